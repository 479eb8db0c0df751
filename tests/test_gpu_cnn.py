"""GPU parity of the warm-start network kernels (BF16 matrix cores) with the FP64 oracle."""
import numpy as np
import pytest

from gpu_util import torch_gpu
from oracle import cnn as OC

pytestmark = pytest.mark.gpu


def _setup(torch, n=2, h=13, w=37, n_cond=2, seed=0):
    rng = np.random.default_rng(seed)
    cin = 1 + n_cond
    theta = np.zeros(OC.param_count(cin))
    o = 0
    for co, ci in OC.layer_shapes(cin):
        k = co * ci * 9
        theta[o:o + k] = rng.standard_normal(k) * np.sqrt(2.0 / (9 * ci))
        o += k
        theta[o:o + co] = 0.05 * rng.standard_normal(co)
        o += co
    theta = theta.astype(np.float32).astype(np.float64)     # exactly what the GPU holds
    f = rng.uniform(0, 1, (n, h, w))
    cond = rng.uniform(-2, 1, (n, n_cond))
    tgt = f + 0.1 * rng.standard_normal((n, h, w))
    return theta, f, cond, tgt


def _net(torch, theta, n_cond):
    from paper_2407_06834_amd.cnn import WarmStartNet
    net = WarmStartNet(n_cond, seed=1)
    net.set_params(theta)
    return net


@pytest.mark.parametrize("shape", [(2, 13, 37), (1, 8, 32), (3, 40, 70)])
def test_forward_matches_oracle(shape):
    torch = torch_gpu()
    theta, f, cond, _ = _setup(torch, *shape)
    net = _net(torch, theta, 2)
    ft = torch.tensor(f, dtype=torch.float32, device="cuda")
    u0 = net.predict(ft, cond).cpu().numpy().astype(np.float64)
    for b in range(shape[0]):
        ref, _ = OC.forward(theta, f[b], cond[b])
        res_g, res_r = u0[b] - f[b], ref - f[b]
        # BF16 activations and weights, FP32 accumulation
        assert np.linalg.norm(res_g - res_r) <= 2e-2 * np.linalg.norm(res_r)
    net.close()


def test_gradient_and_loss_match_oracle():
    torch = torch_gpu()
    theta, f, cond, tgt = _setup(torch, 2, 24, 40, seed=3)
    net = _net(torch, theta, 2)
    ft = torch.tensor(f, dtype=torch.float32, device="cuda")
    tt = torch.tensor(tgt, dtype=torch.float32, device="cuda")
    loss = net.loss_grad(ft, cond, tt)
    g = net.grad().astype(np.float64)
    loss_r, g_r = OC.loss_and_grad(theta, [(f[b], cond[b], tgt[b]) for b in range(2)])
    assert abs(loss - loss_r) <= 2e-2 * loss_r
    o = 0
    for co, ci in OC.layer_shapes(3):
        k = co * ci * 9 + co
        gl, rl = g[o:o + k], g_r[o:o + k]
        assert np.linalg.norm(gl - rl) <= 5e-2 * np.linalg.norm(rl), (co, ci)
        assert float(gl @ rl) / (np.linalg.norm(gl) * np.linalg.norm(rl)) > 0.998
        o += k
    net.close()


def test_adam_step_matches_oracle_and_training_lowers_the_loss():
    torch = torch_gpu()
    theta, f, cond, tgt = _setup(torch, 2, 16, 32, seed=4)
    net = _net(torch, theta, 2)
    ft = torch.tensor(f, dtype=torch.float32, device="cuda")
    tt = torch.tensor(tgt, dtype=torch.float32, device="cuda")
    l0 = net.loss_grad(ft, cond, tt)
    g = net.grad().astype(np.float64)
    net.adam_step(lr=1e-3)
    th1 = net.params().astype(np.float64)
    ref, _, _ = OC.adam_step(theta, g, np.zeros_like(g), np.zeros_like(g), 1, lr=1e-3)
    assert np.max(np.abs(th1 - ref)) < 1e-6
    losses = [l0]
    for _ in range(30):
        losses.append(net.loss_grad(ft, cond, tt))
        net.adam_step(lr=3e-3)
    assert losses[-1] < 0.7 * losses[0]
    net.close()


def test_rejects_bad_arguments():
    torch = torch_gpu()
    from paper_2407_06834_amd import nld
    from paper_2407_06834_amd.cnn import WarmStartNet
    net = WarmStartNet(2)
    with pytest.raises(nld.NldError):
        net.set_params(np.full(net.count, np.nan, dtype=np.float32))
    with pytest.raises(nld.NldError):
        net.adam_step(lr=-1.0)
    net.close()
