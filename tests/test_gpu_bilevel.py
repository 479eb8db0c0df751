"""GPU tests of the kernel update of a plan and of the bilevel outer loop."""
import numpy as np
import pytest

from gpu_util import rel, torch_gpu
from oracle import kernel as OK
from oracle.features import features_from_image as o_features
from oracle.features import window_table as o_windows
from paper_2407_06834_amd.synth import make_image, random_vector

pytestmark = pytest.mark.gpu


def _setup(torch, nld, n=40, seed=230, dtype=None):
    dtype = dtype or torch.float64
    _, f = make_image(seed, n, n, 4, 3, 0.15)
    img = torch.tensor(f, dtype=dtype, device="cuda")
    F = nld.features_from_image(img, 1)
    return f, img, F, nld.window_table(1)


def test_update_kernel_matches_direct_sum_and_round_trips():
    torch = torch_gpu()
    from paper_2407_06834_amd import nld
    f, img, F, wins = _setup(torch, nld)
    s1, w1 = [0.2, 0.25, 0.2, 0.3], [1.0, 0.5, 1.0, 2.0]
    s2, w2 = [0.22, 0.3, 0.21, 0.3], [0.3, 1.5, 0.0, 1.0]
    plan = nld.Plan(F, wins, s1, w1, bandwidth=64, cutoff=8)
    v = torch.tensor(random_vector(5, F.shape[1]), device="cuda")
    y1 = plan.laplacian_matvec(v).clone()
    assert plan.update_kernel(s2, w2)
    y2 = plan.laplacian_matvec(v).clone()
    Fo = o_features(f, 1)
    W = OK.anova_dense(Fo, o_windows(1), s2, w2)
    ref = OK.laplacian_dense(W) @ v.cpu().numpy()
    assert rel(y2.cpu().numpy(), ref) < 1e-6
    # same tables again: the product is reproduced bit for bit
    assert plan.update_kernel(s1, w1)
    assert torch.equal(plan.laplacian_matvec(v), y1)
    # widths that wrap around the torus at the plan's node scaling are refused and leave the
    # plan as it was
    assert not plan.update_kernel([5.0] * 4, w1)
    assert torch.equal(plan.laplacian_matvec(v), y1)
    plan.close()
    # an autotuned plan refuses a width that needs another bandwidth
    auto = nld.Plan(F, wins, [0.1] * 4, [1.0] * 4, cutoff=8)
    M0 = [auto.window_info(l).bandwidth for l in range(4)]
    assert not auto.update_kernel([0.03] * 4, [1.0] * 4)
    assert [auto.window_info(l).bandwidth for l in range(4)] == M0
    auto.close()


def test_update_kernel_solve_equals_fresh_plan_within_tolerance():
    torch = torch_gpu()
    from paper_2407_06834_amd import nld
    f, img, F, wins = _setup(torch, nld, n=48, seed=231)
    plan = nld.Plan(F, wins, [0.1] * 4, [1.0] * 4, bandwidth=64, cutoff=8)
    # a small change of the widths keeps the plan's node scaling ...
    assert plan.update_kernel([0.103, 0.1, 0.098, 0.102], [1.0, 2.0, 0.5, 1.0])
    u1, i1 = plan.pcg_solve(0.7, img.reshape(-1), tol=1e-11)
    fresh = nld.Plan(F, wins, [0.103, 0.1, 0.098, 0.102], [1.0, 2.0, 0.5, 1.0], bandwidth=64, cutoff=8)
    u2, i2 = fresh.pcg_solve(0.7, img.reshape(-1), tol=1e-11)
    assert i1["status"] == "OK" and i2["status"] == "OK"
    assert rel(u1.cpu().numpy(), u2.cpu().numpy()) < 1e-7
    # ... while a large one at this bandwidth asks for a new plan
    assert not plan.update_kernel([0.13] * 4, [1.0] * 4)
    plan.close()
    fresh.close()


def test_projected_gradient_descent_decreases_loss_inside_box():
    torch = torch_gpu()
    from paper_2407_06834_amd import bilevel
    pairs = bilevel.training_set(2, 48, seed0=240)
    prob = bilevel.BilevelProblem(pairs, tol=1e-6)
    L = prob.L
    theta0 = np.concatenate([[0.0], np.log(np.full(L, 0.1)), np.ones(L)])
    J0 = prob.loss(theta0)
    theta, hist = bilevel.projected_gradient_descent(prob, theta0, steps=4)
    Js = [J0] + [h["J"] for h in hist if h["accepted"]]
    assert len(Js) >= 3
    assert all(b <= a for a, b in zip(Js, Js[1:]))
    assert Js[-1] < 0.99 * J0
    assert np.array_equal(theta, bilevel.project(theta, L))
    # the loss of the clean image pair set is below that of the noisy input
    noisy = np.mean([np.sum((f - uc) ** 2) for f, uc in pairs])
    assert Js[-1] < noisy
    prob.close()
