"""The learned warm start on a reduced workload: the network is trained on the GPU on solves the
method generates; on held-out images PCG from the energy-scaled network output reaches the
solution that the oracle's dense Cholesky solve of the exact kernel gives, in no more iterations
than from the zero start (plus one for rounding)."""
import numpy as np
import pytest

from gpu_util import rel, torch_gpu

pytestmark = pytest.mark.gpu


def test_warm_start_matches_the_oracle_solution():
    torch = torch_gpu()
    from oracle import kernel as K
    from oracle import solve as OS
    from oracle.features import features_from_image as o_features
    from paper_2407_06834_amd import nld
    from paper_2407_06834_amd import warmstart as WS
    from paper_2407_06834_amd.cnn import WarmStartNet
    WS.set_alpha_rule("strength")
    data = WS.generate(range(20000, 20064), sides=(256, 384))
    assert len(data) == 64
    net = WarmStartNet(n_cond=10, seed=0)
    losses = WS.train(net, data, steps=1500, crop=128)
    assert sum(losses[-100:]) < 0.5 * sum(losses[:100])
    wins = nld.window_table(WS.RHO)
    for seed in (20100, 20101):
        p = WS.draw_problem(seed, side=48, noise=0.1)
        img = torch.tensor(p["f"], dtype=torch.float32, device="cuda")
        fv = img.reshape(-1)
        F = nld.features_from_image(img, WS.RHO)
        plan = nld.Plan(F, wins, p["sigma"], [1.0] * 9, cutoff=4, matvec_tol=1e-5)
        alpha = WS.problem_alpha(p, plan.degree_vector(), 9.0)
        u0 = net.predict(img.reshape(1, 48, 48), np.array([WS.cond_of(p)])).reshape(-1)
        u_w, i_w = plan.pcg_solve(alpha, fv, u0=u0, tol=1e-6, u0_guard="scaled")
        _, i_z = plan.pcg_solve(alpha, fv, u0=torch.full_like(fv, float(fv.mean())), tol=1e-6)
        u_p, i_p = plan.pcg_solve(alpha, fv, tol=1e-6)
        plan.close()
        assert i_w["status"] == i_p["status"] == "OK" and not i_w["u0_rejected"]
        assert i_w["iters"] <= i_z["iters"] + 1, (i_w, i_z)
        W = K.anova_dense(o_features(p["f"], WS.RHO), wins, p["sigma"], [1.0] * 9)
        u_o = OS.dense_solve(K.system_dense(W, alpha), p["f"].reshape(-1))
        # FP32 arithmetic, product to 1e-5: both solves within 1e-4 of the exact solution
        assert rel(u_w.double().cpu().numpy(), u_o) < 1e-4
        assert rel(u_p.double().cpu().numpy(), u_o) < 1e-4
    net.close()
