"""The paper's outer loops (Sec. 5.5) on a tiny training set: the adjoint gradient in
(lambda, theta) against central differences of GPU solves, Brent against a grid, and
L-BFGS-B with either gradient lowering the loss."""
import math

import numpy as np
import pytest

from gpu_util import torch_gpu

pytestmark = pytest.mark.gpu


def _problem(**kw):
    torch_gpu()
    from paper_2407_06834_amd import outer
    from paper_2407_06834_amd.bilevel import training_set
    pairs = training_set(2, 40, noise=0.15, seed0=77)
    return outer, outer.OuterProblem(pairs, rho=2, **kw)


def test_adjoint_gradient_matches_central_differences():
    outer, prob = _problem(tol=1e-13, maxit=400, matvec_tol=1e-11)
    lam, theta = 0.5, 30.0 ** -2
    J, g = prob.loss_and_grad(lam, theta)
    hl, ht = 1e-4 * lam, 1e-4 * theta
    fd = np.array([(prob.loss(lam + hl, theta) - prob.loss(lam - hl, theta)) / (2 * hl),
                   (prob.loss(lam, theta + ht) - prob.loss(lam, theta - ht)) / (2 * ht)])
    prob.close()
    assert J > 0
    np.testing.assert_allclose(g, fd, rtol=2e-4)


def test_brent_beats_grid():
    outer, prob = _problem()
    r = outer.brent(prob, sigma255=40.0, xatol=1e-6)
    grid = [prob.loss(lam, 40.0 ** -2) for lam in np.logspace(-9, 1, 11)]
    prob.close()
    assert outer.BRENT_BOX[0] <= r["lam"] <= outer.BRENT_BOX[1]
    assert r["J"] <= min(grid) * (1 + 1e-9)


@pytest.mark.parametrize("adjoint", [True, False])
def test_lbfgsb_lowers_the_loss(adjoint):
    outer, prob = _problem()
    x0 = (1.0, 40.0 ** -2)
    J0 = prob.loss(*x0)
    r = outer.lbfgsb(prob, x0, adjoint=adjoint, maxiter=15)
    prob.close()
    assert r["J"] < J0
    assert outer.LAMBDA_BOX[0] <= r["lam"] <= outer.LAMBDA_BOX[1]
    assert outer.THETA_BOX[0] <= r["theta"] <= outer.THETA_BOX[1]


class _OracleOuter:
    """The outer problem of the paper's Sec. 5.5 on the oracle alone: MIS windows from the
    oracle ranking, weights 1/L, exact kernel, dense Cholesky solves; J = mean ||u - u_c||^2."""

    def __init__(self, pairs, rho, mu=1e-2):
        from oracle import mis as OM
        from oracle.features import features_from_image
        self.mu = mu
        self.items = []
        for f, uc in pairs:
            F = features_from_image(f, rho, with_pos=False)
            wins = OM.mis_windows(OM.mis_scores(F, f.reshape(-1)))
            self.items.append((F, wins, f.reshape(-1), uc.reshape(-1)))

    def loss(self, lam, theta):
        from oracle import gradient as OG
        sigma = 1.0 / (255.0 * math.sqrt(theta))
        J = 0.0
        for F, wins, f, uc in self.items:
            L = len(wins)
            u, _ = OG.solve_state(F, wins, [sigma] * L, [1.0 / L] * L, self.mu / lam, f)
            J += float(np.sum((u - uc) ** 2))
        return J / len(self.items)


def _pair_problems():
    torch_gpu()
    from paper_2407_06834_amd import outer
    from paper_2407_06834_amd.bilevel import training_set
    pairs = training_set(2, 20, noise=0.15, seed0=91)
    hip = outer.OuterProblem(pairs, rho=3, tol=1e-13, maxit=400, matvec_tol=1e-11)
    return outer, pairs, hip, _OracleOuter(pairs, rho=3)


def test_outer_objective_and_optima_match_the_oracle():
    """7 x 7 patches in MIS windows (L = 17) on two 20 x 20 crops: the loss of the library's
    solves equals the oracle's exact-kernel loss, and Brent's lambda and L-BFGS-B's (lambda,
    theta) (two-point differences, as in the paper) land on the oracle's optima."""
    outer, pairs, hip, orc = _pair_problems()
    # the GPU ranking cuts the same windows as the oracle's
    assert [list(map(list, w)) for w in hip.wins] == [list(map(list, it[1])) for it in orc.items]
    for lam, s255 in ((1.0, 40.0), (0.05, 25.0), (3.0, 60.0)):
        a, b = hip.loss(lam, s255 ** -2), orc.loss(lam, s255 ** -2)
        assert abs(a - b) <= 1e-7 * b, (lam, s255, a, b)
    rb_h = outer.brent(hip, sigma255=40.0, xatol=1e-7)
    rb_o = outer.brent(orc, sigma255=40.0, xatol=1e-7)
    assert abs(math.log(rb_h["lam"]) - math.log(rb_o["lam"])) < 1e-3, (rb_h, rb_o)
    assert abs(rb_h["J"] - rb_o["J"]) <= 1e-7 * rb_o["J"]
    x0 = (rb_o["lam"], 40.0 ** -2)
    rl_h = outer.lbfgsb(hip, x0, adjoint=False, maxiter=20)
    rl_o = outer.lbfgsb(orc, x0, adjoint=False, maxiter=20)
    hip.close()
    assert abs(rl_h["J"] - rl_o["J"]) <= 1e-6 * rl_o["J"], (rl_h, rl_o)
    assert abs(math.log(rl_h["lam"]) - math.log(rl_o["lam"])) < 1e-2, (rl_h, rl_o)
    assert abs(math.log(rl_h["theta"]) - math.log(rl_o["theta"])) < 1e-2, (rl_h, rl_o)
