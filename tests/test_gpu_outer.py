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
