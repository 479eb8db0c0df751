"""Host logic of the outer loops (paper Sec. 5.5): the change of variables that turns the
adjoint gradient in (log alpha, log sigma_l) into the gradient in (lambda, theta = sigma^-2)."""
import math

import numpy as np

from paper_2407_06834_amd import outer


def test_lambda_theta_chain_rule_against_finite_differences():
    L = 4
    c = np.array([0.7, -0.2, 1.3, 0.4])

    def J_of(alpha, sigmas):
        return (math.log(alpha) - 0.3) ** 2 + float(np.sum(c * (np.log(sigmas) + 1.0) ** 3))

    def grad_of(alpha, sigmas):
        g = np.zeros(1 + 2 * L)
        g[0] = 2.0 * (math.log(alpha) - 0.3)
        g[1:1 + L] = 3.0 * c * (np.log(sigmas) + 1.0) ** 2
        return g

    def F(lam, theta):
        s = outer.sigma_of_theta(theta)
        return J_of(outer.MU / lam, np.full(L, s))

    lam, theta = 3.7, 2.2e-4
    got = outer.lambda_theta_gradient(grad_of(outer.MU / lam, np.full(L, outer.sigma_of_theta(theta))),
                                      lam, theta, L)
    hl, ht = 1e-6 * lam, 1e-6 * theta
    want = np.array([(F(lam + hl, theta) - F(lam - hl, theta)) / (2 * hl),
                     (F(lam, theta + ht) - F(lam, theta - ht)) / (2 * ht)])
    np.testing.assert_allclose(got, want, rtol=1e-7)


def test_units_and_boxes():
    # sigma = 40 on the paper's 0..255 scale is 40/255 on [0, 1]
    assert abs(outer.sigma_of_theta(40.0 ** -2) - 40.0 / 255.0) < 1e-15
    lo, hi = outer.THETA_BOX
    assert abs(outer.sigma_of_theta(lo) - outer.SIGMA_BOX[1]) < 1e-14
    assert abs(outer.sigma_of_theta(hi) - outer.SIGMA_BOX[0]) < 1e-14
    # inside the paper's theta interval [1e-10, 15]
    assert 1e-10 <= lo < hi <= 15.0
