"""Pins of the oracle's solves (paper Sec. 2.4, 4.3, 5.3-5.4): dense Cholesky, the paper's
U-basis deflated Jacobi PCG and its projector form."""
import numpy as np
import pytest

from oracle import kernel as K
from oracle import solve as S
from oracle.features import features_from_image, window_table
from paper_2407_06834_amd.synth import make_image


@pytest.fixture(scope="module")
def prob():
    _, f = make_image(0, 20, 18, 6, 4, 0.1)
    F = features_from_image(f, 1)
    W = K.anova_dense(F, window_table(1), [0.1] * 4, [1.0] * 4)
    return f.reshape(-1), W


def _op(W, alpha):
    A = K.system_dense(W, alpha)
    return A, (lambda v: A @ v)


def test_ubasis_and_projector_iterates_agree(prob):
    f, W = prob
    eta = K.eta_from_degree(K.degree(W), [1.0] * 4)
    A, op = _op(W, 0.5)
    u1, it1, _, h1 = S.pcg_ubasis(op, f, eta, 0.5, 1e-10, 300, record=True)
    u2, it2, _, h2 = S.pcg_projector(op, f, eta, 0.5, 1e-10, 300, record=True)
    assert it1 == it2 and it1 > 3
    for a, b in zip(h1, h2):
        assert np.abs(a - b).max() < 1e-12 * np.abs(f).max()


@pytest.mark.parametrize("alpha", [0.1, 1.0, 10.0])
def test_pcg_matches_cholesky(prob, alpha):
    f, W = prob
    eta = K.eta_from_degree(K.degree(W), [1.0] * 4)
    A, op = _op(W, alpha)
    us = S.dense_solve(A, f)
    u, it, rr, _ = S.pcg_ubasis(op, f, eta, alpha, 1e-12, 500)
    assert rr <= 1e-12
    assert np.linalg.norm(u - us) / np.linalg.norm(us) < 1e-11
    # residual bound: ||A^-1|| <= 1, so ||u - u*|| <= ||r|| <= tol ||f_perp||
    assert np.linalg.norm(u - us) <= 1e-12 * np.linalg.norm(f - f.mean()) * 1.01


def test_maximum_principle_and_mean(prob):
    f, W = prob
    for alpha in (0.01, 1.0, 100.0):
        u = S.dense_solve(K.system_dense(W, alpha), f)
        assert f.min() - 1e-12 <= u.min() and u.max() <= f.max() + 1e-12
        assert abs(u.mean() - f.mean()) < 1e-13


def test_alpha_limits(prob):
    f, W = prob
    u0 = S.dense_solve(K.system_dense(W, 1e-9), f)
    assert np.abs(u0 - f).max() < 1e-5
    uinf = S.dense_solve(K.system_dense(W, 1e9), f)
    assert np.abs(uinf - f.mean()).max() < 1e-4


def test_identical_nodes_closed_form():
    # constant features: W = s 1 1^T, A = I + alpha s (N I - 1 1^T);
    # u = mean(f) 1 + f_perp / (1 + alpha N s), reached in one PCG iteration
    N, s, alpha = 64, 4.0, 0.3
    f = np.random.default_rng(0).standard_normal(N)
    W = s * np.ones((N, N))
    eta = K.eta_from_degree(K.degree(W), [s])
    A = K.system_dense(W, alpha)
    u, it, rr, _ = S.pcg_projector(lambda v: A @ v, f, eta, alpha, 1e-12, 10)
    ref = f.mean() + (f - f.mean()) / (1 + alpha * N * s)
    np.testing.assert_allclose(u, ref, atol=1e-13)
    assert it == 1


def test_constant_image_zero_iterations(prob):
    _, W = prob
    f = np.full(W.shape[0], 0.37)
    eta = K.eta_from_degree(K.degree(W), [1.0] * 4)
    A, op = _op(W, 1.0)
    u, it, _, _ = S.pcg_projector(op, f, eta, 1.0, 1e-10, 50)
    assert it == 0 and np.array_equal(u, f)


def test_deflated_iterations_flat_in_alpha(prob):
    # Sec. 5.4 (comparison of preconditioned iterative methods): once alpha a(L) >> 1,
    # deflated Jacobi PCG keeps a nearly constant iteration count as the regularisation
    # weakens, while plain CG keeps growing
    f, W = prob
    eta = K.eta_from_degree(K.degree(W), [1.0] * 4)
    its_def, its_cg = [], []
    for alpha in (1e2, 1e4, 1e6):
        A, op = _op(W, alpha)
        its_def.append(S.pcg_projector(op, f, eta, alpha, 1e-8, 500)[1])
        its_cg.append(S.cg_plain(op, f, 1e-8, 2000)[1])
    assert max(its_def) - min(its_def) <= 6
    assert its_cg[-1] > 2 * its_def[-1]
