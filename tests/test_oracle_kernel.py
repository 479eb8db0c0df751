"""Pins of the oracle's dense kernel, Laplacian and system (paper Sec. 2.6, 4.2, 4.3).

Each check is a fact the paper (or plain linear algebra) fixes independently of the code:
Laplacian structure, spectral bounds, the Helmert change of basis and its block form."""
import numpy as np
import pytest

from oracle import kernel as K
from oracle import solve as S
from oracle.features import features_from_image, window_table
from paper_2407_06834_amd.synth import make_image


@pytest.fixture(scope="module")
def small():
    _, f = make_image(3, 14, 13, 4, 3, 0.1)
    F = features_from_image(f, 1)
    wins = window_table(1)
    sig = [0.1, 0.15, 0.2, 0.12]
    wts = [1.0, 0.5, 2.0, 1.5]
    W = K.anova_dense(F, wins, sig, wts)
    return f.reshape(-1), F, wins, sig, wts, W


def test_kernel_entry_formula(small):
    _, F, wins, sig, wts, W = small
    i, j = 7, 101
    ref = 0.0
    for win, s, w in zip(wins, sig, wts):
        q = sum((F[d, i] - F[d, j]) ** 2 for d in win)
        ref += w * np.exp(-q / s ** 2)
    assert abs(W[i, j] - ref) < 1e-15
    assert np.allclose(np.diag(W), sum(wts))          # self term sum_l w_l


def test_identical_features_give_rank_one_kernel():
    F = np.ones((5, 40)) * 0.3
    W = K.anova_dense(F, [[0, 1, 2], [3, 4]], [0.1, 0.2], [1.0, 2.0])
    np.testing.assert_array_equal(W, 3.0 * np.ones((40, 40)))


def test_laplacian_structure(small):
    _, _, _, _, wts, W = small
    L = K.laplacian_dense(W)
    assert np.allclose(L, L.T, atol=0)
    assert np.abs(L @ np.ones(L.shape[0])).max() < 1e-12
    ev = np.linalg.eigvalsh(L)
    assert ev[0] > -1e-10 * ev[-1]                     # PSD
    assert ev[1] > 1e-8                                # connected: simple zero eigenvalue
    off = L - np.diag(np.diag(L))
    assert (off <= 0).all()                            # M-matrix sign pattern
    # diagonal of L equals eta = D - sum w (zero-diagonal degree)
    eta = K.eta_from_degree(K.degree(W), wts)
    np.testing.assert_allclose(np.diag(L), eta, rtol=1e-13)


def test_system_spd_with_unit_eigenpair(small):
    _, _, _, _, _, W = small
    A = K.system_dense(W, 0.7)
    one = np.ones(A.shape[0])
    np.testing.assert_allclose(A @ one, one, atol=1e-12)
    assert np.linalg.eigvalsh(A)[0] > 1 - 1e-10


@pytest.mark.parametrize("alpha", [0.05, 1.0, 30.0])
def test_spectral_bounds(small, alpha):
    _, _, _, _, wts, W = small
    N = W.shape[0]
    L = K.laplacian_dense(W)
    eta = K.eta_from_degree(K.degree(W), wts)
    evL = np.linalg.eigvalsh(L)
    rho, aL = evL[-1], evL[1]
    # Sec. 4.2 general spectral bounds: max eta <= rho(L) < 2 max eta
    assert eta.max() <= rho * (1 + 1e-12) and rho < 2 * eta.max()
    # condition number of A = I + alpha L in 1 + alpha max eta [1, 2)
    A = np.eye(N) + alpha * L
    evA = np.linalg.eigvalsh(A)
    kappa = evA[-1] / evA[0]
    assert 1 + alpha * eta.max() * (1 - 1e-12) <= kappa < 1 + 2 * alpha * eta.max()
    # upper bound on algebraic connectivity: a(L) <= N/(N-1) min eta
    assert aL <= N / (N - 1) * eta.min() * (1 + 1e-12)
    # lower bound through any vertex (vertex 0): a(A) >= alpha min_{j != 0} W_j0 + 1
    assert evA[1] >= alpha * W[1:, 0].min() + 1 - 1e-10
    # Jacobi preconditioned spectrum (Sec. 4.3.1)
    P = 1 + alpha * eta
    Ps = 1 / np.sqrt(P)
    evPA = np.linalg.eigvalsh(Ps[:, None] * A * Ps[None, :])
    assert evPA[0] >= 1 / (1 + alpha * eta.max()) * (1 - 1e-12)
    assert evPA[-1] <= min(2.0, N / (N - 1) * rho / aL) * (1 + 1e-12)
    # deflated block pi_2(U^T P^-1 U) pi_2(U^T A U) (Sec. 4.3.2)
    U = S.helmert_dense(N)
    B2 = (U.T @ A @ U)[1:, 1:]
    M2 = (U.T @ np.diag(1 / P) @ U)[1:, 1:]
    ev_def = np.sort(np.linalg.eigvals(M2 @ B2).real)
    assert ev_def[0] > 0
    assert ev_def[0] >= evPA[1] - 1 / (1 + alpha * eta.min()) - 1e-10
    assert ev_def[-1] <= evPA[-1] * (1 + 1e-10)


def test_complete_graph_limit():
    # Sec. 4.3.3: sigma -> infinity gives the complete graph; spectra {1, 1 + alpha N sum w}
    # and, Jacobi preconditioned, {1/(1+alpha(N-1)s), (1+alpha N s)/(1+alpha(N-1)s)}
    N, s, alpha = 30, 3.0, 0.4
    W = s * np.ones((N, N))
    A = K.system_dense(W, alpha)
    ev = np.linalg.eigvalsh(A)
    assert abs(ev[0] - 1) < 1e-12 and np.allclose(ev[1:], 1 + alpha * N * s)
    eta = K.eta_from_degree(K.degree(W), [s])
    P = 1 + alpha * eta
    evp = np.sort(np.linalg.eigvals(np.diag(1 / P) @ A).real)
    np.testing.assert_allclose(evp[0], 1 / (1 + alpha * (N - 1) * s), rtol=1e-12)
    np.testing.assert_allclose(evp[1:], (1 + alpha * N * s) / (1 + alpha * (N - 1) * s),
                               rtol=1e-12)
    # the upper bound on a(L) is attained: a(L) = N/(N-1) min eta
    evL = np.linalg.eigvalsh(K.laplacian_dense(W))
    np.testing.assert_allclose(evL[1], N / (N - 1) * eta.min(), rtol=1e-12)


def test_row_sampled_direct_sum_equals_dense(small):
    fv, F, wins, sig, wts, W = small
    v = np.random.default_rng(5).standard_normal(W.shape[0])
    rows = np.array([0, 5, 77, W.shape[0] - 1])
    np.testing.assert_allclose(K.anova_rows_direct(F, wins, sig, wts, rows, v), (W @ v)[rows],
                               rtol=1e-13)


def test_c_direct_sum_equals_dense(small):
    from oracle import csum
    fv, F, wins, sig, wts, W = small
    v = np.random.default_rng(6).standard_normal(W.shape[0])
    rows = np.arange(W.shape[0])
    np.testing.assert_allclose(csum.anova_rows(F, wins, sig, wts, v, rows), W @ v, rtol=1e-12)
