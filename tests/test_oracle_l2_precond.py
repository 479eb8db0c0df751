"""Pins of the l2 diagonal preconditioners P_b and P_b' of Sec. 4.3.1 (oracle, FP64)."""
import numpy as np

from oracle import kernel as K
from oracle import solve as S
from oracle.features import features_from_image, window_table
from paper_2407_06834_amd.synth import make_image


def _setup(n=14, seed=3, alpha=2.0):
    _, f = make_image(seed, n, n, 3, 2, 0.1)
    F = features_from_image(f, 1)
    wins = window_table(1)
    sig = [0.3, 0.25, 0.4, 0.35]
    wts = [1.0, 0.5, 2.0, 1.5]
    W = K.anova_dense(F, wins, sig, wts)
    D = K.degree(W)
    eta = K.eta_from_degree(D, wts)
    A = K.system_dense(W, alpha)
    return F, f.reshape(-1), wins, sig, wts, eta, A, alpha


def test_squared_gaussian_is_the_gaussian_of_width_sigma_over_sqrt2():
    F, _, wins, sig, wts, *_ = _setup()
    for win, s in zip(wins, sig):
        Ks = K.window_kernel_dense(F, win, s)
        assert np.allclose(Ks * Ks, K.window_kernel_dense(F, win, s / np.sqrt(2.0)), atol=1e-15)


def test_diagonal_ordering_pa_le_pbprime_le_pb_le_sqrt2_pa():
    F, f, wins, sig, wts, eta, A, alpha = _setup()
    pa = K.precond_jacobi(eta, alpha)
    d2 = K.l2_window_degree(F, wins, sig, wts)
    pbp = K.precond_l2_anova(eta, d2, alpha)
    pb = K.precond_l2_full(A)
    assert np.all(pa <= pbp + 1e-12)
    assert np.all(pbp <= pb + 1e-12)
    assert np.all(pb <= np.sqrt(2.0) * pa + 1e-12)
    # with one window the dropped cross terms vanish: P_b' = P_b
    W1 = K.anova_dense(F, wins[:1], sig[:1], wts[:1])
    A1 = K.system_dense(W1, alpha)
    eta1 = K.eta_from_degree(K.degree(W1), wts[:1])
    d21 = K.l2_window_degree(F, wins[:1], sig[:1], wts[:1])
    assert np.allclose(K.precond_l2_anova(eta1, d21, alpha), K.precond_l2_full(A1), rtol=1e-13)


def test_spectrum_of_l2_preconditioned_system_within_the_lemma_bounds():
    F, f, wins, sig, wts, eta, A, alpha = _setup()
    pa = K.precond_jacobi(eta, alpha)
    pbp = K.precond_l2_anova(eta, K.l2_window_degree(F, wins, sig, wts), alpha)
    ea = np.linalg.eigvalsh(A / np.sqrt(np.outer(pa, pa)))
    eb = np.linalg.eigvalsh(A / np.sqrt(np.outer(pbp, pbp)))
    assert eb.min() >= 2 ** -0.5 * ea.min() - 1e-12
    assert eb.max() <= ea.max() + 1e-12


def test_l2_preconditioned_cg_reaches_the_solution_with_and_without_deflation():
    F, f, wins, sig, wts, eta, A, alpha = _setup()
    ref = S.dense_solve(A, f)
    pbp = K.precond_l2_anova(eta, K.l2_window_degree(F, wins, sig, wts), alpha)
    apply_A = lambda v: A @ v
    u1, it1, _, _ = S.pcg_projector(apply_A, f, eta, alpha, 1e-12, 500, P=pbp)
    u2, it2, _ = S.pcg_jacobi(apply_A, f, eta, alpha, 1e-12, 500, P=pbp)
    assert np.linalg.norm(u1 - ref) <= 1e-10 * np.linalg.norm(ref)
    assert np.linalg.norm(u2 - ref) <= 1e-10 * np.linalg.norm(ref)
    assert it1 > 0 and it2 > 0
