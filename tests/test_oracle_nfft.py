"""Pins of the oracle's NFFT fast Gauss summation (paper Sec. 3).

Independent references: brute-force stage definitions on tiny inputs, the exact NDFT,
the Poisson-summation identity, numerical quadrature of the window's Fourier transform,
the directly summed (periodised) Gaussian, and closed-form limits."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import kernel as K
from oracle import nfft
from oracle.features import features_from_image, window_table
from paper_2407_06834_amd.synth import make_image


def test_poisson_summation_coefficients():
    st = 0.07
    x = np.linspace(-0.5, 0.5, 23)
    k = np.arange(-200, 201)
    series = (nfft.gauss_fourier(k, st)[None, :] * np.exp(2j * np.pi * np.outer(x, k))).sum(1).real
    direct = sum(np.exp(-((x + p) / st) ** 2) for p in range(-5, 6))
    np.testing.assert_allclose(series, direct, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("n,M,m", [(64, 32, 4), (128, 64, 6), (64, 48, 5)])
def test_window_fourier_pair_by_quadrature(n, M, m):
    b = nfft.kb_shape(n, M)
    for k in (0, 3, M // 2 - 1):
        re = quad(lambda d: nfft.kb_window(np.array([d]), m, b)[0] * math.cos(2 * math.pi * k * d / n),
                  -m, m, limit=200, epsabs=1e-14, epsrel=1e-13)[0]
        phi = nfft.kb_fourier(np.array([k]), n, m, b)[0]
        assert abs(re - phi) <= 5 * math.exp(-b * m) * phi + 1e-13


def test_window_central_tap_is_one_and_edge_limit():
    b = nfft.kb_shape(128, 64)
    assert abs(nfft.kb_window(np.array([0.0]), 6, b)[0] - 1.0) < 1e-15
    edge = nfft.kb_window(np.array([6.0, 6.0 - 1e-9]), 6, b)
    assert abs(edge[0] - edge[1]) < 1e-6 * edge[0]


def _brute_spread(u, v, n, m, b):
    t, N = u.shape
    g = np.zeros((n,) * t)
    for idx in np.ndindex(*g.shape):
        acc = 0.0
        for j in range(N):
            w = v[j]
            for d in range(t):
                dist = u[d, j] - idx[d]
                dist = dist - n * np.round(dist / n)       # periodic distance
                if dist < -m or dist >= m:
                    w = 0.0
                    break
                w *= nfft.kb_window(np.array([dist]), m, b)[0]
            acc += w
        g[idx] = acc
    return g


def test_spread_and_gather_against_brute_force():
    rng = np.random.default_rng(0)
    n, M, m, t, N = 12, 6, 2, 2, 7
    b = nfft.kb_shape(n, M)
    u = rng.uniform(0, n, size=(t, N))
    v = rng.standard_normal(N)
    g = nfft.spread(u, v, n, m, b)
    np.testing.assert_allclose(g, _brute_spread(u, v, n, m, b), atol=1e-14)
    # gather is the transpose of spread: <gather(h), v> = <h, spread(v)>
    h = rng.standard_normal((n, n))
    lhs = nfft.gather(h, u, m, b) @ v
    rhs = (h * g).sum()
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


def test_convolve_is_circulant_product():
    rng = np.random.default_rng(1)
    n = 10
    g = rng.standard_normal((n, n))
    mults = [rng.uniform(0, 1, n), rng.uniform(0, 1, n)]
    for c in mults:                        # real even spectra
        c[1:] = 0.5 * (c[1:] + c[1:][::-1])
    k = nfft.fft_frequencies(n)
    C = [np.array([[np.sum(mult * np.exp(2j * np.pi * k * (a - bb) / n)).real
                    for bb in range(n)] for a in range(n)]) for mult in mults]
    ref = C[0] @ g @ C[1].T
    np.testing.assert_allclose(nfft.convolve(g, mults), ref, atol=1e-12)


@pytest.mark.parametrize("m", [2, 4, 6])
def test_adjoint_nfft_matches_ndft(m):
    rng = np.random.default_rng(2)
    n, M, t, N = 32, 16, 2, 50
    b = nfft.kb_shape(n, M)
    xt = rng.uniform(-0.45, 0.45, size=(t, N))
    v = rng.standard_normal(N)
    g = nfft.spread(nfft.grid_coords(xt, n), v, n, m, b)
    G = np.fft.fftn(g)
    k = np.arange(-M // 2, M // 2)
    idx = np.mod(k, n)
    Phi = nfft.kb_fourier(k, n, m, b)
    approx = G[np.ix_(idx, idx)] / np.outer(Phi, Phi) * np.outer((-1.0) ** k, (-1.0) ** k)
    exact = nfft.ndft_adjoint(xt, v, M)
    err = np.abs(approx - exact).max() / np.abs(exact).max()
    assert err < {2: 1e-3, 4: 1e-6, 6: 1e-9}[m]


def _window_setup(t, N, seed=3):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 1, size=(t, N))
    return X, rng.standard_normal(N)


@pytest.mark.parametrize("t", [1, 2, 3])
def test_fast_sum_chain(t):
    X, v = _window_setup(t, 300)
    sigma, M, n, m = 0.15, 32, 64, 6
    kept, c, s, st = nfft.torus_scaling(X, sigma, M)
    xt = np.stack([(X[d] - cc) * ss for d, cc, ss in zip(kept, c, s)])
    y_nfft = nfft.fast_gauss_window(X, v, sigma, M, n, m)
    y_trunc = nfft.truncated_fourier_sum(xt, v, st, M)
    y_per = nfft.periodic_gauss_sum(xt, v, st)
    y_dir = K.window_kernel_dense(X, list(range(t)), sigma) @ v
    nrm = np.linalg.norm(y_dir)
    assert np.linalg.norm(y_nfft - y_trunc) / nrm < 1e-10      # window (m) error only
    a = nfft.compression(sigma, 1.0, M)
    sti = sigma * 2 * a
    trunc_bound = math.erfc(math.pi * sti * (M / 2 - 1)) * 300 * t
    assert np.linalg.norm(y_trunc - y_per) / nrm < max(trunc_bound, 1e-13)
    wrap_bound = 2 * math.exp(-((1 - 2 * a) / sti) ** 2) * 300 * t
    assert np.linalg.norm(y_per - y_dir) / nrm < max(wrap_bound, 1e-13)


def test_compression_balances_errors():
    for sigma, R, M in [(0.1, 2.0, 64), (0.05, 2.0, 128), (0.2, 1.0, 32)]:
        a = nfft.compression(sigma, R, M)
        assert 0 < a < 0.5
        st = 2 * a * sigma / R
        assert abs((1 - 2 * a) ** 2 / st ** 2 - (math.pi * st * M / 2) ** 2) < 1e-9 * (
            (1 - 2 * a) ** 2 / st ** 2)


def test_anova_nfft_matches_direct_sum_config1_image():
    _, f = make_image(0, 20, 20, 6, 4, 0.1)
    F = features_from_image(f, 1)
    wins = window_table(1)
    v = np.random.default_rng(7).standard_normal(F.shape[1])
    y = nfft.anova_matvec_nfft(F, wins, [0.1] * 4, [1.0] * 4, v, 64, 128, 6)
    yd = K.anova_matvec_direct(F, wins, [0.1] * 4, [1.0] * 4, v)
    assert np.linalg.norm(y - yd) / np.linalg.norm(yd) < 1e-9
    # M = 32 (the configuration's stated bandwidth) is visibly less accurate
    y32 = nfft.anova_matvec_nfft(F, wins, [0.1] * 4, [1.0] * 4, v, 32, 64, 6)
    assert np.linalg.norm(y32 - yd) / np.linalg.norm(yd) > 1e-7


def test_operator_symmetric_psd():
    X, _ = _window_setup(2, 40, seed=9)
    N = X.shape[1]
    Wt = np.stack([nfft.fast_gauss_window(X, e, 0.2, 16, 32, 4) for e in np.eye(N)], axis=1)
    assert np.abs(Wt - Wt.T).max() < 1e-13 * np.abs(Wt).max()
    assert np.linalg.eigvalsh(0.5 * (Wt + Wt.T))[0] > -1e-12 * np.abs(Wt).max()


def test_wide_kernel_limit():
    X, v = _window_setup(3, 200, seed=11)
    sigma = 100.0
    y = nfft.fast_gauss_window(X, v, sigma, 16, 32, 6)
    yd = K.window_kernel_dense(X, [0, 1, 2], sigma) @ v
    assert np.linalg.norm(y - yd) / np.linalg.norm(yd) < 1e-10
    assert np.abs(y - v.sum()).max() < 3 * 3 / sigma ** 2 * np.abs(v).sum()


def test_identical_nodes_exact():
    X = np.full((3, 25), 0.4)
    v = np.random.default_rng(1).standard_normal(25)
    np.testing.assert_array_equal(nfft.fast_gauss_window(X, v, 0.1, 32, 64, 4),
                                  np.full(25, v.sum()))


def test_dropped_constant_dimension():
    X, v = _window_setup(2, 100, seed=12)
    X3 = np.vstack([X, np.full((1, 100), 0.7)])
    y2 = nfft.fast_gauss_window(X, v, 0.2, 32, 64, 6)
    y3 = nfft.fast_gauss_window(X3, v, 0.2, 32, 64, 6)
    np.testing.assert_array_equal(y2, y3)


def test_sigma_derivative_summation_against_dense():
    from oracle.gradient import sigma_derivative_kernel
    for t in (1, 2, 3):
        X, v = _window_setup(t, 250, seed=20 + t)
        F = X
        y = nfft.fast_sigma_derivative_window(X, v, 0.15, 48, 96, 6)
        yd = sigma_derivative_kernel(F, list(range(t)), 0.15) @ v
        assert np.linalg.norm(y - yd) / np.linalg.norm(yd) < 1e-7


def test_dense_window_matrix_equals_fast_summation_and_is_psd():
    # the dense form B C B^T (entrywise product of per-dimension factors) is the same linear
    # map as the staged summation, symmetric and positive semidefinite, and within the
    # truncation error of the exact Gaussian kernel
    rng = np.random.default_rng(21)
    X = rng.uniform(0.0, 1.0, (3, 150))
    X[2] = 0.37                              # a dropped (constant) dimension
    sigma, M, n, m = 0.15, 32, 64, 6
    Wt = nfft.window_matrix_nfft(X, sigma, M, n, m)
    v = rng.standard_normal(150)
    np.testing.assert_allclose(Wt @ v, nfft.fast_gauss_window(X, v, sigma, M, n, m), atol=1e-11)
    np.testing.assert_allclose(Wt, Wt.T, atol=1e-13)
    assert np.linalg.eigvalsh(Wt).min() > -1e-10 * np.abs(Wt).max()
    Kx = K.window_kernel_dense(X, [0, 1, 2], sigma)
    assert np.abs(Wt - Kx).max() < 1e-5
