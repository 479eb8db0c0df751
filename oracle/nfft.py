"""NFFT-based fast Gauss summation, one window at a time (paper Sec. 3), FP64.

The paper evaluates each subkernel product K_l v with the fast Gauss transform: an adjoint
NFFT of v, a multiplication by Fourier coefficients of a periodic approximation of the
Gaussian, and an NFFT back to the nodes (Sec. 3, discrete Gauss transform and its NFFT
based fast summation).  The paper defers the parameters to the NFFT literature; the
readings used here are:

  torus scaling   per feature dimension: range R = max - min (dimensions with R = 0 are
                  dropped: their kernel factor is exactly 1), centre c = (max + min)/2,
                  compression a = (sqrt(1 + q) - 1)/q with q = 2 pi M sigma^2 / R^2, which
                  balances the wrap-around error exp(-(1-2a)^2/st^2) against the band
                  truncation error exp(-pi^2 st^2 (M/2)^2); scale s = 2a/R, scaled nodes
                  xt = (x - c) s in [-a, a], scaled width st = sigma s.
  coefficients    Poisson summation: the 1-periodisation of exp(-x^2/st^2) has Fourier
                  coefficients bhat_k = sqrt(pi) st exp(-pi^2 st^2 k^2); the band is the
                  symmetric set |k| <= M/2 - 1 (k = -M/2 is dropped so that the operator
                  stays real symmetric).
  window          Kaiser-Bessel pair with shape b = pi (2 - 1/sigma_os), sigma_os = n/M:
                  phi(x) = sinh(b sqrt(m^2 - n^2 x^2)) / (pi sqrt(m^2 - n^2 x^2)) on |x| <= m/n,
                  phihat(k) = I0(m sqrt(b^2 - (2 pi k/n)^2)) / n.  The spreading weights are
                  phi scaled by pi m / sinh(b m) so that the central tap is 1; the scale is
                  undone in the Fourier multiplier.
  grid            n points per dimension; node xt sits at grid coordinate u = n xt + n/2;
                  taps are the 2m cells c = floor(u) - m + 1 ... floor(u) + m (mod n).

With these choices the approximation is W~ = B C B^T, B the spreading matrix and C a real
symmetric circulant with nonnegative spectrum, so W~ is symmetric positive semidefinite.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy.special import i0e


# ----------------------------------------------------------------------------- parameters

def compression(sigma: float, R: float, M: int) -> float:
    """Torus compression a in (0, 1/2) balancing wrap-around against truncation."""
    q = 2.0 * math.pi * M * sigma * sigma / (R * R)
    return (math.sqrt(1.0 + q) - 1.0) / q


def torus_scaling(X: np.ndarray, sigma: float, M: int):
    """Per-dimension scaling of the window's nodes X (t, N) into [-a, a].

    Returns (kept_dims, centres, scales, sigma_tilde) for the dimensions with R > 0."""
    kept, centres, scales, st = [], [], [], []
    for d in range(X.shape[0]):
        lo = float(X[d].min())
        hi = float(X[d].max())
        R = hi - lo
        if R == 0.0:
            continue
        a = compression(sigma, R, M)
        s = 2.0 * a / R
        kept.append(d)
        centres.append(0.5 * (lo + hi))
        scales.append(s)
        st.append(sigma * s)
    return kept, centres, scales, st


def kb_shape(n: int, M: int) -> float:
    return math.pi * (2.0 - M / n)


def kb_window(delta: np.ndarray, m: int, b: float) -> np.ndarray:
    """Spreading weight psi(delta) = m sinh(b z) / (z sinh(b m)), z = sqrt(m^2 - delta^2).

    delta is the distance in grid cells, |delta| <= m.  Evaluated in the overflow-free form
    (m/z) exp(b (z - m)) (1 - exp(-2 b z)) / (1 - exp(-2 b m)), with limit 2 b m exp(-b m) /
    (1 - exp(-2 b m)) at z = 0."""
    delta = np.asarray(delta, dtype=np.float64)
    z = np.sqrt(np.maximum(m * m - delta * delta, 0.0))
    den = -math.expm1(-2.0 * b * m)
    out = np.empty_like(z)
    pos = z > 0
    zp = z[pos]
    out[pos] = (m / zp) * np.exp(b * (zp - m)) * (-np.expm1(-2.0 * b * zp)) / den
    out[~pos] = 2.0 * b * m * math.exp(-b * m) / den
    return out


def kb_fourier(k: np.ndarray, n: int, m: int, b: float) -> np.ndarray:
    """Phi_k = (pi m / sinh(b m)) * n * phihat(k) = pi m I0(x_k) / sinh(b m),
    x_k = m sqrt(b^2 - (2 pi k / n)^2): the Fourier factor the spread grid carries."""
    k = np.asarray(k, dtype=np.float64)
    x = m * np.sqrt(b * b - (2.0 * math.pi * k / n) ** 2)
    # I0(x) = i0e(x) e^x and sinh(bm) = e^{bm} (1 - e^{-2bm}) / 2
    return 2.0 * math.pi * m * i0e(x) * np.exp(x - b * m) / (-math.expm1(-2.0 * b * m))


def gauss_fourier(k: np.ndarray, st: float) -> np.ndarray:
    """Fourier coefficients of the 1-periodised Gaussian exp(-x^2/st^2) (Poisson summation)."""
    k = np.asarray(k, dtype=np.float64)
    return math.sqrt(math.pi) * st * np.exp(-(math.pi * st * k) ** 2)


def fft_frequencies(n: int) -> np.ndarray:
    """Frequency of each FFT index: 0..n/2-1, then -n/2..-1."""
    return np.fft.fftfreq(n, d=1.0 / n)


def conv_multiplier(n: int, M: int, m: int, st: float) -> np.ndarray:
    """Per-dimension Fourier multiplier c_k = bhat_k / Phi_k^2 on |k| <= M/2 - 1, else 0,
    in FFT index order."""
    b = kb_shape(n, M)
    k = fft_frequencies(n)
    c = gauss_fourier(k, st) / kb_fourier(k, n, m, b) ** 2
    c[np.abs(k) > M // 2 - 1] = 0.0
    return c


# ----------------------------------------------------------------------------- stages

def grid_coords(xt: np.ndarray, n: int) -> np.ndarray:
    return n * xt + 0.5 * n


def _taps(u: np.ndarray, n: int, m: int, b: float):
    """For each node and dimension: first tap cell, and the 2m weights (t, N, 2m)."""
    base = np.floor(u).astype(np.int64)  # (t, N)
    offs = np.arange(2 * m)
    cells = base[..., None] - m + 1 + offs  # (t, N, 2m)
    w = kb_window(u[..., None] - cells, m, b)
    return np.mod(cells, n), w


def spread(u: np.ndarray, v: np.ndarray, n: int, m: int, b: float) -> np.ndarray:
    """Adjoint-NFFT spreading g_c = sum_j v_j prod_d psi(u_{j,d} - c_d) on the periodic
    n^t grid (C order: last dimension fastest)."""
    t, N = u.shape
    cells, w = _taps(u, n, m, b)
    g = np.zeros(n ** t)
    # one tap tuple at a time; the (index, weight) pairs are pooled and summed with one
    # bincount per pool (plain summation, only the grouping of the additions differs)
    pool_i, pool_w, pooled = [], [], 0
    for tap in itertools.product(range(2 * m), repeat=t):
        flat = np.zeros(N, dtype=np.int64)
        wt = v.astype(np.float64).copy()
        for d in range(t):
            flat = flat * n + cells[d, :, tap[d]]
            wt = wt * w[d, :, tap[d]]
        pool_i.append(flat)
        pool_w.append(wt)
        pooled += N
        if pooled >= (1 << 23):
            g += np.bincount(np.concatenate(pool_i), weights=np.concatenate(pool_w),
                             minlength=n ** t)
            pool_i, pool_w, pooled = [], [], 0
    if pooled:
        g += np.bincount(np.concatenate(pool_i), weights=np.concatenate(pool_w),
                         minlength=n ** t)
    return g.reshape((n,) * t)


def convolve(g: np.ndarray, mults) -> np.ndarray:
    """Multiply the t-dimensional DFT of g by prod_d c_d(k_d) and transform back with the
    unnormalised inverse DFT (h_c = sum_k H_k e^{+2 pi i k c / n})."""
    G = np.fft.fftn(g)
    t = g.ndim
    for d in range(t):
        shape = [1] * t
        shape[d] = g.shape[d]
        G = G * mults[d].reshape(shape)
    h = np.fft.ifftn(G) * np.prod(g.shape)
    return h.real


def gather(h: np.ndarray, u: np.ndarray, m: int, b: float) -> np.ndarray:
    """NFFT gathering y_j = sum_c h_c prod_d psi(u_{j,d} - c_d)."""
    t, N = u.shape
    n = h.shape[0]
    cells, w = _taps(u, n, m, b)
    hf = h.reshape(-1)
    y = np.zeros(N)
    for tap in itertools.product(range(2 * m), repeat=t):
        flat = np.zeros(N, dtype=np.int64)
        wt = np.ones(N)
        for d in range(t):
            flat = flat * n + cells[d, :, tap[d]]
            wt = wt * w[d, :, tap[d]]
        y += wt * hf[flat]
    return y


# ----------------------------------------------------------------------------- summation

def fast_gauss_window(X: np.ndarray, v: np.ndarray, sigma: float, M: int, n: int, m: int):
    """Approximate (K v)_i = sum_j v_j exp(-||X_i - X_j||^2 / sigma^2) for one window X (t, N):
    scale -> spread -> FFT, multiply, inverse FFT -> gather."""
    kept, centres, scales, st = torus_scaling(X, sigma, M)
    if not kept:                       # identical nodes: K = 1 1^T exactly
        return np.full(X.shape[1], float(np.sum(v)))
    xt = np.stack([(X[d] - c) * s for d, c, s in zip(kept, centres, scales)])
    u = grid_coords(xt, n)
    b = kb_shape(n, M)
    g = spread(u, v, n, m, b)
    h = convolve(g, [conv_multiplier(n, M, m, s_) for s_ in st])
    return gather(h, u, m, b)


def fast_sigma_derivative_window(X, v, sigma, M, n, m):
    """Approximate sum_j v_j (2 r_ij^2 / sigma^2) exp(-r_ij^2 / sigma^2) for one window X (t, N):
    the kernel sigma dK/dsigma.  Its Fourier coefficients follow from those of the Gaussian by
    differentiating the Poisson-summation formula: bhat_k (t - 2 pi^2 sum_d st_d^2 k_d^2), a
    non-separable factor, applied here on the full t-dimensional spectrum."""
    kept, centres, scales, st = torus_scaling(X, sigma, M)
    if not kept:                       # identical nodes: r = 0, the kernel vanishes
        return np.zeros(X.shape[1])
    xt = np.stack([(X[d] - c) * s for d, c, s in zip(kept, centres, scales)])
    u = grid_coords(xt, n)
    b = kb_shape(n, M)
    g = spread(u, v, n, m, b)
    t = len(kept)
    k = fft_frequencies(n)
    G = np.fft.fftn(g)
    factor = np.full(G.shape, float(t))
    for d in range(t):
        shape = [1] * t
        shape[d] = n
        G = G * conv_multiplier(n, M, m, st[d]).reshape(shape)
        factor = factor - 2.0 * math.pi ** 2 * st[d] ** 2 * (k ** 2).reshape(shape)
    h = (np.fft.ifftn(G * factor) * n ** t).real
    return gather(h, u, m, b)


def window_matrix_nfft(X: np.ndarray, sigma: float, M: int, n: int, m: int) -> np.ndarray:
    """The dense N x N matrix of fast_gauss_window for one window X (t, N), for small N.

    The summation is W~ = B C B^T with B the spreading matrix and C the circulant of the
    multiplier; both factor over the kept dimensions (the window is a tensor product of one
    window per dimension, the multiplier a product of per-dimension multipliers), so
    W~ = T_1 o ... o T_t (entrywise product) with T_d = B_d C_d B_d^T, B_d (N x n) the 2m tap
    weights of dimension d and C_d[c, c'] = sum_k c_k e^{2 pi i k (c - c') / n} the real
    circulant of that dimension's multiplier."""
    kept, centres, scales, st = torus_scaling(X, sigma, M)
    N = X.shape[1]
    if not kept:
        return np.ones((N, N))
    b = kb_shape(n, M)
    Wt = np.ones((N, N))
    rows = np.arange(N)
    for d, c, s, s_t in zip(kept, centres, scales, st):
        u = grid_coords(((X[d] - c) * s)[None, :], n)
        cells, w = _taps(u, n, m, b)                      # (1, N, 2m)
        B = np.zeros((N, n))
        for tap in range(2 * m):
            np.add.at(B, (rows, cells[0, :, tap]), w[0, :, tap])
        col = (np.fft.ifft(conv_multiplier(n, M, m, s_t)) * n).real   # C[c, 0] = col[c]
        C = col[(np.arange(n)[:, None] - np.arange(n)[None, :]) % n]
        Wt *= B @ C @ B.T
    return Wt


def anova_matvec_nfft(F, wins, sigmas, weights, v, M, n, m):
    """W~ v = sum_l w_l K~_l v with one fast Gauss summation per window (Sec. 3)."""
    y = np.zeros(F.shape[1])
    for win, s, w in zip(wins, sigmas, weights):
        y += w * fast_gauss_window(F[list(win)], v, s, M, n, m)
    return y


# ----------------------------------------------------------------------------- references

def ndft_adjoint(xt: np.ndarray, v: np.ndarray, M: int) -> np.ndarray:
    """Exact adjoint NDFT ghat_k = sum_j v_j exp(-2 pi i k . xt_j) for k in the full index set
    I_M = {-M/2, ..., M/2-1}^t (paper Sec. 3, NFFT definition), shape (M,)*t."""
    t, N = xt.shape
    k = np.arange(-M // 2, M // 2)
    E = [np.exp(-2j * math.pi * np.outer(k, xt[d])) for d in range(t)]  # (M, N)
    if t == 1:
        return E[0] @ v
    if t == 2:
        return np.einsum("an,bn,n->ab", E[0], E[1], v)
    return np.einsum("an,bn,cn,n->abc", E[0], E[1], E[2], v)


def truncated_fourier_sum(xt: np.ndarray, v: np.ndarray, st, M: int) -> np.ndarray:
    """sum_{|k_d| <= M/2-1} prod_d bhat_{k_d} e^{2 pi i k . xt_i} ghat_k: the band-limited
    periodic kernel the NFFT approximates, evaluated exactly with the NDFT."""
    t, N = xt.shape
    k = np.arange(-M // 2, M // 2)
    ghat = ndft_adjoint(xt, v, M)
    coef = [gauss_fourier(k, s) * (np.abs(k) <= M // 2 - 1) for s in st]
    E = [np.exp(2j * math.pi * np.outer(xt[d], k)) for d in range(t)]  # (N, M)
    if t == 1:
        return (E[0] @ (coef[0] * ghat)).real
    if t == 2:
        H = ghat * np.outer(coef[0], coef[1])
        return np.einsum("na,nb,ab->n", E[0], E[1], H).real
    H = ghat * np.einsum("a,b,c->abc", *coef)
    return np.einsum("na,nb,nc,abc->n", E[0], E[1], E[2], H).real


def periodic_gauss_sum(xt: np.ndarray, v: np.ndarray, st, images: int = 2) -> np.ndarray:
    """sum_j v_j prod_d sum_{p=-images..images} exp(-(xt_i - xt_j + p)^2 / st_d^2): the
    1-periodised Gaussian evaluated directly (wrap-around included)."""
    t, N = xt.shape
    K = np.ones((N, N))
    for d in range(t):
        diff = xt[d][:, None] - xt[d][None, :]
        acc = np.zeros((N, N))
        for p in range(-images, images + 1):
            acc += np.exp(-((diff + p) / st[d]) ** 2)
        K *= acc
    return K @ v
