"""Dense and direct-sum extended Gaussian ANOVA kernel (paper Sec. 2.5-2.6).

Plain definitions, FP64:
  K_l(i, j) = exp(-||F_i[W_l] - F_j[W_l]||^2 / sigma_l^2)       (discrete ANOVA kernel)
  W = sum_l w_l K_l            (the paper's weights are 1/L; general w_l >= 0 here)
  D = W 1,   L = diag(D) - W   (graph Laplacian; its diagonal does not depend on W_ii)
  eta = D - sum_l w_l          (degree with the zero-diagonal convention of the paper)
  A = I + alpha L              (the system (lambda I + mu L) u = lambda f with alpha = mu/lambda)

Diagonal preconditioners of Sec. 4.3.1 in the alpha form (lambda = 1, mu = alpha):
  P_a = I + alpha diag(eta)                                   (Jacobi)
  P_b = diag( (sum_j a_ij^2)^(1/2) )                          (row 2-norms of A)
  P_b' = [ alpha^2 sum_l w_l^2 diag(Gamma_l o Gamma_l 1) + P_a^2 ]^(1/2)
where Gamma_l is K_l with a zero diagonal; P_b' keeps only the L squared window terms of the
square of the window sum (the cross terms are dropped, as the paper does for ANOVA kernels).
"""
from __future__ import annotations

import numpy as np


def window_kernel_dense(F: np.ndarray, win, sigma: float) -> np.ndarray:
    """Dense K_l (N x N) for one window; direct formula."""
    X = F[list(win)].T  # (N, t)
    sq = np.zeros((X.shape[0], X.shape[0]))
    for d in range(X.shape[1]):
        diff = X[:, d][:, None] - X[:, d][None, :]
        sq += diff * diff
    return np.exp(-sq / (sigma * sigma))


def anova_dense(F, wins, sigmas, weights) -> np.ndarray:
    """Dense W = sum_l w_l K_l (self term included)."""
    N = F.shape[1]
    W = np.zeros((N, N))
    for win, s, w in zip(wins, sigmas, weights):
        W += w * window_kernel_dense(F, win, s)
    return W


def laplacian_dense(W: np.ndarray) -> np.ndarray:
    return np.diag(W.sum(axis=1)) - W


def system_dense(W: np.ndarray, alpha: float) -> np.ndarray:
    return np.eye(W.shape[0]) + alpha * laplacian_dense(W)


def degree(W: np.ndarray) -> np.ndarray:
    return W.sum(axis=1)


def eta_from_degree(D: np.ndarray, weights) -> np.ndarray:
    """eta = Gamma 1 with a zero diagonal: the self term sum_l w_l removed."""
    return D - float(np.sum(weights))


def anova_rows_direct(F, wins, sigmas, weights, rows, v, chunk: int = 256) -> np.ndarray:
    """(W v)[rows] by direct O(|rows| N L) summation, chunked over rows."""
    rows = np.asarray(rows)
    out = np.zeros(rows.shape[0])
    for s0 in range(0, rows.shape[0], chunk):
        r = rows[s0:s0 + chunk]
        acc = np.zeros(r.shape[0])
        for win, s, w in zip(wins, sigmas, weights):
            sq = np.zeros((r.shape[0], F.shape[1]))
            for d in win:
                diff = F[d][r][:, None] - F[d][None, :]
                sq += diff * diff
            acc += w * (np.exp(-sq / (s * s)) @ v)
        out[s0:s0 + chunk] = acc
    return out


def anova_matvec_direct(F, wins, sigmas, weights, v, chunk: int = 256) -> np.ndarray:
    """Full W v by direct summation (O(N^2 L)); for small N."""
    return anova_rows_direct(F, wins, sigmas, weights, np.arange(F.shape[1]), v, chunk)


def l2_window_degree(F, wins, sigmas, weights) -> np.ndarray:
    """sum_l w_l^2 (Gamma_l o Gamma_l) 1: squared kernel entries, zero diagonal."""
    N = F.shape[1]
    out = np.zeros(N)
    for win, s, w in zip(wins, sigmas, weights):
        K = window_kernel_dense(F, win, s)
        out += w * w * ((K * K).sum(axis=1) - 1.0)
    return out


def precond_jacobi(eta: np.ndarray, alpha: float) -> np.ndarray:
    return 1.0 + alpha * eta


def precond_l2_anova(eta: np.ndarray, d2: np.ndarray, alpha: float) -> np.ndarray:
    """P_b' from eta and d2 = sum_l w_l^2 (Gamma_l o Gamma_l) 1."""
    return np.sqrt(alpha * alpha * d2 + (1.0 + alpha * eta) ** 2)


def precond_l2_full(A: np.ndarray) -> np.ndarray:
    """P_b: the 2-norms of the rows of A."""
    return np.sqrt((A * A).sum(axis=1))
