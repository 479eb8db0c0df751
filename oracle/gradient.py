"""Bilevel gradient of the denoising loss, dense FP64 (paper Sec. 2.4 optimality system and
Sec. 5.5 parameter learning), written on the discrete system.

Lower level: A(theta) u = f with A = I + alpha L, L = diag(W 1) - W, W = sum_l w_l K_l,
K_l(i, j) = exp(-r_l(i, j)^2 / sigma_l^2).  Upper level (Sec. 5.5, bilevel problem):
J = (1/T) sum_t ||u_t - u_{c,t}||^2 (no factor 1/2).

Adjoint: A p = dJ/du (A is symmetric), dJ/dtheta = -p^T (dA/dtheta) u, which gives
  dJ/dlog(alpha)   = -alpha p^T L u  (= p^T (u - f) because alpha L u = f - u),
  dJ/dw_l          = -alpha p^T L_l u,
  dJ/dlog(sigma_l) = -alpha w_l p^T L_l^s u,
where L_l is the Laplacian of K_l and L_l^s that of sigma_l dK_l/dsigma_l, whose entries are
(2 r^2 / sigma_l^2) exp(-r^2 / sigma_l^2).  (The paper's continuous gradient is stated for the
operator -L; signs are fixed here by the discrete system and pinned by finite differences.)
"""
from __future__ import annotations

import numpy as np

from . import kernel as K
from . import solve as S


def window_sq_dist(F, win):
    X = F[list(win)].T
    sq = np.zeros((X.shape[0], X.shape[0]))
    for d in range(X.shape[1]):
        diff = X[:, d][:, None] - X[:, d][None, :]
        sq += diff * diff
    return sq


def sigma_derivative_kernel(F, win, sigma):
    """sigma dK/dsigma = (2 r^2 / sigma^2) exp(-r^2 / sigma^2) (dense)."""
    r2 = window_sq_dist(F, win) / (sigma * sigma)
    return 2.0 * r2 * np.exp(-r2)


def solve_state(F, wins, sigmas, weights, alpha, f):
    W = K.anova_dense(F, wins, sigmas, weights)
    A = K.system_dense(W, alpha)
    return S.dense_solve(A, f), A


def objective(images, wins, sigmas, weights, alpha):
    """J = (1/T) sum_t ||u_t - u_c,t||^2 for images = [(F_t, f_t, u_c_t)]."""
    T = len(images)
    J = 0.0
    for F, f, uc in images:
        u, _ = solve_state(F, wins, sigmas, weights, alpha, f)
        J += float(np.sum((u - uc) ** 2))
    return J / T


def gradient(images, wins, sigmas, weights, alpha):
    """Returns (J, dJ/dlog alpha, [dJ/dlog sigma_l], [dJ/dw_l]) by the adjoint method."""
    T = len(images)
    L = len(wins)
    J = 0.0
    g_la = 0.0
    g_ls = np.zeros(L)
    g_w = np.zeros(L)
    for F, f, uc in images:
        u, A = solve_state(F, wins, sigmas, weights, alpha, f)
        J += float(np.sum((u - uc) ** 2)) / T
        p = S.dense_solve(A, (2.0 / T) * (u - uc))
        g_la += float(p @ (u - f))
        for l, (win, s, w) in enumerate(zip(wins, sigmas, weights)):
            Kl = K.window_kernel_dense(F, win, s)
            Ks = sigma_derivative_kernel(F, win, s)
            g_w[l] += -alpha * float(p @ (K.laplacian_dense(Kl) @ u))
            g_ls[l] += -alpha * w * float(p @ (K.laplacian_dense(Ks) @ u))
    return J, g_la, g_ls, g_w


def finite_difference_gradient(images, wins, sigmas, weights, alpha, h=1e-5):
    """Central differences of J in (log alpha, log sigma_l, w_l)."""
    L = len(wins)

    def J_of(la, ls, w):
        return objective(images, wins, list(np.exp(ls)), list(w), float(np.exp(la)))

    la0 = np.log(alpha)
    ls0 = np.log(np.asarray(sigmas, dtype=float))
    w0 = np.asarray(weights, dtype=float)
    d_la = (J_of(la0 + h, ls0, w0) - J_of(la0 - h, ls0, w0)) / (2 * h)
    d_ls = np.zeros(L)
    d_w = np.zeros(L)
    for l in range(L):
        e = np.zeros(L)
        e[l] = h
        d_ls[l] = (J_of(la0, ls0 + e, w0) - J_of(la0, ls0 - e, w0)) / (2 * h)
        d_w[l] = (J_of(la0, ls0, w0 + e) - J_of(la0, ls0, w0 - e)) / (2 * h)
    return d_la, d_ls, d_w
