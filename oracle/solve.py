"""Linear solves of the nonlocal system (I + alpha L) u = f, FP64 (paper Sec. 2.6, 4, 5).

  dense_solve          Cholesky solve of the dense SPD system (the paper's dposv baseline,
                       Sec. 5.3).
  helmert_apply /      the orthonormal change of basis U for the eigenvector 1 (paper
  helmert_apply_t      Sec. 4.1.2 general form specialised to v = 1 in Sec. 4.2, the
                       normalised Helmert matrix), in O(N) with the shifted cumulative sums:
                       U x uses the backward (suffix) sum, U^T x the forward (prefix) sum.
                       The forward sum's index range is read as i = 2..N (the printed range
                       stops at N-1, one entry short).
  helmert_dense        U as a dense matrix (small N), for checks.
  q_dense / q_inv_dense / q_apply / q_inv_apply
                       the sparse, non-orthogonal change of basis Q of Sec. 4.1.1 for an
                       eigenvector v (v_1 != 0), its inverse and their O(n) actions.
  pcg_ubasis           the paper's deflated Jacobi-PCG: change of basis with U, x1 = g1
                       (the decoupled eigenvalue of A for the vector 1 is 1 here), CG on the
                       (N-1) block with the preconditioner pi_2(U^T P^-1 U), P = I + alpha
                       diag(eta) (Sec. 4.3.1 Jacobi; Sec. 4.3.2 dense preconditioner), then
                       u = U x (Sec. 5.4).
  pcg_projector        the same iteration written in the original coordinates with the
                       orthogonal projector Pi = I - 1 1^T / N = U_2 U_2^T (equal in exact
                       arithmetic; this is the form the HIP path runs).
  cg_plain / pcg_jacobi  undeflated CG and Jacobi PCG in the original basis (Sec. 5.3, 5.4).

Stopping rule (the paper's "tolerance"): ||r_k||_2 <= tol * ||b||_2 with b the right-hand side
of the block that CG runs on (= f - mean(f) 1 for the deflated forms), r_k the recursive
residual; the initial guess is f (Sec. 5.3).  One iteration = one operator application.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def dense_solve(A: np.ndarray, f: np.ndarray) -> np.ndarray:
    c = scipy.linalg.cho_factor(A, lower=True)
    return scipy.linalg.cho_solve(c, f)


# ----------------------------------------------------------------------------- Helmert U

def _helmert_ab(N: int):
    i = np.arange(2, N + 1, dtype=np.float64)
    a = np.sqrt((i - 1.0) / i)           # a_v for v = 1
    b = 1.0 / np.sqrt(i * (i - 1.0))     # b_v for v = 1
    return a, b


def helmert_apply(x: np.ndarray) -> np.ndarray:
    """U x = SCS_up([x1/sqrt(N); b o x_{2:N}]) - [0; a o x_{2:N}]  (v = 1)."""
    N = x.shape[0]
    a, b = _helmert_ab(N)
    y = np.empty(N)
    y[0] = x[0] / np.sqrt(N)
    y[1:] = b * x[1:]
    # SCS_up(y)_i = y_1 + sum_{j > i} y_j  (i = 1..N; the last entry is y_1)
    suffix = np.concatenate([np.cumsum(y[1:][::-1])[::-1], [0.0]])  # sum_{j >= i+1}, i=1..N
    out = y[0] + suffix
    out[1:] -= a * x[1:]
    return out


def helmert_apply_t(x: np.ndarray) -> np.ndarray:
    """U^T x = [1/sqrt(N); b] o SCS_down(x) - [0; a o x_{2:N}],
    SCS_down(x) = [sum_j x_j; (sum_{j < i} x_j)_{i = 2..N}]."""
    N = x.shape[0]
    a, b = _helmert_ab(N)
    pre = np.cumsum(x)
    out = np.empty(N)
    out[0] = pre[-1] / np.sqrt(N)
    out[1:] = b * pre[:-1] - a * x[1:]
    return out


def helmert_dense(N: int) -> np.ndarray:
    """Dense normalised Helmert matrix: U[:,0] = 1/sqrt(N); column i (1-based, i >= 2) is
    (1_{1:i-1} - (i-1) e_i) / sqrt(i (i-1))."""
    U = np.zeros((N, N))
    U[:, 0] = 1.0 / np.sqrt(N)
    for i in range(2, N + 1):
        U[: i - 1, i - 1] = 1.0
        U[i - 1, i - 1] = -(i - 1.0)
        U[:, i - 1] /= np.sqrt(i * (i - 1.0))
    return U


# ----------------------------------------------------------------------------- Q basis
# The sparse change of basis of paper Sec. 4.1.1 for a real eigenvector v with v_1 != 0:
# q_1 = v and q_i = v_i e_1 - v_1 e_i for i >= 2 (eq. Hermitian_Q_Construction), a symmetric
# bordered matrix whose inverse is v v^T / (v_1 ||v||^2) - diag(0, 1/v_1, ..., 1/v_1)
# (eq. Q_inverse_compact).  Both act in O(n).  For v = 1 these are the matrices of Sec. 4.2
# (eq. QLap).  Q^-1 A Q keeps the eigenvalue of v in its first column with a zero first row,
# but its (n-1) block is not symmetric, so CG runs in the orthonormal (Helmert) basis instead.

def q_dense(v: np.ndarray) -> np.ndarray:
    """Q as a dense matrix: first column and row v, lower-right block -v_1 I (small n)."""
    v = np.asarray(v, dtype=np.float64)
    if v[0] == 0.0:
        raise ValueError("q basis: v_1 must be nonzero")
    n = v.size
    Q = np.zeros((n, n))
    Q[:, 0] = v
    for i in range(1, n):          # column i: v_i e_1 - v_1 e_i
        Q[0, i] = v[i]
        Q[i, i] = -v[0]
    return Q


def q_inv_dense(v: np.ndarray) -> np.ndarray:
    """Q^-1 = v v^T / (v_1 ||v||^2) - diag(0, 1/v_1 ... 1/v_1) (compact form)."""
    v = np.asarray(v, dtype=np.float64)
    if v[0] == 0.0:
        raise ValueError("q basis: v_1 must be nonzero")
    corr = np.full(v.size, 1.0 / v[0])
    corr[0] = 0.0
    return np.outer(v, v) / (v[0] * (v @ v)) - np.diag(corr)


def q_apply(v: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Q u = [<u, v>; u_1 v_{2:n} - v_1 u_{2:n}], O(n)."""
    v = np.asarray(v, dtype=np.float64)
    out = np.empty_like(v)
    out[0] = u @ v
    out[1:] = u[0] * v[1:] - v[0] * u[1:]
    return out


def q_inv_apply(v: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Q^-1 u = (1/v_1) { (<u, v> / ||v||^2) v - [0; u_{2:n}] }, O(n)."""
    v = np.asarray(v, dtype=np.float64)
    out = (u @ v) / (v @ v) * v
    out[1:] -= u[1:]
    return out / v[0]


# ----------------------------------------------------------------------------- CG core

def _pcg(apply_B, apply_Minv, b, y0, tol, maxit, record=None):
    y = y0.copy()
    r = b - apply_B(y)
    bnorm = np.linalg.norm(b)
    history = []
    if np.linalg.norm(r) <= tol * bnorm:
        return y, 0, np.linalg.norm(r) / (bnorm if bnorm > 0 else 1.0), history
    s = apply_Minv(r)
    p = s.copy()
    rho = r @ s
    it = 0
    while it < maxit:
        q = apply_B(p)
        a = rho / (p @ q)
        y = y + a * p
        r = r - a * q
        it += 1
        if record is not None:
            history.append(record(y))
        if np.linalg.norm(r) <= tol * bnorm:
            break
        s = apply_Minv(r)
        rho_new = r @ s
        p = s + (rho_new / rho) * p
        rho = rho_new
    relres = np.linalg.norm(r) / (bnorm if bnorm > 0 else 1.0)
    return y, it, relres, history


def pcg_ubasis(apply_A, f, eta, alpha, tol, maxit, u0=None, record=False):
    """Paper-literal deflated Jacobi PCG in the Helmert basis.  Returns
    (u, iters, relres, iterates) where iterates are mapped back to the original basis."""
    N = f.shape[0]
    if np.all(f == f[0]):              # f_perp = 0: u = f, no iteration
        return f.copy(), 0, 0.0, ([] if record else None)
    u0 = f if u0 is None else u0
    Pinv = 1.0 / (1.0 + alpha * eta)
    g = helmert_apply_t(f)
    x1 = g[0]

    def lift(y):
        return helmert_apply(np.concatenate([[0.0], y]))

    def apply_B(y):
        return helmert_apply_t(apply_A(lift(y)))[1:]

    def apply_Minv(r):
        return helmert_apply_t(Pinv * lift(r))[1:]

    y0 = helmert_apply_t(u0)[1:]
    rec = (lambda y: helmert_apply(np.concatenate([[x1], y]))) if record else None
    y, it, relres, hist = _pcg(apply_B, apply_Minv, g[1:], y0, tol, maxit, rec)
    u = helmert_apply(np.concatenate([[x1], y]))
    return u, it, relres, (hist if record else None)


def pcg_projector(apply_A, f, eta, alpha, tol, maxit, u0=None, record=False, P=None):
    """Deflated diagonally preconditioned CG with the projector Pi = I - 1 1^T/N in the original
    basis: ubar = mean(f), z0 = Pi u0, s = Pi(r / P), u = ubar 1 + z.  P defaults to the Jacobi
    diagonal 1 + alpha eta (P_{U,a}); passing the l2 diagonal gives P_{U,b}.  A constant f
    (f_perp = 0) returns u = f with no iteration."""
    if np.all(f == f[0]):
        return f.copy(), 0, 0.0, ([] if record else None)
    u0 = f if u0 is None else u0
    P = 1.0 + alpha * eta if P is None else P
    ubar = f.mean()

    def proj(x):
        return x - x.mean()

    b = proj(f)
    rec = (lambda z: ubar + z) if record else None
    z, it, relres, hist = _pcg(lambda z: proj(apply_A(z)), lambda r: proj(r / P),
                               b, proj(u0), tol, maxit, rec)
    return ubar + z, it, relres, (hist if record else None)


def cg_plain(apply_A, f, tol, maxit, u0=None):
    u0 = f if u0 is None else u0
    u, it, relres, _ = _pcg(apply_A, lambda r: r, f, u0, tol, maxit)
    return u, it, relres


def pcg_jacobi(apply_A, f, eta, alpha, tol, maxit, u0=None, P=None):
    """Diagonally preconditioned CG without deflation (P_a by default, or a given diagonal)."""
    u0 = f if u0 is None else u0
    P = 1.0 + alpha * eta if P is None else P
    u, it, relres, _ = _pcg(apply_A, lambda r: r / P, f, u0, tol, maxit)
    return u, it, relres


def system_operator(apply_W, D, alpha):
    """v -> v + alpha (D o v - W v): the matrix-free A of the nonlocal system."""
    return lambda v: v + alpha * (D * v - apply_W(v))
