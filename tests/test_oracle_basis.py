"""Pins of the change of basis for the eigenvector 1 (paper Sec. 4.1, 4.2)."""
import numpy as np

from oracle import kernel as K
from oracle import solve as S
from oracle.features import features_from_image, window_table
from paper_2407_06834_amd.synth import make_image


def test_helmert_closed_form():
    N = 9
    U = S.helmert_dense(N)
    np.testing.assert_allclose(U.T @ U, np.eye(N), atol=1e-15)
    np.testing.assert_allclose(U[:, 0], np.full(N, 1 / np.sqrt(N)), rtol=0, atol=1e-16)
    # columns i >= 2 sum to zero (orthogonal to 1) and column 2 = (e1 - e2)/sqrt 2
    np.testing.assert_allclose(U[:, 1:].sum(axis=0), 0, atol=1e-15)
    e = np.zeros(N)
    e[0], e[1] = 1, -1
    np.testing.assert_allclose(U[:, 1], e / np.sqrt(2), atol=1e-16)


def test_scan_forms_equal_dense():
    for N in (2, 3, 17, 256):
        U = S.helmert_dense(N)
        x = np.random.default_rng(N).standard_normal(N)
        np.testing.assert_allclose(S.helmert_apply(x), U @ x, atol=1e-13)
        np.testing.assert_allclose(S.helmert_apply_t(x), U.T @ x, atol=1e-13)


def test_projector_identity():
    N = 50
    U = S.helmert_dense(N)
    Pi = np.eye(N) - np.ones((N, N)) / N
    np.testing.assert_allclose(U[:, 1:] @ U[:, 1:].T, Pi, atol=1e-14)


def test_q_basis_inverse():
    # Q = [1 | (1_{n-1}^T ; -I)] and Q^{-1} = n^{-1} 1 1^T - diag(0, 1_{n-1}) (Sec. 4.2)
    n = 7
    Q = np.zeros((n, n))
    Q[:, 0] = 1
    Q[0, 1:] = 1
    Q[1:, 1:] = -np.eye(n - 1)
    Qi = np.ones((n, n)) / n - np.diag(np.r_[0.0, np.ones(n - 1)])
    np.testing.assert_allclose(Qi @ Q, np.eye(n), atol=1e-14)
    u = np.arange(1.0, n + 1)
    np.testing.assert_allclose(Qi @ u, np.r_[u.mean(), u.mean() - u[1:]], atol=1e-14)


def test_block_form_of_transformed_system():
    _, f = make_image(4, 10, 11, 3, 2, 0.1)
    F = features_from_image(f, 1)
    W = K.anova_dense(F, window_table(1), [0.1] * 4, [1.0] * 4)
    A = K.system_dense(W, 2.0)
    U = S.helmert_dense(A.shape[0])
    B = U.T @ A @ U
    assert abs(B[0, 0] - 1.0) < 1e-12
    assert np.abs(B[0, 1:]).max() < 1e-11 and np.abs(B[1:, 0]).max() < 1e-11


def test_q_basis_general_vector_structure_and_determinant():
    # eq. Hermitian_Q_Construction: symmetric, Q e_1 = v, columns 2..n orthogonal to v;
    # det Q = (v_1 + ||v_{2:n}||^2 / v_1) (-v_1)^(n-1) (eq. detQ)
    rng = np.random.default_rng(3)
    for n in (2, 5, 12):
        v = rng.standard_normal(n)
        v[0] = 0.7
        Q = S.q_dense(v)
        np.testing.assert_array_equal(Q, Q.T)
        np.testing.assert_array_equal(Q[:, 0], v)
        np.testing.assert_allclose(v @ Q[:, 1:], 0.0, atol=1e-14)
        det = (v[0] + (v[1:] @ v[1:]) / v[0]) * (-v[0]) ** (n - 1)
        np.testing.assert_allclose(np.linalg.det(Q), det, rtol=1e-12)


def test_q_inverse_and_linear_time_actions():
    # eq. Q_Inverse / Q_inverse_compact and the O(n) actions, against dense products and a
    # library solve
    rng = np.random.default_rng(4)
    for n in (3, 8, 40):
        v = rng.standard_normal(n)
        v[0] = -1.3
        u = rng.standard_normal(n)
        Q, Qi = S.q_dense(v), S.q_inv_dense(v)
        np.testing.assert_allclose(Qi @ Q, np.eye(n), atol=1e-13)
        np.testing.assert_allclose(S.q_apply(v, u), Q @ u, atol=1e-13)
        np.testing.assert_allclose(S.q_inv_apply(v, u), np.linalg.solve(Q, u), atol=1e-12)


def test_q_basis_of_the_constant_vector():
    # eq. QLap: Q u = [n mean(u); u_1 - u_{2:n}], Q^-1 u = [mean(u); mean(u) - u_{2:n}]
    n = 9
    one = np.ones(n)
    u = np.random.default_rng(5).standard_normal(n)
    np.testing.assert_allclose(S.q_apply(one, u), np.r_[n * u.mean(), u[0] - u[1:]], atol=1e-14)
    np.testing.assert_allclose(S.q_inv_apply(one, u), np.r_[u.mean(), u.mean() - u[1:]],
                               atol=1e-14)
    np.testing.assert_allclose(S.q_inv_dense(one),
                               np.ones((n, n)) / n - np.diag(np.r_[0.0, np.ones(n - 1)]),
                               atol=1e-15)


def test_q_conjugation_isolates_the_eigenvalue():
    # Q^-1 A Q = [lambda, 0; 0, B_2] for the eigenpair (1, 1) of A = I + alpha L (b_1 = 0 since
    # A is symmetric), with a non-symmetric block B_2, and its spectrum is A's without lambda
    _, f = make_image(6, 7, 8, 2, 1, 0.1)
    F = features_from_image(f, 1)
    W = K.anova_dense(F, window_table(1), [0.2] * 4, [1.0] * 4)
    A = K.system_dense(W, 1.5)
    n = A.shape[0]
    one = np.ones(n)
    B = S.q_inv_dense(one) @ A @ S.q_dense(one)
    assert abs(B[0, 0] - 1.0) < 1e-12
    assert np.abs(B[1:, 0]).max() < 1e-11 and np.abs(B[0, 1:]).max() < 1e-11
    assert np.abs(B[1:, 1:] - B[1:, 1:].T).max() > 1e-3
    ev_A = np.sort(np.linalg.eigvalsh(A))
    ev_B = np.sort(np.linalg.eigvals(B[1:, 1:]).real)
    # A's eigenvalue 1 belongs to the vector 1; the rest is the spectrum of B_2
    k = int(np.argmin(np.abs(ev_A - 1.0)))
    np.testing.assert_allclose(ev_B, np.delete(ev_A, k), rtol=1e-9)
