"""Pins of the oracle's bilevel gradient (paper Sec. 2.4, 5.5): central finite differences of
the objective, the closed form of the alpha derivative, and the identity that scaling every
weight by c is the same as scaling alpha by c."""
import numpy as np

from oracle import gradient as G
from oracle import kernel as K
from oracle.features import features_from_image, window_table
from paper_2407_06834_amd.synth import make_image


def _images(T=2, n=12):
    out = []
    for t in range(T):
        uc, f = make_image(200 + t, n, n, 3, 2, 0.15)
        out.append((features_from_image(f, 1), f.reshape(-1), uc.reshape(-1)))
    return out


def test_adjoint_gradient_matches_finite_differences():
    imgs = _images()
    wins = window_table(1)
    sig = [0.1, 0.12, 0.15, 0.2]
    wts = [1.0, 0.7, 1.3, 0.5]
    alpha = 0.8
    J, g_la, g_ls, g_w = G.gradient(imgs, wins, sig, wts, alpha)
    d_la, d_ls, d_w = G.finite_difference_gradient(imgs, wins, sig, wts, alpha, h=1e-5)
    scale = max(abs(g_la), np.abs(g_ls).max(), np.abs(g_w).max())
    assert abs(g_la - d_la) < 1e-6 * scale
    np.testing.assert_allclose(g_ls, d_ls, atol=1e-6 * scale)
    np.testing.assert_allclose(g_w, d_w, atol=1e-6 * scale)
    assert J > 0


def test_alpha_derivative_identities():
    imgs = _images(T=1)
    wins = window_table(1)
    sig, wts, alpha = [0.1] * 4, [1.0, 2.0, 0.5, 1.5], 1.3
    J, g_la, g_ls, g_w = G.gradient(imgs, wins, sig, wts, alpha)
    # alpha multiplies every w_l, so d/dlog alpha = sum_l w_l d/dw_l
    assert abs(g_la - float(np.dot(wts, g_w))) < 1e-10 * abs(g_la)


def test_sigma_derivative_kernel_is_sigma_dK_dsigma():
    uc, f = make_image(7, 8, 8, 2, 1, 0.1)
    F = features_from_image(f, 1)
    win, s, h = [0, 1, 6], 0.13, 1e-6
    num = s * (K.window_kernel_dense(F, win, s + h) - K.window_kernel_dense(F, win, s - h)) / (2 * h)
    np.testing.assert_allclose(G.sigma_derivative_kernel(F, win, s), num, atol=1e-8)
