"""Seeded synthetic grayscale images: the inputs shared by the HIP path and the oracle.

This module holds only the input recipe (no step of the denoising method): a clean
piecewise-constant image of axis-aligned rectangles and discs painted in order, plus
i.i.d. additive Gaussian noise, f = u_c + h with h ~ N(0, s^2 I) as in the paper's
experimental setup (Sec. 5, noisy-image model).  The paper's own test images
(scikit-image samples and private photographs) are not available; these images stand
in for them with the same kind of content: flat regions, jumps, and additive noise.

Recipe (all draws from ``numpy.random.default_rng(seed)``, in this order):
  * background 0;
  * for each rectangle: height U[0.1, 0.5]*n1, width U[0.1, 0.5]*n2 (rounded, >= 1),
    top-left corner uniform over the positions that keep it inside the image,
    intensity U[0, 1]; later shapes overwrite earlier ones;
  * for each disc: centre uniform in the image, radius U[0.05, 0.25]*min(n1, n2),
    intensity U[0, 1];
  * noise: ``noise * rng.standard_normal((n1, n2))`` added once, no clipping.
"""
from __future__ import annotations

import numpy as np


def make_image(seed: int, n1: int, n2: int, n_rect: int, n_disc: int, noise: float):
    """Return ``(u_clean, f_noisy)`` as float64 arrays of shape (n1, n2)."""
    if n1 < 1 or n2 < 1:
        raise ValueError("image sides must be >= 1")
    rng = np.random.default_rng(seed)
    u = np.zeros((n1, n2), dtype=np.float64)
    for _ in range(n_rect):
        h = max(1, int(round(rng.uniform(0.1, 0.5) * n1)))
        w = max(1, int(round(rng.uniform(0.1, 0.5) * n2)))
        r0 = int(rng.integers(0, n1 - h + 1))
        c0 = int(rng.integers(0, n2 - w + 1))
        val = rng.uniform(0.0, 1.0)
        u[r0:r0 + h, c0:c0 + w] = val
    rows = np.arange(n1)[:, None]
    cols = np.arange(n2)[None, :]
    for _ in range(n_disc):
        cr = rng.uniform(0, n1)
        cc = rng.uniform(0, n2)
        rad = rng.uniform(0.05, 0.25) * min(n1, n2)
        val = rng.uniform(0.0, 1.0)
        u[(rows + 0.5 - cr) ** 2 + (cols + 0.5 - cc) ** 2 <= rad * rad] = val
    f = u + noise * rng.standard_normal((n1, n2))
    return u, f


def log_uniform(rng, lo: float, hi: float, size=None):
    """Draw from the log-uniform distribution on [lo, hi]."""
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=size))


def random_vector(seed: int, n: int):
    """A seeded standard-normal test vector of length n (float64)."""
    return np.random.default_rng(seed).standard_normal(n)


# Named workloads: image recipes and kernel parameters of the five configurations.
WORKLOADS = {
    "c1_64": dict(n1=64, n2=64, n_rect=6, n_disc=4, noise=0.1, rho=1, seed=0,
                  sigma=0.1, alpha=0.5, M=32, M_parity=64, m=6, tol=1e-10),
    "c2_512": dict(n1=512, n2=512, n_rect=20, n_disc=12, noise=0.1, rho=2, seed=1,
                   sigmas=(0.05, 0.1, 0.2), alphas=(0.1, 1.0, 10.0), M=64,
                   m_fp32=4, m_fp64=8, tol=1e-6),
}
