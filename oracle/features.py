"""Per-pixel features and window table (paper Sec. 5, patch features; Sec. 2.5, windows).

Features of pixel i (raster index i = row*n2 + col):
  * optional position (col/n2, row/n1), 0-based, in [0, 1);
  * the (2*rho+1)^2 intensities of the square patch of radius rho centred on the pixel,
    in raster order of the offsets (row offset outer, column offset inner), with zeros
    outside the image (the paper pads with zeros near the border).

Windows: the paper ranks features by mutual information and cuts them into groups of at
most three.  Here the grouping is fixed: window 1 = (x, y, centre intensity) when the
position is present; then the remaining patch offsets in raster order, in chunks of 3
(the last chunk may be shorter).
"""
from __future__ import annotations

import numpy as np


def features_from_image(img: np.ndarray, rho: int, with_pos: bool = True) -> np.ndarray:
    """Return the SoA feature matrix F of shape (d, N), float64.  Plain loops over offsets."""
    img = np.asarray(img, dtype=np.float64)
    n1, n2 = img.shape
    N = n1 * n2
    P = 2 * rho + 1
    d = (2 if with_pos else 0) + P * P
    F = np.zeros((d, N), dtype=np.float64)
    rows = np.repeat(np.arange(n1), n2)
    cols = np.tile(np.arange(n2), n1)
    k = 0
    if with_pos:
        F[0] = cols / n2
        F[1] = rows / n1
        k = 2
    for a in range(-rho, rho + 1):
        for b in range(-rho, rho + 1):
            r = rows + a
            c = cols + b
            inside = (r >= 0) & (r < n1) & (c >= 0) & (c < n2)
            col = np.zeros(N)
            col[inside] = img[r[inside], c[inside]]
            F[k] = col
            k += 1
    return F


def window_table(rho: int, with_pos: bool = True):
    """List of windows, each a list of feature column indices (length 1..3)."""
    P = 2 * rho + 1
    base = 2 if with_pos else 0
    centre = base + rho * P + rho
    patch = [base + p for p in range(P * P)]
    wins = []
    if with_pos:
        wins.append([0, 1, centre])
        rest = [c for c in patch if c != centre]
    else:
        rest = patch
    for s in range(0, len(rest), 3):
        wins.append(rest[s:s + 3])
    return wins
