"""FP64 NumPy oracle of the mutual-information feature ranking that forms the windows (paper
Sec. 5, generation of the windows of features; test infrastructure only).

The paper ranks the patch features by their mutual information score (MIS) against the noisy
pixel values f and cuts the ranking into L = ceil(d / 3) windows of at most three features.  It
does not name its estimator.  Reading used here: the plug-in estimate from a joint histogram.

  * Binning: a variable x with minimum lo and maximum hi goes to bin
        b(x) = min(B - 1, floor((x - lo) * s)),  s = B / (hi - lo)  (s = 0 when hi = lo),
    every operation in IEEE double, so that the bin of a value is a fixed decision.
  * Score of feature j against the target y (counts n_ab of the pairs (b(F_j,i), b(y_i)),
    marginals n_a, n_b, N pairs), natural logarithm:
        MIS_j = sum over n_ab > 0 of (n_ab / N) log(N n_ab / (n_a n_b)).
  * Ranking: decreasing score, ties by increasing feature index; windows are consecutive
    triples of the ranking (the last one holds the remainder).
  * Default number of bins: the largest B with B^3 <= N / 4, clamped to [4, 64].

Pins (tests): the score equals scikit-learn's contingency-table mutual information of the same
bin labels; MIS(y, y) equals the entropy of the binned y; an exact product distribution scores
0; a bijective relabelling keeps the entropy; a bivariate Gaussian approaches
-log(1 - r^2) / 2; features of growing noise rank in order; the window counts of the paper.
"""
from __future__ import annotations

import numpy as np


def default_bins(N: int) -> int:
    B = 1
    while (B + 1) ** 3 <= N // 4:
        B += 1
    return int(min(64, max(4, B)))


def bin_index(x: np.ndarray, B: int) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    lo, hi = float(x.min()), float(x.max())
    s = B / (hi - lo) if hi > lo else 0.0
    b = np.floor((x - lo) * s).astype(np.int64)
    return np.minimum(b, B - 1)


def joint_counts(bx: np.ndarray, by: np.ndarray, B: int) -> np.ndarray:
    c = np.zeros((B, B), dtype=np.int64)
    np.add.at(c, (bx, by), 1)
    return c


def mutual_information(counts: np.ndarray) -> float:
    N = counts.sum()
    na = counts.sum(axis=1)
    nb = counts.sum(axis=0)
    mi = 0.0
    for a in range(counts.shape[0]):
        for b in range(counts.shape[1]):
            c = counts[a, b]
            if c > 0:
                mi += c / N * np.log(N * c / (na[a] * nb[b]))
    return float(mi)


def mis_scores(F: np.ndarray, y: np.ndarray, B: int | None = None) -> np.ndarray:
    """Scores of the feature rows F (d, N) against the target y (N)."""
    F = np.asarray(F, dtype=np.float64)
    B = default_bins(F.shape[1]) if B is None else B
    by = bin_index(y, B)
    return np.array([mutual_information(joint_counts(bin_index(F[j], B), by, B))
                     for j in range(F.shape[0])])


def ranking(scores) -> list[int]:
    return sorted(range(len(scores)), key=lambda j: (-float(scores[j]), j))


def mis_windows(scores, size: int = 3) -> list[list[int]]:
    order = ranking(scores)
    return [order[s:s + size] for s in range(0, len(order), size)]
