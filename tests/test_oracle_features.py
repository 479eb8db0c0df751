"""Pins of the oracle's feature construction and window grouping (paper Sec. 5)."""
import os

import numpy as np

from oracle.features import features_from_image, window_table

GOLD = os.path.join(os.path.dirname(__file__), "golden", "features_2x3_rho1.txt")


def test_features_hand_worked_example():
    img = np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0]])
    F = features_from_image(img, 1)
    assert F.shape == (11, 6)
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        head, *vals = line.split()
        i = int(head.split("=")[1])
        np.testing.assert_allclose(F[:, i], np.array(vals, dtype=float), rtol=0, atol=1e-15)


def test_window_counts_match_paper_and_configs():
    # paper Sec. 5.2: 49 patch features (7x7) -> 16 windows of three and one of one
    w = window_table(3, with_pos=False)
    assert sorted(len(x) for x in w) == [1] + [3] * 16
    # 3x3 patch + position: 11 dims in windows of 3,3,3,2
    assert [len(x) for x in window_table(1)] == [3, 3, 3, 2]
    # 5x5 patch + position: 27 dims in 9 windows of 3
    assert [len(x) for x in window_table(2)] == [3] * 9
    # every feature used exactly once
    for rho in (1, 2, 3):
        cols = sorted(c for x in window_table(rho) for c in x)
        assert cols == list(range(2 + (2 * rho + 1) ** 2))


def test_first_window_is_position_and_centre():
    w = window_table(2)
    assert w[0] == [0, 1, 2 + 2 * 5 + 2]
