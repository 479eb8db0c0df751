"""Pins of the oracle's mutual-information ranking (paper Sec. 5, windows of features)."""
import math

import numpy as np
from sklearn.metrics import mutual_info_score

from oracle import mis
from oracle.features import features_from_image
from paper_2407_06834_amd.synth import make_image


def test_score_matches_contingency_library():
    rng = np.random.default_rng(1)
    x = rng.normal(size=5000)
    y = 0.6 * x + rng.normal(size=5000)
    B = 16
    bx, by = mis.bin_index(x, B), mis.bin_index(y, B)
    got = mis.mutual_information(mis.joint_counts(bx, by, B))
    assert abs(got - mutual_info_score(bx, by)) < 1e-12


def test_binning_edges():
    x = np.array([0.0, 0.25, 0.5, 0.999, 1.0])
    assert mis.bin_index(x, 4).tolist() == [0, 1, 2, 3, 3]
    assert mis.bin_index(np.full(7, 3.5), 8).tolist() == [0] * 7       # constant -> one bin


def test_self_information_is_entropy():
    rng = np.random.default_rng(2)
    y = rng.integers(0, 5, size=3000).astype(float)
    B = 5
    by = mis.bin_index(y, B)
    p = np.bincount(by, minlength=B) / y.size
    H = -sum(q * math.log(q) for q in p if q > 0)
    assert abs(mis.mis_scores(y[None], y, B)[0] - H) < 1e-12
    # a bijective relabelling of the bins keeps all the information
    z = 4.0 - y
    assert abs(mis.mis_scores(z[None], y, B)[0] - H) < 1e-12


def test_product_distribution_scores_zero():
    # every pair (a, b) of a 6 x 6 grid exactly 7 times: independent, MI exactly 0
    a, b = np.meshgrid(np.arange(6.0), np.arange(6.0), indexing="ij")
    x = np.repeat(a.ravel(), 7)
    y = np.repeat(b.ravel(), 7)
    assert abs(mis.mis_scores(x[None], y, 6)[0]) < 1e-14


def test_gaussian_closed_form():
    rng = np.random.default_rng(3)
    r = 0.8
    n = 400000
    x = rng.normal(size=n)
    y = r * x + math.sqrt(1 - r * r) * rng.normal(size=n)
    got = mis.mis_scores(x[None], y, 40)[0]
    want = -0.5 * math.log(1 - r * r)
    # binning lowers the estimate slightly, the finite sample raises it; both are small here
    assert abs(got - want) < 0.03


def test_noisier_features_rank_lower():
    rng = np.random.default_rng(4)
    y = rng.uniform(size=20000)
    F = np.stack([y + s * rng.normal(size=y.size) for s in (0.4, 0.0, 0.1, 1.0, 0.02)])
    sc = mis.mis_scores(F, y, 16)
    assert mis.ranking(sc) == [1, 4, 2, 0, 3]


def test_windows_on_patches():
    _, f = make_image(5, 48, 40, 6, 4, 0.1)
    F = features_from_image(f, 3, with_pos=False)
    sc = mis.mis_scores(F, f.ravel())
    wins = mis.mis_windows(sc)
    # 49 features -> 16 windows of three and one of one, each feature once
    assert [len(w) for w in wins] == [3] * 16 + [1]
    assert sorted(sum(wins, [])) == list(range(49))
    # the centre pixel is the target itself: it ranks first
    assert wins[0][0] == 24
    # ties broken by index, scores non-increasing along the ranking
    order = sum(wins, [])
    assert all(sc[order[k]] >= sc[order[k + 1]] for k in range(48))
    F = features_from_image(f, 5, with_pos=False)
    assert len(mis.mis_windows(mis.mis_scores(F, f.ravel()))) == 41


def test_default_bins():
    assert mis.default_bins(16) == 4
    assert mis.default_bins(4096) == 10          # 10^3 <= 1024 < 11^3
    assert mis.default_bins(262144) == 40        # 40^3 = 64000 <= 65536 < 41^3
    assert mis.default_bins(1 << 22) == 64
