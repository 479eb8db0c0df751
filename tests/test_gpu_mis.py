"""GPU parity of the mutual-information feature ranking (paper Sec. 5, windows of features)."""
import numpy as np
import pytest

from gpu_util import torch_gpu
from oracle import mis as OM
from oracle.features import features_from_image as o_features
from paper_2407_06834_amd.synth import make_image

pytestmark = pytest.mark.gpu


def _run(n1, n2, rho, with_pos, dtype, bins, seed=0):
    torch = torch_gpu()
    from paper_2407_06834_amd import nld
    _, f = make_image(seed, n1, n2, 6, 4, 0.1)
    img = torch.tensor(f, dtype=dtype, device="cuda")
    F = nld.features_from_image(img, rho, with_pos=with_pos)
    wins, sc = nld.mis_window_table(F, img.reshape(-1), bins=bins)
    # the oracle bins the same stored values (FP32 values are exact in FP64)
    fo = img.double().cpu().numpy()
    Fo = o_features(fo, rho, with_pos=with_pos)
    B = OM.default_bins(n1 * n2) if bins == 0 else bins
    so = OM.mis_scores(Fo, fo.ravel(), B)
    return np.array(sc), so, wins, OM.mis_windows(so)


def _same_windows(sc, so, wins, wo, tol=1e-12):
    # rankings must agree except between scores closer than the tolerance
    order, oracle = sum(wins, []), sum(wo, [])
    assert sorted(order) == sorted(oracle)
    for k, (a, b) in enumerate(zip(order, oracle)):
        if a != b:
            assert abs(so[a] - so[b]) <= tol, (k, a, b)
    assert [len(w) for w in wins] == [len(w) for w in wo]


@pytest.mark.parametrize("n1,n2,rho,with_pos,bins", [
    (64, 48, 3, False, 0),        # 49 features, auto bins (9), one row block per group
    (37, 53, 1, True, 7),         # ragged, position features, odd bin count
    (300, 280, 5, False, 64),     # 121 features over 61 groups of two, many row blocks
    (129, 131, 2, True, 2),       # two bins
])
@pytest.mark.parametrize("fp64", [True, False])
def test_scores_and_windows_match_oracle(n1, n2, rho, with_pos, bins, fp64):
    torch = torch_gpu()
    sc, so, wins, wo = _run(n1, n2, rho, with_pos, torch.float64 if fp64 else torch.float32, bins)
    np.testing.assert_allclose(sc, so, rtol=0, atol=1e-12)
    _same_windows(sc, so, wins, wo)


def test_special_rows():
    torch = torch_gpu()
    from paper_2407_06834_amd import nld
    rng = np.random.default_rng(3)
    y = rng.uniform(size=5000)
    rows = np.stack([np.full(5000, 0.25), y, 1.0 - y, rng.uniform(size=5000)])
    F = torch.tensor(rows, device="cuda")
    sc = nld.mis_scores(F, torch.tensor(y, device="cuda"), bins=16).cpu().numpy()
    so = OM.mis_scores(rows, y, 16)
    np.testing.assert_allclose(sc, so, rtol=0, atol=1e-12)
    assert sc[0] == 0.0                            # a constant feature carries nothing
    assert abs(sc[1] - sc[2]) < 1e-12              # bin relabelling keeps the information
    # one pixel: every row is constant
    one = nld.mis_scores(torch.ones(3, 1, device="cuda", dtype=torch.float64),
                         torch.ones(1, device="cuda", dtype=torch.float64))
    assert one.cpu().tolist() == [0.0, 0.0, 0.0]


def test_deterministic():
    torch = torch_gpu()
    from paper_2407_06834_amd import nld
    _, f = make_image(9, 200, 200, 6, 4, 0.1)
    img = torch.tensor(f, dtype=torch.float32, device="cuda")
    F = nld.features_from_image(img, 3, with_pos=False)
    a = nld.mis_scores(F, img.reshape(-1))
    b = nld.mis_scores(F, img.reshape(-1))
    assert torch.equal(a, b)
