"""The allocation-free entry point mis_scores_noalloc against mis_scores (C ABI, GPU): equal
scores bit for bit on two calls in a row, the second on a smaller input, and the size limit of
its static scratch rejected on the host."""
import numpy as np
import pytest

from gpu_util import torch_gpu

pytestmark = pytest.mark.gpu


def _inputs(torch, nld, seed, n1, n2, rho, dtype):
    from paper_2407_06834_amd.synth import make_image
    _, f = make_image(seed, n1, n2, 5, 3, 0.1)
    img = torch.tensor(f, dtype=dtype, device="cuda")
    return nld.features_from_image(img, rho), img.reshape(-1).contiguous()


@pytest.mark.parametrize("dtype_name", ["float32", "float64"])
def test_noalloc_scores_equal_allocating_scores_twice(dtype_name):
    torch = torch_gpu()
    from paper_2407_06834_amd import nld
    dtype = getattr(torch, dtype_name)
    # first a larger problem (49 + 2 features, 16 bins), then a smaller one (9 + 2, 7 bins): the
    # second call must not see the first one's histograms
    for seed, n1, n2, rho, bins in ((61, 96, 80, 3, 16), (62, 33, 21, 1, 7)):
        F, y = _inputs(torch, nld, seed, n1, n2, rho, dtype)
        ref = nld.mis_scores(F, y, bins)
        out = torch.full((F.shape[0],), float("nan"), dtype=torch.float64, device="cuda")
        got = nld.mis_scores_noalloc(F, y, bins, out=out)
        torch.cuda.synchronize()
        assert got.data_ptr() == out.data_ptr()
        assert torch.equal(got, ref), (seed, (got - ref).abs().max().item())
        assert torch.isfinite(got).all() and (got >= -1e-12).all()


def test_noalloc_default_bins_and_size_limit():
    torch = torch_gpu()
    from paper_2407_06834_amd import nld
    F, y = _inputs(torch, nld, 63, 64, 64, 2, torch.float32)
    assert torch.equal(nld.mis_scores_noalloc(F, y), nld.mis_scores(F, y))
    # 4 (d + 1) + d B^2 words must fit 2^20: d = 27 at B = 64 needs 110704 words (fits);
    # 300 features at 64 bins need 1230004 words: rejected before any launch
    big = torch.zeros((300, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(nld.NldError) as e:
        nld.mis_scores_noalloc(big, torch.zeros(64, dtype=torch.float32, device="cuda"), 64)
    assert e.value.status == nld.NLD_E_INVAL and "scratch" in str(e.value)
