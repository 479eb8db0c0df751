"""The C ABI library loads, exports every entry point declared in include/nld.h, and rejects
invalid arguments on the host before any launch (no GPU needed for these paths)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("nld.h", "nld_cnn.h")]
LIB = os.path.join(ROOT, "paper_2407_06834_amd", "libnld.so")


def _declared():
    text = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"^(?:nld_status|const char\*|int64_t)\s+(\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2407_06834_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert {"nfft_plan", "nfft_plan_destroy", "anova_matvec", "laplacian_matvec", "pcg_solve",
            "degree_vector", "features_from_image", "nld_last_error"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    from paper_2407_06834_amd import cnn, nld
    assert set(nld.SYMBOLS) <= set(names)
    assert set(cnn.SYMBOLS) <= set(names)
    assert {"cnn_create", "cnn_predict", "cnn_loss_grad", "cnn_adam_step"} <= set(names)


def test_invalid_arguments_rejected_on_host(lib):
    from paper_2407_06834_amd import nld
    L = nld.load()
    err = lambda: L.nld_last_error().decode()
    h = ctypes.c_void_p()
    wd = (ctypes.c_int32 * 1)(3)
    wf = (ctypes.c_int32 * 3)(0, 1, 2)
    sg = (ctypes.c_double * 1)(0.1)
    wt = (ctypes.c_double * 1)(1.0)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    base = dict(n_windows=1, win_dim=wd, win_feat=wf, sigma=sg, weight=wt, bandwidth=64,
                win_bandwidth=None, cutoff=4, oversampling=2.0, matvec_tol=1e-6, prec=0)

    def plan(N=100, d=3, **kw):
        desc = nld.KernelDesc(**{**base, **kw})
        return L.nfft_plan(ctypes.byref(h), fake, N, d, ctypes.byref(desc), None)

    assert plan(N=0) == nld.NLD_E_INVAL and "N" in err()
    assert plan(d=2) == nld.NLD_E_INVAL and "feature index" in err()
    assert plan(bandwidth=63) == nld.NLD_E_INVAL
    assert plan(cutoff=9) == nld.NLD_E_INVAL
    assert plan(oversampling=1.0) == nld.NLD_E_INVAL
    assert plan(max_grid=100) == nld.NLD_E_INVAL and "max_grid" in err()
    assert plan(prec=7) == nld.NLD_E_INVAL
    assert plan(tile=12) == nld.NLD_E_INVAL and "tile" in err()
    assert plan(n_windows=0) == nld.NLD_E_INVAL
    sg[0] = -1.0
    assert plan() == nld.NLD_E_INVAL and "sigma" in err()
    sg[0] = 0.1
    wt[0] = float("nan")
    assert plan() == nld.NLD_E_INVAL and "weight" in err()
    wt[0] = 1.0
    wd[0] = 4
    assert plan() == nld.NLD_E_INVAL and "dimension" in err()
    wd[0] = 3
    assert h.value is None
    assert L.nfft_plan_destroy(None) == nld.NLD_E_INVAL
    opts = nld.PcgOpts(1e-6, 10, 0, 1, 1, 0, 0)
    info = nld.PcgInfo()
    assert L.pcg_solve(None, 1.0, fake, fake, ctypes.byref(opts), ctypes.byref(info), None) == nld.NLD_E_INVAL
    assert L.features_from_image(fake, 0, 4, 1, 1, 0, fake, None) == nld.NLD_E_INVAL
    assert L.features_from_image(fake, 4, 4, -1, 1, 0, fake, None) == nld.NLD_E_INVAL
    assert L.anova_matvec(None, fake, fake, None) == nld.NLD_E_INVAL
    one = (ctypes.c_double * 1)(1.0)
    ptrs = (ctypes.c_void_p * 1)(0x1000)
    infos = (nld.PcgInfo * 1)()
    assert L.pcg_solve_batched(ptrs, one, ptrs, ptrs, 0, ctypes.byref(opts), infos, None) == nld.NLD_E_INVAL
    nulls = (ctypes.c_void_p * 1)(None)
    assert L.pcg_solve_batched(nulls, one, ptrs, ptrs, 1, ctypes.byref(opts), infos, None) == nld.NLD_E_INVAL
    assert "null" in err()
    assert L.nfft_plan_update_kernel(None, one, one, None) == nld.NLD_E_INVAL
    grad = (ctypes.c_double * 3)()
    assert L.adjoint_solve(None, 1.0, fake, fake, fake, fake, grad, ctypes.byref(opts),
                           ctypes.byref(info), None) == nld.NLD_E_INVAL
    assert L.mis_scores(None, 10, 2, fake, 0, 0, fake, None) == nld.NLD_E_INVAL and "null" in err()
    assert L.mis_scores(fake, 0, 2, fake, 0, 0, fake, None) == nld.NLD_E_INVAL
    assert L.mis_scores(fake, 10, 0, fake, 0, 0, fake, None) == nld.NLD_E_INVAL
    assert L.mis_scores(fake, 10, 2, fake, 0, 1, fake, None) == nld.NLD_E_INVAL and "bins" in err()
    assert L.mis_scores(fake, 10, 2, fake, 0, 65, fake, None) == nld.NLD_E_INVAL
    assert L.mis_scores(fake, 10, 2, fake, 3, 8, fake, None) == nld.NLD_E_INVAL
    from paper_2407_06834_amd import cnn
    C = cnn._lib()
    assert C.cnn_create(None, 2, 0) == nld.NLD_E_INVAL
    hh = ctypes.c_void_p()
    assert C.cnn_create(ctypes.byref(hh), 40, 0) == nld.NLD_E_INVAL and hh.value is None
    assert C.cnn_param_count(None) == -1
    assert C.cnn_predict(None, fake, fake, 1, 4, 4, fake, None) == nld.NLD_E_INVAL
