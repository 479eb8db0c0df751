"""Empirical autotuner for the NFFT parameters of a workload class.

For every class (an image side with its sample image and kernel widths) the tuner builds
candidate plans over the grid of

    cutoff m           {3, 4, 5} (FP32) or {5, 6, 7, 8} (FP64)
    oversampling       {2, 4}  (grid n = next power of two >= oversampling * M, n <= 256)
    3-D tile extent    {8, 16}

with the bandwidth M of every window left to the plan's error model (it depends on sigma_l and
the data range, not on timing).  Each candidate is measured twice on the GPU: the mean time of
one Laplacian product (HIP events on the current stream) and its relative error against the
library's own high-accuracy product (FP64, m = 8, the same M) on a seeded random vector.
Candidates above the error target are discarded.  Plans solved together in one batch share
one cutoff, so the tuner first picks the m that minimises the summed time of all classes
(weighted by how many plans each class has), then the fastest (oversampling, tile) per class
at that m.

No reference implementation is involved: accuracy is judged against the library's own product
at the highest cutoff, which differs from the exact summation only by the bandwidth
truncation that the error model already bounds.
"""
from __future__ import annotations

import dataclasses
import json
import math

import torch

from . import nld


@dataclasses.dataclass
class Candidate:
    cutoff: int
    oversampling: float
    tile: int
    ms: float
    err: float


def _time_product(plan: nld.Plan, v: torch.Tensor, reps: int = 8) -> float:
    out = torch.empty_like(v)
    for _ in range(2):
        plan.laplacian_matvec(v, out=out)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        plan.laplacian_matvec(v, out=out)
    stop.record()
    stop.synchronize()
    return start.elapsed_time(stop) / reps


class Autotuner:
    def __init__(self, dtype=torch.float32, matvec_tol: float | None = None, rho: int = 1,
                 reps: int = 8):
        self.dtype = dtype
        self.matvec_tol = matvec_tol if matvec_tol is not None else (
            1e-4 if dtype == torch.float32 else 1e-6)
        self.rho = rho
        self.reps = reps
        self.windows = nld.window_table(rho)
        self.results: dict[str, list[Candidate]] = {}

    def cutoffs(self):
        return (3, 4, 5) if self.dtype == torch.float32 else (5, 6, 7, 8)

    def measure_class(self, key: str, img: torch.Tensor, sigma, weight) -> list[Candidate]:
        """All feasible candidates of one class, with time and error."""
        L = len(self.windows)
        F = nld.features_from_image(img.to(self.dtype), self.rho)
        F64 = nld.features_from_image(img.to(torch.float64), self.rho)
        g = torch.Generator(device="cpu").manual_seed(12345)
        v64 = torch.randn(F.shape[1], generator=g, dtype=torch.float64).cuda()
        v = v64.to(self.dtype)
        # bandwidths from the plan's error model (independent of m, n and the tile)
        probe = nld.Plan(F, self.windows, sigma, weight, matvec_tol=self.matvec_tol, cutoff=2)
        M = [probe.window_info(l).bandwidth for l in range(L)]
        probe.close()
        ref = nld.Plan(F64, self.windows, sigma, weight, win_bandwidth=M, bandwidth=M[0],
                       cutoff=8, matvec_tol=self.matvec_tol)
        y_ref = ref.anova_matvec(v64)
        ref.close()
        nrm = float(torch.linalg.vector_norm(y_ref))
        out = []
        for m in self.cutoffs():
            for os_ in (2.0, 4.0):
                if max(2 ** math.ceil(math.log2(os_ * Mi)) for Mi in M) > 256:
                    continue
                for tile in (8, 16):
                    try:
                        p = nld.Plan(F, self.windows, sigma, weight, win_bandwidth=M,
                                     bandwidth=M[0], cutoff=m, oversampling=os_, tile=tile,
                                     matvec_tol=self.matvec_tol)
                    except nld.NldError:
                        continue
                    y = p.anova_matvec(v).to(torch.float64)
                    err = float(torch.linalg.vector_norm(y - y_ref)) / max(nrm, 1e-300)
                    ms = _time_product(p, v, self.reps)
                    p.close()
                    out.append(Candidate(m, os_, tile, ms, err))
        self.results[key] = out
        return out

    def choose(self, counts: dict[str, int]):
        """counts: plans per measured class.  Returns (m, {key: plan kwargs})."""
        best_m, best_total = None, math.inf
        for m in self.cutoffs():
            total = 0.0
            for key, cnt in counts.items():
                ok = [c for c in self.results[key] if c.cutoff == m and c.err <= self.matvec_tol]
                if not ok:
                    total = math.inf
                    break
                total += cnt * min(c.ms for c in ok)
            if total < best_total:
                best_m, best_total = m, total
        if best_m is None:
            raise RuntimeError("autotune: no candidate meets the error target")
        picks = {}
        for key in counts:
            ok = [c for c in self.results[key] if c.cutoff == best_m and c.err <= self.matvec_tol]
            c = min(ok, key=lambda c: c.ms)
            picks[key] = dict(cutoff=c.cutoff, oversampling=c.oversampling, tile=c.tile,
                              matvec_tol=self.matvec_tol)
        return best_m, picks

    def report(self) -> str:
        return json.dumps({k: [dataclasses.asdict(c) for c in v] for k, v in self.results.items()})


def tune_classes(samples: dict[str, tuple], counts: dict[str, int], dtype=torch.float32,
                 matvec_tol: float | None = None, rho: int = 1):
    """samples: key -> (image tensor (n1, n2), sigma list, weight list).  Returns
    (tuner, m, picks) with picks[key] the keyword arguments of nld.Plan for that class."""
    tuner = Autotuner(dtype=dtype, matvec_tol=matvec_tol, rho=rho)
    for key, (img, sigma, weight) in samples.items():
        tuner.measure_class(key, img, sigma, weight)
    m, picks = tuner.choose(counts)
    return tuner, m, picks


__all__ = ["Autotuner", "Candidate", "tune_classes"]
