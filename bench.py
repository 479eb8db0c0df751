"""Benchmark: NFFT nonlocal denoising of a 512 x 512 synthetic image on one MI355X.

One step = the whole hot path over one image: features (5x5 patch + position, 27 dims),
for each kernel width sigma in {0.05, 0.1, 0.2} a plan over 9 windows of 3 features
(torus scaling, tile sort, Fourier multipliers) and the degree vector, and for each
alpha in {0.1, 1, 10} one deflated Jacobi-PCG solve of (I + alpha L) u = f to relative
residual 1e-6: 9 denoised images per step.  value = 9 * N / step time (Mpixel/s).

Printed as one JSON line; also carries the roofline of the dominant operation (the NFFT
Laplacian product inside CG, timed with HIP events by the library on the solve's stream)
and a CPU baseline (the FP64 NFFT oracle, one product timed on the host, extrapolated).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f32|f64] [--no-cpu-baseline]
                    [--profile-copy]

`roofline.traffic` is the HBM traffic of one product measured with rocprofv3 counters
(FETCH_SIZE and WRITE_SIZE summed over the product's kernels, each scaled by what the counter
reads for a device copy of 256 MiB; --profile-copy runs that copy after the timed steps); it is
reported only while the kernel sources hash to the value recorded with the measurement.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes of one FP32 Laplacian product on this workload, from the rocprofv3 counter runs kept
# in profiles/nfft_laplacian_512_fp32_hbm_traffic.md, valid for the kernel sources of that hash
TRAFFIC = {"sha1": "6418c9213667ee5024d0887cd5988a2525a911c2", "bytes": 834913906}
KERNEL_SOURCES = ("paper_2407_06834_amd/csrc/nfft.hip", "paper_2407_06834_amd/csrc/plan.hip",
                  "paper_2407_06834_amd/csrc/nld_internal.h", "paper_2407_06834_amd/csrc/nld_device.h")


def kernel_sha1() -> str:
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()
N1 = N2 = 512
RHO = 2
SIGMAS = (0.05, 0.1, 0.2)
ALPHAS = (0.1, 1.0, 10.0)
M = 64
TOL = 1e-6


def matvec_bytes(N: int, L: int, t: int, G: int, b: int) -> int:
    """Algorithmic HBM bytes of one Laplacian product: per window, node coordinates and
    node index read twice, the input read, the window result written and read once, the
    grid written by the spread, read and written by each of the t convolution passes and
    read by the gather; plus the epilogue (D in FP64, v in, result out)."""
    per_window = N * (2 * t * b + 8 + 3 * b) + G * b * (2 + 2 * t)
    return L * per_window + N * (8 + 2 * b)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", choices=("f32", "f64"), default="f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-copy", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (asked for --gpus {args.gpus}); "
              "independent solves would shard across GPUs with no communication, but no "
              "multi-GPU path is built or measured here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2407_06834_amd import nld
    from paper_2407_06834_amd.synth import make_image

    nld.load()
    dev = torch.device("cuda:0")
    dtype = torch.float32 if args.dtype == "f32" else torch.float64
    m = 4 if args.dtype == "f32" else 8
    _, f = make_image(1, N1, N2, 20, 12, 0.1)
    img = torch.tensor(f, dtype=dtype, device=dev)
    fv = img.reshape(-1)
    N = N1 * N2
    wins = nld.window_table(RHO)
    L = len(wins)
    u = torch.empty_like(fv)
    stream = torch.cuda.current_stream()

    def step(record):
        F = nld.features_from_image(img, RHO)
        for sigma in SIGMAS:
            plan = nld.Plan(F, wins, [sigma] * L, [1.0] * L, bandwidth=M, cutoff=m)
            for alpha in ALPHAS:
                _, info = plan.pcg_solve(alpha, fv, tol=TOL, maxit=500, out=u, timing=record)
                if record is not None:
                    record.append((sigma, alpha, info))
            plan.close()

    for _ in range(args.warmup):
        step(None)
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(infos)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    if args.profile_copy:
        a = torch.ones(64 * 1024 * 1024, device=dev)   # 256 MiB, the counters' scale reference
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    mpix = 9 * N / (ms_step * 1e-3) / 1e6
    bad = [i for i in infos if i[2]["status"] != "OK"]

    # roofline of the NFFT Laplacian product (dominant operation): algorithmic bytes over the
    # mean duration of the products timed inside the solves of the timed steps
    b = 4 if args.dtype == "f32" else 8
    n_grid = 2 * M
    bytes_mv = matvec_bytes(N, L, 3, n_grid ** 3, b)
    timed = [(i["ms_matvec"], i["matvecs_timed"]) for _, _, i in infos if i["matvecs_timed"] > 0]
    ms_mv = sum(a * k for a, k in timed) / max(1, sum(k for _, k in timed))
    achieved = bytes_mv / (ms_mv * 1e-3) / 1e9 if ms_mv > 0 else 0.0
    iters = [i["iters"] for _, _, i in infos]

    out = {
        "metric": "Mpixel/s denoised at rel-res 1e-6 (plain deflated Jacobi PCG); matvec GB/s",
        "value": round(mpix, 4),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": "512x512 synthetic image (20 rectangles, 12 discs, noise 0.1), 5x5 "
                        "patch + position features in 9 windows of 3, sigma in {0.05,0.1,0.2} x "
                        "alpha in {0.1,1,10}, M=64, n=128, m=%d, deflated Jacobi PCG to 1e-6" % m,
            "pixels_per_step": 9 * N,
            "mean_iters": round(float(np.mean(iters)), 2),
            "solves_not_converged": len(bad),
        },
        "roofline": {
            "kernel": "NFFT Laplacian product (spread, fold, 3 FFT passes, gather, reduce)",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": (round(TRAFFIC["bytes"] / 1e9, 4)
                        if TRAFFIC["sha1"] is not None and TRAFFIC["sha1"] == kernel_sha1() and
                        args.dtype == "f32" else None),
            "traffic_unit": "GB per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "bytes_per_launch": bytes_mv,
            "ms_per_launch": round(ms_mv, 4),
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(f, wins, m, iters)
    print(json.dumps(out), flush=True)


def cpu_baseline(f, wins, m, iters):
    """The FP64 NFFT oracle as it stands: the fast Gauss summation of one window (of the 9) at
    sigma = 0.1 timed on one host core, extrapolated to a solve as 9 windows per product and
    (iterations + 2) products per solve."""
    import numpy as np

    from oracle import nfft as ON
    from oracle.features import features_from_image as o_features

    F = o_features(f, RHO)
    v = np.random.default_rng(0).standard_normal(F.shape[1])
    t0 = time.perf_counter()
    ON.fast_gauss_window(F[wins[1]], v, 0.1, M, 2 * M, m)
    t_win = time.perf_counter() - t0
    t_mv = t_win * len(wins)
    solves = [(it + 2) * t_mv for it in iters]
    sec_per_solve = float(np.mean(solves))
    N = F.shape[1]
    return {"value": round(N / sec_per_solve / 1e6, 6), "unit": "Mpixel/s", "cores": 1,
            "kind": "oracle",
            "sample": "FP64 NFFT fast Gauss summation of one 3-dim window (512x512 nodes, M=64, "
                      "n=128, m=%d) in numpy on one host core, %.1f s; extrapolated to a solve as "
                      "9 windows per product and (iterations + 2) products at the GPU's mean "
                      "iteration count" % (m, t_win)}


if __name__ == "__main__":
    main()
