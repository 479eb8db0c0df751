"""Benchmark: learned warm start vs plain deflated PCG on 2048 x 2048 synthetic images, one MI355X.

One step = one 2048 x 2048 evaluation image (seeded: 20 rectangles, 12 discs, noise 0.1;
sigma_l ~ U[0.05, 0.2] per window and a smoothing strength s ~ logU[0.3, 30] drawn per image,
alpha = s / mean(eta) with eta the plan's zero-diagonal degree; --alpha-rule absolute draws
alpha ~ logU[0.05, 20] instead) through the whole hot path three times:
  plain  features (5x5 patch + position, 27 dims), plan over 9 windows of 3 (torus scaling, tile
         sort, Fourier multipliers, bandwidth per window for a 1e-4 product, window cutoff m = 3,
         grids of at most 128 points per dimension, FP32 with FP64 reductions) and degree vector,
         then deflated Jacobi PCG from u0 = f to relative residual 1e-6;
  warm   the same features, plan and degree vector, the warm-start network (BF16 MFMA kernels)
         predicting u0 from (f, alpha, sigma_l), then the same PCG from the energy-optimal
         multiple b Pi u0 of its output (no extra product; a non-finite u0 is replaced by f).
  zero   control without the network: the same PCG from u = mean(f) 1.
value = Mpixel/s of the warm path (pixels / (plan + network + PCG time)); the plain path's
Mpixel/s and the ratio are in `config`.  Both solves run on the same plan; the plan time counts in
both.  Inputs are uploaded before the timed region.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--weights FILE] [--no-cpu-baseline]
                    [--no-c2] [--profile-copy]

`roofline` is the Laplacian product inside the timed solves (event-timed by the library on the
solve's stream).  `roofline_c2` is the 512 x 512 FP32 product, where the byte model is HBM-bound
(9 windows, M = 64, n = 128, m = 4), timed the same way in a short section after the timed steps
(--no-c2 skips it).  `traffic` fields are HBM bytes from rocprofv3 counters (FETCH_SIZE +
WRITE_SIZE, copy-scaled), reported only while the kernel sources hash to the recorded value.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
SIDE = 2048
RHO = 2
TOL = 1e-6
EVAL_SEED0 = 300
WEIGHTS = os.path.join(ROOT, "paper_2407_06834_amd", "weights", "warmstart_c5.npy")
# grids are capped at 128 points per dimension (windows with M = 96 oversample by 4/3)
MAX_GRID = 128
# window cutoff (2m taps per dimension): on the evaluation images m = 3 keeps the product within
# 1.4e-5 relative L2 (2.6e-5 per entry) of the exact sums, the FP32 target being 1e-4
CUTOFF = 3

# HBM bytes per product from the rocprofv3 counter runs in profiles/ (valid for the kernel
# sources of the recorded hash)
TRAFFIC = {
    # the 512^2 section of the default command
    "c2_512": {"sha1": "67c7509276541b855a3db617b879f069a34afa7c", "bytes": 809209161},
    # the timed images of the default command (seeds 301..304, --steps 4 --warmup 1)
    "c5_2048": {"sha1": "67c7509276541b855a3db617b879f069a34afa7c", "bytes": 5634581115, "cutoff": 3},
}
KERNEL_SOURCES = ("paper_2407_06834_amd/csrc/nfft.hip", "paper_2407_06834_amd/csrc/plan.hip",
                  "paper_2407_06834_amd/csrc/nld_internal.h", "paper_2407_06834_amd/csrc/nld_device.h")


def kernel_sha1() -> str:
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def product_bytes(N: int, grids, b: int = 4) -> int:
    """Algorithmic HBM bytes of one Laplacian product: per 3-D window with n^3 grid cells, node
    coordinates and node index read twice, the input read, the window result written and read
    once, the grid written by the spread, read and written by each of the 3 convolution passes
    and read by the gather; plus the epilogue (D in FP64, v in, result out)."""
    t = 3
    return sum(N * (2 * t * b + 8 + 3 * b) + (n ** 3) * b * (2 + 2 * t) for n in grids) + \
        N * (8 + 2 * b)


def product_flops(N: int, grids, m: int = 4) -> float:
    """Algorithmic FLOPs of one product: 2 flops per tap in spreading and in gathering
    ((2m)^3 taps per node and window), and per window 3 passes of n^2 lines, each a real
    circulant convolution of 5 n log2 n + n flops."""
    import math
    w3 = (2 * m) ** 3
    return float(sum(4 * N * w3 + 3 * n * n * (5 * n * math.log2(n) + n) for n in grids))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--weights", default=WEIGHTS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c2", action="store_true")
    ap.add_argument("--profile-copy", action="store_true")
    ap.add_argument("--cutoff", type=int, default=CUTOFF, help="window cutoff m of the plans")
    ap.add_argument("--alpha-rule", choices=("strength", "absolute"), default="strength",
                    help="strength: alpha = s / mean(eta), s ~ logU[0.3, 30] (default); "
                         "absolute: alpha ~ logU[0.05, 20]")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (asked for --gpus {args.gpus}); "
              "independent solves would shard across GPUs with no communication, but no "
              "multi-GPU path is built or measured here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2407_06834_amd import nld
    from paper_2407_06834_amd.cnn import WarmStartNet
    from paper_2407_06834_amd import warmstart as WS
    from paper_2407_06834_amd.warmstart import cond_of, draw_problem, problem_alpha

    nld.load()
    if not os.path.exists(args.weights):
        raise SystemExit(f"bench.py: network weights not found at {args.weights} "
                         "(python -m paper_2407_06834_amd.warmstart --save FILE writes them)")
    net = WarmStartNet(n_cond=10, seed=0)
    net.set_params(np.load(args.weights))
    wins = nld.window_table(RHO)
    L = len(wins)
    N = SIDE * SIDE

    # inputs: seeded evaluation images, uploaded before the timed region
    total = args.warmup + args.steps
    probs = [draw_problem(EVAL_SEED0 + k, side=SIDE, noise=0.1) for k in range(total)]
    imgs = [torch.tensor(p["f"], dtype=torch.float32, device="cuda") for p in probs]
    WS.set_alpha_rule(args.alpha_rule)
    conds = [np.array([cond_of(p)]) for p in probs]
    torch.cuda.synchronize()

    def step(k, rec):
        p, img = probs[k], imgs[k]
        fv = img.reshape(-1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = nld.features_from_image(img, RHO)
        plan = nld.Plan(F, wins, p["sigma"], [1.0] * L, cutoff=args.cutoff, matvec_tol=1e-4,
                        max_grid=MAX_GRID)
        alpha = problem_alpha(p, plan.degree_vector(), float(L))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, ip = plan.pcg_solve(alpha, fv, tol=TOL, maxit=1000, timing=rec is not None)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        u0 = net.predict(img.reshape(1, SIDE, SIDE), conds[k]).reshape(-1)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        _, iw = plan.pcg_solve(alpha, fv, u0=u0, tol=TOL, maxit=1000,
                               timing=rec is not None, u0_guard="scaled")
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        # control without the network: the zero start u = mean(f) 1
        _, iz = plan.pcg_solve(alpha, fv, u0=torch.full_like(fv, float(fv.mean())), tol=TOL,
                               maxit=1000)
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        grids = [plan.window_info(l).grid for l in range(L)]
        plan.close()
        if rec is not None:
            rec.append(dict(plan=t1 - t0, plain=t2 - t1, net=t3 - t2, warm=t4 - t3, zero=t5 - t4,
                            ip=ip, iw=iw, iz=iz, grids=grids, alpha=alpha))

    for k in range(args.warmup):
        step(k, None)
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.warmup, total):
        step(k, recs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps

    t_plain = sum(r["plan"] + r["plain"] for r in recs)
    t_warm = sum(r["plan"] + r["net"] + r["warm"] for r in recs)
    t_zero = sum(r["plan"] + r["zero"] for r in recs)
    mpix_plain = N * len(recs) / t_plain / 1e6
    mpix_warm = N * len(recs) / t_warm / 1e6
    mpix_zero = N * len(recs) / t_zero / 1e6
    bad = sum(1 for r in recs for i in (r["ip"], r["iw"], r["iz"]) if i["status"] != "OK")

    # dominant kernel: the Laplacian product inside the timed solves
    nb = nf = ms = 0.0
    for r in recs:
        for i in (r["ip"], r["iw"]):
            k = i["matvecs_timed"]
            nb += k * product_bytes(N, r["grids"])
            nf += k * product_flops(N, r["grids"], args.cutoff)
            ms += k * i["ms_matvec"]
    n_prod = sum(i["matvecs_timed"] for r in recs for i in (r["ip"], r["iw"]))
    sha = kernel_sha1()
    tr = TRAFFIC["c5_2048"]
    out = {
        "metric": "Mpixel/s denoised at rel-res 1e-6, learned warm-start vs plain PCG; matvec GB/s",
        "value": round(mpix_warm, 4),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "2048x2048 synthetic images (20 rectangles, 12 discs, noise 0.1; seeds "
                        "%d..%d), %s, sigma_l ~ U[0.05,0.2], 5x5 patch + "
                        "position in 9 windows of 3, FP32 NFFT (m=%d, bandwidth per window for a "
                        "1e-4 product, grids of at most 128^3) with FP64 reductions, deflated "
                        "Jacobi PCG to 1e-6; warm "
                        "start from the 5-layer BF16 network vs plain PCG from u0=f"
                        % (EVAL_SEED0 + args.warmup, EVAL_SEED0 + total - 1,
                           "alpha = s / mean(eta), s ~ logU[0.3,30]" if args.alpha_rule ==
                           "strength" else "alpha ~ logU[0.05,20]", args.cutoff),
            "alpha_mean": round(float(np.mean([r["alpha"] for r in recs])), 8),
            "value_is": "warm-start path: plan + degree + network + PCG",
            "mpix_warm": round(mpix_warm, 4),
            "mpix_plain": round(mpix_plain, 4),
            "speedup_warm_vs_plain": round(t_plain / t_warm, 4),
            "mean_iters_plain": round(float(np.mean([r["ip"]["iters"] for r in recs])), 2),
            "mean_iters_warm": round(float(np.mean([r["iw"]["iters"] for r in recs])), 2),
            "mpix_zero_start": round(mpix_zero, 4),
            "mean_iters_zero_start": round(float(np.mean([r["iz"]["iters"] for r in recs])), 2),
            "zero_start_note": "control without the network: PCG from u = mean(f) 1",
            "u0_rejected": int(sum(r["iw"]["u0_rejected"] for r in recs)),
            "ms_plan_mean": round(1e3 * float(np.mean([r["plan"] for r in recs])), 3),
            "ms_net_mean": round(1e3 * float(np.mean([r["net"] for r in recs])), 3),
            "pixels_per_step": N,
            "solves_not_converged": bad,
        },
        "roofline": {
            "kernel": "NFFT Laplacian product at 2048x2048 (spread, fold, FFT passes, gather, "
                      "reduce), inside the timed solves",
            "bound": "alu",
            "achieved": round(nf / (ms * 1e-3) / 1e12, 3) if ms > 0 else 0.0,
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(nf / (ms * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS, 4) if ms > 0 else 0.0,
            "traffic": (round(tr["bytes"] / 1e9, 4) if tr["sha1"] == sha and tr["bytes"] and
                        (args.steps, args.warmup) == (4, 1) and args.alpha_rule == "strength"
                        and args.cutoff == tr["cutoff"] else None),
            "traffic_unit": "GB per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "flops_per_launch": round(nf / max(1, n_prod)),
            "bytes_per_launch": round(nb / max(1, n_prod)),
            "hbm_gbs": round(nb / (ms * 1e-3) / 1e9, 1) if ms > 0 else 0.0,
            "hbm_frac": round(nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if ms > 0 else 0.0,
            "ms_per_launch": round(ms / max(1, n_prod), 4),
            "launches": n_prod,
        },
    }
    if not args.no_c2:
        out["roofline_c2"] = c2_product(nld, torch, sha)
    if args.profile_copy:
        a = torch.ones(64 * 1024 * 1024, device="cuda")   # 256 MiB, the counters' scale reference
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(probs[args.warmup], out["config"], args.cutoff)
    net.close()
    print(json.dumps(out), flush=True)


def c2_product(nld, torch, sha):
    """The 512 x 512 FP32 product, where the byte model is HBM-bound (image seed 1: 20 rectangles,
    12 discs, noise 0.1; 9 windows, sigma 0.1, M = 64, n = 128, m = 4), event-timed by the
    library inside two deflated PCG solves (alpha = 1, tol 1e-6)."""
    from paper_2407_06834_amd.synth import make_image
    _, f = make_image(1, 512, 512, 20, 12, 0.1)
    img = torch.tensor(f, dtype=torch.float32, device="cuda")
    F = nld.features_from_image(img, RHO)
    wins = nld.window_table(RHO)
    plan = nld.Plan(F, wins, [0.1] * 9, [1.0] * 9, bandwidth=64, cutoff=4)
    plan.pcg_solve(1.0, img.reshape(-1), tol=TOL, maxit=500)
    _, info = plan.pcg_solve(1.0, img.reshape(-1), tol=TOL, maxit=500, timing=True)
    plan.close()
    N = 512 * 512
    bts = product_bytes(N, [128] * 9)
    ms = info["ms_matvec"]
    tr = TRAFFIC["c2_512"]
    return {"kernel": "NFFT Laplacian product at 512x512 (9 windows, M=64, n=128, m=4, FP32)",
            "bound": "hbm", "achieved": round(bts / (ms * 1e-3) / 1e9, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(bts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": (round(tr["bytes"] / 1e9, 4) if tr["sha1"] == sha else None),
            "traffic_unit": "GB per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "bytes_per_launch": bts, "ms_per_launch": round(ms, 4),
            "launches": info["matvecs_timed"], "timed": "after the timed steps"}


def cpu_baseline(p, cfg, m):
    """The FP64 NFFT oracle as it stands, on a bounded sample: the fast Gauss summation of one
    3-dim window (window 2 of 9, that image's sigma) over the central 128x128 and 512x512 crops
    of the first timed image's features, M = 64, n = 128, cutoff m as in the timed plans, median of 3 on one thread and
    on all host threads; the time per node-window is fitted as a + b N on the two crops and
    extrapolated to a solve: 9 windows x 2048^2 nodes per product, (mean iterations + 2)
    products per solve (plain path)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import nfft as ON
    from oracle.features import features_from_image as o_features

    f = p["f"]
    c0 = SIDE // 2
    crops = {}
    for h in (128, 512):
        sub = f[c0 - h // 2:c0 + h // 2, c0 - h // 2:c0 + h // 2]
        crops[h] = o_features(sub, RHO)[[3, 4, 5]]      # window 2 of the fixed grouping
    sig = p["sigma"][1]
    rng = np.random.default_rng(0)

    def med(threads):
        ts = {}
        with threadpool_limits(limits=threads):
            for h, X in crops.items():
                v = rng.standard_normal(X.shape[1])
                runs = []
                for _ in range(3):
                    t0 = time.perf_counter()
                    ON.fast_gauss_window(X, v, sig, 64, 128, m)
                    runs.append(time.perf_counter() - t0)
                ts[h] = statistics.median(runs)
        n1, n2 = 128 * 128, 512 * 512
        b = (ts[512] - ts[128]) / (n2 - n1)
        a = ts[128] - b * n1
        t_prod = 9 * (a + b * SIDE * SIDE)
        t_solve = (cfg["mean_iters_plain"] + 2) * t_prod
        return SIDE * SIDE / t_solve / 1e6, ts

    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    v1, ts1 = med(1)
    vall, tsall = med(ncores)
    return {"value": round(vall, 7), "unit": "Mpixel/s", "cores": ncores, "kind": "oracle",
            "value_1core": round(v1, 7), "cpu": cpu_model(),
            "sample": "FP64 NFFT oracle (numpy): one window's fast Gauss summation on the central "
                      "128^2 and 512^2 crops, M=64, n=128, m=%d, median of 3 (%.2f s / %.2f s on 1 "
                      "thread, %.2f s / %.2f s on %d); a + b N fit extrapolated to 9 windows x "
                      "2048^2 nodes per product and (plain mean iterations + 2) products per solve"
                      % (m, ts1[128], ts1[512], tsall[128], tsall[512], ncores)}


if __name__ == "__main__":
    main()
