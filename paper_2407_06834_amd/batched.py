"""Batched denoising of many images of uneven sizes on one GPU.

Workload: `count` seeded synthetic images (20 rectangles, 12 discs, noise std 0.1) with sides
drawn uniformly from {128, 256, 384, 512, 768, 1024}, each with its own alpha ~ logU[0.05, 20]
and window widths sigma_l ~ U[0.05, 0.2]; 3x3 patch + position features in 4 windows; FP32
NFFT with FP64 CG reductions; deflated Jacobi PCG to relative residual 1e-6.

The NFFT cutoff, oversampling and 3-D tile extent come from the autotuner (one sample image
per side, timed before the measured run); the bandwidth of every window comes from the
plan's error model.  The measured run builds every plan (features, scaling, sort,
schedules) and then solves all images with one pcg_solve_batched call.  Reported: aggregate
Mpixel/s = sum of N over the wall time of plans + solves, and p50 / p99 of the per-solve
latency, measured from the start of the run to the moment the solve was seen finished.  The
same plans solved one after another with pcg_solve give the sequential baseline.

    python -m paper_2407_06834_amd.batched [--count 64] [--no-sequential]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

from . import autotune, nld
from .synth import make_image

SIDES = (128, 256, 384, 512, 768, 1024)


def make_problems(count: int = 64, seed0: int = 100):
    probs = []
    for k in range(count):
        rng = np.random.default_rng(seed0 + k)
        side = int(rng.choice(SIDES))
        alpha = float(np.exp(rng.uniform(np.log(0.05), np.log(20.0))))
        sigma = [float(x) for x in rng.uniform(0.05, 0.2, 4)]
        _, f = make_image(seed0 + k, side, side, 20, 12, 0.1)
        probs.append(dict(side=side, alpha=alpha, sigma=sigma, f=f))
    return probs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-sequential", action="store_true")
    args = ap.parse_args()
    nld.load()
    dtype = torch.float32
    probs = make_problems(args.count)
    for p in probs:
        p["img"] = torch.tensor(p["f"], dtype=dtype, device="cuda")
    windows = nld.window_table(1)
    ones = [1.0] * len(windows)

    # ---- autotuning: one sample per side
    t0 = time.perf_counter()
    samples, counts = {}, {}
    for p in probs:
        key = str(p["side"])
        counts[key] = counts.get(key, 0) + 1
        if key not in samples:
            samples[key] = (p["img"], p["sigma"], ones)
    tuner, m, picks = autotune.tune_classes(samples, counts, dtype=dtype)
    t_tune = time.perf_counter() - t0
    print(json.dumps({"autotune_s": round(t_tune, 2), "cutoff": m, "picks": picks}), flush=True)

    def build_plans():
        plans = []
        for p in probs:
            F = nld.features_from_image(p["img"], 1)
            kw = picks[str(p["side"])]
            try:
                plans.append(nld.Plan(F, windows, p["sigma"], ones, **kw))
            except nld.NldError:
                # a narrower kernel than the class sample's needs a larger M: oversampling 2
                plans.append(nld.Plan(F, windows, p["sigma"], ones, **{**kw, "oversampling": 2.0}))
        return plans

    # ---- warm-up (kernel loading), then the measured batched run
    warm = build_plans()[:2]
    nld.pcg_solve_batched(warm, [p["alpha"] for p in probs[:2]],
                          [p["img"].reshape(-1) for p in probs[:2]], tol=args.tol)
    for w in warm:
        w.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plans = build_plans()
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    fs = [p["img"].reshape(-1) for p in probs]
    us, infos, st = nld.pcg_solve_batched(plans, [p["alpha"] for p in probs], fs, tol=args.tol,
                                          maxit=1000)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    total_px = sum(p["side"] ** 2 for p in probs)
    lat = np.array([t_plan * 1e3 + i["ms_solve"] for i in infos])
    out = {
        "workload": f"{args.count} images, sides U{{128..1024}}, alpha logU[0.05,20], sigma_l "
                    "U[0.05,0.2], 3x3 patch + position in 4 windows, FP32 NFFT, FP64 CG "
                    f"reductions, tol {args.tol}",
        "pixels": total_px,
        "mpixel_per_s": round(total_px / t_all / 1e6, 3),
        "wall_ms": round(t_all * 1e3, 1),
        "plans_ms": round(t_plan * 1e3, 1),
        "solve_ms": round((t_all - t_plan) * 1e3, 1),
        "latency_p50_ms": round(float(np.percentile(lat, 50)), 1),
        "latency_p99_ms": round(float(np.percentile(lat, 99)), 1),
        "iters_mean": round(float(np.mean([i["iters"] for i in infos])), 2),
        "iters_max": int(max(i["iters"] for i in infos)),
        "not_converged": sum(i["status"] != "OK" for i in infos),
        "cutoff": m,
    }
    if not args.no_sequential:
        # the same plans solved one at a time (plans reused: only the solves are repeated)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        seq_lat = []
        maxdiff = 0.0
        for p, plan, f, u in zip(probs, plans, fs, us):
            u1, info = plan.pcg_solve(p["alpha"], f, tol=args.tol, maxit=1000)
            seq_lat.append((time.perf_counter() - t1) * 1e3)
            maxdiff = max(maxdiff, float(torch.max(torch.abs(u1 - u))))
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t1
        out["sequential_solve_ms"] = round(t_seq * 1e3, 1)
        out["sequential_mpixel_per_s_incl_plans"] = round(total_px / (t_seq + t_plan) / 1e6, 3)
        out["sequential_latency_p50_ms"] = round(float(np.percentile(np.array(seq_lat) + t_plan * 1e3, 50)), 1)
        out["sequential_latency_p99_ms"] = round(float(np.percentile(np.array(seq_lat) + t_plan * 1e3, 99)), 1)
        out["batched_vs_sequential_max_abs_diff"] = maxdiff
    print(json.dumps(out), flush=True)
    for plan in plans:
        plan.close()


if __name__ == "__main__":
    main()
