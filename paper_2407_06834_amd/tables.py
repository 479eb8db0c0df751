"""The paper's three measurement protocols (Sec. 5.2-5.4) on seeded synthetic stand-ins.

Images: seeded grayscale images (rectangles and discs, intensities in [0, 1], noise std 0.1) of
sides 64 ... 1024, standing in for the paper's scaled test images.  Features: patches without
position (Sec. 5.2); windows from the mutual-information ranking of the features against the
noisy pixels, as in the paper (7x7 patches: 16 x 3 + 1 = 17 windows; 11x11 patches:
40 x 3 + 1 = 41 windows; `--windows fixed` for the fixed grouping); window weights 1/L as in
the paper; widths sigma / 255 for the paper's 0..255 intensities; FP64 throughout;
alpha = mu / lambda.

  operator    L = 17, sigma = 50: time of the features and their ranking, plan set-up time (scaling, sort,
              schedules, degree vector) and the time of one product W v.
  solution    L = 17, sigma = 50, mu = 1e-2, lambda = 1e-1: PCG from x0 = f, tolerance 1e-7,
              at most 200 iterations; iterations, time, and the condition estimate
              2 alpha max(eta) + 1.
  iterations  L = 41, sigma = 30, mu = 1e-2, lambda in {1, 1e-3, 1e-6, 1e-9}: iterations of CG
              with no preconditioner, P_a and P_b' in the original basis and in the U basis,
              tolerance 1e-8, at most 30 iterations ("x" when not converged).

    python -m paper_2407_06834_amd.tables [--sides 64,128,256,512,1024] [--only iterations]
                                          [--all-lambdas] [--windows mis|fixed]
"""
from __future__ import annotations

import argparse
import json
import time

import torch

from . import nld
from .synth import make_image

LAMBDAS = (1.0, 1e-3, 1e-6, 1e-9)        # the columns the paper prints; --all-lambdas: 10^-i, i = 0..9
COLUMNS = (("none", False), ("jacobi", False), ("l2", False), ("none", True), ("jacobi", True),
           ("l2", True))


def _image(side: int, seed: int = 7):
    _, f = make_image(seed, side, side, 8, 5, 0.1)
    return torch.tensor(f, dtype=torch.float64, device="cuda")


WINDOWS = "mis"


def _windows(F, img, rho):
    if WINDOWS == "mis":
        return nld.mis_window_table(F, img.reshape(-1))[0]
    return nld.window_table(rho, with_pos=False)


def _plan(img, rho: int, sigma255: float, tol: float, times=None, **plan_kw):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F = nld.features_from_image(img, rho, with_pos=False)
    wins = _windows(F, img, rho)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L = len(wins)
    plan = nld.Plan(F, wins, [sigma255 / 255.0] * L, [1.0 / L] * L, matvec_tol=tol, **plan_kw)
    if times is not None:
        plan.degree_vector()
        torch.cuda.synchronize()
        times.update(mis_ms=round((t1 - t0) * 1e3, 2),
                     setup_ms=round((time.perf_counter() - t1) * 1e3, 2))
    return plan, L


def operator_table(sides):
    rows = []
    _plan(_image(sides[0]), 3, 50.0, 1e-7, {})[0].close()     # first-use costs out of the timings
    for side in sides:
        img = _image(side)
        times = {}
        plan, L = _plan(img, 3, 50.0, 1e-7, times)
        v = torch.randn(side * side, dtype=torch.float64, device="cuda")
        out = torch.empty_like(v)
        plan.anova_matvec(v, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 5
        for _ in range(reps):
            plan.anova_matvec(v, out=out)
        torch.cuda.synchronize()
        t_mv = (time.perf_counter() - t0) / reps
        rows.append(dict(side=side, n=side * side, windows=L, **times,
                         product_ms=round(t_mv * 1e3, 3)))
        plan.close()
    return rows


def solution_table(sides):
    rows = []
    alpha = 1e-2 / 1e-1
    for side in sides:
        img = _image(side)
        plan, L = _plan(img, 3, 50.0, 1e-7)
        plan.degree_vector()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, info = plan.pcg_solve(alpha, img.reshape(-1), tol=1e-7, maxit=200, precond=False,
                                 deflate=False)
        torch.cuda.synchronize()
        rows.append(dict(side=side, n=side * side, kappa_est=info["kappa_est"], iters=info["iters"],
                         status=info["status"], solve_ms=round((time.perf_counter() - t0) * 1e3, 2)))
        plan.close()
    return rows


def iterations_table(sides, lambdas=LAMBDAS, plan_kw=None):
    """plan_kw: fixed summation parameters (bandwidth, cutoff); default: chosen for 1e-9."""
    rows = []
    for side in sides:
        img = _image(side)
        plan, L = _plan(img, 5, 30.0, 1e-9, **(plan_kw or {}))
        row = dict(side=side, n=side * side, windows=L)
        for lam in lambdas:
            alpha = 1e-2 / lam
            its = []
            for pre, defl in COLUMNS:
                _, info = plan.pcg_solve(alpha, img.reshape(-1), tol=1e-8, maxit=30, precond=pre,
                                         deflate=defl)
                its.append(info["iters"] if info["status"] == "OK" else "x")
            row[f"lambda={lam:g}"] = its
        rows.append(row)
        plan.close()
    return rows


def markdown(rows, keys):
    out = ["| " + " | ".join(keys) + " |", "|" + "---|" * len(keys)]
    for r in rows:
        out.append("| " + " | ".join(str(r[k]) for k in keys) + " |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sides", default="64,128,256,512,1024")
    ap.add_argument("--only", default="")
    ap.add_argument("--all-lambdas", action="store_true")
    ap.add_argument("--windows", choices=("mis", "fixed"), default="mis")
    args = ap.parse_args()
    global WINDOWS
    WINDOWS = args.windows
    sides = [int(x) for x in args.sides.split(",")]
    nld.load()
    todo = args.only.split(",") if args.only else ["operator", "solution", "iterations"]
    if "operator" in todo:
        r = operator_table(sides)
        print(json.dumps({"operator": r}), flush=True)
        print(markdown(r, ["side", "n", "windows", "mis_ms", "setup_ms", "product_ms"]), flush=True)
    if "solution" in todo:
        r = solution_table(sides)
        print(json.dumps({"solution": r}), flush=True)
        print(markdown(r, ["side", "n", "kappa_est", "iters", "status", "solve_ms"]), flush=True)
    if "iterations" in todo:
        lambdas = tuple(10.0 ** -i for i in range(10)) if args.all_lambdas else LAMBDAS
        r = iterations_table(sides, lambdas)
        print(json.dumps({"iterations": r}), flush=True)
        keys = ["side", "n"] + [f"lambda={lam:g}" for lam in lambdas]
        print("columns per lambda: " + ", ".join(f"{p}{' U' if d else ''}" for p, d in COLUMNS))
        print(markdown(r, keys), flush=True)


if __name__ == "__main__":
    main()
