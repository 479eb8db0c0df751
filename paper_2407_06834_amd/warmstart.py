"""Learned warm start for the deflated Jacobi PCG: training data from the method itself,
training on the GPU, evaluation against plain PCG.

1. Data: seeded synthetic images (20 rectangles, 12 discs) with sides drawn from
   {256, 384, 512, 768, 1024}, noise std ~ U[0.05, 0.2], alpha ~ logU[0.05, 20] and
   sigma_l ~ U[0.05, 0.2] per window; 5x5 patch + position features in 9 windows; each image
   is solved to relative residual 1e-6 by batched PCG (FP32 NFFT).  The pairs (f, u*) and the
   parameters stay in GPU memory.
2. Training: random 128 x 128 crops (same crop of f and u*), batches of 16, mean squared error
   of u0 = f + net(f, cond) against u*, Adam; all layers run in the library's BF16 matrix-core
   kernels.  cond = (log alpha / 3, (log sigma_l - log 0.1) / 0.7) so every input channel is of
   order one.
3. Evaluation: seeded 2048 x 2048 images (alpha, sigma_l drawn as in training), one plan per
   image, PCG from u0 = f (plain) and from the energy-optimal multiple of the network output
   (warm, use_u0 = 3 of pcg_solve), both to relative residual 1e-6 against ||f_perp||; the zero
   start u = mean(f) 1 (no network) is run beside as a control.  Throughput counts plan,
   degree vector, network and PCG.

    python -m paper_2407_06834_amd.warmstart [--train 2000] [--eval 32] [--eval-side 2048]
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np
import torch

from . import nld
from .cnn import WarmStartNet
from .synth import make_image

TRAIN_SIDES = (256, 384, 512, 768, 1024)
# grids are capped at 128 points per dimension (windows with M = 96 oversample by 4/3)
MAX_GRID = 128
# window cutoff of the plans (2m taps per dimension); the product stays within 1e-4 at m = 3
CUTOFF = 3
RHO = 2


# How alpha is drawn.  "strength": the smoothing strength s = alpha * mean(eta) is drawn
# log-uniformly in [0.3, 30] and alpha = s / mean(eta) with eta the plan's zero-diagonal degree,
# so that images of every size are denoised to a similar degree.  "absolute": alpha itself is
# drawn log-uniformly in [0.05, 20]; with unit window weights the degree grows with the number
# of pixels (the patch windows have no position, every pixel of similar patch is a neighbour),
# and at 2048 x 2048 the solution is then the constant image mean(f) 1 to within 1e-4 of
# ||f - mean f||, whatever the network predicts.
ALPHA_RULE = "strength"
ABS_RANGE = (0.05, 20.0)
STRENGTH_RANGE = (0.3, 30.0)


def draw_problem(seed: int, side: int | None = None, sides=TRAIN_SIDES, noise=None):
    rng = np.random.default_rng(seed)
    s = int(rng.choice(sides)) if side is None else side
    nz = float(rng.uniform(0.05, 0.2)) if noise is None else noise
    alpha = float(np.exp(rng.uniform(np.log(ABS_RANGE[0]), np.log(ABS_RANGE[1]))))
    sigma = [float(x) for x in rng.uniform(0.05, 0.2, 9)]
    # the same uniform draw placed in the strength range
    t = (math.log(alpha) - math.log(ABS_RANGE[0])) / math.log(ABS_RANGE[1] / ABS_RANGE[0])
    strength = math.exp(math.log(STRENGTH_RANGE[0]) + t * math.log(STRENGTH_RANGE[1] /
                                                                    STRENGTH_RANGE[0]))
    uc, f = make_image(seed, s, s, 20, 12, nz)
    return dict(side=s, alpha=alpha, strength=strength, sigma=sigma, f=f, seed=seed)


def set_alpha_rule(rule: str):
    global ALPHA_RULE
    if rule not in ("strength", "absolute"):
        raise ValueError(rule)
    ALPHA_RULE = rule


def problem_alpha(p, D: torch.Tensor, wsum: float) -> float:
    """alpha of problem p under ALPHA_RULE; D is the plan's degree vector (FP64, device)."""
    if ALPHA_RULE == "absolute":
        return p["alpha"]
    return p["strength"] / (float(D.mean()) - wsum)


def cond_of(p):
    """Network conditioning: log of the drawn alpha (absolute rule) or strength, and the
    windows' log widths, each scaled to order one."""
    x = p["alpha"] if ALPHA_RULE == "absolute" else p["strength"]
    return [math.log(x) / 3.0] + [(math.log(s) - math.log(0.1)) / 0.7 for s in p["sigma"]]


def generate(seeds, sides=TRAIN_SIDES, batch=16, tol=1e-6, log=None):
    """Solves every problem; returns a list of dicts with GPU tensors f, u and cond."""
    wins = nld.window_table(RHO)
    probs = [draw_problem(s, sides=sides) for s in seeds]
    # batch problems of equal side together
    probs.sort(key=lambda p: p["side"])
    out = []
    for b0 in range(0, len(probs), batch):
        chunk = probs[b0:b0 + batch]
        plans, fs, alphas = [], [], []
        for p in chunk:
            img = torch.tensor(p["f"], dtype=torch.float32, device="cuda")
            F = nld.features_from_image(img, RHO)
            plan = nld.Plan(F, wins, p["sigma"], [1.0] * 9, cutoff=CUTOFF, matvec_tol=1e-4,
                            max_grid=MAX_GRID)
            alphas.append(problem_alpha(p, plan.degree_vector(), 9.0))
            plans.append(plan)
            fs.append(img.reshape(-1))
        us, infos, st = nld.pcg_solve_batched(plans, alphas, fs, tol=tol, maxit=1000)
        for p, f, u, i, pl in zip(chunk, fs, us, infos, plans):
            pl.close()
            if i["status"] != "OK":
                continue
            n = p["side"]
            out.append(dict(f=f.reshape(n, n), u=u.reshape(n, n), side=n, cond=cond_of(p)))
        if log:
            log({"generated": len(out), "of": len(probs)})
    return out


def train(net: WarmStartNet, data, steps=6000, crop=128, batch=16, lr=1e-3, seed=0, log=None):
    g = torch.Generator(device="cpu").manual_seed(seed)
    losses = []
    for it in range(steps):
        idx = torch.randint(len(data), (batch,), generator=g).tolist()
        fb, tb, cb = [], [], []
        for k in idx:
            d = data[k]
            n = d["side"]
            y = int(torch.randint(n - crop + 1, (1,), generator=g))
            x = int(torch.randint(n - crop + 1, (1,), generator=g))
            fb.append(d["f"][y:y + crop, x:x + crop])
            tb.append(d["u"][y:y + crop, x:x + crop])
            cb.append(d["cond"])
        f = torch.stack(fb).contiguous()
        t = torch.stack(tb).contiguous()
        loss = net.loss_grad(f, np.array(cb), t)
        rate = lr if it < 2 * steps // 3 else lr * 0.3
        net.adam_step(lr=rate)
        losses.append(loss)
        if log and (it % 500 == 0 or it == steps - 1):
            log({"step": it, "loss": float(np.mean(losses[-100:]))})
    return losses


def evaluate(net: WarmStartNet, seeds, side=2048, tol=1e-6, log=None):
    wins = nld.window_table(RHO)
    rows = []
    for s in seeds:
        p = draw_problem(s, side=side, noise=0.1)
        img = torch.tensor(p["f"], dtype=torch.float32, device="cuda")
        fv = img.reshape(-1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = nld.features_from_image(img, RHO)
        plan = nld.Plan(F, wins, p["sigma"], [1.0] * 9, cutoff=CUTOFF, matvec_tol=1e-4,
                            max_grid=MAX_GRID)
        alpha = problem_alpha(p, plan.degree_vector(), 9.0)
        torch.cuda.synchronize()
        t_plan = time.perf_counter() - t0
        t0 = time.perf_counter()
        u_plain, i_plain = plan.pcg_solve(alpha, fv, tol=tol, maxit=1000)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        t0 = time.perf_counter()
        u0 = net.predict(img.reshape(1, side, side), np.array([cond_of(p)]))
        torch.cuda.synchronize()
        t_net = time.perf_counter() - t0
        t0 = time.perf_counter()
        u_warm, i_warm = plan.pcg_solve(alpha, fv, u0=u0.reshape(-1), tol=tol, maxit=1000,
                                        u0_guard="scaled")
        torch.cuda.synchronize()
        t_warm = time.perf_counter() - t0
        # control: the zero start u = mean(f) 1 (no network)
        t0 = time.perf_counter()
        _, i_zero = plan.pcg_solve(alpha, fv, u0=torch.full_like(fv, float(fv.mean())),
                                   tol=tol, maxit=1000)
        torch.cuda.synchronize()
        t_zero = time.perf_counter() - t0
        plan.close()
        fperp = float(torch.linalg.vector_norm(fv.double() - fv.double().mean()))
        row = dict(seed=s, alpha=alpha, iters_plain=i_plain["iters"], iters_warm=i_warm["iters"],
                   iters_zero=i_zero["iters"], ms_plan=t_plan * 1e3, ms_plain=t_plain * 1e3,
                   ms_net=t_net * 1e3, ms_warm=t_warm * 1e3, ms_zero=t_zero * 1e3,
                   u0_rejected=i_warm["u0_rejected"],
                   status=(i_plain["status"], i_warm["status"], i_zero["status"]),
                   zero_start_err_rel=float(torch.linalg.vector_norm(u_plain.double() - fv.double().mean())) / fperp,
                   diff_rel=float(torch.linalg.vector_norm((u_warm - u_plain).double())) / fperp,
                   u0_err_rel=float(torch.linalg.vector_norm((u0.reshape(-1) - u_plain).double())) / fperp)
        rows.append(row)
        if log:
            log(row)
    n_px = side * side * len(rows)
    t_p = sum(r["ms_plan"] + r["ms_plain"] for r in rows) / 1e3
    t_w = sum(r["ms_plan"] + r["ms_net"] + r["ms_warm"] for r in rows) / 1e3
    t_z = sum(r["ms_plan"] + r["ms_zero"] for r in rows) / 1e3
    return dict(images=len(rows), side=side,
                iters_plain=float(np.mean([r["iters_plain"] for r in rows])),
                iters_warm=float(np.mean([r["iters_warm"] for r in rows])),
                iters_zero=float(np.mean([r["iters_zero"] for r in rows])),
                mpix_plain=n_px / t_p / 1e6, mpix_warm=n_px / t_w / 1e6, speedup=t_p / t_w,
                mpix_zero=n_px / t_z / 1e6,
                zero_start_err_rel_max=max(r["zero_start_err_rel"] for r in rows),
                ms_net_mean=float(np.mean([r["ms_net"] for r in rows])),
                max_diff_rel=max(r["diff_rel"] for r in rows),
                u0_err_rel_mean=float(np.mean([r["u0_err_rel"] for r in rows])))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--eval", type=int, default=32)
    ap.add_argument("--eval-side", type=int, default=2048)
    ap.add_argument("--save", default="")
    ap.add_argument("--alpha-rule", choices=("strength", "absolute"), default=ALPHA_RULE)
    args = ap.parse_args()
    set_alpha_rule(args.alpha_rule)
    nld.load()

    def log(rec):
        print(json.dumps(rec), flush=True)

    t0 = time.perf_counter()
    data = generate(range(10000, 10000 + args.train), log=log)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    net = WarmStartNet(n_cond=10, seed=0)
    t0 = time.perf_counter()
    losses = train(net, data, steps=args.steps, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    if args.save:
        np.save(args.save, net.params())
    del data
    torch.cuda.empty_cache()
    res = evaluate(net, range(300, 300 + args.eval), side=args.eval_side, log=log)
    res.update(train_solves=args.train, gen_s=round(t_gen, 1), train_steps=args.steps,
               train_s=round(t_train, 1), final_loss=float(np.mean(losses[-200:])))
    print(json.dumps(res), flush=True)
    net.close()


if __name__ == "__main__":
    main()
