"""Write the FP64 reference solution of a 256 x 256 denoising problem, from the oracle alone.

    python tests/golden/make_solution_256.py      # about 20-30 minutes on 8 host cores

Problem (the 512 x 512 benchmark configuration's recipe at a side the exact operator still
handles): the seeded synthetic image of 20 rectangles and 12 discs with noise 0.1, 5 x 5
patch + position features in 9 windows of 3 (fixed grouping), sigma_l = 0.1, weights 1,
alpha = 1.  The system (I + alpha L) u = f of paper Sec. 2.6 is solved with the exact
kernel: every product W v is the direct O(N^2) sum of the ANOVA kernel (oracle.csum, FP64),
D = W 1, eta = D - sum_l w_l, and the solver is the paper-literal deflated Jacobi PCG in the
Helmert basis (Sec. 4.2, 4.3.1, 5.4; oracle.solve.pcg_ubasis) run to relative residual 1e-12,
so the stored u is within 1e-12 ||f - mean f|| of the exact solution (||A^-1|| <= 1).

Writes solution_256_s01_a1.npy (u, float64, raster order) and solution_256_s01_a1.txt
(parameters, iterations, residuals).  Uses nothing but oracle/ and the input recipe.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import csum  # noqa: E402
from oracle import solve as OS  # noqa: E402
from oracle.features import features_from_image, window_table  # noqa: E402
from paper_2407_06834_amd.synth import make_image  # noqa: E402

SIDE = 256
SEED = 1
RHO = 2
SIGMA = 0.1
ALPHA = 1.0
TOL = 1e-12
NAME = "solution_256_s01_a1"


def problem():
    """The inputs both sides start from: noisy image, features, windows, widths, weights."""
    _, f = make_image(SEED, SIDE, SIDE, 20, 12, 0.1)
    F = features_from_image(f, RHO)
    wins = window_table(RHO)
    L = len(wins)
    return f, F, wins, [SIGMA] * L, [1.0] * L


def main():
    f, F, wins, sig, wt = problem()
    N = F.shape[1]
    rows = np.arange(N, dtype=np.int64)
    t0 = time.time()
    calls = [0]

    def W(v):
        calls[0] += 1
        y = csum.anova_rows(F, wins, sig, wt, v, rows)
        print(f"  direct product {calls[0]}: {time.time() - t0:.0f} s", flush=True)
        return y

    D = W(np.ones(N))
    eta = D - sum(wt)
    A = OS.system_operator(W, D, ALPHA)
    fv = f.reshape(-1)
    u, it, relres, _ = OS.pcg_ubasis(A, fv, eta, ALPHA, TOL, 400)
    r = fv - A(u)
    fperp = fv - fv.mean()
    true_rel = float(np.linalg.norm(r) / np.linalg.norm(fperp))
    np.save(os.path.join(HERE, NAME + ".npy"), u)
    with open(os.path.join(HERE, NAME + ".txt"), "w") as fh:
        fh.write(f"# FP64 exact-kernel solution, written by make_solution_256.py (oracle only)\n"
                 f"side {SIDE}\nseed {SEED}\nrects 20\ndiscs 12\nnoise 0.1\nrho {RHO}\n"
                 f"windows {len(wins)}\nsigma {SIGMA}\nweight 1\nalpha {ALPHA}\n"
                 f"tol {TOL}\niterations {it}\nrelres_recursive {relres:.3e}\n"
                 f"relres_true {true_rel:.3e}\nmean_u {u.mean():.17g}\nmean_f {fv.mean():.17g}\n")
    print(f"done: {it} iterations, recursive {relres:.2e}, true {true_rel:.2e}, "
          f"{time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
