"""Experimental order of convergence on the GPU (Sec. 3.4).

The level-set mean-curvature flow with the exact solution
u = (x1^2 + x2^2 + x3^2 + x4^2 - 1)/6 + t on [-L, L]^4, G = 1, eps = h^2,
tau = T/steps, Dirichlet data from the exact solution, no rescaling; the
error is sqrt(sum_n tau * sum_P h^4 (u^n_P - u(x_P, t_n))^2).  Grid: cell
centres x_i = -L + (i - 1/2) h, ghost centres one h outside; the ghosts of
u^{n-1} hold the exact solution at t_{n-1}, the new level's Dirichlet data is
the exact solution at t_n.

Every time step runs in libsubsurf4d.so (subsurf4d_step_dirichlet); torch
only holds the arrays, builds the boundary data of the test problem and sums
the error.
"""
from __future__ import annotations

import time

import numpy as np

from paper_2111_11866_amd import binding as B

# (N, steps) of the paper's table: tau proportional to h^2
PAPER_LEVELS = ((10, 1), (20, 4), (40, 16), (80, 64), (160, 256))


def run(N, steps, T=0.0625, L=1.25, omega=1.5, tol=1e-11, precision=B.FP64, device="cuda", log=None):
    import torch

    h = 2.0 * L / N
    n = (N, N, N, N)
    x = torch.tensor(-L + (np.arange(N + 2) - 0.5) * h, dtype=torch.float64, device=device)
    r2 = (x.view(-1, 1, 1, 1) ** 2 + x.view(1, -1, 1, 1) ** 2 + x.view(1, 1, -1, 1) ** 2
          + x.view(1, 1, 1, -1) ** 2)
    base = (r2 - 1.0) / 6.0                       # exact solution at t = 0 (padded)
    del r2
    tau = T / steps
    G = torch.ones((4,) + B.padded_shape(n), dtype=torch.float64, device=device)
    u = base.clone()
    ub = torch.empty_like(base)
    ws = B.alloc_workspace(n, 0, precision)
    sp = B.StepParams(eps=h * h, tau=tau, omega=omega, tol=tol, max_iter=100000, rescale=False,
                      precision=precision, refine_tol=tol)
    err2 = 0.0
    its = []
    t0 = time.perf_counter()
    for s in range(1, steps + 1):
        torch.add(base, s * tau, out=ub)          # boundary data of the new level
        r = B.step_dirichlet(n, h, G, ub, None, 0, None, u, sp, ws)
        if r["status"] != 0:
            raise RuntimeError(f"EOC step {s} of N={N}: status {r['status']}")
        its.append(r["iterations"])
        e = u[1:-1, 1:-1, 1:-1, 1:-1] - ub[1:-1, 1:-1, 1:-1, 1:-1]
        err2 += tau * h ** 4 * float(torch.sum(e * e))
        if log and (s % 16 == 0 or s == steps):
            log(f"[eoc] N={N} step {s}/{steps}: {r['iterations']} iterations, {time.perf_counter() - t0:.1f}s")
    torch.cuda.synchronize()
    return float(np.sqrt(err2)), its, time.perf_counter() - t0


def table(levels=PAPER_LEVELS, log=None, **kw):
    rows = []
    prev = None
    for N, steps in levels:
        err, its, sec = run(N, steps, log=log, **kw)
        eoc = None if prev is None else float(np.log2(prev / err))
        rows.append(dict(n=N, steps=steps, h=2.5 / N, error=err, eoc=eoc, iterations_mean=float(np.mean(its)),
                         seconds=sec))
        prev = err
        if log:
            log(f"[eoc] N={N}: error {err:.6e} eoc {eoc} ({sec:.1f}s)")
    return rows


def main():
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser(description="EOC table of Sec. 3.4 on the GPU")
    ap.add_argument("--max-n", type=int, default=160)
    ap.add_argument("--mixed", action="store_true", help="mixed-precision steps refined to the same tol")
    args = ap.parse_args()
    levels = [lv for lv in PAPER_LEVELS if lv[0] <= args.max_n]
    rows = table(levels, log=lambda m: print(m, file=sys.stderr, flush=True),
                 precision=B.MIXED if args.mixed else B.FP64)
    print(json.dumps(rows))


if __name__ == "__main__":
    main()
