"""Ground state by multi-guess selection (Sec. 3): Algorithm 1 (through the cascade of
Algorithm 2) from each of the paper's ten starting states, run as one batch of solves on every
grid, and the converged state of lowest energy kept.

    python -m paper_2603_05194_amd.guesses --example table2 [--grid 256 256 256] [--levels 4]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import BEC_FP32, BEC_FP64, bec_pcg_default_opts, make_params
from . import multigrid as MG

# Ex. 3.2 of Sec. 3 (U-shape vortex line): gamma = (1, 1, 0.05), beta = 1000, lambda = -300,
# n = z, Omega = 0.75 on [-10,10]^2 x [-100,100].
TABLE2 = dict(a=(10.0, 10.0, 100.0), gamma=(1.0, 1.0, 0.05), beta=1000.0, lam=-300.0, ndip=(0.0, 0.0, 1.0),
              omega=0.75)


def lowest_energy(n, a, gamma, beta, lam, ndip, omega, levels=4, precision=BEC_FP32, opts=None, log=None):
    """Runs the ten guesses of Sec. 3 through `levels` grids of the cascade ending at n and
    returns (index of the lowest-energy converged state, its field on grid n, records per guess
    of the finest level, per-level records)."""
    import bec_inputs as bi
    p = make_params(gamma, beta, lam, ndip, omega)
    nl0 = MG.levels(n, levels)[0]
    g0 = bi.paper_guesses(nl0, a, gamma, beta, omega)
    phi, recs = MG.solve(n, a, [p] * len(g0), g0, precision=precision, opts=opts, count=levels, log=log)
    fine = recs[-1]
    ok = [k for k, r in enumerate(fine) if r["status"] == 0]
    best = min(ok, key=lambda k: fine[k]["E"]) if ok else None
    return best, (phi[best] if best is not None else None), fine, recs


def main(argv=None):
    import bec_inputs as bi
    ap = argparse.ArgumentParser()
    ap.add_argument("--example", default="table2", choices=["table2"])
    ap.add_argument("--grid", type=int, nargs=3, default=[256, 256, 256])
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--fp64", action="store_true")
    args = ap.parse_args(argv)
    log = lambda s: print(s, file=sys.stderr, flush=True)
    ex = TABLE2
    o = bec_pcg_default_opts()
    o.max_iter = 200000
    t0 = time.perf_counter()
    best, _, fine, recs = lowest_energy(tuple(args.grid), ex["a"], ex["gamma"], ex["beta"], ex["lam"], ex["ndip"],
                                        ex["omega"], args.levels, BEC_FP64 if args.fp64 else BEC_FP32, o, log)
    rows = [dict(guess=name, **r) for name, r in zip(bi.PAPER_GUESS_NAMES, fine)]
    print(json.dumps(dict(grid=args.grid, levels=args.levels, seconds=time.perf_counter() - t0, best=best,
                          best_guess=bi.PAPER_GUESS_NAMES[best] if best is not None else None, rows=rows)))


if __name__ == "__main__":
    main()
