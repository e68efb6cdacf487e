"""FP32-bulk / FP64-polish PCG against plain FP64 PCG on one workload, from the same guess.

Reports for both solves the time, iterations, E and mu, and for the mixed result its distance to
the FP64 ground state: dE, dmu, the density difference max| |phi_m|^2 - |phi_64|^2 | / max |phi_64|^2
(after both are normalised), and the FP64 residual ||H phi - mu phi||_inf of the mixed state
evaluated by the FP64 apply (Sec. 2.3 residual; the mixed path itself is the project's addition).

    python -m paper_2603_05194_amd.mixed [--workload cigar_128] [--max-iter K] [--switch-res R]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

from . import BEC_FP32, BEC_FP64, BecGrid, bec_pcg_default_opts, make_params


def compare(w, max_iter=None, log=None, switch_res=None):
    import torch
    import bec_inputs as bi
    p = make_params(w.gamma, w.beta, w.lam, w.ndip, w.omega)
    opts = bec_pcg_default_opts()
    if max_iter:
        opts.max_iter = max_iter
    if switch_res:
        opts.switch_res = switch_res
    guess = torch.from_numpy(bi.initial_guess(w)).to("cuda")
    out = {}
    states = {}
    for name, prec in (("fp64", BEC_FP64), ("mixed", BEC_FP32)):
        g = BecGrid(w.n, w.a, precision=prec)
        g.ensure_symbol()
        phi = guess.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = g.pcg_solve(p, phi, opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = dict(seconds=dt, iters=r.iters, fp32_iters=r.fp32_iters, status=r.status, res_inf=r.res_inf,
                         E=r.e.E, mu=r.e.mu)
        states[name] = phi
        if log:
            log(f"{name}: {dt:.2f}s iters {r.iters} (fp32 {r.fp32_iters}) status {r.status} E {r.e.E:.13f}")
        del g
    g64 = BecGrid(w.n, w.a)
    h, mu = g64.apply_H(p, states["mixed"])
    res = float((h - mu * states["mixed"]).abs().max())
    d64 = states["fp64"].abs() ** 2
    dm = states["mixed"].abs() ** 2
    out["mixed_vs_fp64"] = dict(dE=out["mixed"]["E"] - out["fp64"]["E"], dmu=out["mixed"]["mu"] - out["fp64"]["mu"],
                                density_rel_linf=float((dm - d64).abs().max() / d64.abs().max()),
                                fp64_residual_of_mixed_state=res,
                                speedup=out["fp64"]["seconds"] / out["mixed"]["seconds"])
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="cigar_128")
    ap.add_argument("--max-iter", type=int, default=None)
    ap.add_argument("--switch-res", type=float, default=None,
                    help="residual at which the mixed solve switches to FP64 (library default 1e-5)")
    args = ap.parse_args(argv)
    os.environ.setdefault("BEC_PROGRESS", "30")
    import bec_inputs as bi
    w = bi.WORKLOADS[args.workload]
    log = lambda s: print(s, file=sys.stderr, flush=True)
    res = compare(w, args.max_iter, log, args.switch_res)
    print(json.dumps(dict(workload=args.workload, n=list(w.n), switch_res=args.switch_res, **res)))


if __name__ == "__main__":
    main()
