"""Batched parameter sweeps of ground states and the critical rotation frequency.

A sweep of solves on several grid sizes groups the solves by grid (same box and grid within a
group: one launch per phase serves all of its solves). By default the groups run in one call of
bec_pcg_solve_ragged, side by side on streams of their own; --serial runs one group after
another. The critical rotation frequency for each dipolar strength is the first Omega at which
the ground state carries a vortex, read as <L_z> = -E_rot / Omega >= 1/2 (Sec. 3, critical
rotational frequency study).

    python -m paper_2603_05194_amd.sweep [--quick] [--max-iter K] [--fp64] [--serial]
                                         [--autotune [--tile-cache F]]
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from collections import OrderedDict

import numpy as np

from . import BEC_FP32, BEC_FP64, BecGrid, bec_pcg_default_opts, make_params, pcg_solve_ragged


def group_by_grid(workloads):
    groups = OrderedDict()
    for i, w in enumerate(workloads):
        groups.setdefault((tuple(w.n), tuple(w.a)), []).append(i)
    return groups


def _record(r, w, n, dt, tiles, tune_s):
    lz = -r.e.Erot / w.omega if w.omega != 0 else 0.0
    return dict(name=w.name, n=list(n), omega=w.omega, lam=w.lam, beta=w.beta, status=r.status, iters=r.iters,
                fp32_iters=r.fp32_iters, res_inf=r.res_inf, E=r.e.E, mu=r.e.mu, Erot=r.e.Erot, Lz=lz,
                batch_seconds=dt, tiles=list(tiles), tune_seconds=tune_s)


def run_sweep(workloads, guesses, precision=BEC_FP32, opts=None, log=None, autotune=False, tile_cache=None,
              ragged=True):
    """Solve every workload, grouped by grid. `guesses[i]` is a complex128 numpy array.
    ragged: all groups in one bec_pcg_solve_ragged call (batch_seconds is then the whole call's
    time); else one batched solve per group, one after another.
    With `autotune`, each grid's line tiles and kernel variants are searched (or read from
    `tile_cache`) on its initial guesses first; the search time is reported apart (tune_seconds).
    Returns one dict per workload with status, iterations, energies and <L_z>."""
    import torch
    opts = opts or bec_pcg_default_opts()
    out = [None] * len(workloads)
    if ragged:
        groups = list(group_by_grid(workloads).items())
        grids, plists, phis, tunes, tiles_all = [], [], [], [], []
        for (n, a), idx in groups:
            g = BecGrid(n, a, precision=precision, batch=len(idx))
            params = [make_params(workloads[i].gamma, workloads[i].beta, workloads[i].lam, workloads[i].ndip,
                                  workloads[i].omega) for i in idx]
            ph = torch.from_numpy(np.stack([guesses[i] for i in idx])).to(g.device)
            tune_s, tiles = 0.0, (1, 1, 1)
            if autotune:
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                tiles, _ = g.autotune(params, ph.to(g.cdtype), reps=3, cache=tile_cache, log=log)
                g.autotune_kernels(params, ph.clone(), iters=10, cache=tile_cache, log=log)
                tune_s = time.perf_counter() - t1
            grids.append(g)
            plists.append(params)
            phis.append(ph)
            tunes.append(tune_s)
            tiles_all.append(tiles)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = pcg_solve_ragged(grids, plists, phis, opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        for gi, ((n, a), idx) in enumerate(groups):
            for k, i in enumerate(idx):
                out[i] = _record(res[gi][k], workloads[i], n, dt, tiles_all[gi], tunes[gi])
            if log:
                rs = res[gi]
                log(f"grid {n}: {len(idx)} solves, iterations {min(r.iters for r in rs)}..{max(r.iters for r in rs)}, "
                    f"converged {sum(r.status == 0 for r in rs)}/{len(idx)}")
        if log:
            log(f"ragged call over {len(groups)} grids: {dt:.1f}s")
        return out
    for (n, a), idx in group_by_grid(workloads).items():
        t0 = time.perf_counter()
        g = BecGrid(n, a, precision=precision, batch=len(idx))
        params = [make_params(workloads[i].gamma, workloads[i].beta, workloads[i].lam, workloads[i].ndip,
                              workloads[i].omega) for i in idx]
        phis = torch.from_numpy(np.stack([guesses[i] for i in idx])).to(g.device)
        tune_s, tiles = 0.0, (1, 1, 1)
        if autotune:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            tiles, _ = g.autotune(params, phis.to(g.cdtype), reps=3, cache=tile_cache, log=log)
            tune_s = time.perf_counter() - t1
            t0 += tune_s
        res = g.pcg_solve_batched(params, phis, opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        for k, i in enumerate(idx):
            out[i] = _record(res[k], workloads[i], n, dt, tiles, tune_s)
        if log:
            log(f"grid {n}: {len(idx)} solves in {dt:.1f}s, iterations {min(res[k].iters for k in range(len(idx)))}"
                f"..{max(res[k].iters for k in range(len(idx)))}, converged "
                f"{sum(r.status == 0 for r in res)}/{len(idx)}")
        del g
    return out


def critical_omega(results):
    """Per dipolar strength: the first Omega (ascending) with <L_z> >= 1/2 among the converged
    solves (status 0; results without a status count as converged), and its bracket. Solves that
    did not converge are left out and listed."""
    by_lam = OrderedDict()
    for r in results:
        by_lam.setdefault(r["lam"], []).append(r)
    out = OrderedDict()
    for lam, rs in by_lam.items():
        rs = sorted(rs, key=lambda r: r["omega"])
        ok = [r for r in rs if r.get("status", 0) == 0]
        oc, lo = None, None
        for i, r in enumerate(ok):
            if r["Lz"] >= 0.5:
                oc = r["omega"]
                lo = ok[i - 1]["omega"] if i > 0 else 0.0
                break
        out[lam] = dict(omega_c=oc, bracket=[lo, oc], Lz=[round(r["Lz"], 6) for r in ok],
                        omegas=[r["omega"] for r in ok],
                        not_converged=[r["omega"] for r in rs if r.get("status", 0) != 0])
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="quarter-size grids")
    ap.add_argument("--fp64", action="store_true", help="FP64 only (default: FP32 bulk + FP64 polish)")
    ap.add_argument("--max-iter", type=int, default=20000)
    ap.add_argument("--autotune", action="store_true", help="search the line tiles of each grid first")
    ap.add_argument("--tile-cache", default=None, help="JSON file of searched line tiles (read and written)")
    ap.add_argument("--serial", action="store_true", help="one batched solve per grid, one after another")
    args = ap.parse_args(argv)
    import bec_inputs as bi
    ws = bi.batched_sweep(quick=args.quick)
    guesses = [bi.initial_guess(w) for w in ws]
    o = bec_pcg_default_opts()
    o.max_iter = args.max_iter
    log = lambda s: print(s, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    res = run_sweep(ws, guesses, BEC_FP64 if args.fp64 else BEC_FP32, o, log, args.autotune, args.tile_cache,
                    ragged=not args.serial)
    total = time.perf_counter() - t0
    oc = critical_omega(res)
    print(json.dumps({"seconds": total, "solves": len(res), "converged": sum(r["status"] == 0 for r in res),
                      "critical_omega": oc, "results": res}))


if __name__ == "__main__":
    main()
