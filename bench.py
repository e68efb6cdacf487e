"""North-star benchmark: FP64 PCG-ATKM (Algorithm 1) on the 256x256x64 pancake workload on one
MI355X: time to ground state, PCG iterations/s, H phi applies/s, the dominant kernel's HBM
roofline fraction inside the iteration, the learned + mixed-precision path against plain FP64,
and the CPU oracle timed on the host cores.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--block B] [--budget S] [--no-cpu] [--no-learned]
                [--with-mixed] [--solve-iters N] [--quick]

* A step is a block of B (default 1000) FP64 PCG iterations of the pancake workload, continuing
  from the previous block's iterate (the first block starts from the seed-0 random-phase guess);
  W untimed blocks, then K timed ones give ms_per_step and iterations/s. Inputs are resident in
  HBM before the timed region.
* `value` is the time of one full FP64 solve from the seed-0 guess (--seed) to
  ||H phi - mu phi||_inf <= 1e-8.
  Its iteration cap comes from the wall budget (--budget seconds from the start of the script,
  default 540) and the measured iteration rate, so the JSON line is always printed; a capped
  solve is reported as such (`solve.status`).
* The solver runs passes that do not depend on each other on a second stream (graph branches);
  the timed blocks and `value` use it. Kernel durations taken beside other kernels include the
  sharing of the GPU, so the roofline kernel is taken from an event-timed profile of 50
  iterations launched in order on one stream (bec_pcg_profile, every launch with start and stop
  events of its own): the launch site with the largest kernel time per iteration; achieved =
  algorithmic bytes per launch / mean duration. Three more blocks on one stream give the rate
  without the branches (pcg_iters_per_s_one_stream).
* The learned legs (network + spectral interpolation + FP32 bulk + FP64 polish, all inside the
  timed region) run only if the budget allows: `learned` starts from the network's modulus with
  the phase of the FP64 solve's seed-0 guess, `learned_network` from the network's field. A
  speed-up against the FP64 solve is reported only when both end in the same state
  (|dE| <= 1e-10 |E|).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

T_START = time.monotonic()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "s to ground state (res≤1e-8) at 256²×64; H·φ/s; mixed+learned vs plain FP64"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(f"[bench {time.monotonic() - T_START:7.1f}s]", *a, file=sys.stderr, flush=True)


def pass_bytes(which, n, csize):
    """Algorithmic HBM bytes of one launch of a padded ATKM pass (complex values of csize bytes):
    y forward: read the [Nx][Ny][Nz+1] z half spectrum, write the [Nx][2Ny][Nz+1] buffer;
    x pass (forward, S' multiply, inverse): read + write the [Nx][2Ny][Nz+1] buffer and read the
    FP64 symbol octant [Nx+1][Ny+1][Nz+1] once; dual x Parseval: read two such buffers + octant."""
    nx, ny, nz = n
    zh = nx * ny * (nz + 1) * csize
    yb = nx * 2 * ny * (nz + 1) * csize
    octant = (nx + 1) * (ny + 1) * (nz + 1) * 8
    return {"y_fwd": zh + yb, "x_pass": 2 * yb + octant, "x_pars2": 2 * yb + octant}[which]


def site_bytes(site, n, csize, lam=True):
    """Algorithmic HBM bytes of one launch at each launch site of a PCG iteration (bec_pcg_profile):
    every field read and written once. N-grid complex fields are N*csize bytes, real fields
    N*csize/2; Z = [Nx][Ny][Nz+1] and Y = [Nx][2Ny][Nz+1] half spectra; the symbol octant is FP64."""
    nx, ny, nz = n
    N = nx * ny * nz
    c, r = N * csize, N * csize // 2
    Z = nx * ny * (nz + 1) * csize
    Y = nx * 2 * ny * (nz + 1) * csize
    octant = (nx + 1) * (ny + 1) * (nz + 1) * 8
    Phi = r if lam else 0
    return {
        "prec_z": 4 * c + Phi,             # read H phi, phi, Phi; write r, W
        "prec_y": 2 * c,                   # W in place
        "prec_x": 2 * c,
        "prec_zi": 6 * c + Phi,            # read W, phi, Phi, r_prev, H phi, p_prev; write P r (r is formed again)
        "dir_z": 4 * c + Phi + 2 * Z,      # read phi, P r, p_prev, Phi; write p, Z1, Z2
        "y_fwd": Z + Y,
        "x_pars2": 2 * Y + octant,
        "p_lines": c,                      # read p (Parseval only)
        "retract": 3 * c + Z,              # retraction in the z R2C of |phi|^2: read phi, p; write phi, Z1
        "atkm_z": c + Z,                   # read phi; write Z1
        "x_atkm": 2 * Y + octant,          # Y1 in place + symbol
        "y_inv": Y + Z,
        "atkm_zi": Z + r,                  # read Z1; write Phi
        "h_z": 2 * c,                      # read phi; write acc
        "h_y": 3 * c,                      # read phi, acc; write acc
        "h_x": 3 * c + Phi,                # read phi, acc, Phi; write H phi
    }.get(site, 0)


# HBM bytes per launch and site from rocprofv3 FETCH_SIZE / WRITE_SIZE (FETCH_SIZE scaled by the
# copy-kernel calibration factor 2.0, WRITE_SIZE by 1.0), taken with the kernel sources hashing to
# MEASURED_TRAFFIC_SRC; the roofline's traffic is null once the sources have changed.
MEASURED_TRAFFIC_SRC = "955e154b7ff25205"
MEASURED_TRAFFIC = {
    "atkm_z": 136.4e6, "y_fwd": 214.2e6, "x_atkm": 324.9e6, "y_inv": 220.4e6,
    "atkm_zi": 126.8e6, "h_z": 134.4e6, "h_y": 201.6e6, "h_x": 268.8e6,
    "prec_z": 302.2e6, "prec_y": 134.3e6, "prec_x": 134.4e6, "prec_zi": 436.6e6,
    "dir_z": 440.9e6, "x_pars2": 337.5e6, "p_lines": 67.3e6, "retract": 270.6e6,
}


def kernel_src_hash():
    m = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h", "ops.inc", "special.inc", "pcg.inc", "regfft.h", "fft.h", "common.h",
              "lines.h"):
        with open(os.path.join(ROOT, "paper_2603_05194_amd", "csrc", f), "rb") as fh:
            m.update(fh.read())
    return m.hexdigest()[:16]


def cpu_baseline(w, warm_iters=2, timed_iters=20, applies=5):
    """The CPU oracle on the host cores, a bounded sample of the same workload: the symbol (timed,
    excluded), the median of `applies` H applies, and the oracle's Algorithm 1 from the seed-0
    guess for warm_iters + timed_iters iterations, each iteration timed on its own; s/iteration is
    the median of the timed ones (the first warm_iters are warm-up)."""
    import numpy as np
    import bec_inputs as bi
    from oracle import spectral, symbol
    from oracle.energy import Model
    from oracle.grid import Grid
    from oracle.pcg import pcg
    t0 = time.perf_counter()
    uh = symbol.symbol_full_by_octant(Grid(w.n, w.a))
    t_sym = time.perf_counter() - t0
    m = Model.from_workload(w, uhat_full=uh)
    phi0 = bi.initial_guess(w)
    ta = []
    for _ in range(applies):
        t0 = time.perf_counter()
        m.H(phi0)
        ta.append(time.perf_counter() - t0)
    stamps = []
    t_start = time.perf_counter()
    pcg(m, phi0, tol_res=0.0, max_iter=warm_iters + timed_iters, on_iter=lambda n: stamps.append(time.perf_counter()))
    per = np.diff(np.array([t_start] + stamps))[warm_iters:]
    cpu = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cores": spectral.WORKERS, "s_per_iter": float(np.median(per)), "s_per_apply": float(np.median(ta)),
            "iters_timed": int(per.size), "warmup_iters": warm_iters, "applies_timed": applies,
            "symbol_s": t_sym, "cpu_model": cpu, "numpy": np.__version__}


def cpu_line(c, gpu_iters):
    """The cpu_baseline object: oracle s/iteration times the GPU's FP64 iteration count."""
    return {"value": c["s_per_iter"] * gpu_iters, "unit": "s", "cores": c["cores"], "kind": "oracle",
            "sample": f"oracle (FP64 NumPy/SciPy FFT, {c['cores']} threads) on the same workload: Algorithm 1 "
                      f"from the seed-0 guess, {c['warmup_iters']} warm-up iterations, then the median of "
                      f"{c['iters_timed']} timed iterations = {c['s_per_iter']:.2f} s/iteration, times the GPU FP64 "
                      f"iteration count {gpu_iters} = extrapolated time to ground state; H apply (median of "
                      f"{c['applies_timed']}) {c['s_per_apply']:.2f} s; symbol {c['symbol_s']:.1f} s excluded",
            "extrapolated": True, **c}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed blocks of --block PCG iterations")
    ap.add_argument("--warmup", type=int, default=5, help="untimed blocks before the timed ones")
    ap.add_argument("--block", type=int, default=1000, help="PCG iterations per step")
    ap.add_argument("--budget", type=float, default=540.0, help="wall seconds from the start for the whole run")
    ap.add_argument("--profile-iters", type=int, default=50)
    ap.add_argument("--solve-iters", type=int, default=None,
                    help="cap the full solve (profiling runs; the result is then not a ground state)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--with-mixed", action="store_true", help="also time mixed precision from the plain guess")
    ap.add_argument("--quick", action="store_true", help="reduced grid (for testing the script)")
    ap.add_argument("--seed", type=int, default=0,
                    help="random-phase guess of the full solve and of the learned starts (the timed blocks use seed 0)")
    ap.add_argument("--learned-starts", default="envelope,network",
                    help="comma-separated learned starts to run: envelope, network")
    ap.add_argument("--one-stream", action="store_true",
                    help="every solve without the second stream (for kernel traces whose durations are each "
                         "kernel's own)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs a solve on one GPU; --gpus must be 1"}))
        sys.exit(2)
    deadline = T_START + args.budget

    # the library prints a progress line to stderr every 30 s of a long solve
    os.environ.setdefault("BEC_PROGRESS", "30")
    import numpy as np
    import torch
    import bec_inputs as bi
    import paper_2603_05194_amd as bec

    w = bi.WORKLOADS["pancake_256"]
    if args.quick:
        w = w.with_grid((64, 64, 16))
    n = w.n
    p = bec.make_params(w.gamma, w.beta, w.lam, w.ndip, w.omega)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"torch ready; grid {n}")

    t0 = time.perf_counter()
    g = bec.BecGrid(n, w.a)
    g.ensure_symbol()
    torch.cuda.synchronize()
    t_symbol = time.perf_counter() - t0
    log(f"workspace + symbol {t_symbol:.3f}s")

    def guess(seed):
        ws = bi.Workload(**{**w.to_dict(), "seed": seed})
        return torch.from_numpy(bi.initial_guess(ws)).to(dev)

    # ---------------------------------------------------------------- timed blocks
    ob = bec.bec_pcg_default_opts()
    ob.tol_res_inf = 0.0          # fixed-length blocks
    ob.max_iter = args.block
    if args.one_stream:
        ob.branches = 0
    phi_b = guess(0)
    torch.cuda.synchronize()
    for i in range(args.warmup):
        r = g.pcg_solve(p, phi_b, ob)
        log(f"warmup block {i}: iters {r.iters} res {r.res_inf:.2e} E {r.e.E:.12f}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    blocks = [g.pcg_solve(p, phi_b, ob) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_blocks = time.perf_counter() - t0
    it_blocks = sum(r.iters for r in blocks)
    ms_per_step = 1e3 * t_blocks / args.steps
    it_per_s = it_blocks / t_blocks
    log(f"{args.steps} blocks of {args.block}: {t_blocks:.3f}s, {it_per_s:.1f} it/s, res {blocks[-1].res_inf:.2e}")

    # ---------------------------------------------------------------- per-kernel profile in the iteration
    prof = g.pcg_profile(p, phi_b, args.profile_iters, concurrent=False)
    sites = {}
    for name, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        b = site_bytes(name, n, 16, w.lam != 0.0)
        avg = ms / cnt
        sites[name] = {"us_per_iter": 1e3 * ms / args.profile_iters, "launches_per_iter": cnt / args.profile_iters,
                       "avg_us": 1e3 * avg, "bytes_per_launch": b,
                       "achieved_GBs": (b / (avg * 1e-3) / 1e9) if b else None}
    kern_us = sum(s["us_per_iter"] for s in sites.values())
    dom = max((k for k in sites if sites[k]["bytes_per_launch"]), key=lambda k: sites[k]["us_per_iter"])
    for k, s in sorted(sites.items(), key=lambda kv: -kv[1]["us_per_iter"]):
        log(f"  {k:9s} {s['us_per_iter']:8.1f} us/it  {s['avg_us']:7.1f} us/launch  "
            + (f"{s['achieved_GBs']:6.0f} GB/s" if s["achieved_GBs"] else ""))
    log(f"kernel time per iteration {kern_us:.1f} us (one stream); dominant {dom}")
    o1 = bec.bec_pcg_default_opts()
    o1.tol_res_inf = 0.0
    o1.max_iter = args.block
    o1.branches = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it1 = sum(g.pcg_solve(p, phi_b, o1).iters for _ in range(3))
    torch.cuda.synchronize()
    it_per_s_1 = it1 / (time.perf_counter() - t0)
    log(f"one stream: {it_per_s_1:.1f} it/s")

    t_apply_ms = g.time_stage(p, phi_b, 2, reps=20)
    t_atkm_ms = g.time_stage(p, phi_b, 1, reps=20)
    t_copy_ms = g.time_stage(p, phi_b, 4, reps=50)
    copy_gbs = 2 * 16 * n[0] * n[1] * n[2] / (t_copy_ms * 1e-3) / 1e9
    log(f"H apply {t_apply_ms:.3f} ms, ATKM {t_atkm_ms:.3f} ms, copy {copy_gbs:.0f} GB/s")
    del phi_b

    # ---------------------------------------------------------------- CPU oracle baseline
    cpu = None
    if not args.no_cpu:
        try:
            cpu = cpu_baseline(w)
            log(f"cpu baseline {cpu['s_per_iter']:.2f} s/iter on {cpu['cores']} threads")
        except Exception as e:   # the baseline never hides the GPU result
            cpu = {"error": repr(e)}

    # ---------------------------------------------------------------- time to ground state
    opts = bec.bec_pcg_default_opts()
    reserve = 15.0
    cap = int(max(1000, it_per_s * (deadline - time.monotonic() - reserve)))
    opts.max_iter = min(cap, 2_000_000) if args.solve_iters is None else args.solve_iters
    if args.one_stream:
        opts.branches = 0
    phi = guess(args.seed)
    torch.cuda.synchronize()
    log(f"full FP64 solve from the seed-{args.seed} guess, iteration cap {opts.max_iter}")
    t0 = time.perf_counter()
    ref = g.pcg_solve(p, phi, opts)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    converged = ref.status == bec.BEC_OK
    log(f"solve: status {ref.status} iters {ref.iters} {t_solve:.3f}s res {ref.res_inf:.2e} E {ref.e.E:.13f}")
    if cpu and "s_per_iter" in cpu:
        cpu = cpu_line(cpu, ref.iters)

    # ---------------------------------------------------------------- learned + mixed precision
    # Two learned starts, each FP32 bulk + FP64 polish with everything from the network call on
    # inside the timed region: "envelope" (the network's modulus with the phase of the seed-0
    # guess the FP64 solve starts from; formed on the host) and "network" (the network's field).
    learned, learned_network = None, None
    if not args.no_learned:
        from paper_2603_05194_amd import learned as L
        net = L.load_default()
        draw = np.array([w.beta, w.lam / w.beta, w.omega, w.gamma[2], math.acos(w.ndip[2]),
                         math.atan2(w.ndip[1], w.ndip[0])])
        gm = bec.BecGrid(n, w.a, precision=bec.BEC_FP32)
        gm.ensure_symbol()
        g0 = bi.initial_guess(bi.Workload(**{**w.to_dict(), "seed": args.seed}))
        for mode in [m for m in ("envelope", "network") if m in args.learned_starts.split(",")]:
            left = deadline - time.monotonic()
            need = 0.45 * t_solve + 20.0
            if left < need:
                leg = {"start": mode, "skipped": f"wall budget: {left:.0f}s left, about {need:.0f}s needed"}
                log(leg["skipped"])
            else:
                ol = bec.bec_pcg_default_opts()
                ol.max_iter = int(max(1000, it_per_s * 1.5 * (deadline - time.monotonic() - reserve)))
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                phil = L.predict(net, [draw], n)[0].contiguous()
                if mode == "envelope":
                    phil = torch.from_numpy(L.envelope_start(phil.cpu().numpy(), g0, n, w.a)).to(dev)
                torch.cuda.synchronize()
                t_net = time.perf_counter() - t0
                rl = gm.pcg_solve(p, phil, ol)
                torch.cuda.synchronize()
                tl = time.perf_counter() - t0
                dE = rl.e.E - ref.e.E
                same = converged and rl.status == bec.BEC_OK and abs(dE) <= 1e-10 * abs(ref.e.E)
                leg = {"start": mode, "s_to_ground_state": tl, "network_and_interp_s": t_net, "iters": rl.iters,
                       "fp32_iters": rl.fp32_iters, "status": rl.status, "E": rl.e.E, "dE_vs_fp64": dE,
                       "same_state": same, "speedup_vs_fp64": (t_solve / tl) if same else None,
                       "note": None if same else "ends in another state than the FP64 solve (|dE| > 1e-10|E|) "
                                                 "or did not converge: no speed-up is claimed"}
                log(f"mixed+learned ({mode}): {tl:.3f}s iters {rl.iters} (fp32 {rl.fp32_iters}) dE {dE:.2e} "
                    f"same {same}")
            if mode == "envelope":
                learned = leg
            else:
                learned_network = leg
        del gm, net

    mixed = None
    if args.with_mixed and deadline - time.monotonic() > 0.6 * t_solve:
        gm = bec.BecGrid(n, w.a, precision=bec.BEC_FP32)
        gm.ensure_symbol()
        phim = guess(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rm = gm.pcg_solve(p, phim, opts)
        torch.cuda.synchronize()
        tm = time.perf_counter() - t0
        dE = rm.e.E - ref.e.E
        same = converged and rm.status == bec.BEC_OK and abs(dE) <= 1e-10 * abs(ref.e.E)
        mixed = {"s_to_ground_state": tm, "iters": rm.iters, "fp32_iters": rm.fp32_iters, "status": rm.status,
                 "dE_vs_fp64": dE, "same_state": same, "speedup_vs_fp64": (t_solve / tm) if same else None}
        log(f"mixed: {tm:.3f}s iters {rm.iters} (fp32 {rm.fp32_iters}) dE {dE:.2e}")
        del gm

    ds = sites[dom]
    src_ok = dom in MEASURED_TRAFFIC and MEASURED_TRAFFIC_SRC == kernel_src_hash()
    out = {
        "metric": METRIC,
        "value": t_solve,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"pancake trap {n[0]}x{n[1]}x{n[2]} on [-16,16]^2x[-2,2], gamma=(1,1,20), "
                               f"beta=2000, lambda=600, n=(sin30,0,cos30), Omega=0.9, random-phase Gaussian guess "
                               f"seed {args.seed}; value: FP64 PCG-ATKM to ||r||_inf<=1e-8; step: {args.block} FP64 PCG "
                               f"iterations",
                   "grid": list(n), "padded": [2 * v for v in n], "tol_res_inf": 1e-8, "block_iters": args.block,
                   "seed": args.seed},
        "solve": {"status": ref.status, "converged": converged, "iters": ref.iters, "res_inf": ref.res_inf,
                  "E": ref.e.E, "mu": ref.e.mu, "iter_cap": opts.max_iter,
                  "note": None if converged else "iteration cap from the wall budget reached: not a ground state"},
        "pcg_iters_per_s": it_per_s,
        "pcg_iters_per_s_one_stream": it_per_s_1,
        "hphi_per_s": 1e3 / t_apply_ms,
        "atkm_per_s": 1e3 / t_atkm_ms,
        "kernel_us_per_iter": kern_us,
        "symbol_precompute_s": t_symbol,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": ds["achieved_GBs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": ds["achieved_GBs"] / HBM_PEAK_GBS,
                     "traffic": MEASURED_TRAFFIC[dom] if src_ok else None,
                     "algorithmic_bytes": ds["bytes_per_launch"], "avg_us": ds["avg_us"],
                     "launches_per_iter": ds["launches_per_iter"]},
        "sites": sites,
        "copy_GBs": copy_gbs,
        "learned": learned,
        "learned_network": learned_network,
        "mixed": mixed,
        "cpu_baseline": cpu,
        "wall_s": time.monotonic() - T_START,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
