"""Learned initial guess for Algorithm 1: training-set generation with the batched solver,
training with the library's network kernels, and inference (network -> coarse field ->
spectral interpolation -> unit mass).

The network maps six problem parameters (beta, lambda/beta, Omega, gamma_z, theta_n, phi_n),
gamma_x = gamma_y = 1, dipole axis n = (sin theta cos phi, sin theta sin phi, cos theta), to a
complex 32 x 32 x 16 field on the box [-16,16]^2 x [-a_z, a_z]. The z half-width follows the
trap: a_z = 2 sqrt(20 / g), evaluated at the lower edge g of the gamma_z band that holds the
problem (bands 20 * 2^(k/3)), so that all problems of a band share one box and grid and can be
solved in one batch. gamma_z = 20 gives a_z = 2.

Targets are ground states computed by this library's own PCG on the 64 x 64 x 32 grid of the
same box, phase-fixed (bec_gauge_fix) and truncated to the 32 x 32 x 16 Fourier modes
(bec_interp_spectral). At inference the coarse output is interpolated to the target grid by
the same spectral interpolation and normalised; Algorithm 1 then runs from it.

    python -m paper_2603_05194_amd.learned --train 2000 --out weights.npz [--eval-grid 128 128 32]

The shipped weights (data/mlp_weights.npz) were made with the defaults: 2000 training draws
(seeds 0..1999) solved to ||r||_inf <= 1e-8 on 64 x 64 x 32, Adam with step 1e-3 decayed by
cosine to 5e-5 over 1500 epochs of batch 64, initial weights from seed 0.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import BEC_FP32, BEC_FP64, BecGrid, Mlp, bec_pcg_default_opts, make_params

import os

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "mlp_weights.npz")
DIMS = (6, 512, 32768)
COARSE = (32, 32, 16)
TRAIN_N = (64, 64, 32)
XY_HALF = 16.0
GZ_RANGE = (4.0, 40.0)


def gz_band(gz: float) -> int:
    """Index k of the band [20 * 2^(k/3), 20 * 2^((k+1)/3)) holding gamma_z."""
    return int(math.floor(3.0 * math.log2(gz / 20.0) + 1e-12))


def box_for(gz: float):
    lo = 20.0 * 2.0 ** (gz_band(gz) / 3.0)
    return (XY_HALF, XY_HALF, 2.0 * math.sqrt(20.0 / lo))


def features(draw) -> np.ndarray:
    """Affine map of (beta, lambda/beta, Omega, gamma_z, theta, phi) from their sampling
    ranges onto [-1, 1]."""
    beta, ratio, om, gz, th, ph = (float(v) for v in draw)
    return np.array([(beta - 1600.0) / 1400.0, (ratio - 0.4) / 0.4, (om - 0.475) / 0.475,
                     (gz - 22.0) / 18.0, (th - math.pi / 4) / (math.pi / 4), (ph - math.pi / 2) / (math.pi / 2)],
                    dtype=np.float32)


def physical(draw):
    beta, ratio, om, gz, th, ph = (float(v) for v in draw)
    nd = (math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th))
    return dict(gamma=(1.0, 1.0, gz), beta=beta, lam=ratio * beta, ndip=nd, omega=om)


def params_of(draw):
    p = physical(draw)
    return make_params(p["gamma"], p["beta"], p["lam"], p["ndip"], p["omega"])


def plain_guess(draw, n):
    import bec_inputs as bi
    p = physical(draw)
    return bi.guess_d(tuple(n), box_for(p["gamma"][2]), p["gamma"], p["omega"])


def by_band(draws):
    groups = {}
    for i, d in enumerate(draws):
        groups.setdefault(gz_band(float(d[3])), []).append(i)
    return groups


def solve_batch(draws, n, guesses, precision, opts):
    """Batched Algorithm 1 for draws of one band on grid n. Returns (fields [B, *n] tensor,
    results, seconds)."""
    import torch
    a = box_for(float(draws[0][3]))
    g = BecGrid(n, a, precision=precision, batch=len(draws))
    phis = torch.from_numpy(np.ascontiguousarray(np.stack(guesses))).to(g.device)
    t0 = time.perf_counter()
    res = g.pcg_solve_batched([params_of(d) for d in draws], phis, opts)
    torch.cuda.synchronize()
    return g, phis, res, time.perf_counter() - t0


def boundary_ratio(phis):
    """max |phi| on the six boundary planes over max |phi|, per field (data check only, on the host)."""
    m = np.abs(phis.cpu().numpy() if hasattr(phis, "cpu") else np.asarray(phis))
    planes = [m[:, 0], m[:, -1], m[:, :, 0], m[:, :, -1], m[:, :, :, 0], m[:, :, :, -1]]
    edge = np.stack([p.reshape(p.shape[0], -1).max(1) for p in planes]).max(0)
    return edge / m.reshape(m.shape[0], -1).max(1)


def generate(draws, max_iter=4000, batch=64, tol=1e-8, log=None):
    """Training targets for `draws`: float32 [len, 32768] (complex64 32x32x16 interleaved),
    per-draw status, and the boundary-ratio check."""
    import torch
    T = np.zeros((len(draws), DIMS[2]), dtype=np.float32)
    info = [None] * len(draws)
    opts = bec_pcg_default_opts()
    opts.max_iter = int(max_iter)
    opts.tol_res_inf = tol
    for band, idx in sorted(by_band(draws).items()):
        for s in range(0, len(idx), batch):
            part = idx[s:s + batch]
            ds = [draws[i] for i in part]
            gs = [plain_guess(d, TRAIN_N) for d in ds]
            g, phis, res, dt = solve_batch(ds, TRAIN_N, gs, BEC_FP32, opts)
            br = boundary_ratio(phis)
            g.gauge_fix_([params_of(d) for d in ds], phis)
            gc = BecGrid(COARSE, g.a, batch=len(ds))
            coarse = g.interp_to(gc, phis, out_precision=BEC_FP32)
            torch.cuda.synchronize()
            T[part] = coarse.reshape(len(ds), -1).view(torch.float32).cpu().numpy()
            for k, i in enumerate(part):
                r = res[k]
                info[i] = dict(status=r.status, iters=r.iters, res=r.res_inf, E=r.e.E, boundary=float(br[k]))
            if log:
                its = [res[k].iters for k in range(len(ds))]
                log(f"band {band} (a_z={g.a[2]:.3f}): {len(ds)} solves in {dt:.1f}s, iterations "
                    f"{min(its)}..{max(its)}, converged {sum(r.status == 0 for r in res)}/{len(ds)}")
            del g, gc, phis, coarse
    return T, info


def train(X, T, epochs=1500, batch=64, lr=1e-3, seed=0, log=None, X_val=None, T_val=None):
    """Adam on the mean squared error; step size decays by cosine to lr/20. Returns the
    network and the per-epoch losses."""
    import torch
    import bec_inputs as bi
    net = Mlp(*DIMS)
    net.load_params(bi.mlp_init(DIMS, seed))
    dX = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    dT = torch.from_numpy(np.ascontiguousarray(T, dtype=np.float32)).cuda()
    n = X.shape[0]
    rng = np.random.default_rng(seed + 1)
    hist = []
    steps = epochs * ((n + batch - 1) // batch)
    k = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = rng.permutation(n).astype(np.int32)
        losses = []
        for s in range(0, n, batch):
            idx = torch.from_numpy(perm[s:s + batch]).cuda()
            frac = k / max(1, steps - 1)
            losses.append(net.loss_grad(dX, dT, idx=idx))
            net.adam_step(lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * frac))))
            k += 1
        torch.cuda.synchronize()
        ep_loss = float(torch.cat(losses).mean().item())
        rec = dict(epoch=ep, loss=ep_loss)
        if X_val is not None and (ep % 25 == 0 or ep == epochs - 1):
            rec["val"] = evaluate_loss(net, X_val, T_val)
        hist.append(rec)
        if log and (ep % 25 == 0 or ep == epochs - 1):
            log(f"epoch {ep}: loss {ep_loss:.4e}" + (f" val {rec['val']:.4e}" if "val" in rec else "")
                + f" ({time.perf_counter() - t0:.1f}s)")
    return net, hist


def evaluate_loss(net, X, T):
    """Mean squared error of the network on (X, T) by the loss kernel (overwrites net.grads)."""
    import torch
    dX = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    dT = torch.from_numpy(np.ascontiguousarray(T, dtype=np.float32)).cuda()
    return float(net.loss_grad(dX, dT).item())


def predict(net, draws, n):
    """Initial guesses on grid n for draws of one gamma_z band: complex128 [B, *n], unit mass."""
    import torch
    a = box_for(float(draws[0][3]))
    assert all(gz_band(float(d[3])) == gz_band(float(draws[0][3])) for d in draws)
    X = torch.from_numpy(np.stack([features(d) for d in draws])).cuda()
    y = net.forward(X)
    coarse = y.view(torch.complex64).reshape((len(draws),) + COARSE).contiguous()
    gc = BecGrid(COARSE, a, batch=len(draws))
    gf = BecGrid(n, a, batch=len(draws))
    fine = gc.interp_to(gf, coarse)
    gf.normalize_(fine)
    return fine


def envelope_start(learned, plain, n, a):
    """The network's modulus with the plain guess's phase, at unit mass (host arrays; h^3 from the
    box half-widths a): the start that keeps the network's envelope but not its vortex layout."""
    h3 = 8.0 * a[0] * a[1] * a[2] / (n[0] * n[1] * n[2])
    f = np.abs(learned) * np.exp(1j * np.angle(plain))
    return f / math.sqrt(h3 * float(np.sum(np.abs(f) ** 2)))


def evaluate(net, draws, n, precision=BEC_FP32, max_iter=200000, log=None, start="network"):
    """Algorithm 1 from the plain guess (phi_d of the trap Gaussian) and from the network's
    guess, for every draw, batched per gamma_z band. Returns one record per draw with the
    iterations, final energies and status of both runs, and the wall time of both batches.
    start="envelope": the learned run starts from envelope_start (network modulus, plain phase);
    forming it on the host is counted in the learned start's time."""
    import torch
    opts = bec_pcg_default_opts()
    opts.max_iter = int(max_iter)
    rows = [None] * len(draws)
    for band, idx in sorted(by_band(draws).items()):
        ds = [draws[i] for i in idx]
        gs = [plain_guess(d, n) for d in ds]
        g0, _, r0, t0 = solve_batch(ds, n, gs, precision, opts)
        del g0
        torch.cuda.synchronize()
        tp = time.perf_counter()
        lg = predict(net, ds, n)
        torch.cuda.synchronize()
        starts = list(lg.cpu().numpy())
        if start == "envelope":
            a = box_for(float(ds[0][3]))
            starts = [envelope_start(f, pl, n, a) for f, pl in zip(starts, gs)]
        t_pred = time.perf_counter() - tp
        g1, _, r1, t1 = solve_batch(ds, n, starts, precision, opts)
        t1 += t_pred            # the network and the interpolation belong to the learned start's time
        del g1
        for k, i in enumerate(idx):
            rows[i] = dict(band=band, draw=[float(v) for v in draws[i]],
                           plain=dict(status=r0[k].status, iters=r0[k].iters, E=r0[k].e.E, mu=r0[k].e.mu),
                           learned=dict(status=r1[k].status, iters=r1[k].iters, E=r1[k].e.E, mu=r1[k].e.mu),
                           plain_batch_s=t0, learned_batch_s=t1, batch=len(ds))
        if log:
            log(f"eval band {band}: {len(ds)} draws, plain {t0:.1f}s (iters median "
                f"{np.median([r.iters for r in r0]):.0f}), learned {t1:.1f}s (iters median "
                f"{np.median([r.iters for r in r1]):.0f})")
        torch.cuda.synchronize()
    return rows


def diagnose(net, draws, n, precision=BEC_FP32, max_iter=15000, log=None):
    """Where the learned start gains or loses, for draws of one gamma_z band: Algorithm 1 from four
    starts per draw, all in one batch: the plain guess, the network's guess, the network's modulus
    with the plain guess's phase ("envelope"), and the plain modulus with the network's phase
    ("phase"). The mixed starts are formed on the host and brought to unit mass there. Returns one
    record per draw: iterations, status and final energy per start, and each final energy's
    difference from the plain start's."""
    import torch
    assert all(gz_band(float(d[3])) == gz_band(float(draws[0][3])) for d in draws)
    a = box_for(float(draws[0][3]))
    h3 = 8.0 * a[0] * a[1] * a[2] / (n[0] * n[1] * n[2])
    plain = [plain_guess(d, n) for d in draws]
    learned = predict(net, draws, n).cpu().numpy()
    starts, kinds = [], ("plain", "learned", "envelope", "phase")
    for k in range(len(draws)):
        pl, le = plain[k], learned[k]
        pha = np.abs(pl) * np.exp(1j * np.angle(le))
        starts += [pl, le, envelope_start(le, pl, n, a), pha / math.sqrt(h3 * float(np.sum(np.abs(pha) ** 2)))]
    opts = bec_pcg_default_opts()
    opts.max_iter = int(max_iter)
    reps = [d for d in draws for _ in kinds]
    g, _, res, t = solve_batch(reps, n, starts, precision, opts)
    del g
    torch.cuda.synchronize()
    rows = []
    for k, d in enumerate(draws):
        r = {kind: res[4 * k + j] for j, kind in enumerate(kinds)}
        e0 = r["plain"].e.E
        rows.append(dict(draw=[float(v) for v in d], band=gz_band(float(d[3])),
                         **{kind: dict(status=x.status, iters=x.iters, E=x.e.E, dE=x.e.E - e0)
                            for kind, x in r.items()}))
        if log:
            log(f"diagnose draw {k}: " + "  ".join(f"{kind} {x.iters} it dE {x.e.E - e0:+.2e}"
                                                   f"{'' if x.status == 0 else ' (st %d)' % x.status}"
                                                   for kind, x in r.items()))
    if log:
        log(f"diagnose band {gz_band(float(draws[0][3]))}: {len(draws)} draws x 4 starts in {t:.1f}s")
    return rows


def summarize(rows, rel_tol=1e-10):
    """Gain of the learned guess: median iteration ratio, batch-time ratio, and the count of
    draws where it ends at a higher energy (a loss of the network) or a lower one."""
    ok = [r for r in rows if r["plain"]["status"] == 0 and r["learned"]["status"] == 0]
    ratio = [r["learned"]["iters"] / max(1, r["plain"]["iters"]) for r in ok]
    worse = sum(r["learned"]["E"] > r["plain"]["E"] + rel_tol * abs(r["plain"]["E"]) for r in ok)
    better = sum(r["learned"]["E"] < r["plain"]["E"] - rel_tol * abs(r["plain"]["E"]) for r in ok)
    bands = {}
    for r in rows:
        bands.setdefault(r["band"], (r["plain_batch_s"], r["learned_batch_s"]))
    tp = sum(v[0] for v in bands.values())
    tl = sum(v[1] for v in bands.values())
    return dict(draws=len(rows), both_converged=len(ok),
                iters_plain_median=float(np.median([r["plain"]["iters"] for r in ok])) if ok else None,
                iters_learned_median=float(np.median([r["learned"]["iters"] for r in ok])) if ok else None,
                iter_ratio_median=float(np.median(ratio)) if ok else None,
                learned_fewer_iters=sum(v < 1 for v in ratio), plain_seconds=tp, learned_seconds=tl,
                time_ratio=tl / tp if tp > 0 else None, higher_energy=worse, lower_energy=better)


def save(net, path, meta=None):
    """BF16 weights (the values the kernels use) plus FP32 biases, as an .npz file."""
    o = net.offsets()
    pb = net.params_bf16.cpu().numpy().view(np.uint16)
    p = net.params.cpu().numpy()
    arrs = {}
    for k, (a, b) in o.items():
        arrs[k] = p[a:b] if k.startswith("b") else pb[a:b]
    np.savez(path, dims=np.array(net.dims), meta=json.dumps(meta or {}), **arrs)


def load_default():
    """The shipped network (data/mlp_weights.npz)."""
    return load(WEIGHTS)


def load(path):
    """Network with the saved weights (BF16 weights widened to FP32 masters)."""
    z = np.load(path, allow_pickle=False)
    dims = tuple(int(v) for v in z["dims"])
    net = Mlp(*dims)
    parts = []
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        v = z[k]
        if k.startswith("W"):
            v = (v.astype(np.uint32) << 16).view(np.float32)
        parts.append(v.astype(np.float32))
    net.load_params(np.concatenate(parts))
    return net


def time_step(batch=256, steps=50, warmup=3):
    """Wall time of one training step (loss gradient + Adam) of the shipped architecture on a
    synthetic batch; returns seconds per step and the GEMM rate over the step."""
    import bec_inputs as bi
    import torch
    net = Mlp(*DIMS)
    net.load_params(bi.mlp_init(DIMS, 0))
    rng = np.random.default_rng(0)
    x = torch.from_numpy(rng.uniform(-1, 1, (batch, DIMS[0])).astype(np.float32)).to(net.device)
    t = torch.from_numpy((0.01 * rng.standard_normal((batch, DIMS[2]))).astype(np.float32)).to(net.device)
    for _ in range(warmup):
        net.loss_grad(x, t)
        net.adam_step(1e-3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.loss_grad(x, t)
        net.adam_step(1e-3)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    d_in, d_h, d_out = DIMS
    flops = 3 * 2 * batch * (d_h * d_h + d_h * d_out)   # forward + two backward products per layer
    return dict(batch=batch, steps=steps, ms_per_step=dt * 1e3, gemm_tflops=flops / dt / 1e12)


def main(argv=None):
    import bec_inputs as bi
    ap = argparse.ArgumentParser()
    ap.add_argument("--time-step", type=int, default=0, metavar="B",
                    help="only time training steps at batch B on a synthetic batch and exit")
    ap.add_argument("--eval-only", action="store_true",
                    help="skip training: evaluate the shipped network on the held-out draws at --eval-grid")
    ap.add_argument("--train", type=int, default=2000, help="training draws (seeds 0..)")
    ap.add_argument("--val", type=int, default=64, help="held-out draws (seeds 10^6..)")
    ap.add_argument("--val-start", type=int, default=0, help="first held-out seed offset (--eval-only)")
    ap.add_argument("--max-iter", type=int, default=4000)
    ap.add_argument("--epochs", type=int, default=1500)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-grid", type=int, nargs=3, default=None,
                    help="also solve the held-out draws from plain and learned guesses on this grid")
    ap.add_argument("--drop", type=float, default=1e-2, help="drop draws with boundary |phi| above this x max")
    ap.add_argument("--out", default=None)
    ap.add_argument("--diagnose-bands", type=int, nargs="*", default=None,
                    help="only run diagnose() on the held-out draws of these gamma_z bands at --eval-grid")
    ap.add_argument("--diag-per-band", type=int, default=4)
    ap.add_argument("--start", choices=("network", "envelope"), default="network",
                    help="learned start of --eval-only: the network's field, or its modulus with the plain phase")
    args = ap.parse_args(argv)
    if args.time_step:
        print(json.dumps(time_step(args.time_step)), flush=True)
        return
    if args.diagnose_bands is not None:
        grid = tuple(args.eval_grid or (256, 256, 64))
        log = lambda s: print(s, file=sys.stderr, flush=True)
        net = load_default()
        val = [bi.mlp_param_draw(10 ** 6 + s) for s in range(100)]
        out = []
        for band in args.diagnose_bands:
            ds = [d for d in val if gz_band(float(d[3])) == band][:args.diag_per_band]
            if ds:
                out += diagnose(net, ds, grid, max_iter=args.max_iter, log=log)
        print(json.dumps(dict(diagnose=dict(grid=list(grid), max_iter=args.max_iter, rows=out))), flush=True)
        return
    if args.eval_only:
        grid = tuple(args.eval_grid or (256, 256, 64))
        log = lambda s: print(s, file=sys.stderr, flush=True)
        val = [bi.mlp_param_draw(10 ** 6 + s) for s in range(args.val_start, args.val_start + args.val)]
        rows = evaluate(load_default(), val, grid, max_iter=args.max_iter, log=log, start=args.start)
        print(json.dumps(dict(eval=dict(grid=list(grid), max_iter=args.max_iter, start=args.start,
                                        summary=summarize(rows), rows=rows))), flush=True)
        return
    log = lambda s: print(s, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    draws = [bi.mlp_param_draw(s) for s in range(args.train)]
    val = [bi.mlp_param_draw(10 ** 6 + s) for s in range(args.val)]
    T, info = generate(draws, args.max_iter, log=log)
    Tv, infov = generate(val, args.max_iter, log=log)
    t_gen = time.perf_counter() - t0
    keep = [i for i, r in enumerate(info) if r["boundary"] <= args.drop]
    keepv = [i for i, r in enumerate(infov) if r["boundary"] <= args.drop]
    br = np.array([r["boundary"] for r in info])
    log(f"boundary ratio quantiles (10/50/90/max): {np.quantile(br, [0.1, 0.5, 0.9, 1.0])}; kept {len(keep)}/{len(info)}")
    X = np.stack([features(draws[i]) for i in keep])
    Xv = np.stack([features(val[i]) for i in keepv]) if keepv else None
    Tvk = Tv[keepv] if keepv else None
    net, hist = train(X, T[keep], epochs=args.epochs, batch=args.batch, lr=args.lr, log=log, X_val=Xv, T_val=Tvk)
    summary = dict(train=len(draws), kept=len(keep), dropped_frac=1 - len(keep) / len(draws),
                   val=len(val), val_kept=len(keepv), gen_seconds=t_gen,
                   converged=sum(r["status"] == 0 for r in info),
                   boundary_quantiles=[float(v) for v in np.quantile(br, [0.1, 0.5, 0.9, 1.0])],
                   iters_median=float(np.median([r["iters"] for r in info])),
                   final_loss=hist[-1]["loss"], final_val=hist[-1].get("val"),
                   seconds=time.perf_counter() - t0)
    if args.out:
        save(net, args.out, summary)
    out = dict(summary=summary, history=hist)
    if args.eval_grid:
        rows = evaluate(net, [val[i] for i in keepv], tuple(args.eval_grid), log=log)
        out["eval"] = dict(grid=args.eval_grid, summary=summarize(rows), rows=rows)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
