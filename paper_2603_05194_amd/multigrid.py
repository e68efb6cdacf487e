"""Cascadic multigrid PCG-ATKM (Algorithm 2): Algorithm 1 on a coarse grid, spectral
interpolation of its ground state to the grid refined by two per axis, Algorithm 1 again,
up to the target grid. The paper runs three levels, from N/4 points per axis to N
(Sec. 3, set-up of the numerical results).

Each level's solve stops by the same rule as the finest one; the interpolated state is scaled
back to unit mass (dropping the Nyquist modes changes the mass slightly).
"""
from __future__ import annotations

import time

import numpy as np

from . import BEC_FP64, BecGrid, bec_pcg_default_opts


def levels(n, count=3):
    """Grids of the cascade, coarsest first: N / 2^(count-1-i) per axis."""
    out = []
    for i in range(count):
        f = 2 ** (count - 1 - i)
        lv = tuple(int(v) // f for v in n)
        if any(v * f != int(n[d]) or v < 4 or v % 2 for d, v in enumerate(lv)):
            raise ValueError(f"grid {tuple(n)} cannot be coarsened {count - 1} times by 2 (even sizes >= 4)")
        out.append(lv)
    return out


def solve(n, a, params, guess, precision=BEC_FP64, opts=None, count=3, log=None, coarse_opts=None):
    """Algorithm 2 on grid n (box half-widths a).

    `params` is one bec_params, or a list of them to run a batch of solves through the cascade
    together (one launch per phase on every level). `guess` is the complex128 initial guess on
    the coarsest grid ([Nx][Ny][Nz], or [batch][Nx][Ny][Nz] for a list of params): a device
    tensor, a numpy array, or a callable guess(nl) returning a numpy array. Returns (phi on grid n as a torch
    tensor, per-level records: one dict per level, or one list of dicts per level for a batch)."""
    import torch
    batched = isinstance(params, (list, tuple))
    plist = list(params) if batched else [params]
    B = len(plist)
    opts = opts or bec_pcg_default_opts()
    coarse_opts = coarse_opts or opts
    grids = levels(n, count)
    recs = []
    phi = None
    prev = None
    for li, nl in enumerate(grids):
        g = BecGrid(nl, a, precision=precision, batch=B)
        if prev is None:
            if torch.is_tensor(guess):
                phi = guess
            else:
                arr = guess if isinstance(guess, np.ndarray) else guess(nl)
                phi = torch.from_numpy(np.ascontiguousarray(arr)).to(g.device)
            phi = phi.reshape((B,) + tuple(nl)).contiguous()
        else:
            phi = prev.interp_to(g, phi)
            g.normalize_(phi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = g.pcg_solve_batched(plist, phi, opts if li == len(grids) - 1 else coarse_opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        lv = [dict(grid=list(nl), status=r.status, iters=r.iters, fp32_iters=r.fp32_iters, res=r.res_inf, E=r.e.E,
                   mu=r.e.mu, virial=r.e.virial, seconds=dt) for r in res]
        recs.append(lv if batched else lv[0])
        if log:
            log(f"level {li} {nl}: iterations {min(r.iters for r in res)}..{max(r.iters for r in res)}, {dt:.2f}s, "
                f"E min {min(r.e.E for r in res):.12f}")
        prev = g
    return (phi if batched else phi[0]), recs
