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
    """Algorithm 2 on grid n (box half-widths a) for one parameter set.

    `guess` is the complex128 initial guess on the coarsest grid: a device tensor, or a
    callable guess(nl) returning a numpy array. Returns (phi on grid n as a torch tensor,
    per-level records)."""
    import torch
    opts = opts or bec_pcg_default_opts()
    coarse_opts = coarse_opts or opts
    grids = levels(n, count)
    recs = []
    phi = None
    prev = None
    for li, nl in enumerate(grids):
        g = BecGrid(nl, a, precision=precision)
        if prev is None:
            phi = guess if torch.is_tensor(guess) else torch.from_numpy(np.ascontiguousarray(guess(nl))).to(g.device)
            assert tuple(phi.shape) == tuple(nl)
        else:
            phi = prev.interp_to(g, phi)
            g.normalize_(phi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = g.pcg_solve(params, phi, opts if li == len(grids) - 1 else coarse_opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        recs.append(dict(grid=list(nl), status=r.status, iters=r.iters, fp32_iters=r.fp32_iters, res=r.res_inf,
                         E=r.e.E, mu=r.e.mu, seconds=dt))
        if log:
            log(f"level {li} {nl}: {r.iters} iterations, {dt:.2f}s, E {r.e.E:.12f}, res {r.res_inf:.2e}")
        prev = g
    return phi, recs
