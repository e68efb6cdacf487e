"""Relative errors of Sec. 3 (accuracy study) between a computed state and a reference on the same
grid: E2 with the global phase removed, and E2~, which also removes the rotation about z that best
aligns the two (for vortex states in traps symmetric about z). The rotation runs in the library
(bec_rotate_z, three Fourier shears); the minimisation over the angle is a scan over the period
followed by golden-section refinement.
"""
from __future__ import annotations

import math


def e2(u, ref):
    """||u - kappa ref|| / ||ref||, kappa = <u, ref> / <ref, ref>; u and ref are device tensors (or
    host arrays), the sums are taken on the host in FP64."""
    import numpy as np
    a = _host(u).ravel()
    b = _host(ref).ravel()
    kappa = np.vdot(b, a) / np.vdot(b, b)
    return float(np.linalg.norm(a - kappa * b) / np.linalg.norm(b))


def _host(t):
    import numpy as np
    return t.detach().cpu().numpy() if hasattr(t, "detach") else np.asarray(t)


def e2_tilde(grid, u, ref, period=2.0 * math.pi, scan=72, tol=1e-9):
    """min over alpha of e2(u(R_alpha x), ref) and the minimising alpha; `grid` is the BecGrid of
    u (batch 1, N_x = N_y, a_x = a_y)."""
    ref = _host(ref)
    f = lambda al: e2(grid.rotate_z(u, al), ref)
    step = period / scan
    vals = [f(i * step) for i in range(scan)]
    i = min(range(scan), key=lambda k: vals[k])
    lo, hi = (i - 1) * step, (i + 1) * step
    g = (math.sqrt(5.0) - 1.0) / 2.0
    c, d = hi - g * (hi - lo), lo + g * (hi - lo)
    fc, fd = f(c), f(d)
    while hi - lo > tol:
        if fc < fd:
            hi, d, fd = d, c, fc
            c = hi - g * (hi - lo)
            fc = f(c)
        else:
            lo, c, fc = c, d, fd
            d = lo + g * (hi - lo)
            fd = f(d)
    al = 0.5 * (lo + hi)
    return f(al), al
