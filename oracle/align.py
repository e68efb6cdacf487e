"""Rotation about z and the rotation-aligned relative error of Sec. 3 (accuracy study).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3 measures a computed state against a reference by the relative l2 error after removing the
global phase, and, for vortex states in a trap that is symmetric about z, after the rotation
that best aligns the two; the paper evaluates the rotated field with an FFT shear-decomposition
rotation. Here:
  rotate_z(u, grid, alpha)[x] = u(R_alpha x): three one-axis Fourier shifts (the grid
      function's Fourier series along one axis evaluated at shifted points), with
      R_alpha = S_x(t) S_y(s) S_x(t), t = -tan(alpha/2), s = sin(alpha), split into equal parts
      of at most pi/2; the Nyquist frequency is kept as -pi N/(2a);
  e2(u, ref) = ||u - kappa ref|| / ||ref||, kappa = <u, ref> / <ref, ref>;
  e2_tilde(u, ref, grid) = min over alpha of e2(rotate_z(u, alpha), ref), by a scan over the
      period followed by golden-section refinement.
"""
from __future__ import annotations

import math

import numpy as np


def _shift(u, axis, d_of_other, a):
    """u(s + d) along `axis` with d depending on the index along the other in-plane axis."""
    n = u.shape[axis]
    k = np.fft.fftfreq(n, 1.0 / n)
    nu = math.pi * k / a
    U = np.fft.fft(u, axis=axis)
    if axis == 0:
        ph = np.exp(1j * nu[:, None, None] * d_of_other[None, :, None])
    else:
        ph = np.exp(1j * nu[None, :, None] * d_of_other[:, None, None])
    return np.fft.ifft(U * ph, axis=axis)


def rotate_z(u, grid, alpha):
    u = np.asarray(u, dtype=np.complex128)
    parts = max(1, int(math.ceil(abs(alpha) / (0.5 * math.pi) - 1e-12)))
    a = alpha / parts
    t, s = -math.tan(0.5 * a), math.sin(a)
    x, y = grid.x[0], grid.x[1]
    for _ in range(parts):
        u = _shift(u, 0, t * y, grid.a[0])
        u = _shift(u, 1, s * x, grid.a[1])
        u = _shift(u, 0, t * y, grid.a[0])
    return u


def e2(u, ref):
    u = np.asarray(u)
    ref = np.asarray(ref)
    kappa = np.vdot(ref, u) / np.vdot(ref, ref)
    return float(np.linalg.norm(u - kappa * ref) / np.linalg.norm(ref))


def e2_tilde(u, ref, grid, period=2.0 * math.pi, scan=72, tol=1e-9):
    f = lambda al: e2(rotate_z(u, grid, al), ref)
    angles = np.arange(scan) * period / scan
    vals = [f(al) for al in angles]
    i = int(np.argmin(vals))
    lo, hi = angles[i] - period / scan, angles[i] + period / scan
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
