"""Spectral interpolation between two grids on one box, unit-mass scaling and the global
phase fix (Algorithm 2, step 2; Sec. 2.1, eqs. "Fourphi", "FourphiCo"; Sec. 3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading: Algorithm 2 interpolates a ground state to a refined mesh without naming the
interpolant. Here it is the grid function's own Fourier series (eq. "Fourphi") evaluated on
the new points, keeping the modes with |f| < min(N_src, N_dst)/2 per axis; the Nyquist mode
(f = -N/2) of either grid is dropped because its series term is not real-symmetric. On a
coarser grid the same rule truncates the series.
"""
from __future__ import annotations

import numpy as np


def _signed(k, n):
    return k if k < n // 2 else k - n


def resample(u, n_dst):
    """Fourier-series resampling of the 3-D grid function u to n_dst points per axis."""
    u = np.asarray(u, dtype=np.complex128)
    ns = u.shape
    c = np.fft.fftn(u) / u.size                         # coefficients of eq. "FourphiCo"
    out = np.zeros(tuple(n_dst), dtype=np.complex128)
    idx = []
    for a in range(3):
        lim = min(ns[a], n_dst[a]) // 2
        pairs = [(kd, f % ns[a]) for kd in range(n_dst[a]) for f in [_signed(kd, n_dst[a])] if abs(f) < lim]
        idx.append(pairs)
    for kx, sx in idx[0]:
        for ky, sy in idx[1]:
            kz = np.array([p[0] for p in idx[2]])
            sz = np.array([p[1] for p in idx[2]])
            out[kx, ky, kz] = c[sx, sy, sz]
    return np.fft.ifftn(out) * out.size                  # sum_k c_k exp(i nu_k (x + a))


def normalize(u, h3):
    """u / ||u|| with ||u||^2 = h3 sum |u|^2 (the constraint of eq. "groundDef")."""
    u = np.asarray(u, dtype=np.complex128)
    return u / np.sqrt(h3 * np.sum(np.abs(u) ** 2))


def gauge_fix(u, grid, gamma):
    """u times the unit complex number that makes sum u G real and positive,
    G = exp(-(gamma_x x^2 + gamma_y y^2 + gamma_z z^2)/2) on the grid points."""
    X, Y, Z = grid.mesh()
    G = np.exp(-0.5 * (gamma[0] * X ** 2 + gamma[1] * Y ** 2 + gamma[2] * Z ** 2))
    z = np.sum(np.asarray(u) * G)
    if z == 0:
        return np.asarray(u, dtype=np.complex128)
    return np.asarray(u, dtype=np.complex128) * (np.conj(z) / abs(z))
