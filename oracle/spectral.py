"""Fourier pseudo-spectral operators on the grid (Sec. 2.1, eqs. "Fourphi",
"FourphiCo", "Laplacian").

The discrete coefficients are phi_hat_k = (1/N) sum_j phi_j conj(W_k(x_j)) with
W_k(x_j) = exp(i nu_k (x_j + a)) = exp(2 pi i k j / N): a plain DFT, i.e.
numpy's fftn divided by N. Derivatives multiply the coefficients by i nu_k,
the Laplacian by -|nu|^2, and are evaluated back on the grid.
L_z = -i (x [[d_y]] - y [[d_x]]).
"""
from __future__ import annotations

import os
import numpy as np
import scipy.fft as sfft

WORKERS = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)


def fftn(u, axes=None):
    return sfft.fftn(u, axes=axes, workers=WORKERS)


def ifftn(u, axes=None):
    return sfft.ifftn(u, axes=axes, workers=WORKERS)


def neg_half_laplacian(grid, u):
    """-1/2 [[Delta]] u = ifftn( 1/2 |nu|^2 fftn(u) )."""
    NX, NY, NZ = grid.nu_mesh()
    return ifftn(0.5 * (NX * NX + NY * NY + NZ * NZ) * fftn(u))


def deriv(grid, u, axis):
    """[[d_axis]] u = ifftn( i nu_axis fftn(u) ), nu at k = -N/2 kept literally."""
    shape = [1, 1, 1]
    shape[axis] = grid.n[axis]
    nu = grid.nu[axis].reshape(shape)
    return sfft.ifft(1j * nu * sfft.fft(u, axis=axis, workers=WORKERS), axis=axis, workers=WORKERS)


def Lz(grid, u):
    """[[L_z]] u = -i ( x [[d_y]] u - y [[d_x]] u )."""
    X, Y, _ = grid.mesh()
    return -1j * (X * deriv(grid, u, 1) - Y * deriv(grid, u, 0))


def trap(grid, gamma):
    """V = 1/2 (gx^2 x^2 + gy^2 y^2 + gz^2 z^2) on the grid (eq. "Vpoten")."""
    X, Y, Z = grid.mesh()
    return 0.5 * (gamma[0] ** 2 * X * X + gamma[1] ** 2 * Y * Y + gamma[2] ** 2 * Z * Z)
