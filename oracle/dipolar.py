"""Dipolar potential by the anisotropic truncated kernel method (Sec. 2.2).

Phi = U_dip * rho = -rho - 3 U * (d_nn rho)           (eq. "DDI2Cou3D")

On the twofold padded grid d_nn becomes -(n.nu)^2 in Fourier space, so

    Phi[rho] = -rho + Re( IDFT_{2N}( S . DFT_{2N}( pad(rho) ) ) ) restricted to D,
    S_k = 3 (n . nu_k)^2 U_k                            (eqs. "fouriercoeff", "U_TrunFour")

Readings:
 * pad() puts rho at the corner [0, N_a) of a zero 2N_a array and the result is read
   back from the same corner. The paper centres D in the twofold box; a circular
   shift of the padded grid changes nothing.
 * -rho is added in physical space (not folded into S).
 * Nyquist planes of the padded grid: the cross terms n_a n_b nu_a nu_b (a != b) are
   set to zero where nu_a or nu_b is the Nyquist frequency, so that S is real and even
   and the result real; the real part of the inverse transform is taken.
"""
from __future__ import annotations

import numpy as np

from . import spectral
from .symbol import symbol_full


def dipolar_symbol(grid, ndip, uhat_full=None):
    """S_k = 3 (n.nu_k)^2 U_k on the padded grid, FFT order, Nyquist cross terms zeroed."""
    if uhat_full is None:
        uhat_full = symbol_full(grid)
    pg = grid.padded()
    nu = pg.nu_mesh()
    nyq = [np.zeros(pg.n, dtype=bool) for _ in range(3)]
    ks = np.meshgrid(*pg.k, indexing="ij")
    for d in range(3):
        nyq[d] = ks[d] == -grid.n[d]
    nn = np.zeros(pg.n)
    for d in range(3):
        nn += ndip[d] ** 2 * nu[d] ** 2
    for d in range(3):
        for e in range(d + 1, 3):
            cross = 2.0 * ndip[d] * ndip[e] * nu[d] * nu[e]
            cross[nyq[d] | nyq[e]] = 0.0
            nn += cross
    return 3.0 * nn * uhat_full


def pad(grid, rho):
    pg = grid.padded()
    out = np.zeros(pg.n, dtype=rho.dtype)
    nx, ny, nz = grid.n
    out[:nx, :ny, :nz] = rho
    return out


def crop(grid, u):
    nx, ny, nz = grid.n
    return u[:nx, :ny, :nz]


def conv_part(grid, S, rho):
    """Re IDFT_{2N}(S DFT_{2N}(pad rho)) on D: the truncated-kernel convolution."""
    return np.real(crop(grid, spectral.ifftn(S * spectral.fftn(pad(grid, rho)))))


def potential(grid, S, rho):
    """Phi[rho] = -rho + Re IDFT_{2N}(S DFT_{2N}(pad rho)) on D."""
    return -rho + conv_part(grid, S, rho)


def normalize_axis(ndip, tol=1e-12):
    n = np.asarray(ndip, dtype=np.float64)
    nrm = float(np.sqrt(np.sum(n * n)))
    if abs(nrm - 1.0) > tol:
        raise ValueError("dipole axis must be a unit vector")
    return n / nrm
