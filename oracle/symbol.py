"""Fourier integral of the truncated Coulomb kernel on the twofold box (Sec. 2.2,
eq. "FUk"; computed once per box and grid, Remark after eq. "U_TrunFour").

    U_k = int_{D_{2L xi}} U(y) exp(-i nu_k . y) dy,   U(y) = 1/(4 pi |y|),

with nu_k = pi k / (2 a_a) for k in the index set of the 2N_a-point padded grid.

Reading (garbled passage): the paper writes the integrand with conj(W_k^{2L}(y)),
i.e. with an extra phase exp(-i nu (2 L xi)). By the convolution theorem the
kernel's transform carries no such offset, so U_k above has none. With the
phase the potential of a Gaussian is off by O(1); without it, it matches the
analytic potential to spectral accuracy.

Evaluation (the paper treats this as a sum-of-Gaussians black box): use the exact
identity 1/|y| = (2/sqrt(pi)) int_0^inf exp(-s^2 |y|^2) ds, which separates:

    U_k = 1/(2 pi^{3/2}) int_0^inf prod_a I(s; nu_a, b_a) ds,  b_a = 2 a_a,
    I(s; nu, b) = int_{-b}^{b} exp(-s^2 y^2) cos(nu y) dy.

The s-integral uses s = exp(tau) and the trapezoid rule with step 0.1 on
tau in [-40, 25]. I is the closed form sqrt(pi)/s exp(-nu^2/(4 s^2)) when
s b > 6.5 (neglected tail erfc(6.5) ~ 4e-20), else Gauss-Legendre on [-b, b]
with ceil(|nu| b / 2) + 80 nodes.
"""
from __future__ import annotations

import math
import numpy as np
import scipy.special as sps

TAU_LO, TAU_HI, TAU_STEP = -40.0, 25.0, 0.1
SB_CUT = 6.5


def tau_nodes():
    m = int(round((TAU_HI - TAU_LO) / TAU_STEP)) + 1
    tau = TAU_LO + TAU_STEP * np.arange(m)
    w = np.full(m, TAU_STEP)
    w[0] *= 0.5
    w[-1] *= 0.5
    return tau, w


_GL_CACHE = {}


def _gauss_legendre(n):
    if n not in _GL_CACHE:
        _GL_CACHE[n] = sps.roots_legendre(n)
    return _GL_CACHE[n]


def box_integral_1d(s, nu, b):
    """I(s; nu, b) = int_{-b}^{b} exp(-s^2 y^2) cos(nu y) dy for an array of s and one nu."""
    s = np.asarray(s, dtype=np.float64)
    out = np.empty_like(s)
    big = s * b > SB_CUT
    sb = s[big]
    out[big] = math.sqrt(math.pi) / sb * np.exp(-nu * nu / (4.0 * sb * sb))
    small = ~big
    if np.any(small):
        nq = int(math.ceil(abs(nu) * b / 2.0)) + 80
        t, wt = _gauss_legendre(nq)
        y = b * t                      # nodes on [-b, b]
        ss = s[small][:, None]
        f = np.exp(-(ss * ss) * (y * y)[None, :]) * np.cos(nu * y)[None, :]
        out[small] = b * (f @ wt)
    return out


def axis_tables(n_pad, a_pad):
    """Per-axis tables T[m, i] = I(exp(tau_m); nu_i, b) for the n_pad frequencies of
    one axis of the padded grid in FFT order (nu_i = pi k_i / a_pad, b = a_pad)."""
    tau, _ = tau_nodes()
    s = np.exp(tau)
    k = np.fft.fftfreq(n_pad, 1.0 / n_pad)
    nu = math.pi * k / a_pad
    T = np.empty((tau.size, n_pad))
    for i in range(n_pad):
        T[:, i] = box_integral_1d(s, nu[i], a_pad)
    return T


def symbol_full(grid, chunk=4):
    """U_k on the whole padded grid (2Nx, 2Ny, 2Nz), FFT order, FP64."""
    pg = grid.padded()
    tau, w = tau_nodes()
    coef = w * np.exp(tau) / (2.0 * math.pi ** 1.5)
    Tx, Ty, Tz = (axis_tables(pg.n[d], pg.a[d]) for d in range(3))
    out = np.empty(pg.n)
    Tyz = Ty[:, :, None] * Tz[:, None, :]            # [m, ky, kz]
    for i0 in range(0, pg.n[0], chunk):
        blk = (coef[:, None] * Tx[:, i0:i0 + chunk])[:, :, None, None] * Tyz[:, None, :, :]
        out[i0:i0 + chunk] = np.sum(blk, axis=0)      # pairwise summation over m
    return out


def symbol_full_by_octant(grid, chunk=4):
    """U_k on the whole padded grid from its values at k_a = 0..N_a: I(s; nu, b) is even in nu
    (cos is even), so U_k depends on |k_a| only. Same sums as symbol_full, 8x fewer of them."""
    pg = grid.padded()
    tau, w = tau_nodes()
    coef = w * np.exp(tau) / (2.0 * math.pi ** 1.5)
    T = [axis_tables(pg.n[d], pg.a[d])[:, : grid.n[d] + 1] for d in range(3)]
    nx, ny, nz = (v + 1 for v in grid.n)
    oct_ = np.empty((nx, ny, nz))
    Tyz = T[1][:, :, None] * T[2][:, None, :]
    for i0 in range(0, nx, chunk):
        blk = (coef[:, None] * T[0][:, i0:i0 + chunk])[:, :, None, None] * Tyz[:, None, :, :]
        oct_[i0:i0 + chunk] = np.sum(blk, axis=0)
    idx = [np.abs(np.fft.fftfreq(pg.n[d], 1.0 / pg.n[d])).astype(int) for d in range(3)]
    return oct_[np.ix_(idx[0], idx[1], idx[2])]


def symbol_at(grid, kx, ky, kz):
    """U_k for given padded-grid FFT-order indices (arrays of equal length)."""
    pg = grid.padded()
    tau, w = tau_nodes()
    coef = w * np.exp(tau) / (2.0 * math.pi ** 1.5)
    idx = (np.asarray(kx), np.asarray(ky), np.asarray(kz))
    cols = []
    for d in range(3):
        uniq, inv = np.unique(idx[d], return_inverse=True)
        k = np.fft.fftfreq(pg.n[d], 1.0 / pg.n[d])[uniq]
        s = np.exp(tau)
        T = np.stack([box_integral_1d(s, math.pi * kk / pg.a[d], pg.a[d]) for kk in k], axis=1)
        cols.append(T[:, inv])
    prod = coef[:, None] * cols[0] * cols[1] * cols[2]
    return np.sum(prod, axis=0)


def octant(full, grid):
    """The values at k_a = 0..N_a of each padded axis (the symbol is even in each nu_a)."""
    nx, ny, nz = grid.n
    return np.ascontiguousarray(full[: nx + 1, : ny + 1, : nz + 1])
