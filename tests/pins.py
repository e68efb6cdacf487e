"""Independent references that pin the oracle: closed forms, textbook routines and
brute-force definitions written out from the mathematics, sharing no arithmetic with
oracle/ (they never call it).

 * dft_matrices: the 1-D coefficient map and its inverse built entry by entry from the
   Fourier basis W_k(x) = exp(i nu_k (x + a)), k in {-N/2..N/2-1} (Sec. 2.1).
 * box_coulomb_F: int_{[0,a]x[0,b]x[0,c]} dV/|y| in closed form; U_0 = (2/pi) F(2ax,2ay,2az).
 * gaussian_potential: Phi(x) of a normalised anisotropic Gaussian density via a 1-D
   integral over the Gaussian-identity parameter s (derived from 1/|y| = 2/sqrt(pi) int e^{-s^2 y^2}).
 * gaussian_dipolar_J: int Phi rho for that Gaussian via a 1-D integral over t
   (from 1/|k|^2 = int_0^inf e^{-t k^2} dt in Fourier space).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.integrate as si


def dft_matrices(N, a):
    """F[k, j] = (1/N) conj(W_k(x_j)), B[j, k] = W_k(x_j), natural order k = -N/2..N/2-1."""
    h = 2.0 * a / N
    x = -a + h * np.arange(N)
    k = np.arange(-N // 2, N // 2)
    nu = math.pi * k / a
    W = np.exp(1j * np.outer(x + a, nu))        # W[j, k]
    return W.conj().T / N, W, nu, x


def apply_axis(M, u, axis):
    u = np.moveaxis(u, axis, 0)
    out = np.tensordot(M, u, axes=(1, 0))
    return np.moveaxis(out, 0, axis)


def box_coulomb_F(a, b, c):
    r = math.sqrt(a * a + b * b + c * c)
    return (b * c * math.asinh(a / math.hypot(b, c)) + a * c * math.asinh(b / math.hypot(a, c))
            + a * b * math.asinh(c / math.hypot(a, b))
            - 0.5 * a * a * math.atan(b * c / (a * r)) - 0.5 * b * b * math.atan(a * c / (b * r))
            - 0.5 * c * c * math.atan(a * b / (c * r)))


def gaussian_density(X, Y, Z, sig):
    out = 1.0
    for C, s in zip((X, Y, Z), sig):
        out = out * np.exp(-C * C / (2 * s * s)) / math.sqrt(2 * math.pi * s * s)
    return out


def gaussian_potential(X, Y, Z, sig, n, dtau=0.02, lo=-30.0, hi=12.0):
    """Phi(x) = -rho - 3/(2 pi^{3/2}) int_0^inf C(s) [4 (sum a n x)^2 - 2 sum a n^2] e^{-sum a x^2} ds,
    a_i(s) = s^2/(1 + 2 s^2 sig_i^2), C(s) = prod (1 + 2 s^2 sig_i^2)^{-1/2}; s = e^tau, trapezoid."""
    rho = gaussian_density(X, Y, Z, sig)
    acc = np.zeros(X.shape)
    taus = np.arange(lo, hi + dtau / 2, dtau)
    for tau in taus:
        s = math.exp(tau)
        a = [s * s / (1 + 2 * s * s * sg * sg) for sg in sig]
        C = 1.0
        for sg in sig:
            C /= math.sqrt(1 + 2 * s * s * sg * sg)
        lin = a[0] * n[0] * X + a[1] * n[1] * Y + a[2] * n[2] * Z
        quad = a[0] * X * X + a[1] * Y * Y + a[2] * Z * Z
        acc += s * C * (4 * lin * lin - 2 * (a[0] * n[0] ** 2 + a[1] * n[1] ** 2 + a[2] * n[2] ** 2)) * np.exp(-quad)
    return -rho - 3.0 / (2 * math.pi ** 1.5) * dtau * acc


def gaussian_dipolar_J(sig, n):
    """J = int Phi rho = (2pi)^{-3} [3 pi^{3/2} int_0^inf prod (sig^2+t)^{-1/2} sum n^2/(2(sig^2+t)) dt
    - pi^{3/2} / (sx sy sz)]."""
    def f(t):
        c = [s * s + t for s in sig]
        return (1.0 / math.sqrt(c[0] * c[1] * c[2])) * sum(n[i] ** 2 / (2 * c[i]) for i in range(3))
    val, _ = si.quad(f, 0.0, math.inf, epsabs=0, epsrel=2e-14, limit=400)
    return (3 * math.pi ** 1.5 * val - math.pi ** 1.5 / (sig[0] * sig[1] * sig[2])) / (2 * math.pi) ** 3
