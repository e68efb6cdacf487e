"""Uniform grid on an anisotropic box and its Fourier frequencies (Sec. 2.1).

Box D = prod_a [-a_a, a_a] with a_a = L xi_a; N_a even; h_a = 2 a_a / N_a;
x_j = -a_a + j h_a, j = 0..N_a-1 (the right end point is excluded).
Fourier index set k in {-N/2, ..., N/2-1}; nu_k = pi k / a_a.
Arrays are stored with index j (physical) or in FFT order (k = 0..N/2-1, -N/2..-1),
which is numpy's fftfreq order; nu at k = -N/2 is kept literally as -pi N/(2a).
"""
from __future__ import annotations

import math
import numpy as np


class Grid:
    def __init__(self, n, a):
        n = tuple(int(v) for v in n)
        a = tuple(float(v) for v in a)
        if any(v < 2 or v % 2 for v in n):
            raise ValueError("grid sizes must be even")
        if any(v <= 0 for v in a):
            raise ValueError("box half-widths must be positive")
        self.n, self.a = n, a
        self.h = tuple(2.0 * a[d] / n[d] for d in range(3))
        self.h3 = self.h[0] * self.h[1] * self.h[2]
        self.x = [-a[d] + np.arange(n[d]) * self.h[d] for d in range(3)]
        # k in numpy fftfreq order, nu_k = pi k / a (Sec. 2.1, W_k^L)
        self.k = [np.fft.fftfreq(n[d], 1.0 / n[d]) for d in range(3)]
        self.nu = [math.pi * self.k[d] / a[d] for d in range(3)]

    @property
    def shape(self):
        return self.n

    @property
    def size(self):
        return self.n[0] * self.n[1] * self.n[2]

    def mesh(self):
        return np.meshgrid(*self.x, indexing="ij")

    def nu_mesh(self):
        return np.meshgrid(*self.nu, indexing="ij")

    def padded(self):
        """The twofold box D_{2L xi} with 2N_a points (Sec. 2.2, eq. FourSeriB3):
        same mesh size, frequencies nu^p_k = pi k / (2 a_a), k in fftfreq(2N_a)."""
        return Grid(tuple(2 * v for v in self.n), tuple(2.0 * v for v in self.a))
