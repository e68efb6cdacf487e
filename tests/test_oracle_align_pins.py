"""CPU pins of the oracle's rotation about z and of the rotation-aligned error: exact quarter
turns (index permutation), closed-form rotated Gaussians, inverse rotations, and invariances of
the error measure."""
import math

import numpy as np
import pytest

from oracle import align as oa
from oracle.grid import Grid


def gauss(grid, x0, y0, sx=1.0, sy=0.7):
    X, Y, Z = grid.mesh()
    return np.exp(-((X - x0) ** 2) / (2 * sx ** 2) - ((Y - y0) ** 2) / (2 * sy ** 2) - Z ** 2).astype(np.complex128)


def test_quarter_turn_is_an_index_permutation():
    g = Grid((32, 32, 8), (6.0, 6.0, 3.0))
    rng = np.random.default_rng(0)
    u = rng.standard_normal(g.n) + 1j * rng.standard_normal(g.n)
    r = oa.rotate_z(u, g, math.pi / 2)
    N = 32
    ref = np.empty_like(u)
    for j in range(N):
        for k in range(N):
            ref[j, k] = u[(N - k) % N, j]          # u(-y, x)
    assert np.max(np.abs(r - ref)) <= 1e-12 * np.max(np.abs(u))


@pytest.mark.parametrize("alpha", [0.3, -1.1, 2.0, math.pi])
def test_rotated_gaussian_closed_form(alpha):
    # the shears act on the periodic extension, so the field must have decayed within a margin
    # of the largest shift (|y| tan(alpha/2) where it is not negligible) of the box edge
    g = Grid((96, 96, 8), (12.0, 12.0, 4.0))
    x0, y0 = 0.5, -0.3
    r = oa.rotate_z(gauss(g, x0, y0), g, alpha)
    # u(R x) for an anisotropic Gaussian: evaluate at the rotated points directly
    X, Y, Z = g.mesh()
    ca, sa = math.cos(alpha), math.sin(alpha)
    Xr, Yr = ca * X - sa * Y, sa * X + ca * Y
    ref = np.exp(-((Xr - x0) ** 2) / 2 - ((Yr - y0) ** 2) / (2 * 0.49) - Z ** 2)
    assert np.max(np.abs(r - ref)) <= 1e-10


def test_rotation_and_its_inverse_cancel():
    g = Grid((48, 48, 8), (8.0, 8.0, 4.0))
    u = gauss(g, 0.7, 1.1) * np.exp(1j * 0.4 * gauss(g, -1.0, 0.0).real)
    back = oa.rotate_z(oa.rotate_z(u, g, 0.9), g, -0.9)
    assert np.max(np.abs(back - u)) <= 1e-10


def test_error_measures():
    g = Grid((40, 40, 8), (8.0, 8.0, 4.0))
    ref = gauss(g, 1.2, 0.5)
    assert oa.e2(np.exp(0.8j) * ref, ref) <= 1e-14
    u = oa.rotate_z(ref, g, -0.7)          # u(x) = ref(R_-0.7 x), so u(R_0.7 x) = ref(x)
    e, al = oa.e2_tilde(u, ref, g)
    assert e <= 1e-8 and abs(al - 0.7) <= 1e-6
    assert oa.e2(u, ref) > 0.1
