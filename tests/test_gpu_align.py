"""GPU rotation about z (bec_rotate_z) against the oracle's shear rotation and exact quarter
turns, and the rotation-aligned error of Table 1 (Sec. 3, Example 3.1, Case I, Omega = 0.85,
two vortices) against the printed values."""
import json
import math
import os

import numpy as np
import pytest

import paper_2603_05194_amd as bec
from oracle import align as oa
from oracle.grid import Grid
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_table1.json")))


def smooth_field(g, seed):
    rng = np.random.default_rng(seed)
    X, Y, Z = g.mesh()
    u = np.zeros(g.n, dtype=np.complex128)
    for _ in range(4):
        x0, y0 = rng.uniform(-2, 2, 2)
        c = rng.standard_normal() + 1j * rng.standard_normal()
        u += c * np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / 2.0 - Z ** 2)
    return u


@pytest.mark.parametrize("alpha", [0.3, -1.1, 2.0, math.pi, 7.0])
def test_rotation_matches_oracle(alpha):
    n, a = (96, 96, 8), (12.0, 12.0, 4.0)
    g = bec.BecGrid(n, a, batch=2)
    G = Grid(n, a)
    u = np.stack([smooth_field(G, 1), smooth_field(G, 2)])
    got = host(g.rotate_z(dev(u), alpha))
    for b in range(2):
        ref = oa.rotate_z(u[b], G, alpha)
        assert np.max(np.abs(got[b] - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_quarter_turn_is_exact():
    n, a = (32, 32, 8), (6.0, 6.0, 3.0)
    g = bec.BecGrid(n, a)
    rng = np.random.default_rng(3)
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    r = host(g.rotate_z(dev(u), math.pi / 2))
    k = np.arange(32)
    ref = u[(32 - k) % 32][:, :, :].transpose(1, 0, 2)   # ref[j, k] = u[(N - k) % N, j]
    assert np.max(np.abs(r - ref)) <= 1e-12 * np.max(np.abs(u))


def test_rotation_aligned_error_two_vortices():
    """E2~ of Example 3.1, Case I, Omega = 0.85 (two vortices; in the isotropic trap any rotation of
    the ground state about z is equally a ground state), against our 256^3 state sampled on the
    coarse grids. The alignment must remove the rotation (E2~ << E2) and E2~ must fall spectrally
    with N. The printed Table 1 values (7.9153e-4 at 64^3, 1.4546e-7 at 128^3) are reported beside
    ours; they differ by a factor of about three and are not asserted (parity unpinned: the paper's
    minimiser and reference are not specified beyond fmincon and 512^3)."""
    from paper_2603_05194_amd import align as A
    from paper_2603_05194_amd import guesses as Gs
    c = GOLD["cases"]["I"]
    a, gam = tuple(c["box_half_widths"]), tuple(c["gamma"])
    o = bec.bec_pcg_default_opts()
    o.max_iter = 200000
    o.tol_res_inf = 1e-12
    print("Case I Omega 0.85: 256^3 reference", flush=True)
    _, ref, fine, _ = Gs.lowest_energy((256, 256, 256), a, gam, 100.0, 80.0, (0.0, 0.0, 1.0), 0.85, levels=3,
                                       precision=bec.BEC_FP64, opts=o)
    printed = GOLD["E2"]["I"].get("0.85", {"64": 7.9153e-04, "128": 1.4546e-07})
    got = {}
    for n in (64, 128):
        _, phi, _, _ = Gs.lowest_energy((n, n, n), a, gam, 100.0, 80.0, (0.0, 0.0, 1.0), 0.85, levels=3,
                                        precision=bec.BEC_FP64, opts=o)
        s = 256 // n
        pg = ref[::s, ::s, ::s].contiguous()
        g = bec.BecGrid((n, n, n), a)
        e, al = A.e2_tilde(g, phi.contiguous(), pg, period=math.pi)
        plain = A.e2(phi, pg)
        got[n] = e
        print(f"N {n}: E2~ {e:.5e} at alpha {al:.6f} (printed {printed[str(n)]:.5e}); E2 without rotation {plain:.3e}")
        assert e <= 1e-2 * plain
    assert got[128] <= 1e-2 * got[64]
