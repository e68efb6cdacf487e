"""GPU parity of the operator kernels against the oracle (and numpy's FFT for the transform):
3-D FFT, truncated-kernel symbol, ATKM dipolar potential, H phi, energy parts."""
import math

import numpy as np
import pytest

import bec_inputs as bi
import paper_2603_05194_amd as bec
from oracle import symbol as osym, dipolar as odip
from oracle.energy import Model
from oracle.grid import Grid
from tests.gpu_util import dev, host, rel_max, params_of

pytestmark = pytest.mark.gpu

SHAPES = [(8, 12, 16), (32, 32, 32), (24, 40, 10), (64, 64, 16), (96, 32, 48), (20, 12, 18), (16, 20, 50)]


@pytest.mark.parametrize("n", SHAPES)
def test_fft3d_matches_numpy(n):
    g = bec.BecGrid(n, (1.0, 1.0, 1.0))
    rng = np.random.default_rng(11)
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    fw = host(g.fft3d(dev(u), -1))
    assert rel_max(fw, np.fft.fftn(u)) < 1e-14 * max(8, math.log2(np.prod(n)))
    bw = host(g.fft3d(dev(u), +1))
    assert rel_max(bw, np.fft.ifftn(u) * np.prod(n)) < 1e-14 * max(8, math.log2(np.prod(n)))


@pytest.mark.parametrize("n,a", [((32, 32, 32), (8.0, 8.0, 4.0)), ((12, 20, 8), (3.0, 5.0, 2.0)),
                                 ((16, 16, 64), (4.0, 4.0, 24.0))])
def test_symbol_matches_oracle(n, a):
    g = bec.BecGrid(n, a)
    got = host(g.symbol())
    ref = osym.octant(osym.symbol_full(Grid(n, a)), Grid(n, a))
    assert got.shape == ref.shape
    # both sides sum the same O(U_0)-sized quadrature terms: the error is absolute, at the
    # rounding level of U_0, also where U_k itself is small
    assert rel_max(got, ref) < 1e-13


CASES = [
    ("small_32", None),
    ("small_32", (20, 12, 18)),
    ("pancake_256", (32, 32, 8)),
    ("cigar_128", (16, 16, 32)),
]


def _case(name, n):
    w = bi.WORKLOADS[name]
    n = tuple(n or w.n)
    m = Model.from_workload(w, n=n)
    phi = bi.initial_guess(w, n)
    return w, n, m, phi


@pytest.mark.parametrize("name,n", CASES)
def test_dipolar_matches_oracle(name, n):
    w, n, m, phi = _case(name, n)
    g = bec.BecGrid(n, w.a)
    got = host(g.dipolar(params_of(m), dev(phi)))
    ref = m.Phi(np.abs(phi) ** 2)
    assert rel_max(got, ref) < 1e-12


@pytest.mark.parametrize("name,n", CASES)
def test_apply_H_matches_oracle(name, n):
    w, n, m, phi = _case(name, n)
    g = bec.BecGrid(n, w.a)
    h, mu, Phi = g.apply_H(params_of(m), dev(phi), want_Phi=True)
    ref = m.H(phi)
    assert rel_max(host(h), ref) < 1e-12
    e = m.energies(phi)
    assert abs(float(host(mu)[0]) - e.mu) < 1e-12 * abs(e.mu)
    assert rel_max(host(Phi), m.Phi(np.abs(phi) ** 2)) < 1e-12


@pytest.mark.parametrize("name,n", CASES)
def test_energy_matches_oracle(name, n):
    w, n, m, phi = _case(name, n)
    g = bec.BecGrid(n, w.a)
    got = g.energy(params_of(m), dev(phi))
    ref = m.energies(phi).as_dict()
    scale = sum(abs(ref[k]) for k in ("Ekin", "Epot", "Eint", "Edip", "Erot"))
    for k in ("E", "Ekin", "Epot", "Eint", "Edip", "Erot", "mu", "mass", "virial"):
        assert abs(got[k] - ref[k]) < 1e-12 * scale, (k, got[k], ref[k])


def test_apply_H_random_field_all_terms():
    """A rough random field (all Fourier modes populated, Nyquist included)."""
    n, a = (16, 12, 20), (3.0, 2.0, 2.5)
    m = Model(n, a, (1.0, 1.7, 2.3), 37.0, -21.0, (0.3, -0.4, math.sqrt(1 - 0.25)), 0.7)
    rng = np.random.default_rng(5)
    phi = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    phi = bi.normalize(phi, n, a)
    g = bec.BecGrid(n, a)
    h, mu = g.apply_H(params_of(m), dev(phi))
    assert rel_max(host(h), m.H(phi)) < 1e-12


@pytest.mark.parametrize("name,n", [("small_32", None), ("pancake_256", (64, 64, 16))])
def test_generic_and_power_of_two_paths_agree(name, n, monkeypatch):
    """The compile-time power-of-two FFT kernels and the generic mixed-radix kernels give the
    same H phi and energies (both within the oracle tolerance)."""
    w, n, m, phi = _case(name, n)
    out = []
    for flag in ("1", "0"):
        monkeypatch.setenv("BEC_GENERIC_FFT", flag)
        g = bec.BecGrid(n, w.a)
        h, mu = g.apply_H(params_of(m), dev(phi))
        out.append((host(h), g.energy(params_of(m), dev(phi))))
    assert rel_max(out[0][0], out[1][0]) < 1e-13
    for k in ("E", "mu", "Edip"):
        assert abs(out[0][1][k] - out[1][1][k]) < 1e-13 * abs(out[1][1][k]) + 1e-15


MIXED_RADIX = [(96, 48, 160), (192, 20, 48), (160, 8, 96), (48, 16, 16)]


@pytest.mark.parametrize("n", MIXED_RADIX)
def test_mixed_radix_register_fft_matches_numpy(n):
    """Register kernels for 3 2^p and 5 2^p lengths (radix-3/5 stage, then radix 2 and 4)."""
    g = bec.BecGrid(n, (1.0, 1.0, 1.0))
    rng = np.random.default_rng(12)
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    print(f"fft3d {n}", flush=True)
    assert rel_max(host(g.fft3d(dev(u), -1)), np.fft.fftn(u)) < 1e-14 * math.log2(np.prod(n))
    assert rel_max(host(g.fft3d(dev(u), +1)), np.fft.ifftn(u) * np.prod(n)) < 1e-14 * math.log2(np.prod(n))


@pytest.mark.parametrize("n", [(96, 48, 160), (192, 160, 8)])
def test_mixed_radix_apply_H_matches_oracle_and_generic(n, monkeypatch):
    """H phi on grids whose N-grid and padded lengths (2N) are all 3 2^p or 5 2^p: register and
    runtime-length kernels agree, both match the oracle, in FP64; FP32 within its rounding."""
    a = (6.0, 4.0, 5.0)
    m = Model(n, a, (1.0, 1.4, 0.8), 60.0, -30.0, (0.6, 0.0, 0.8), 0.5)
    rng = np.random.default_rng(7)
    X, Y, Z = Grid(n, a).mesh()
    env = np.exp(-0.5 * (X ** 2 + 1.4 * Y ** 2 + 0.8 * Z ** 2))
    phi = bi.normalize(env * (1 + 0.1 * rng.standard_normal(n)) * np.exp(0.3j * rng.standard_normal(n)), n, a)
    ref = m.H(phi)
    out = []
    for flag in ("1", "0"):
        monkeypatch.setenv("BEC_GENERIC_FFT", flag)
        g = bec.BecGrid(n, a)
        print(f"apply_H {n} generic={flag}", flush=True)
        h, mu = g.apply_H(params_of(m), dev(phi))
        out.append(host(h))
        assert rel_max(out[-1], ref) < 1e-12
    assert rel_max(out[0], out[1]) < 1e-13
    monkeypatch.setenv("BEC_GENERIC_FFT", "0")
    g32 = bec.BecGrid(n, a, precision=bec.BEC_FP32)
    h32, _ = g32.apply_H(params_of(m), dev(phi.astype(np.complex64)))
    assert rel_max(host(h32), ref) < 2e-5
