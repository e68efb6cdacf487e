"""Parity at full size against the oracle on the whole grid (the oracle's symbol comes from its
octant form, a few seconds on the host). For the pancake, 256 x 256 x 64 (padded 512 x 512 x 128),
in the kernels and launch shapes the bench times: the symbol, the ATKM potential, H phi, mu and
the energy parts, the first PCG iterations (Algorithm 1) in FP64, and H phi in FP32. For the
cigar, 128 x 128 x 256: H phi and the energies in FP64 and H phi in FP32."""
import numpy as np
import pytest

import bec_inputs as bi
import paper_2603_05194_amd as bec
from oracle import symbol as osym
from oracle.energy import Model
from oracle.grid import Grid
from oracle.pcg import pcg
from tests.gpu_util import dev, host, params_of, rel_max, torch_mod

pytestmark = pytest.mark.gpu

W = bi.WORKLOADS["pancake_256"]


@pytest.fixture(scope="module")
def full():
    torch_mod()
    print("oracle symbol and model at 256x256x64", flush=True)
    uh = osym.symbol_full_by_octant(Grid(W.n, W.a))
    m = Model.from_workload(W, uhat_full=uh)
    phi0 = bi.initial_guess(W)
    return m, uh, phi0


def test_symbol_full_size(full):
    m, uh, _ = full
    g = bec.BecGrid(W.n, W.a)
    got = host(g.symbol())
    ref = osym.octant(uh, Grid(W.n, W.a))
    assert got.shape == ref.shape == (257, 257, 65)
    assert rel_max(got, ref) < 1e-13


def test_apply_H_and_energy_full_size(full):
    m, _, phi0 = full
    g = bec.BecGrid(W.n, W.a)
    print("apply_H 256x256x64", flush=True)
    h, mu, Phi = g.apply_H(params_of(m), dev(phi0), want_Phi=True)
    assert rel_max(host(Phi), m.Phi(np.abs(phi0) ** 2)) < 1e-12
    assert rel_max(host(h), m.H(phi0)) < 1e-12
    e = m.energies(phi0).as_dict()
    assert abs(float(host(mu)[0]) - e["mu"]) < 1e-12 * abs(e["mu"])
    got = g.energy(params_of(m), dev(phi0))
    scale = sum(abs(e[k]) for k in ("Ekin", "Epot", "Eint", "Edip", "Erot"))
    for k in ("E", "Ekin", "Epot", "Eint", "Edip", "Erot", "mu", "mass"):
        assert abs(got[k] - e[k]) < 1e-12 * scale, (k, got[k], e[k])


def test_first_iterations_full_size(full):
    torch = torch_mod()
    m, _, phi0 = full
    k = 3
    print(f"oracle pcg {k} iterations at 256x256x64", flush=True)
    ro = pcg(m, phi0, max_iter=k)
    g = bec.BecGrid(W.n, W.a)
    o = bec.bec_pcg_default_opts()
    o.max_iter = k
    phi = dev(phi0.copy())
    r = g.pcg_solve(params_of(m), phi, o)
    torch.cuda.synchronize()
    assert r.status == bec.BEC_ENOTCONV and r.iters == k
    assert abs(r.e.E - ro.energies.E) < 1e-12 * abs(ro.energies.E)
    assert np.max(np.abs(host(phi) - ro.phi)) < 1e-10 * np.max(np.abs(ro.phi))
    assert r.halvings == ro.halvings and r.psd_resets == ro.resets


def test_apply_H_fp32_full_size(full):
    m, _, phi0 = full
    g = bec.BecGrid(W.n, W.a, precision=bec.BEC_FP32)
    h, _ = g.apply_H(params_of(m), dev(phi0.astype(np.complex64)))
    assert rel_max(host(h), m.H(phi0)) < 2e-5


def test_cigar_full_size_apply_and_energy():
    torch_mod()
    w = bi.WORKLOADS["cigar_128"]
    print("oracle model at 128x128x256", flush=True)
    m = Model.from_workload(w, uhat_full=osym.symbol_full_by_octant(Grid(w.n, w.a)))
    phi0 = bi.initial_guess(w)
    ref = m.H(phi0)
    g = bec.BecGrid(w.n, w.a)
    h, mu = g.apply_H(params_of(m), dev(phi0))
    assert rel_max(host(h), ref) < 1e-12
    e = m.energies(phi0).as_dict()
    got = g.energy(params_of(m), dev(phi0))
    scale = sum(abs(e[k]) for k in ("Ekin", "Epot", "Eint", "Edip", "Erot"))
    for k in ("E", "Ekin", "Epot", "Eint", "Edip", "Erot", "mu"):
        assert abs(got[k] - e[k]) < 1e-12 * scale, (k, got[k], e[k])
    g32 = bec.BecGrid(w.n, w.a, precision=bec.BEC_FP32)
    h32, _ = g32.apply_H(params_of(m), dev(phi0.astype(np.complex64)))
    assert rel_max(host(h32), ref) < 2e-5
