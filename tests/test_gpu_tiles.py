"""Line tiles of the runtime-length FFT kernels and their autotuner: tiles change only which block
handles which lines, so fields are bit-identical and reductions agree to rounding; H phi under
tuned tiles still matches the oracle; the search result is applied, reported and cached."""
import json
import math

import numpy as np
import pytest

import bec_inputs as bi
import paper_2603_05194_amd as bec
from oracle.energy import Model
from tests.gpu_util import dev, host, rel_max, params_of, torch_mod

pytestmark = pytest.mark.gpu

N, A = (24, 20, 12), (3.0, 2.5, 2.0)     # every axis and its padded length off the register kernels


def _model():
    return Model(N, A, (1.0, 1.3, 2.1), 40.0, -25.0, (0.3, -0.4, math.sqrt(1 - 0.25)), 0.6)


def _field(seed=3):
    rng = np.random.default_rng(seed)
    return bi.normalize(rng.standard_normal(N) + 1j * rng.standard_normal(N), N, A)


@pytest.mark.parametrize("div", [(2, 1, 1), (1, 4, 1), (1, 1, 2), (16, 16, 16), (4, 2, 8)])
def test_tiles_leave_fields_bit_identical(div):
    torch_mod()
    m, phi = _model(), _field()
    g = bec.BecGrid(N, A)
    assert g.line_tiles() == ((1, 1, 1), (1, 1, 1))
    h0, mu0, Phi0 = g.apply_H(params_of(m), dev(phi), want_Phi=True)
    e0 = g.energy(params_of(m), dev(phi))
    print(f"tiles {div}", flush=True)
    g.set_line_tiles(div)
    assert g.line_tiles()[0] == div
    h1, mu1, Phi1 = g.apply_H(params_of(m), dev(phi), want_Phi=True)
    e1 = g.energy(params_of(m), dev(phi))
    assert np.array_equal(host(h0), host(h1))
    assert np.array_equal(host(Phi0), host(Phi1))
    assert abs(float(host(mu1)[0]) - float(host(mu0)[0])) <= 1e-14 * abs(float(host(mu0)[0]))
    for k in ("E", "Ekin", "Edip", "Erot", "mu"):
        assert abs(e1[k] - e0[k]) <= 1e-14 * abs(e0[k]) + 1e-16, k
    assert rel_max(host(h1), m.H(phi)) < 1e-12


def test_bad_divisors_rejected():
    torch_mod()
    g = bec.BecGrid(N, A)
    for bad in ((3, 1, 1), (0, 1, 1), (1, 32, 1), (1, 1, -2)):
        with pytest.raises(RuntimeError):
            g.set_line_tiles(bad)
    assert g.line_tiles()[0] == (1, 1, 1)


def test_autotune_applies_choice_and_caches(tmp_path):
    torch = torch_mod()
    m, phi = _model(), _field(4)
    g = bec.BecGrid(N, A)
    cache = str(tmp_path / "tiles.json")
    print("autotune", flush=True)
    div, ms = g.autotune(params_of(m), dev(phi), reps=3, cache=cache)
    assert all(d in (1, 2, 4, 8, 16) for d in div) and ms > 0
    assert g.line_tiles()[0] == div
    h, mu = g.apply_H(params_of(m), dev(phi))
    assert rel_max(host(h), m.H(phi)) < 1e-12
    store = json.load(open(cache))
    assert store[g.tile_key()]["div"] == list(div)
    g2 = bec.BecGrid(N, A)
    div2, ms2 = g2.autotune(params_of(m), dev(phi), cache=cache)
    assert div2 == div and ms2 is None and g2.line_tiles()[0] == div
    torch.cuda.synchronize()


def test_autotune_skips_register_only_grids():
    torch_mod()
    w = bi.WORKLOADS["small_32"]
    n = (32, 32, 32)
    m = Model.from_workload(w, n=n)
    g = bec.BecGrid(n, w.a)
    assert g.line_tiles() == ((1, 1, 1), (0, 0, 0))
    div, ms = g.autotune(params_of(m), dev(bi.initial_guess(w, n)))
    assert div == (1, 1, 1) and ms is None


def test_batched_mixed_solve_with_tuned_tiles():
    """A batch of two FP32-bulk solves on a runtime-length grid after tuning reaches the same
    energies as with the default tiles (to the solver tolerance)."""
    torch = torch_mod()
    n, a = (24, 24, 12), (6.0, 6.0, 3.0)
    ms_ = [Model(n, a, (1.0, 1.0, 4.0), 80.0, 20.0 * k, (0.0, 0.0, 1.0), 0.3) for k in (1, 2)]
    X, Y, Z = np.meshgrid(*[-a[i] + np.arange(n[i]) * (2 * a[i] / n[i]) for i in range(3)], indexing="ij")
    phi0 = bi.normalize(np.exp(-0.5 * (X ** 2 + Y ** 2 + 4.0 * Z ** 2)).astype(complex), n, a)
    phis = np.stack([phi0, phi0])
    out = []
    for tune in (False, True):
        g = bec.BecGrid(n, a, precision=bec.BEC_FP32, batch=2)
        if tune:
            div, _ = g.autotune([params_of(m) for m in ms_], dev(phis.astype(np.complex64)), reps=2)
            print(f"tuned {div}", flush=True)
        res = g.pcg_solve_batched([params_of(m) for m in ms_], dev(phis))
        torch.cuda.synchronize()
        assert all(r.status == 0 for r in res)
        out.append([r.e.E for r in res])
    for e0, e1 in zip(*out):
        assert abs(e1 - e0) <= 1e-9 * abs(e0)
