"""GPU checks of the drivers built on the solver: the cascadic multigrid of Algorithm 2, the
learned initial guess (shipped weights, save/load, a solve from its guess) and the batched
sweep. Results are compared with the oracle's solve of the same problem where one exists."""
import math
import os

import numpy as np
import pytest

import bec_inputs as bi
import paper_2603_05194_amd as bec
from oracle.energy import Model
from oracle.pcg import pcg
from tests.gpu_util import dev, host, params_of, torch_mod

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small32_oracle():
    w = bi.WORKLOADS["small_32"]
    m = Model.from_workload(w)
    return w, m, pcg(m, bi.initial_guess(w))


def test_multigrid_reaches_a_ground_state(small32_oracle):
    from paper_2603_05194_amd import multigrid as MG
    w, m, ro = small32_oracle
    print("multigrid small_32, 2 levels", flush=True)
    phi, recs = MG.solve(w.n, w.a, params_of(m), lambda nl: bi.initial_guess(w, nl), count=2)
    phi = host(phi)
    assert [r["grid"] for r in recs] == [[16, 16, 16], [32, 32, 32]]
    assert all(r["status"] == bec.BEC_OK and r["res"] <= 1e-8 for r in recs)
    # a critical point of the oracle's energy on the unit sphere, at or below the direct solve
    e = m.energies(phi)
    assert abs(e.mass - 1.0) < 1e-12
    assert np.max(np.abs(m.H(phi) - e.mu * phi)) <= 1.01e-8
    assert e.E <= ro.energies.E * (1 + 1e-10)
    print(f"multigrid E {e.E:.14f} direct oracle E {ro.energies.E:.14f}")


def test_shipped_network_prediction_is_a_unit_mass_field():
    from paper_2603_05194_amd import learned as L
    net = L.load_default()
    assert net.dims == L.DIMS
    draws = [bi.mlp_param_draw(10 ** 6 + s) for s in range(40)]
    band = L.gz_band(draws[0][3])
    ds = [d for d in draws if L.gz_band(d[3]) == band][:3]
    fine = host(L.predict(net, ds, (64, 64, 16)))
    a = L.box_for(ds[0][3])
    h3 = (2 * a[0] / 64) * (2 * a[1] / 64) * (2 * a[2] / 16)
    assert fine.shape == (len(ds), 64, 64, 16) and np.all(np.isfinite(fine))
    for b in range(len(ds)):
        assert h3 * np.sum(np.abs(fine[b]) ** 2) == pytest.approx(1.0, abs=1e-12)


def test_save_load_roundtrip(tmp_path):
    torch = torch_mod()
    from paper_2603_05194_amd import learned as L
    dims = (6, 64, 128)
    net = bec.Mlp(*dims)
    net.load_params(bi.mlp_init(dims, 4))
    x = torch.from_numpy(np.random.default_rng(1).uniform(-1, 1, (5, 6)).astype(np.float32)).cuda()
    y0 = host(net.forward(x))
    path = os.path.join(tmp_path, "w.npz")
    L.save(net, path)
    net2 = L.load(path)
    assert net2.dims == dims
    assert np.array_equal(host(net2.forward(x)), y0)


def test_solve_from_learned_guess_converges():
    from paper_2603_05194_amd import learned as L
    net = L.load_default()
    d = bi.mlp_param_draw(10 ** 6 + 7)
    n = (64, 64, 32)
    phi = L.predict(net, [d], n)
    g = bec.BecGrid(n, L.box_for(d[3]), precision=bec.BEC_FP32, batch=1)
    r = g.pcg_solve_batched([L.params_of(d)], phi.contiguous())
    print(f"learned guess: {r[0].iters} iterations, E {r[0].e.E:.12f}")
    assert r[0].status == bec.BEC_OK and r[0].res_inf <= 1e-8


def test_quick_sweep_groups_and_extracts():
    from paper_2603_05194_amd import sweep as S
    ws = bi.batched_sweep(quick=True)
    pick = [ws[0], ws[1], ws[15], ws[16], ws[17]]
    o = bec.bec_pcg_default_opts()
    o.max_iter = 3000
    res = S.run_sweep(pick, [bi.initial_guess(w) for w in pick], bec.BEC_FP32, o)
    assert len(res) == 5 and all(r is not None for r in res)
    for r, w in zip(res, pick):
        assert r["n"] == list(w.n) and math.isfinite(r["E"]) and math.isfinite(r["Lz"])
    oc = S.critical_omega(res)
    assert set(oc) == {w.lam for w in pick}
