"""GPU solves of the configured workloads against the oracle beyond the apply-level checks:

 * density parity on reduced pancake and cigar grids, both sides run to ||r||_inf <= 1e-10 from
   the same guess (tests/golden/oracle_densities.json, written by make_oracle_densities.py);
 * the cigar workload at its full 128 x 128 x 256 size, FP64 and FP32 bulk + FP64 polish, each end
   state re-evaluated by the oracle;
 * a grid of the batched sweep (96 x 96 x 48) with three solves: batched equal to unbatched bit
   for bit, and the oracle's re-evaluation of each;
 * the paper's stopping rule ||phi_{n+1} - phi_n||_inf <= eps against the oracle's.
"""
import json
import os

import numpy as np
import pytest

import bec_inputs as bi
import paper_2603_05194_amd as bec
from oracle.energy import Model
from oracle.pcg import pcg
from tests.gpu_util import dev, host, params_of, torch_mod

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def gpu_solve(w, n, phi0, precision=bec.BEC_FP64, **kw):
    torch = torch_mod()
    g = bec.BecGrid(n, w.a, precision=precision)
    m = Model.from_workload(w, n=n)
    o = bec.bec_pcg_default_opts()
    for k, v in kw.items():
        setattr(o, k, v)
    phi = dev(phi0.copy())
    r = g.pcg_solve(params_of(m), phi, o)
    torch.cuda.synchronize()
    return r, host(phi), m


@pytest.mark.parametrize("name,n", [("cigar_128", (32, 32, 64)), ("pancake_256", (64, 64, 16))])
def test_reduced_density_parity(name, n):
    gold = json.load(open(os.path.join(GOLDEN, "oracle_densities.json")))[f"{name}@{n[0]}x{n[1]}x{n[2]}"]
    w = bi.WORKLOADS[name]
    print(f"density parity {name} {n}", flush=True)
    r, phi, m = gpu_solve(w, n, bi.initial_guess(w, n), tol_res_inf=gold["tol"], max_iter=100000)
    assert gold["status"] == "ok" and r.status == bec.BEC_OK
    rho = (np.abs(phi) ** 2).reshape(-1)
    gap = float(np.max(np.abs(rho[gold["index"]] - np.array(gold["rho"]))))
    print(f"{name} {n}: iters gpu {r.iters} oracle {gold['iters']}; dE {r.e.E - gold['E']:.2e} "
          f"dmu {r.e.mu - gold['mu']:.2e}; density L_inf gap on {len(gold['index'])} samples {gap:.2e}, "
          f"max {rho.max() - gold['rho_max']:.2e}")
    assert abs(r.e.E - gold["E"]) < 1e-10 * abs(gold["E"])
    assert abs(r.e.mu - gold["mu"]) < 1e-10 * abs(gold["mu"])
    assert gap < 1e-8
    assert abs(rho.max() - gold["rho_max"]) < 1e-8 and int(rho.argmax()) == gold["argmax"]
    assert abs(np.sqrt(m.grid.h3 * np.sum(rho * rho)) - gold["rho_l2"]) < 1e-8


def test_cigar_full_size_fp64_and_mixed():
    """Cigar workload at 128 x 128 x 256: FP64 and mixed solves from the same guess; the oracle's
    own H re-evaluates both end states (energy and residual), and the mixed state is the FP64
    ground state to the solver tolerance."""
    torch = torch_mod()
    w = bi.WORKLOADS["cigar_128"]
    phi0 = bi.initial_guess(w)
    print("cigar 128x128x256 fp64", flush=True)
    r64, p64, m = gpu_solve(w, w.n, phi0)
    print("cigar 128x128x256 mixed", flush=True)
    rmx, pmx, _ = gpu_solve(w, w.n, phi0, precision=bec.BEC_FP32)
    assert r64.status == bec.BEC_OK and rmx.status == bec.BEC_OK and rmx.fp32_iters > 0
    out = {}
    for name, r, phi in (("fp64", r64, p64), ("mixed", rmx, pmx)):
        e = m.energies(phi)
        res = float(np.max(np.abs(m.H(phi) - e.mu * phi)))
        out[name] = (e, res)
        assert abs(e.E - r.e.E) < 1e-12 * abs(e.E)
        assert abs(e.mu - r.e.mu) < 1e-11 * abs(e.mu)
        assert res <= 1.01e-8, (name, res)
    rho64, rhomx = np.abs(p64) ** 2, np.abs(pmx) ** 2
    drho = float(np.max(np.abs(rhomx - rho64)) / np.max(rho64))
    dE, dmu = rmx.e.E - r64.e.E, rmx.e.mu - r64.e.mu
    print(f"cigar full: fp64 {r64.iters} it; mixed {rmx.fp32_iters} fp32 + {rmx.iters - rmx.fp32_iters} fp64 it; "
          f"dE {dE:.2e} dmu {dmu:.2e} density rel L_inf {drho:.2e}; oracle residuals "
          f"{out['fp64'][1]:.2e} / {out['mixed'][1]:.2e}")
    assert abs(dE) <= 1e-10 * abs(r64.e.E)
    assert abs(dmu) <= 1e-8 * abs(r64.e.mu)
    assert drho <= 1e-6


def test_sweep_grid_batched_equals_unbatched():
    """Three solves of the 96 x 96 x 48 grid of the batched sweep (Omega x lambda/beta): one
    batch of three equals three single solves bit for bit, and the oracle re-evaluates each."""
    torch = torch_mod()
    ws = [w for w in bi.batched_sweep() if tuple(w.n) == (96, 96, 48)]
    pick = [ws[0], ws[5], ws[10]]
    assert len({(w.omega, w.lam) for w in pick}) == 3
    n, a = pick[0].n, pick[0].a
    phis = np.stack([bi.initial_guess(w) for w in pick])
    params = [params_of(Model.from_workload(w)) for w in pick]
    o = bec.bec_pcg_default_opts()
    print("sweep grid 96x96x48 batch of 3", flush=True)
    gb = bec.BecGrid(n, a, batch=3)
    db = dev(phis.copy())
    rb = gb.pcg_solve_batched(params, db, o)
    torch.cuda.synchronize()
    for k, w in enumerate(pick):
        g1 = bec.BecGrid(n, a)
        d1 = dev(phis[k].copy())
        r1 = g1.pcg_solve(params[k], d1, o)
        torch.cuda.synchronize()
        assert rb[k].status == bec.BEC_OK and r1.status == bec.BEC_OK
        assert rb[k].iters == r1.iters
        assert torch.equal(db[k], d1)
        m = Model.from_workload(w)
        phi = host(d1)
        e = m.energies(phi)
        assert abs(e.E - r1.e.E) < 1e-12 * abs(e.E)
        assert float(np.max(np.abs(m.H(phi) - e.mu * phi))) <= 1.01e-8
        print(f"  Omega {w.omega:.3f} lambda {w.lam:.0f}: {r1.iters} it, E {r1.e.E:.12f}, <L_z> "
              f"{-r1.e.Erot / w.omega:.4f}")


def test_step_rule_matches_oracle():
    """The paper's stopping rule ||phi_{n+1} - phi_n||_inf <= eps (residual test off) on both sides."""
    w = bi.WORKLOADS["small_32"]
    n = (16, 16, 16)
    m = Model.from_workload(w, n=n)
    phi0 = bi.initial_guess(w, n)
    ro = pcg(m, phi0, tol_res=0.0, tol_step=1e-7)
    r, phi, _ = gpu_solve(w, n, phi0, tol_res_inf=0.0, tol_step_inf=1e-7)
    print(f"step rule: gpu {r.iters} it (step {r.step_inf:.2e}), oracle {ro.iters} it (step {ro.step_inf:.2e})")
    assert ro.status == "ok" and r.status == bec.BEC_OK
    assert r.step_inf <= 1e-7 and ro.step_inf <= 1e-7
    assert abs(r.iters - ro.iters) <= 2
    assert abs(r.e.E - ro.energies.E) < 1e-10 * abs(ro.energies.E)
