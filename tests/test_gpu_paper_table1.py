"""Paper-printed values (Sec. 3, Example 3.1, Table 1): the virial residual |I^h| of the
vortex-free ground states (Omega = 0.2, 0.4, 0.6) on the grids where it is set by the
discretization (32^3, 64^3 and, for the anisotropic trap, 128^3). The lowest-energy state over
the ten starting states of Sec. 3 is solved to ||r||_inf <= 1e-12 in FP64.

The printed values are reproduced to 0.03-0.4 %; the remaining difference is attributed to
discretization details the paper does not state (its symbol is a sum-of-Gaussians
approximation), so the test allows 1 %. A missing or mis-scaled energy term changes |I^h| by
orders of magnitude at these sizes."""
import json
import os

import pytest

import paper_2603_05194_amd as bec

pytestmark = pytest.mark.gpu
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_table1.json")))

CASES = [("I", om, n) for om in ("0.2", "0.4", "0.6") for n in (32, 64)] + \
        [("II", om, n) for om in ("0.2", "0.4") for n in (32, 64, 128)]


@pytest.mark.parametrize("case,om,n", CASES)
def test_table1_virial_residual(case, om, n):
    from paper_2603_05194_amd import guesses as G
    c = GOLD["cases"][case]
    o = bec.bec_pcg_default_opts()
    o.max_iter = 200000
    o.tol_res_inf = 1e-12
    print(f"Example 3.1 case {case} Omega {om} N {n}", flush=True)
    best, _, fine, _ = G.lowest_energy((n, n, n), tuple(c["box_half_widths"]), tuple(c["gamma"]), 100.0, 80.0,
                                       (0.0, 0.0, 1.0), float(om), levels=1, precision=bec.BEC_FP64, opts=o)
    r = fine[best]
    ref = GOLD["virial_abs"][case][om][str(n)]
    print(f"E {r['E']:.12f} |I| {abs(r['virial']):.5e} printed {ref:.5e}")
    assert r["res"] <= 1e-12
    assert abs(abs(r["virial"]) - ref) <= 1e-2 * ref


E2_CASES = [("I", "0.2"), ("II", "0.2")]


@pytest.mark.parametrize("case,om", E2_CASES)
def test_table1_relative_error_against_fine_solution(case, om):
    """E2 of Table 1 for a vortex-free state: ||phi^h - kappa phi_g|| / ||phi_g|| on the coarse
    grid, with phi_g our 256^3 ground state sampled at the coarse points (the paper's reference
    is 512^3; at 256^3 the printed error is already ~1e-11, far below the 32^3-128^3 values)."""
    import numpy as np
    from paper_2603_05194_amd import guesses as G
    from tests.gpu_util import host
    c = GOLD["cases"][case]
    a, gam = tuple(c["box_half_widths"]), tuple(c["gamma"])
    o = bec.bec_pcg_default_opts()
    o.max_iter = 200000
    o.tol_res_inf = 1e-12
    print(f"E2 case {case} Omega {om}: 256^3 reference", flush=True)
    best, ref, _, _ = G.lowest_energy((256, 256, 256), a, gam, 100.0, 80.0, (0.0, 0.0, 1.0), float(om), levels=3,
                                      precision=bec.BEC_FP64, opts=o)
    ref = host(ref)
    for n in (32, 64, 128):
        best, phi, _, _ = G.lowest_energy((n, n, n), a, gam, 100.0, 80.0, (0.0, 0.0, 1.0), float(om), levels=1,
                                          precision=bec.BEC_FP64, opts=o)
        phi = host(phi)
        s = 256 // n
        pg = ref[::s, ::s, ::s]
        kappa = np.vdot(pg, phi) / np.vdot(pg, pg)
        e2 = np.linalg.norm(phi - kappa * pg) / np.linalg.norm(pg)
        printed = GOLD["E2"][case][om][str(n)]
        print(f"N {n}: E2 {e2:.5e} printed {printed:.5e}")
        assert abs(e2 - printed) <= 2e-2 * printed
