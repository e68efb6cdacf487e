"""Launch-shape variants of the register kernels (bec_set_kernel_variants, bec_autotune_kernels):
fields are bit for bit those of the default shape, sums agree to rounding, and a short solve
under the tuner's choice tracks the default one; the oracle checks the apply."""
import numpy as np
import pytest

import bec_inputs as bi
import paper_2603_05194_amd as bec
from oracle.energy import Model
from tests.gpu_util import dev, host, params_of, rel_max, torch_mod

pytestmark = pytest.mark.gpu

# 256-point padded y lines (128-wide grid, no variants) and 512-point padded x lines (variants)
GRIDS = [("pancake_256", (256, 128, 16)), ("cigar_128", (160, 160, 32))]


@pytest.mark.parametrize("name,n", GRIDS)
@pytest.mark.parametrize("prec", [bec.BEC_FP64, bec.BEC_FP32])
def test_variants_leave_fields_bit_identical(name, n, prec):
    torch = torch_mod()
    w = bi.WORKLOADS[name]
    m = Model.from_workload(w, n=n)
    p = params_of(m)
    phi0 = bi.initial_guess(w, n)
    g = bec.BecGrid(n, w.a, precision=prec)
    g.ensure_symbol()
    x = dev(phi0).to(g.cdtype)
    ref_h, ref_mu, ref_Phi = g.apply_H(p, x, want_Phi=True)
    if prec == bec.BEC_FP64:
        assert rel_max(host(ref_h), m.H(phi0)) < 1e-12
    for v in range(1, bec.BEC_KERNEL_VARIANTS):
        print(f"{name} {n} prec {prec} variant {v}", flush=True)
        g.set_kernel_variants([v] * len(bec.SITES))
        h, mu, Phi = g.apply_H(p, x, want_Phi=True)
        torch.cuda.synchronize()
        assert torch.equal(h, ref_h) and torch.equal(Phi, ref_Phi), v
        assert abs(mu.item() - ref_mu.item()) <= 1e-13 * abs(ref_mu.item())


@pytest.mark.parametrize("name,n", GRIDS)
def test_variants_track_default_iterations(name, n):
    """Every pass of Algorithm 1 under every variant (the Parseval pass and the wide tiles
    included): the iterate after 12 FP64 iterations is the default's to rounding."""
    torch = torch_mod()
    w = bi.WORKLOADS[name]
    m = Model.from_workload(w, n=n)
    p = params_of(m)
    phi0 = bi.initial_guess(w, n)
    g = bec.BecGrid(n, w.a)
    g.ensure_symbol()
    o = bec.bec_pcg_default_opts()
    o.max_iter = 12
    o.tol_res_inf = 0.0
    ref = dev(phi0)
    r0 = g.pcg_solve(p, ref, o)
    for v in range(1, bec.BEC_KERNEL_VARIANTS):
        print(f"{name} {n} iterations, variant {v} on every site", flush=True)
        g.set_kernel_variants([v] * len(bec.SITES))
        x = dev(phi0)
        r = g.pcg_solve(p, x, o)
        torch.cuda.synchronize()
        assert r.iters == r0.iters == 12
        assert abs(r.e.E - r0.e.E) < 1e-13 * abs(r0.e.E), v
        assert float((x - ref).abs().max()) < 1e-11, v


def test_tuned_solve_tracks_default():
    torch = torch_mod()
    w = bi.WORKLOADS["pancake_256"]
    n = (128, 128, 32)
    m = Model.from_workload(w, n=n)
    p = params_of(m)
    phi0 = bi.initial_guess(w, n)
    g = bec.BecGrid(n, w.a)
    g.ensure_symbol()
    o = bec.bec_pcg_default_opts()
    o.max_iter = 200
    a = dev(phi0)
    ra = g.pcg_solve(p, a, o)
    chosen, times = g.autotune_kernels(p, dev(phi0), iters=5)
    print(f"tuned variants {chosen}")
    assert set(chosen) <= set(bec.SITES) and times
    # the Parseval pass has one shape variant (bit 0); no other value can be chosen there
    assert chosen.get("x_pars2", 0) in (0, 1)
    g.set_kernel_variants([3] * len(bec.SITES))      # every shape change that exists on this grid
    b = dev(phi0)
    rb = g.pcg_solve(p, b, o)
    torch.cuda.synchronize()
    assert ra.iters == rb.iters == 200
    assert abs(ra.e.E - rb.e.E) < 1e-12 * abs(ra.e.E)
    assert float((a - b).abs().max()) < 1e-9


def test_autotune_kernels_checks_the_scratch_field():
    """The tuner reads and overwrites batch x N complex128 values also on FP32 grids: a field of
    another type or shape is refused before anything runs."""
    torch = torch_mod()
    w = bi.WORKLOADS["small_32"]
    n = (32, 32, 16)
    m = Model.from_workload(w, n=n)
    p = params_of(m)
    g = bec.BecGrid(n, w.a, precision=bec.BEC_FP32, batch=2)
    with pytest.raises(ValueError):
        g.autotune_kernels([p, p], torch.zeros((2,) + n, dtype=torch.complex64, device="cuda"), iters=2)
    with pytest.raises(ValueError):
        g.autotune_kernels([p, p], torch.zeros(n, dtype=torch.complex128, device="cuda"), iters=2)
