"""The allocation-free H apply (bec_apply_H_static, static device scratch) against bec_apply_H on
a caller-owned workspace, through the C ABI: the same kernels on the same inputs give the same
H phi, Phi and mu bit for bit. Two calls in a row, the second on a smaller grid, then the first
grid again; a grid whose workspace exceeds the static scratch is rejected. The oracle's H phi
is checked as well."""
import numpy as np
import pytest

import bec_inputs as bi
import paper_2603_05194_amd as bec
from oracle.energy import Model
from tests.gpu_util import torch_mod, dev, host, rel_max

pytestmark = pytest.mark.gpu


def _both(w, n):
    torch = torch_mod()
    phi = dev(bi.initial_guess(w, n))
    p = bec.make_params(w.gamma, w.beta, w.lam, w.ndip, w.omega)
    g = bec.BecGrid(n, w.a)
    h_ref, mu_ref, Phi_ref = g.apply_H(p, phi, want_Phi=True)
    h = torch.empty_like(phi)
    Phi = torch.empty(n, dtype=torch.float64, device="cuda")
    mu = torch.empty(1, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream()
    print(f"static apply {n}", flush=True)
    bec.bec_apply_H_static(bec.make_desc(n, w.a), p, phi.data_ptr(), h.data_ptr(), Phi.data_ptr(), mu.data_ptr(),
                           s.cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(h, h_ref), float((h - h_ref).abs().max())
    assert torch.equal(Phi, Phi_ref)
    assert torch.equal(mu, mu_ref)
    ref = Model.from_workload(w, n=n).H(bi.initial_guess(w, n))
    assert rel_max(host(h), ref) < 1e-12
    return h


def test_static_apply_matches_workspace_apply():
    w = bi.WORKLOADS["pancake_256"]
    _both(w, (32, 32, 16))
    _both(w, (16, 16, 8))            # smaller grid: the static workspace is carved again
    _both(w, (32, 32, 16))
    ws = bi.WORKLOADS["small_32"]
    _both(ws, (24, 24, 24))          # another box, another symbol


def test_static_apply_rejects_oversized_grid():
    torch = torch_mod()
    w = bi.WORKLOADS["pancake_256"]
    n = (128, 128, 64)
    p = bec.make_params(w.gamma, w.beta, w.lam, w.ndip, w.omega)
    x = torch.zeros(8, dtype=torch.complex128, device="cuda")
    with pytest.raises(bec.BecError) as ei:
        bec.bec_apply_H_static(bec.make_desc(n, w.a), p, x.data_ptr(), x[4:].data_ptr())
    assert ei.value.code == bec.BEC_EINVAL and "static scratch" in str(ei.value)
    assert bec.bec_static_scratch_bytes() == 64 << 20
