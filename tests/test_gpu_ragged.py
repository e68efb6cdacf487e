"""Uneven grids in one call (bec_pcg_solve_ragged): solves of the batched sweep's four grids
(96x96x48, 128x128x48, 160x160x64, 192x192x64), two per grid, give bit for bit the results of one
batched solve per grid; FP64 and FP32 bulk + FP64 polish."""
import numpy as np
import pytest

import bec_inputs as bi
import paper_2603_05194_amd as bec
from oracle.energy import Model
from tests.gpu_util import host, params_of, torch_mod

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [bec.BEC_FP64, bec.BEC_FP32])
def test_ragged_equals_per_grid_batches(prec):
    torch = torch_mod()
    from paper_2603_05194_amd.sweep import group_by_grid
    ws = bi.batched_sweep()
    groups = list(group_by_grid(ws).items())
    assert len(groups) == 4
    picks = [(n, a, [ws[i] for i in idx[:2]]) for (n, a), idx in groups]
    o = bec.bec_pcg_default_opts()
    o.max_iter = 1500
    grids, plists, phis, refs = [], [], [], []
    for n, a, sel in picks:
        pl = [params_of(Model.from_workload(w)) for w in sel]
        guess = np.stack([bi.initial_guess(w) for w in sel])
        print(f"per-grid batch {n}", flush=True)
        g1 = bec.BecGrid(n, a, precision=prec, batch=len(sel))
        d1 = torch.from_numpy(guess.copy()).cuda()
        r1 = g1.pcg_solve_batched(pl, d1, o)
        torch.cuda.synchronize()
        refs.append((r1, d1))
        grids.append(bec.BecGrid(n, a, precision=prec, batch=len(sel)))
        plists.append(pl)
        phis.append(torch.from_numpy(guess.copy()).cuda())
    print("ragged call over the four grids", flush=True)
    res = bec.pcg_solve_ragged(grids, plists, phis, o)
    torch.cuda.synchronize()
    for (r1, d1), rr, dr, (n, a, sel) in zip(refs, res, phis, picks):
        for k in range(len(sel)):
            assert rr[k].status == r1[k].status and rr[k].iters == r1[k].iters, (n, k)
            assert rr[k].fp32_iters == r1[k].fp32_iters
            assert rr[k].e.E == r1[k].e.E and rr[k].e.mu == r1[k].e.mu
        assert torch.equal(dr, d1), n
        print(f"  {n}: iterations {[r.iters for r in rr]}, status {[r.status for r in rr]}")


def test_ragged_rejects_repeated_handles():
    torch = torch_mod()
    w = bi.batched_sweep()[0]
    g = bec.BecGrid(w.n, w.a)
    p = [params_of(Model.from_workload(w))]
    x = torch.from_numpy(bi.initial_guess(w)[None].copy()).cuda()
    with pytest.raises(bec.BecError) as ei:
        bec.pcg_solve_ragged([g, g], [p, p], [x, x])
    assert ei.value.code == bec.BEC_EINVAL
