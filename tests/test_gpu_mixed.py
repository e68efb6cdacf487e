"""The mixed-precision comparison (FP32 bulk + FP64 polish against plain FP64 from the same guess)
on a reduced cigar grid: the mixed result is the FP64 ground state to the solver tolerance."""
import pytest

import bec_inputs as bi
from tests.gpu_util import torch_mod

pytestmark = pytest.mark.gpu


def test_mixed_reaches_fp64_ground_state_reduced_cigar():
    torch_mod()
    from paper_2603_05194_amd import mixed
    w = bi.WORKLOADS["cigar_128"].with_grid((32, 32, 64))
    print(f"mixed vs fp64 on {w.n}", flush=True)
    out = mixed.compare(w)
    assert out["fp64"]["status"] == 0 and out["mixed"]["status"] == 0
    assert out["mixed"]["fp32_iters"] > 0
    d = out["mixed_vs_fp64"]
    E = out["fp64"]["E"]
    assert abs(d["dE"]) <= 1e-10 * abs(E)
    assert abs(d["dmu"]) <= 1e-8 * abs(out["fp64"]["mu"])
    assert d["density_rel_linf"] <= 1e-7
    assert d["fp64_residual_of_mixed_state"] <= 1.5e-8
