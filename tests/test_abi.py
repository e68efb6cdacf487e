"""CPU checks of the C ABI: the library loads, exports every symbol the public header declares,
and rejects bad arguments before touching a GPU."""
import ctypes as C
import os
import re

import pytest

import paper_2603_05194_amd as bec

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    syms = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            syms |= set(re.findall(r"\b(bec_[a-z0-9_]+)\s*\(", txt))
    return sorted(syms)


def test_library_exports_header_symbols():
    lib = bec._lib()
    syms = header_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(lib, s), s
    assert set(bec.EXPORTS) >= set(syms)


def test_struct_layouts_match_header():
    assert C.sizeof(bec.bec_grid_desc) == 40
    assert C.sizeof(bec.bec_params) == 8 * 9
    assert C.sizeof(bec.bec_energies) == 8 * 9


def test_validation_without_gpu():
    lib = bec._lib()
    out = C.c_size_t(0)
    good = bec.make_desc((32, 32, 16), (8, 8, 4))
    assert lib.bec_workspace_bytes(C.byref(good), 0, C.byref(out)) == 0 and out.value > 0
    for n, a in [((31, 32, 16), (8, 8, 4)), ((32, 2, 16), (8, 8, 4)), ((32, 32, 14), (8, 8, 4)),
                 ((32, 32, 16), (8, -1, 4)), ((32, 32, 4096), (8, 8, 4))]:
        d = bec.make_desc(n, a)
        assert lib.bec_workspace_bytes(C.byref(d), 0, C.byref(out)) == bec.BEC_EINVAL
        assert len(lib.bec_last_error()) > 0
    assert lib.bec_workspace_bytes(None, 0, C.byref(out)) == bec.BEC_EINVAL
    assert lib.bec_workspace_bytes(C.byref(good), 7, C.byref(out)) == bec.BEC_EINVAL
    h = C.c_void_p()
    assert lib.bec_init_grid(C.byref(good), 0, None, 0, None, C.byref(h)) == bec.BEC_EINVAL
    assert lib.bec_init_grid(C.byref(good), 0, C.c_void_p(4096), 16, None, C.byref(h)) == bec.BEC_ENOMEM
    assert lib.bec_init_grid(C.byref(good), 0, C.c_void_p(4097), 1 << 40, None, C.byref(h)) == bec.BEC_EINVAL
    assert lib.bec_apply_H(None, None, None, None, None, None) == bec.BEC_EINVAL
    o = bec.bec_pcg_default_opts()
    assert o.tol_res_inf == 1e-8 and o.max_halvings == 30 and o.t_default == 0.3
    assert bec._lib().bec_status_string(bec.BEC_ENOTCONV) == b"not converged"


def test_mlp_abi_validation_without_gpu():
    lib = bec._lib()
    assert bec.bec_mlp_param_count(6, 512, 32768) == 512 * 6 + 512 + 512 * 512 + 512 + 32768 * 512 + 32768
    assert lib.bec_mlp_param_count(0, 512, 32768) == 0
    net = bec.bec_mlp(6, 512, 32768, 256, 256, 256, 256, 256, 256, 256)
    out = C.c_size_t(0)
    assert lib.bec_mlp_scratch_bytes(C.byref(net), 4, C.byref(out)) == 0 and out.value > 4 * 32768 * 4
    assert lib.bec_mlp_scratch_bytes(C.byref(net), 0, C.byref(out)) == bec.BEC_EINVAL
    bad = bec.bec_mlp(6, 500, 32768, 256, 256, 256, 256, 256, 256, 256)
    assert lib.bec_mlp_scratch_bytes(C.byref(bad), 4, C.byref(out)) == bec.BEC_EINVAL
    assert len(lib.bec_mlp_last_error()) > 0
    nul = bec.bec_mlp(6, 512, 32768, None, 256, 256, 256, 256, 256, 256)
    assert lib.bec_mlp_sync(C.byref(nul), None) == bec.BEC_EINVAL
    # scratch too small: rejected before any launch
    assert lib.bec_mlp_forward(C.byref(net), 4, C.c_void_p(256), None, C.c_void_p(256), C.c_void_p(256), 16,
                               None) == bec.BEC_ENOMEM
    assert lib.bec_mlp_adam_step(C.byref(net), 1e-3, 0.9, 0.999, 1e-8, 0, None) == bec.BEC_EINVAL
    g = lib.bec_gemm_bf16_nt
    assert g(4, 4, 12, C.c_void_p(256), 16, C.c_void_p(256), 16, C.c_void_p(256), 4, None, 1, None, None) == bec.BEC_EINVAL
    assert g(4, 4, 16, C.c_void_p(258), 16, C.c_void_p(256), 16, C.c_void_p(256), 4, None, 1, None, None) == bec.BEC_EINVAL
    assert g(4, 4, 256, C.c_void_p(256), 256, C.c_void_p(256), 256, C.c_void_p(256), 4, None, 2, None, None) == bec.BEC_EINVAL


def test_interp_validation_without_gpu():
    lib = bec._lib()
    assert lib.bec_interp_spectral(None, None, None, 0, None, 0) == bec.BEC_EINVAL
    assert lib.bec_normalize(None, None) == bec.BEC_EINVAL
    assert lib.bec_gauge_fix(None, None, None) == bec.BEC_EINVAL
