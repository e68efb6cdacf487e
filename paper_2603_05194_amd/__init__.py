"""MI355X-native PCG-ATKM ground states of rotating dipolar BECs.

Thin ctypes binding over libbec.so (HIP kernels for gfx950 + C ABI, see include/bec.h).
The functions named bec_* marshal arguments only; every step of the computation runs in
the library's kernels. torch provides device memory and the stream.

The library must be built (python -m paper_2603_05194_amd.build); importing the binding
without it raises at first use, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbec.so")

BEC_OK, BEC_EINVAL, BEC_ENOMEM, BEC_EHIP, BEC_ENOTCONV, BEC_ENUMERIC, BEC_ESTALL = 0, -1, -2, -3, -4, -5, -6
BEC_FP64, BEC_FP32 = 0, 1
BEC_MIXED = BEC_FP32      # the same precision mode under the name the mixed-precision path goes by
# launch sites of one PCG iteration (bec_pcg_profile), in the order of the BEC_SITE_* enum
SITES = ("control", "finish", "prec_z", "prec_y", "prec_x", "prec_zi", "dir_z", "y_fwd", "x_pars2", "p_lines",
         "retract", "atkm_z", "x_atkm", "y_inv", "atkm_zi", "h_z", "h_y", "h_x", "other")
BEC_NSITES = len(SITES)
BEC_KERNEL_VARIANTS = 8   # launch-shape variants per site, 0 .. 7 (include/bec.h)


class bec_grid_desc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("a", C.c_double * 3)]


class bec_params(C.Structure):
    _fields_ = [("gamma", C.c_double * 3), ("beta", C.c_double), ("lambda_", C.c_double),
                ("n", C.c_double * 3), ("omega", C.c_double)]


class bec_energies(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("E", "Ekin", "Epot", "Eint", "Edip", "Erot", "mu", "mass", "virial")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class bec_pcg_opts(C.Structure):
    _fields_ = [("tol_res_inf", C.c_double), ("tol_step_inf", C.c_double), ("max_iter", C.c_int32),
                ("max_halvings", C.c_int32), ("t_default", C.c_double), ("tau_E_ulps", C.c_double),
                ("switch_res", C.c_double), ("check_every", C.c_int32), ("debug_flags", C.c_int32),
                ("debug_t", C.c_double), ("debug_c2", C.c_double), ("stall_window", C.c_int32),
                ("use_graph", C.c_int32), ("switch_relative", C.c_int32), ("branches", C.c_int32)]


class bec_pcg_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("halvings", C.c_int32),
                ("psd_resets", C.c_int32), ("forced_accepts", C.c_int32), ("fp32_iters", C.c_int32),
                ("res_inf", C.c_double), ("step_inf", C.c_double), ("e", bec_energies)]


class bec_mlp(C.Structure):
    _fields_ = [("d_in", C.c_int32), ("d_h", C.c_int32), ("d_out", C.c_int32), ("params", C.c_void_p),
                ("params_bf16", C.c_void_p), ("w2t_bf16", C.c_void_p), ("w3t_bf16", C.c_void_p),
                ("grads", C.c_void_p), ("adam_m", C.c_void_p), ("adam_v", C.c_void_p)]


class BecError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = (_lib().bec_mlp_last_error() if where.startswith(("bec_mlp", "bec_gemm")) else _lib().bec_last_error())
        super().__init__(f"{where}: {code} ({_lib().bec_status_string(code).decode()}): {msg.decode()}")


_LIB = None
_SIGS = {
    "bec_status_string": (C.c_char_p, [C.c_int]),
    "bec_last_error": (C.c_char_p, []),
    "bec_version": (C.c_int, []),
    "bec_workspace_bytes": (C.c_int, [C.POINTER(bec_grid_desc), C.c_int, C.POINTER(C.c_size_t)]),
    "bec_workspace_bytes_batched": (C.c_int, [C.POINTER(bec_grid_desc), C.c_int, C.c_int, C.POINTER(C.c_size_t)]),
    "bec_init_grid_batched": (C.c_int, [C.POINTER(bec_grid_desc), C.c_int, C.c_int, C.c_void_p, C.c_size_t,
                                        C.c_void_p, C.POINTER(C.c_void_p)]),
    "bec_grid_batch": (C.c_int, [C.c_void_p]),
    "bec_pcg_solve_batched": (C.c_int, [C.c_void_p, C.POINTER(bec_params), C.c_void_p, C.POINTER(bec_pcg_opts),
                                        C.POINTER(bec_pcg_result)]),
    "bec_init_grid": (C.c_int, [C.POINTER(bec_grid_desc), C.c_int, C.c_void_p, C.c_size_t, C.c_void_p,
                                C.POINTER(C.c_void_p)]),
    "bec_destroy_grid": (C.c_int, [C.c_void_p]),
    "bec_atkm_symbol": (C.c_int, [C.c_void_p, C.c_void_p]),
    "bec_dipolar": (C.c_int, [C.c_void_p, C.POINTER(bec_params), C.c_void_p, C.c_void_p]),
    "bec_apply_H": (C.c_int, [C.c_void_p, C.POINTER(bec_params), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "bec_energy": (C.c_int, [C.c_void_p, C.POINTER(bec_params), C.c_void_p, C.c_void_p, C.c_int]),
    "bec_apply_H_static": (C.c_int, [C.POINTER(bec_grid_desc), C.POINTER(bec_params), C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p]),
    "bec_static_scratch_bytes": (C.c_int, [C.POINTER(C.c_size_t)]),
    "bec_pcg_solve": (C.c_int, [C.c_void_p, C.POINTER(bec_params), C.c_void_p, C.POINTER(bec_pcg_opts),
                                C.POINTER(bec_pcg_result)]),
    "bec_pcg_default_opts": (C.c_int, [C.POINTER(bec_pcg_opts)]),
    "bec_pcg_solve_ragged": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int,
                                       C.POINTER(bec_pcg_opts), C.POINTER(bec_pcg_result)]),
    "bec_fft3d": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "bec_time_stage": (C.c_int, [C.c_void_p, C.POINTER(bec_params), C.c_void_p, C.c_int, C.c_int,
                                 C.POINTER(C.c_double)]),
    "bec_pcg_profile": (C.c_int, [C.c_void_p, C.POINTER(bec_params), C.c_void_p, C.c_int, C.c_int,
                                  C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "bec_interp_spectral": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_int]),
    "bec_normalize": (C.c_int, [C.c_void_p, C.c_void_p]),
    "bec_gauge_fix": (C.c_int, [C.c_void_p, C.POINTER(bec_params), C.c_void_p]),
    "bec_rotate_z": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double]),
    "bec_set_kernel_variants": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "bec_get_kernel_variants": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "bec_autotune_kernels": (C.c_int, [C.c_void_p, C.POINTER(bec_params), C.c_void_p, C.c_int, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "bec_set_line_tiles": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "bec_get_line_tiles": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "bec_autotune_line_tiles": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.POINTER(C.c_int32),
                                          C.POINTER(C.c_double)]),
    # learned initial guess (include/bec_mlp.h)
    "bec_mlp_last_error": (C.c_char_p, []),
    "bec_mlp_param_count": (C.c_size_t, [C.c_int, C.c_int, C.c_int]),
    "bec_mlp_scratch_bytes": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_size_t)]),
    "bec_mlp_sync": (C.c_int, [C.c_void_p, C.c_void_p]),
    "bec_mlp_forward": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                  C.c_void_p]),
    "bec_mlp_loss_grad": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_size_t, C.c_void_p]),
    "bec_mlp_adam_step": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32,
                                    C.c_void_p]),
    "bec_gemm_bf16_nt": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_void_p,
                                   C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
}
EXPORTS = tuple(_SIGS)


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2603_05194_amd.build`")
        # torch ships its own HIP runtime under the same soname. Importing torch first makes the
        # loader bind libbec.so to that copy; loading libbec.so first would pull in a second
        # runtime that sees none of the memory or streams torch hands over.
        import torch  # noqa: F401
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def _check(rc, where, ok=(BEC_OK,)):
    if rc not in ok:
        raise BecError(rc, where)
    return rc


# ------------------------------------------------------------------ raw binding (same names)
def bec_workspace_bytes(desc: bec_grid_desc, precision: int) -> int:
    out = C.c_size_t(0)
    _check(_lib().bec_workspace_bytes(C.byref(desc), precision, C.byref(out)), "bec_workspace_bytes")
    return out.value


def bec_workspace_bytes_batched(desc: bec_grid_desc, precision: int, batch: int) -> int:
    out = C.c_size_t(0)
    _check(_lib().bec_workspace_bytes_batched(C.byref(desc), precision, batch, C.byref(out)),
           "bec_workspace_bytes_batched")
    return out.value


def bec_init_grid(desc, precision, d_ws, ws_bytes, stream):
    h = C.c_void_p()
    _check(_lib().bec_init_grid(C.byref(desc), precision, C.c_void_p(d_ws), ws_bytes, C.c_void_p(stream),
                                C.byref(h)), "bec_init_grid")
    return h


def bec_init_grid_batched(desc, precision, batch, d_ws, ws_bytes, stream):
    h = C.c_void_p()
    _check(_lib().bec_init_grid_batched(C.byref(desc), precision, batch, C.c_void_p(d_ws), ws_bytes,
                                        C.c_void_p(stream), C.byref(h)), "bec_init_grid_batched")
    return h


def bec_destroy_grid(h):
    return _lib().bec_destroy_grid(h)


def bec_atkm_symbol(h, d_out=None):
    _check(_lib().bec_atkm_symbol(h, C.c_void_p(d_out) if d_out else None), "bec_atkm_symbol")


def bec_dipolar(h, params, d_phi, d_Phi):
    _check(_lib().bec_dipolar(h, _params_arg(params), C.c_void_p(d_phi), C.c_void_p(d_Phi)), "bec_dipolar")


def bec_apply_H(h, params, d_phi, d_hphi, d_Phi=None, d_mu=None):
    _check(_lib().bec_apply_H(h, _params_arg(params), C.c_void_p(d_phi), C.c_void_p(d_hphi),
                              C.c_void_p(d_Phi) if d_Phi else None, C.c_void_p(d_mu) if d_mu else None),
           "bec_apply_H")


def bec_apply_H_static(desc, params, d_phi, d_hphi, d_Phi=None, d_mu=None, stream=None):
    _check(_lib().bec_apply_H_static(C.byref(desc), C.byref(params), C.c_void_p(d_phi), C.c_void_p(d_hphi),
                                     C.c_void_p(d_Phi) if d_Phi else None, C.c_void_p(d_mu) if d_mu else None,
                                     C.c_void_p(stream) if stream else None), "bec_apply_H_static")


def bec_static_scratch_bytes() -> int:
    out = C.c_size_t(0)
    _check(_lib().bec_static_scratch_bytes(C.byref(out)), "bec_static_scratch_bytes")
    return out.value


def _params_arg(params):
    """One bec_params or a ctypes array of them (batched grids)."""
    if isinstance(params, bec_params):
        return C.byref(params)
    return C.cast(params, C.POINTER(bec_params))


def bec_energy(h, params, d_phi, batch=1):
    out = (bec_energies * batch)()
    _check(_lib().bec_energy(h, _params_arg(params), C.c_void_p(d_phi), C.cast(out, C.c_void_p), 1), "bec_energy")
    return out[0] if batch == 1 else list(out)


def bec_pcg_default_opts() -> bec_pcg_opts:
    o = bec_pcg_opts()
    _check(_lib().bec_pcg_default_opts(C.byref(o)), "bec_pcg_default_opts")
    return o


def bec_pcg_solve(h, params, d_phi, opts=None) -> bec_pcg_result:
    res = bec_pcg_result()
    rc = _lib().bec_pcg_solve(h, C.byref(params), C.c_void_p(d_phi), C.byref(opts) if opts is not None else None,
                              C.byref(res))
    _check(rc, "bec_pcg_solve", ok=(BEC_OK, BEC_ENOTCONV, BEC_ENUMERIC))
    return res


def bec_pcg_solve_batched(h, params_array, d_phi, batch, opts=None):
    res = (bec_pcg_result * batch)()
    rc = _lib().bec_pcg_solve_batched(h, _params_arg(params_array), C.c_void_p(d_phi),
                                      C.byref(opts) if opts is not None else None, res)
    _check(rc, "bec_pcg_solve_batched", ok=(BEC_OK, BEC_ENOTCONV, BEC_ENUMERIC))
    return list(res)


def bec_pcg_solve_ragged(handles, params_arrays, d_phis, batches, opts=None):
    """handles, params_arrays (ctypes bec_params arrays), device pointers and batch sizes per grid;
    returns the results of every solve in grid order."""
    k = len(handles)
    hs = (C.c_void_p * k)(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    ps = (C.c_void_p * k)(*[C.cast(a, C.c_void_p).value for a in params_arrays])
    ds = (C.c_void_p * k)(*d_phis)
    res = (bec_pcg_result * sum(batches))()
    rc = _lib().bec_pcg_solve_ragged(hs, ps, ds, k, C.byref(opts) if opts is not None else None, res)
    _check(rc, "bec_pcg_solve_ragged", ok=(BEC_OK, BEC_ENOTCONV, BEC_ENUMERIC))
    return list(res)


def pcg_solve_ragged(grids, params_lists, phis_list, opts=None):
    """Algorithm 1 on several BecGrid objects of different sizes in one call (see
    bec_pcg_solve_ragged). params_lists[k]: the grid's bec_params list; phis_list[k]: its
    contiguous complex128 [batch, Nx, Ny, Nz] tensor (overwritten). Returns one result list per grid."""
    arrays = []
    for g, pl, ph in zip(grids, params_lists, phis_list):
        assert len(pl) == g.batch and ph.is_contiguous() and ph.dtype == g.torch.complex128
        assert tuple(ph.shape) == (g.batch,) + g.n
        if any(p.lambda_ != 0.0 for p in pl):
            g.ensure_symbol()
        arrays.append((bec_params * g.batch)(*pl))
    flat = bec_pcg_solve_ragged([g.handle for g in grids], arrays, [ph.data_ptr() for ph in phis_list],
                                [g.batch for g in grids], opts)
    out, k = [], 0
    for g in grids:
        out.append(flat[k:k + g.batch])
        k += g.batch
    return out


def bec_fft3d(h, d_in, d_out, direction):
    _check(_lib().bec_fft3d(h, C.c_void_p(d_in), C.c_void_p(d_out), direction), "bec_fft3d")


def bec_time_stage(h, params, d_phi, which, reps) -> float:
    ms = C.c_double(0.0)
    _check(_lib().bec_time_stage(h, _params_arg(params), C.c_void_p(d_phi), which, reps, C.byref(ms)), "bec_time_stage")
    return ms.value


def bec_pcg_profile(h, params, d_phi, iters, flags=0):
    """{site name: (total ms, launches)} over `iters` eagerly launched, event-timed iterations
    (flags bit 0: with the solver's second stream)."""
    ms, cnt = (C.c_double * BEC_NSITES)(), (C.c_int32 * BEC_NSITES)()
    _check(_lib().bec_pcg_profile(h, _params_arg(params), C.c_void_p(d_phi), iters, flags, ms, cnt),
           "bec_pcg_profile")
    return {SITES[i]: (ms[i], cnt[i]) for i in range(BEC_NSITES)}


def bec_set_kernel_variants(h, variants):
    arr = (C.c_int32 * BEC_NSITES)(*[int(v) for v in variants])
    _check(_lib().bec_set_kernel_variants(h, arr), "bec_set_kernel_variants")


def bec_get_kernel_variants(h):
    arr = (C.c_int32 * BEC_NSITES)()
    _check(_lib().bec_get_kernel_variants(h, arr), "bec_get_kernel_variants")
    return tuple(arr)


def bec_autotune_kernels(h, params, d_phi, iters):
    """(variants, ms_default, ms_best), each a tuple over the launch sites."""
    v, d, b = (C.c_int32 * BEC_NSITES)(), (C.c_double * BEC_NSITES)(), (C.c_double * BEC_NSITES)()
    _check(_lib().bec_autotune_kernels(h, _params_arg(params), C.c_void_p(d_phi), iters, v, d, b),
           "bec_autotune_kernels")
    return tuple(v), tuple(d), tuple(b)


def bec_set_line_tiles(h, div):
    arr = (C.c_int32 * 3)(*[int(v) for v in div])
    _check(_lib().bec_set_line_tiles(h, arr), "bec_set_line_tiles")


def bec_get_line_tiles(h):
    """(divisors, tunable flags), each a tuple over (x, y, z)."""
    d, t = (C.c_int32 * 3)(), (C.c_int32 * 3)()
    _check(_lib().bec_get_line_tiles(h, d, t), "bec_get_line_tiles")
    return tuple(d), tuple(t)


def bec_autotune_line_tiles(h, params, d_phi, reps):
    d, ms = (C.c_int32 * 3)(), C.c_double(0.0)
    _check(_lib().bec_autotune_line_tiles(h, _params_arg(params), C.c_void_p(d_phi), reps, d, C.byref(ms)),
           "bec_autotune_line_tiles")
    return tuple(d), ms.value


def bec_interp_spectral(h_src, h_dst, d_in, in_precision, d_out, out_precision):
    _check(_lib().bec_interp_spectral(h_src, h_dst, C.c_void_p(d_in), in_precision, C.c_void_p(d_out), out_precision),
           "bec_interp_spectral")


def bec_normalize(h, d_phi):
    _check(_lib().bec_normalize(h, C.c_void_p(d_phi)), "bec_normalize")


def bec_gauge_fix(h, params, d_phi):
    _check(_lib().bec_gauge_fix(h, _params_arg(params), C.c_void_p(d_phi)), "bec_gauge_fix")


def bec_rotate_z(h, d_in, d_out, alpha):
    _check(_lib().bec_rotate_z(h, C.c_void_p(d_in), C.c_void_p(d_out), alpha), "bec_rotate_z")


def bec_mlp_param_count(d_in, d_h, d_out) -> int:
    return int(_lib().bec_mlp_param_count(d_in, d_h, d_out))


def bec_mlp_scratch_bytes(net: bec_mlp, batch) -> int:
    out = C.c_size_t(0)
    _check(_lib().bec_mlp_scratch_bytes(C.byref(net), batch, C.byref(out)), "bec_mlp_scratch_bytes")
    return out.value


def bec_mlp_sync(net, stream):
    _check(_lib().bec_mlp_sync(C.byref(net), C.c_void_p(stream)), "bec_mlp_sync")


def bec_mlp_forward(net, batch, d_x, d_idx, d_y, d_scratch, scratch_bytes, stream):
    _check(_lib().bec_mlp_forward(C.byref(net), batch, C.c_void_p(d_x), C.c_void_p(d_idx) if d_idx else None,
                                  C.c_void_p(d_y), C.c_void_p(d_scratch), scratch_bytes, C.c_void_p(stream)),
           "bec_mlp_forward")


def bec_mlp_loss_grad(net, batch, d_x, d_target, d_idx, d_y, d_loss, d_scratch, scratch_bytes, stream):
    _check(_lib().bec_mlp_loss_grad(C.byref(net), batch, C.c_void_p(d_x), C.c_void_p(d_target),
                                    C.c_void_p(d_idx) if d_idx else None, C.c_void_p(d_y) if d_y else None,
                                    C.c_void_p(d_loss), C.c_void_p(d_scratch), scratch_bytes, C.c_void_p(stream)),
           "bec_mlp_loss_grad")


def bec_mlp_adam_step(net, lr, beta1, beta2, eps, t, stream):
    _check(_lib().bec_mlp_adam_step(C.byref(net), lr, beta1, beta2, eps, t, C.c_void_p(stream)), "bec_mlp_adam_step")


def bec_gemm_bf16_nt(M, N, K, d_A, lda, d_B, ldb, d_C, ldc, d_bias, splits, d_part, stream):
    _check(_lib().bec_gemm_bf16_nt(M, N, K, C.c_void_p(d_A), lda, C.c_void_p(d_B), ldb, C.c_void_p(d_C), ldc,
                                   C.c_void_p(d_bias) if d_bias else None, splits,
                                   C.c_void_p(d_part) if d_part else None, C.c_void_p(stream)), "bec_gemm_bf16_nt")


# ------------------------------------------------------------------ torch-facing helpers
def make_desc(n, a) -> bec_grid_desc:
    d = bec_grid_desc()
    for i in range(3):
        d.n[i] = int(n[i])
        d.a[i] = float(a[i])
    return d


def make_params(gamma, beta, lam, ndip, omega) -> bec_params:
    p = bec_params()
    for i in range(3):
        p.gamma[i] = float(gamma[i])
        p.n[i] = float(ndip[i])
    p.beta, p.lambda_, p.omega = float(beta), float(lam), float(omega)
    return p


class BecGrid:
    """Owns a torch-allocated workspace and a library handle for one box/grid."""

    def __init__(self, n, a, precision=BEC_FP64, device="cuda", stream=None, batch=1):
        import torch
        self.torch = torch
        self.n, self.a = tuple(int(v) for v in n), tuple(float(v) for v in a)
        self.precision = precision
        self.batch = int(batch)
        self.desc = make_desc(self.n, self.a)
        self.ws_bytes = bec_workspace_bytes_batched(self.desc, precision, self.batch)
        self.device = torch.device(device)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = s
        self.handle = bec_init_grid_batched(self.desc, precision, self.batch, base + off, self.ws_bytes,
                                            s.cuda_stream)
        self._symbol = False

    def close(self):
        if getattr(self, "handle", None):
            bec_destroy_grid(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def cdtype(self):
        return self.torch.complex128 if self.precision == BEC_FP64 else self.torch.complex64

    @property
    def rdtype(self):
        return self.torch.float64 if self.precision == BEC_FP64 else self.torch.float32

    def symbol(self):
        torch = self.torch
        out = torch.empty((self.n[0] + 1, self.n[1] + 1, self.n[2] + 1), dtype=torch.float64, device=self.device)
        bec_atkm_symbol(self.handle, out.data_ptr())
        self._symbol = True
        return out

    def ensure_symbol(self):
        if not self._symbol:
            bec_atkm_symbol(self.handle, None)
            self._symbol = True

    def _field(self, phi):
        assert phi.is_contiguous() and phi.dtype == self.cdtype and tuple(phi.shape) == self.n, \
            f"field must be contiguous {self.cdtype} of shape {self.n}"
        return phi

    def fft3d(self, u, direction=-1):
        u = self._field(u)
        out = self.torch.empty_like(u)
        bec_fft3d(self.handle, u.data_ptr(), out.data_ptr(), direction)
        return out

    def dipolar(self, params, phi):
        self.ensure_symbol()
        phi = self._field(phi)
        out = self.torch.empty(self.n, dtype=self.rdtype, device=self.device)
        bec_dipolar(self.handle, params, phi.data_ptr(), out.data_ptr())
        return out

    def apply_H(self, params, phi, want_Phi=False):
        if params.lambda_ != 0.0:
            self.ensure_symbol()
        phi = self._field(phi)
        h = self.torch.empty_like(phi)
        Phi = self.torch.empty(self.n, dtype=self.rdtype, device=self.device) if want_Phi else None
        mu = self.torch.empty(1, dtype=self.torch.float64, device=self.device)
        bec_apply_H(self.handle, params, phi.data_ptr(), h.data_ptr(), Phi.data_ptr() if want_Phi else None,
                    mu.data_ptr())
        return (h, mu, Phi) if want_Phi else (h, mu)

    def apply_H_batched(self, params_list, phis):
        """H phi for every solve: phis is a contiguous [batch, Nx, Ny, Nz] tensor."""
        assert len(params_list) == self.batch and tuple(phis.shape) == (self.batch,) + self.n
        assert phis.is_contiguous() and phis.dtype == self.cdtype
        if any(p.lambda_ != 0.0 for p in params_list):
            self.ensure_symbol()
        arr = (bec_params * self.batch)(*params_list)
        h = self.torch.empty_like(phis)
        mu = self.torch.empty(self.batch, dtype=self.torch.float64, device=self.device)
        bec_apply_H(self.handle, arr, phis.data_ptr(), h.data_ptr(), None, mu.data_ptr())
        return h, mu

    def energy_batched(self, params_list, phis):
        assert len(params_list) == self.batch and tuple(phis.shape) == (self.batch,) + self.n
        if any(p.lambda_ != 0.0 for p in params_list):
            self.ensure_symbol()
        arr = (bec_params * self.batch)(*params_list)
        return [e.as_dict() for e in bec_energy(self.handle, arr, phis.data_ptr(), self.batch)]

    def energy(self, params, phi) -> dict:
        if params.lambda_ != 0.0:
            self.ensure_symbol()
        phi = self._field(phi)
        return bec_energy(self.handle, params, phi.data_ptr()).as_dict()

    def time_stage(self, params, phi, which, reps=10):
        self.ensure_symbol()
        return bec_time_stage(self.handle, params, self._field(phi).data_ptr(), which, reps)

    def pcg_profile(self, params, phi, iters, concurrent=False):
        """Per launch site (total ms, launches) over `iters` iterations from phi (updated in place);
        concurrent: with the solver's second stream."""
        if params.lambda_ != 0.0:
            self.ensure_symbol()
        assert self.batch == 1
        assert phi.is_contiguous() and phi.dtype == self.torch.complex128 and tuple(phi.shape) == self.n
        return bec_pcg_profile(self.handle, params, phi.data_ptr(), iters, 1 if concurrent else 0)

    def set_line_tiles(self, div):
        """Per-axis (x, y, z) divisors of the runtime-length FFT kernels' lines per block."""
        bec_set_line_tiles(self.handle, div)

    def line_tiles(self):
        """((div_x, div_y, div_z), (tunable_x, tunable_y, tunable_z))."""
        return bec_get_line_tiles(self.handle)

    def kernel_variants(self):
        return dict(zip(SITES, bec_get_kernel_variants(self.handle)))

    def set_kernel_variants(self, variants):
        """variants: a {site: variant} dict (missing sites 0) or a sequence over SITES."""
        if isinstance(variants, dict):
            variants = [int(variants.get(s, 0)) for s in SITES]
        bec_set_kernel_variants(self.handle, variants)

    def autotune_kernels(self, params, phi_scratch, iters=10, cache=None, log=None):
        """Pick the launch-shape variant of each launch site (bec_autotune_kernels) by timing
        `iters` iterations per variant from phi_scratch (overwritten). With `cache` (a JSON file) a
        stored choice for this device, precision and grid is applied without timing, and a new
        search is stored. Returns ({site: variant}, {site: (ms default, ms chosen)} or None)."""
        import json
        import os
        key = "kernels|" + self.tile_key()
        store = {}
        if cache and os.path.exists(cache):
            with open(cache) as fh:
                store = json.load(fh)
            if key in store:
                self.set_kernel_variants(store[key]["variants"])
                return dict(store[key]["variants"]), None
        self.ensure_symbol()
        # the library reads and overwrites batch x N complex128 values here, on FP32 grids too
        shapes = ((self.batch,) + self.n,) + ((self.n,) if self.batch == 1 else ())
        if not (phi_scratch.is_contiguous() and phi_scratch.dtype == self.torch.complex128
                and tuple(phi_scratch.shape) in shapes):
            raise ValueError(f"phi_scratch must be a contiguous complex128 tensor of shape {shapes[-1]}")
        if self.batch > 1 or not isinstance(params, bec_params):
            params = (bec_params * self.batch)(*params)
        v, d, b = bec_autotune_kernels(self.handle, params, phi_scratch.data_ptr(), iters)
        chosen = {s: v[i] for i, s in enumerate(SITES) if v[i]}
        times = {s: (d[i], b[i]) for i, s in enumerate(SITES) if d[i] > 0}
        if log:
            for s, (a, c) in times.items():
                if s in chosen:
                    log(f"kernel variant {key} {s}: {chosen[s]} ({a * 1e3:.1f} -> {c * 1e3:.1f} us per iteration)")
        if cache:
            store[key] = dict(variants=chosen, ms={s: list(t) for s, t in times.items()})
            os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
            tmp = cache + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(store, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return chosen, times

    def tile_key(self):
        torch = self.torch
        dev = torch.cuda.get_device_name(self.device)
        prec = "fp64" if self.precision == BEC_FP64 else "fp32"
        return f"{dev}|{prec}|{self.n[0]}x{self.n[1]}x{self.n[2]}|batch{self.batch}"

    def autotune(self, params, phis, reps=5, cache=None, log=None):
        """Search the line tiles (bec_autotune_line_tiles) on `phis` (one field, or [batch, ...] for
        a batched grid, in the grid's precision) and leave the fastest on the grid. With `cache`
        (a JSON file) a stored choice for this device, precision, grid and batch is applied
        without timing, and a new search is stored. Returns (divisors, ms or None)."""
        import json
        import os
        key = self.tile_key()
        store = {}
        if cache and os.path.exists(cache):
            with open(cache) as fh:
                store = json.load(fh)
            if key in store:
                div = tuple(store[key]["div"])
                self.set_line_tiles(div)
                return div, None
        if not any(self.line_tiles()[1]):
            return self.line_tiles()[0], None
        self.ensure_symbol()
        assert phis.is_contiguous() and phis.dtype == self.cdtype
        assert phis.numel() == self.batch * self.n[0] * self.n[1] * self.n[2]
        if self.batch > 1 or not isinstance(params, bec_params):
            params = (bec_params * self.batch)(*params)
        div, ms = bec_autotune_line_tiles(self.handle, params, phis.data_ptr(), reps)
        if log:
            log(f"line tiles {key}: divisors {div}, {ms:.3f} ms per apply + Parseval pass")
        if cache:
            store[key] = dict(div=list(div), ms=ms)
            os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
            tmp = cache + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(store, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return div, ms

    def interp_to(self, dst: "BecGrid", phis, out_precision=BEC_FP64):
        """Spectral interpolation of `batch` fields on this grid to grid `dst` (same box).
        phis: complex128 or complex64 tensor [batch, Nx, Ny, Nz] (or [Nx, Ny, Nz] for batch 1)."""
        torch = self.torch
        assert phis.is_contiguous() and phis.dtype in (torch.complex128, torch.complex64)
        assert phis.numel() == self.batch * self.n[0] * self.n[1] * self.n[2]
        in_prec = BEC_FP64 if phis.dtype == torch.complex128 else BEC_FP32
        shape = ((self.batch,) if phis.dim() == 4 else ()) + dst.n
        out = torch.empty(shape, dtype=torch.complex128 if out_precision == BEC_FP64 else torch.complex64,
                          device=self.device)
        bec_interp_spectral(self.handle, dst.handle, phis.data_ptr(), in_prec, out.data_ptr(), out_precision)
        return out

    def normalize_(self, phis):
        assert phis.is_contiguous() and phis.dtype == self.torch.complex128
        assert phis.numel() == self.batch * self.n[0] * self.n[1] * self.n[2]
        bec_normalize(self.handle, phis.data_ptr())
        return phis

    def rotate_z(self, phis, alpha):
        """phis(R_alpha x) for the batch (complex128, [batch, Nx, Ny, Nz] or [Nx, Ny, Nz])."""
        assert phis.is_contiguous() and phis.dtype == self.torch.complex128
        assert phis.numel() == self.batch * self.n[0] * self.n[1] * self.n[2]
        out = self.torch.empty_like(phis)
        bec_rotate_z(self.handle, phis.data_ptr(), out.data_ptr(), float(alpha))
        return out

    def gauge_fix_(self, params_list, phis):
        assert phis.is_contiguous() and phis.dtype == self.torch.complex128
        assert phis.numel() == self.batch * self.n[0] * self.n[1] * self.n[2] and len(params_list) == self.batch
        arr = (bec_params * self.batch)(*params_list)
        bec_gauge_fix(self.handle, arr, phis.data_ptr())
        return phis

    def pcg_solve(self, params, phi, opts=None):
        if params.lambda_ != 0.0:
            self.ensure_symbol()
        assert self.batch == 1
        assert phi.is_contiguous() and phi.dtype == self.torch.complex128 and tuple(phi.shape) == self.n
        return bec_pcg_solve(self.handle, params, phi.data_ptr(), opts)

    def pcg_solve_batched(self, params_list, phis, opts=None):
        """params_list: `batch` bec_params; phis: contiguous complex128 tensor [batch, Nx, Ny, Nz]."""
        assert len(params_list) == self.batch
        if any(p.lambda_ != 0.0 for p in params_list):
            self.ensure_symbol()
        assert phis.is_contiguous() and phis.dtype == self.torch.complex128
        assert tuple(phis.shape) == (self.batch,) + self.n
        arr = (bec_params * self.batch)(*params_list)
        return bec_pcg_solve_batched(self.handle, arr, phis.data_ptr(), self.batch, opts)


class Mlp:
    """The learned-initial-guess network on torch-allocated buffers (include/bec_mlp.h).

    `params` is the packed FP32 master vector [W1 b1 W2 b2 W3 b3]; set it with load_params."""

    def __init__(self, d_in=6, d_h=512, d_out=32768, device="cuda", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.dims = (int(d_in), int(d_h), int(d_out))
        P = bec_mlp_param_count(*self.dims)
        self.P = P
        f32 = dict(dtype=torch.float32, device=self.device)
        self.params = torch.zeros(P, **f32)
        self.grads = torch.zeros(P, **f32)
        self.adam_m = torch.zeros(P, **f32)
        self.adam_v = torch.zeros(P, **f32)
        self.params_bf16 = torch.zeros(P, dtype=torch.int16, device=self.device)
        self.w2t = torch.zeros(d_h * d_h, dtype=torch.int16, device=self.device)
        self.w3t = torch.zeros(d_h * d_out, dtype=torch.int16, device=self.device)
        self.net = bec_mlp(d_in, d_h, d_out, self.params.data_ptr(), self.params_bf16.data_ptr(), self.w2t.data_ptr(),
                           self.w3t.data_ptr(), self.grads.data_ptr(), self.adam_m.data_ptr(), self.adam_v.data_ptr())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._scratch = None
        self.step_count = 0

    def offsets(self):
        d_in, d_h, d_out = self.dims
        o = {}
        k = 0
        for name, size in (("W1", d_h * d_in), ("b1", d_h), ("W2", d_h * d_h), ("b2", d_h), ("W3", d_out * d_h),
                           ("b3", d_out)):
            o[name] = (k, k + size)
            k += size
        return o

    def load_params(self, flat):
        """flat: FP32 host or device vector of length P (copied), then BF16 copies refreshed."""
        t = self.torch.as_tensor(flat, dtype=self.torch.float32)
        assert t.numel() == self.P
        self.params.copy_(t.reshape(-1).to(self.device))
        self.adam_m.zero_()
        self.adam_v.zero_()
        self.step_count = 0
        bec_mlp_sync(self.net, self.stream.cuda_stream)

    def scratch(self, batch):
        """Scratch for `batch` rows; the need is not monotone in the batch, so it is asked each time."""
        nbytes = bec_mlp_scratch_bytes(self.net, batch)
        if self._scratch is None or self._scratch.numel() < nbytes:
            self._scratch = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device)
        return self._scratch

    def forward(self, x, idx=None, batch=None):
        torch = self.torch
        batch = int(batch if batch is not None else (idx.numel() if idx is not None else x.shape[0]))
        assert x.dtype == torch.float32 and x.is_contiguous()
        y = torch.empty((batch, self.dims[2]), dtype=torch.float32, device=self.device)
        sc = self.scratch(batch)
        bec_mlp_forward(self.net, batch, x.data_ptr(), idx.data_ptr() if idx is not None else None, y.data_ptr(),
                        sc.data_ptr(), sc.numel(), self.stream.cuda_stream)
        return y

    def loss_grad(self, x, target, idx=None, batch=None, want_y=False):
        torch = self.torch
        batch = int(batch if batch is not None else (idx.numel() if idx is not None else x.shape[0]))
        assert x.dtype == torch.float32 and target.dtype == torch.float32
        y = torch.empty((batch, self.dims[2]), dtype=torch.float32, device=self.device) if want_y else None
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        sc = self.scratch(batch)
        bec_mlp_loss_grad(self.net, batch, x.data_ptr(), target.data_ptr(), idx.data_ptr() if idx is not None else None,
                          y.data_ptr() if y is not None else None, loss.data_ptr(), sc.data_ptr(), sc.numel(),
                          self.stream.cuda_stream)
        return (loss, y) if want_y else loss

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        bec_mlp_adam_step(self.net, lr, beta1, beta2, eps, self.step_count, self.stream.cuda_stream)
