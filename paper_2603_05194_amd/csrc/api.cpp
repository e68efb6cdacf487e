// C ABI of the PCG-ATKM library: validation, workspace carving, FFT plans, entry points.
#include <hip/hip_runtime.h>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/bec.h"
#include "impl.h"

using namespace bec;

struct bec_grid_s : public Grid {};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(Grid* g, hipError_t e, const char* where) {
    if (g) g->poisoned = 1;
    return fail(BEC_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

bool good_size(int n) {
    if (n < 4 || n > 2048 || (n & 1)) return false;
    int m = n;
    for (int f : {2, 3, 5})
        while (m % f == 0) m /= f;
    return m == 1;
}

int validate_desc(const bec_grid_desc* d) {
    if (!d) return fail(BEC_EINVAL, "grid descriptor is NULL");
    for (int i = 0; i < 3; ++i) {
        if (!good_size(d->n[i])) return fail(BEC_EINVAL, "N must be even, in [4, 2048] and 2^i 3^j 5^k");
        if (!(d->a[i] > 0.0) || !std::isfinite(d->a[i])) return fail(BEC_EINVAL, "box half-width must be positive");
    }
    if ((long)d->n[0] * d->n[1] * d->n[2] * 8L >= (1L << 31) * 4L)
        return fail(BEC_EINVAL, "grid too large");
    return BEC_OK;
}

int validate_params(const bec_params* p, Params& out) {
    if (!p) return fail(BEC_EINVAL, "params is NULL");
    const double nn = std::sqrt(p->n[0] * p->n[0] + p->n[1] * p->n[1] + p->n[2] * p->n[2]);
    if (!(std::fabs(nn - 1.0) <= 1e-12)) return fail(BEC_EINVAL, "dipole axis must be a unit vector");
    for (int i = 0; i < 3; ++i) {
        if (!(p->gamma[i] > 0.0) || !std::isfinite(p->gamma[i])) return fail(BEC_EINVAL, "trap frequencies must be positive");
        out.gamma[i] = p->gamma[i];
        out.nd[i] = p->n[i] / nn;
    }
    if (!std::isfinite(p->beta) || !std::isfinite(p->lambda) || !std::isfinite(p->omega))
        return fail(BEC_EINVAL, "non-finite parameter");
    out.beta = p->beta;
    out.lam = p->lambda;
    out.omega = p->omega;
    return BEC_OK;
}

std::vector<int> factor(int n) {
    std::vector<int> r;
    while (n % 8 == 0) { r.push_back(8); n /= 8; }
    while (n % 4 == 0) { r.push_back(4); n /= 4; }
    while (n % 2 == 0) { r.push_back(2); n /= 2; }
    while (n % 3 == 0) { r.push_back(3); n /= 3; }
    while (n % 5 == 0) { r.push_back(5); n /= 5; }
    return r;
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t state, partials, uhat, symscr, tw64, tw32, f64, f32, total;
    size_t partials_cap, symscr_doubles;
};

int tiles_of(const Geo& g) { return g.ntiles; }

Geo make_geo(int axis, int d0, int d1, int d2, int nfft, int dual) {
    Geo g;
    std::memset(&g, 0, sizeof(g));
    g.axis = axis;
    int L = kTileElems / nfft;
    if (dual) L /= 2;
    if (L < 1) L = 1;
    if (axis == 2) {
        g.n_outer = d0 * d1;
        g.n_inner = 1;
        if (L > g.n_outer) L = g.n_outer;
        g.L = L;
        g.tpo = 1;
        g.ntiles = (g.n_outer + L - 1) / L;
        g.dA = d1;
    } else if (axis == 1) {
        g.n_outer = d0;
        g.n_inner = d2;
        if (L > d2) L = d2;
        g.L = L;
        g.tpo = (d2 + L - 1) / L;
        g.ntiles = d0 * g.tpo;
    } else {
        g.n_outer = 1;
        g.n_inner = d1 * d2;
        if (L > g.n_inner) L = g.n_inner;
        g.L = L;
        g.tpo = (g.n_inner + L - 1) / L;
        g.ntiles = g.tpo;
        g.dB = d2;
    }
    return g;
}

Layout layout(const int n[3], int precision) {
    Layout L;
    const size_t N = (size_t)n[0] * n[1] * n[2];
    const size_t Nz1 = (size_t)n[0] * n[1] * (n[2] + 1);
    const size_t Ny2 = (size_t)n[0] * 2 * n[1] * (n[2] + 1);
    // partials: generous bound on tiles x slots of one reducing kernel
    size_t maxt = 0;
    maxt = std::max(maxt, (size_t)make_geo(0, n[0], 2 * n[1], n[2] + 1, 2 * n[0], 1).ntiles);
    maxt = std::max(maxt, (size_t)make_geo(0, n[0], n[1], n[2], n[0], 0).ntiles);
    maxt = std::max(maxt, (size_t)make_geo(1, n[0], n[1], n[2], n[1], 0).ntiles);
    maxt = std::max(maxt, (size_t)make_geo(2, n[0], n[1], n[2], n[2], 0).ntiles);
    maxt = std::max(maxt, N / kThreads + 1);
    L.partials_cap = maxt * kMaxRed + 1024;
    const int ms = 651;
    size_t sd = 2 * ms;
    for (int d = 0; d < 3; ++d) sd += (size_t)ms * (n[d] + 1) + 2 * ((size_t)std::ceil(M_PI * n[d] / 2.0) + 80);
    L.symscr_doubles = sd;
    size_t tw = 0;
    for (int d = 0; d < 3; ++d) tw += al((size_t)n[d] * 16) + al((size_t)2 * n[d] * 16);
    size_t off = 0;
    L.state = off; off += al(sizeof(DevState));
    L.partials = off; off += al(L.partials_cap * sizeof(double));
    L.uhat = off; off += al((size_t)(n[0] + 1) * (n[1] + 1) * (n[2] + 1) * sizeof(double));
    L.symscr = off; off += al(sd * sizeof(double));
    L.tw64 = off; off += tw;
    L.tw32 = off; off += precision ? tw / 2 + 6 * 256 : 0;
    auto fields_bytes = [&](size_t cs) {
        return 8 * al(N * 2 * cs) + 2 * al(N * cs) + 2 * al(Nz1 * 2 * cs) + 2 * al(Ny2 * 2 * cs);
    };
    L.f64 = off; off += fields_bytes(8);
    L.f32 = off; off += precision ? fields_bytes(4) : 0;
    L.total = off + 256;
    return L;
}

template <typename R> void carve_fields(Fields<R>& f, char*& p, const int n[3]) {
    const size_t N = (size_t)n[0] * n[1] * n[2];
    const size_t Nz1 = (size_t)n[0] * n[1] * (n[2] + 1);
    const size_t Ny2 = (size_t)n[0] * 2 * n[1] * (n[2] + 1);
    auto take = [&](size_t bytes) { char* q = p; p += al(bytes); return q; };
    f.hphi = (cpx<R>*)take(N * sizeof(cpx<R>));
    f.acc = (cpx<R>*)take(N * sizeof(cpx<R>));
    f.r0 = (cpx<R>*)take(N * sizeof(cpx<R>));
    f.r1 = (cpx<R>*)take(N * sizeof(cpx<R>));
    f.pr = (cpx<R>*)take(N * sizeof(cpx<R>));
    f.p = (cpx<R>*)take(N * sizeof(cpx<R>));
    f.w = (cpx<R>*)take(N * sizeof(cpx<R>));
    f.phi = (cpx<R>*)take(N * sizeof(cpx<R>));
    f.Phi = (R*)take(N * sizeof(R));
    f.Phi_aux = (R*)take(N * sizeof(R));
    f.z1 = (cpx<R>*)take(Nz1 * sizeof(cpx<R>));
    f.z2 = (cpx<R>*)take(Nz1 * sizeof(cpx<R>));
    f.y1 = (cpx<R>*)take(Ny2 * sizeof(cpx<R>));
    f.y2 = (cpx<R>*)take(Ny2 * sizeof(cpx<R>));
}

template <typename R> int make_plan(Grid& g, FftPlan& pl, int n, char*& twp) {
    std::memset(&pl, 0, sizeof(pl));
    pl.n = n;
    std::vector<int> r = factor(n);
    if ((int)r.size() > kMaxStages) return fail(BEC_EINVAL, "FFT length has too many factors");
    pl.nst = (int)r.size();
    for (size_t i = 0; i < r.size(); ++i) pl.radix[i] = r[i];
    std::vector<cpx<R>> tw(n);
    for (int t = 0; t < n; ++t) {
        const long double ang = -2.0L * 3.14159265358979323846264338327950288L * t / n;
        tw[t].x = (R)std::cos(ang);
        tw[t].y = (R)std::sin(ang);
    }
    hipError_t e = hipMemcpy(twp, tw.data(), n * sizeof(cpx<R>), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(&g, e, "twiddle upload");
    pl.tw = twp;
    twp += al((size_t)n * sizeof(cpx<R>));
    return BEC_OK;
}

template <typename R> int make_plans(Grid& g, Fields<R>& f, char* twp) {
    int rc;
    if ((rc = make_plan<R>(g, f.pz, g.n[2], twp))) return rc;
    if ((rc = make_plan<R>(g, f.py, g.n[1], twp))) return rc;
    if ((rc = make_plan<R>(g, f.px, g.n[0], twp))) return rc;
    if ((rc = make_plan<R>(g, f.pzp, 2 * g.n[2], twp))) return rc;
    if ((rc = make_plan<R>(g, f.pyp, 2 * g.n[1], twp))) return rc;
    if ((rc = make_plan<R>(g, f.pxp, 2 * g.n[0], twp))) return rc;
    return BEC_OK;
}

int check_grid(bec_grid g) {
    if (!g) return fail(BEC_EINVAL, "grid handle is NULL");
    if (g->poisoned) return fail(BEC_EHIP, "handle unusable after an earlier HIP error");
    return BEC_OK;
}

int check_launch(Grid* g, const char* where) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(g, e, where);
    return BEC_OK;
}

// ------------------------------------------------------------------ PCG driver
// Runs Algorithm 1 with all scalar decisions on the device. The host enqueues iterations
// (eagerly for the first two, then as a captured two-iteration HIP graph) on a private
// non-blocking stream and reads the device state every check_every iterations.
struct HostPoll { int done, status, iter; double res; };

int read_state(Grid& g, DevState& hs) {
    hipError_t e = hipMemcpyAsync(&hs, g.st, sizeof(DevState), hipMemcpyDeviceToHost, g.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g.stream);
    if (e != hipSuccess) return hip_fail(&g, e, "state readback");
    return BEC_OK;
}

template <typename R>
int pcg_phase(Grid& g, Fields<R>& f, const Params& p, cpx<R>* phi, const bec_pcg_opts& o, bool stall_stop,
              DevState& hs) {
    int rc;
    launch_pcg_start<R>(g, f, p, phi);
    if ((rc = check_launch(&g, "pcg start"))) return rc;
    const int every = o.check_every;
    long it = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double best = 1e300;
    long best_it = 0;
    int polls_since = 0;
    const char* prog = std::getenv("BEC_PROGRESS");
    const double prog_every = prog ? std::atof(prog) : 0.0;
    double last_print = 0.0;
    auto now = []() { return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count(); };
    if (prog_every > 0) last_print = now();
    for (;;) {
        if (o.use_graph && it >= 2 && (it & 1) == 0) {
            if (!exec) {
                hipError_t e = hipStreamBeginCapture(g.stream, hipStreamCaptureModeThreadLocal);
                if (e != hipSuccess) return hip_fail(&g, e, "begin capture");
                launch_pcg_iteration<R>(g, f, p, phi, 0);
                launch_pcg_iteration<R>(g, f, p, phi, 1);
                e = hipStreamEndCapture(g.stream, &graph);
                if (e != hipSuccess) return hip_fail(&g, e, "end capture");
                e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                if (e != hipSuccess) return hip_fail(&g, e, "graph instantiate");
            }
            hipError_t e = hipGraphLaunch(exec, g.stream);
            if (e != hipSuccess) return hip_fail(&g, e, "graph launch");
            it += 2;
        } else {
            launch_pcg_iteration<R>(g, f, p, phi, (int)(it & 1));
            it += 1;
        }
        if ((rc = check_launch(&g, "pcg iteration"))) break;
        if (it % every == 0 || it < 2) {
            if ((rc = read_state(g, hs))) break;
            if (prog_every > 0 && now() - last_print >= prog_every) {
                std::fprintf(stderr, "[bec] %s iter %d res %.3e E %.15f\n", sizeof(R) == 4 ? "fp32" : "fp64", hs.iter,
                             hs.res_inf, hs.E);
                std::fflush(stderr);
                last_print = now();
            }
            if (hs.done) break;
            if (stall_stop) {
                // FP32 phase: leave when ||r||_inf has not dropped below 0.9x its best value
                // for stall_window iterations (FP32 rounding floor reached)
                if (hs.res_inf < 0.9 * best) { best = hs.res_inf; best_it = hs.iter; }
                else if (hs.iter - best_it >= o.stall_window) break;
                (void)polls_since;
            }
        }
    }
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    if (rc) return rc;
    return read_state(g, hs);
}

int pcg_solve(Grid& g, const Params& p, cpx<double>* phi, const bec_pcg_opts& o, bec_pcg_result* res) {
    hipStream_t user = g.stream;
    hipStream_t ps = nullptr;
    hipEvent_t ev = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&ps, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, user);
    if (e == hipSuccess) e = hipStreamWaitEvent(ps, ev, 0);
    if (e != hipSuccess) return hip_fail(&g, e, "solve stream");
    g.stream = ps;
    const long N = (long)g.n[0] * g.n[1] * g.n[2];
    CtlOpts co;
    co.tol_res = o.tol_res_inf; co.tol_step = o.tol_step_inf; co.t_default = o.t_default; co.tau_ulps = o.tau_E_ulps;
    co.dbg_t = o.debug_t; co.dbg_c2 = o.debug_c2; co.max_iter = o.max_iter; co.max_halv = o.max_halvings;
    co.dbg_flags = o.debug_flags; co.fp32 = g.precision;
    DevState hs;
    std::memset(&hs, 0, sizeof(hs));
    int rc = BEC_OK;
    int fp32_iters = 0;
    // clear reductions and the CG memory buffers once (outside any captured graph)
    e = hipMemsetAsync(g.st->red, 0, sizeof(g.st->red), g.stream);
    if (e == hipSuccess) e = hipMemsetAsync(g.f64.p, 0, N * sizeof(cpx<double>), g.stream);
    if (e == hipSuccess) e = hipMemsetAsync(g.f64.r1, 0, N * sizeof(cpx<double>), g.stream);
    if (e != hipSuccess) rc = hip_fail(&g, e, "solve init");
    if (!rc && g.precision == BEC_FP32) {
        // FP32 bulk phase: stop at ||r||_inf <= switch_res or when the residual stalls
        co.tol_res = std::max(o.switch_res, o.tol_res_inf);
        launch_ctl_init(g, co);
        e = hipMemsetAsync(g.f32.p, 0, N * sizeof(cpx<float>), g.stream);
        if (e == hipSuccess) e = hipMemsetAsync(g.f32.r1, 0, N * sizeof(cpx<float>), g.stream);
        if (e != hipSuccess) rc = hip_fail(&g, e, "solve init");
        if (!rc) {
            launch_to_f32(g, phi, g.f32.phi);
            rc = pcg_phase<float>(g, g.f32, p, g.f32.phi, o, true, hs);
        }
        if (!rc) {
            fp32_iters = hs.iter;
            if (hs.status == BEC_ENUMERIC) {
                // keep the caller's guess untouched; fall through to the FP64 phase from it
            } else {
                launch_to_f64_normalized(g, g.f32.phi, phi);
            }
            launch_ctl_phase(g, o.tol_res_inf, o.max_iter);
            rc = check_launch(&g, "phase switch");
        }
        if (!rc) rc = pcg_phase<double>(g, g.f64, p, phi, o, false, hs);
    } else if (!rc) {
        launch_ctl_init(g, co);
        rc = pcg_phase<double>(g, g.f64, p, phi, o, false, hs);
    }
    hipStreamSynchronize(ps);
    g.stream = user;
    hipEventDestroy(ev);
    hipStreamDestroy(ps);
    if (rc) return rc;
    res->status = hs.status == 0 ? BEC_OK : hs.status;
    res->iters = hs.iter;
    res->halvings = hs.halvings;
    res->psd_resets = hs.resets;
    res->forced_accepts = hs.forced;
    res->fp32_iters = fp32_iters;
    res->res_inf = hs.res_inf;
    res->step_inf = hs.step_inf;
    res->e.E = hs.E; res->e.Ekin = hs.Ekin; res->e.Epot = hs.Epot; res->e.Eint = hs.Eint;
    res->e.Edip = hs.Edip; res->e.Erot = hs.Erot; res->e.mu = hs.mu; res->e.mass = hs.mass;
    res->e.virial = 2 * hs.Ekin - 2 * hs.Epot + 3 * hs.Eint + 3 * hs.Edip;
    if (res->status != BEC_OK) g_last_error = bec_status_string(res->status);
    return res->status;
}

}  // namespace

extern "C" {

const char* bec_status_string(int s) {
    switch (s) {
        case BEC_OK: return "ok";
        case BEC_EINVAL: return "invalid argument";
        case BEC_ENOMEM: return "workspace too small";
        case BEC_EHIP: return "HIP error";
        case BEC_ENOTCONV: return "not converged";
        case BEC_ENUMERIC: return "non-finite value";
        case BEC_ESTALL: return "stalled";
        default: return "unknown status";
    }
}

const char* bec_last_error(void) { return g_last_error.c_str(); }

int bec_version(void) { return 1; }

int bec_workspace_bytes(const bec_grid_desc* desc, int precision, size_t* bytes) {
    int rc = validate_desc(desc);
    if (rc) return rc;
    if (!bytes) return fail(BEC_EINVAL, "bytes is NULL");
    if (precision != BEC_FP64 && precision != BEC_FP32) return fail(BEC_EINVAL, "bad precision");
    *bytes = layout(desc->n, precision).total;
    return BEC_OK;
}

int bec_init_grid(const bec_grid_desc* desc, int precision, void* d_ws, size_t ws_bytes, void* stream, bec_grid* out) {
    int rc = validate_desc(desc);
    if (rc) return rc;
    if (!out || !d_ws) return fail(BEC_EINVAL, "NULL workspace or output handle");
    if (precision != BEC_FP64 && precision != BEC_FP32) return fail(BEC_EINVAL, "bad precision");
    if (((uintptr_t)d_ws) & 255) return fail(BEC_EINVAL, "workspace must be 256-byte aligned");
    Layout L = layout(desc->n, precision);
    if (ws_bytes < L.total) return fail(BEC_ENOMEM, "workspace smaller than bec_workspace_bytes");
    bec_grid g = new bec_grid_s();
    for (int i = 0; i < 3; ++i) {
        g->n[i] = desc->n[i];
        g->a[i] = desc->a[i];
        g->h[i] = 2.0 * desc->a[i] / desc->n[i];
    }
    g->h3 = g->h[0] * g->h[1] * g->h[2];
    g->precision = precision;
    g->stream = (hipStream_t)stream;
    g->ws = (char*)d_ws;
    g->ws_bytes = ws_bytes;
    g->st = (DevState*)(g->ws + L.state);
    g->done_flag = &g->st->done;
    g->partials = (double*)(g->ws + L.partials);
    g->partials_cap = L.partials_cap;
    g->uhat = (double*)(g->ws + L.uhat);
    g->sym_scratch = (double*)(g->ws + L.symscr);
    g->sym_scratch_bytes = L.symscr_doubles * sizeof(double);
    char* p = g->ws + L.f64;
    carve_fields<double>(g->f64, p, g->n);
    if (precision) {
        p = g->ws + L.f32;
        carve_fields<float>(g->f32, p, g->n);
    }
    const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    g->gz = make_geo(2, nx, ny, nz, nz, 0);
    g->gy = make_geo(1, nx, ny, nz, ny, 0);
    g->gx = make_geo(0, nx, ny, nz, nx, 0);
    g->g_ay = make_geo(1, nx, ny, nz + 1, 2 * ny, 0);
    g->g_ayi = g->g_ay;
    g->g_ax = make_geo(0, nx, 2 * ny, nz + 1, 2 * nx, 0);
    g->g_ax2 = make_geo(0, nx, 2 * ny, nz + 1, 2 * nx, 1);
    g->zf_L = std::max(1, kTileElems / (2 * nz));
    if (const char* e = std::getenv("BEC_GENERIC_FFT")) g->use_rf = std::atoi(e) ? 0 : 1;
    g->zf2_L = g->zf_L;
    g->zi_L = g->zf_L;
    if ((rc = make_plans<double>(*g, g->f64, g->ws + L.tw64))) { delete g; return rc; }
    if (precision && (rc = make_plans<float>(*g, g->f32, g->ws + L.tw32))) { delete g; return rc; }
    hipError_t e = hipMemsetAsync(g->st, 0, sizeof(DevState), g->stream);
    if (e != hipSuccess) { int r2 = hip_fail(g, e, "init state"); delete g; return r2; }
    *out = g;
    return BEC_OK;
}

int bec_destroy_grid(bec_grid g) {
    if (!g) return BEC_OK;
    if (g->graph) hipGraphExecDestroy(g->graph);
    delete g;
    return BEC_OK;
}

int bec_atkm_symbol(bec_grid g, double* d_out) {
    int rc = check_grid(g);
    if (rc) return rc;
    std::vector<double> scratch;
    launch_symbol(*g, scratch);
    if ((rc = check_launch(g, "symbol"))) return rc;
    g->have_symbol = true;
    if (d_out) {
        const size_t bytes = (size_t)(g->n[0] + 1) * (g->n[1] + 1) * (g->n[2] + 1) * sizeof(double);
        hipError_t e = hipMemcpyAsync(d_out, g->uhat, bytes, hipMemcpyDeviceToDevice, g->stream);
        if (e != hipSuccess) return hip_fail(g, e, "symbol copy");
    }
    return BEC_OK;
}

int bec_dipolar(bec_grid g, const bec_params* pp, const void* d_phi, void* d_Phi) {
    int rc = check_grid(g);
    if (rc) return rc;
    Params p;
    if ((rc = validate_params(pp, p))) return rc;
    if (!d_phi || !d_Phi) return fail(BEC_EINVAL, "NULL field pointer");
    if (!g->have_symbol) return fail(BEC_EINVAL, "bec_atkm_symbol has not been called on this grid");
    if (g->precision == BEC_FP64)
        launch_atkm<double>(*g, g->f64, p, (const cpx<double>*)d_phi, (double*)d_Phi, nullptr);
    else
        launch_atkm<float>(*g, g->f32, p, (const cpx<float>*)d_phi, (float*)d_Phi, nullptr);
    return check_launch(g, "dipolar");
}

int bec_apply_H(bec_grid g, const bec_params* pp, const void* d_phi, void* d_hphi, void* d_Phi, double* d_mu) {
    int rc = check_grid(g);
    if (rc) return rc;
    Params p;
    if ((rc = validate_params(pp, p))) return rc;
    if (!d_phi || !d_hphi) return fail(BEC_EINVAL, "NULL field pointer");
    if (d_phi == d_hphi) return fail(BEC_EINVAL, "d_hphi must not alias d_phi");
    if (p.lam != 0.0 && !g->have_symbol) return fail(BEC_EINVAL, "bec_atkm_symbol has not been called on this grid");
    launch_set_params(*g, p);
    if (g->precision == BEC_FP64) {
        double* Phi = d_Phi ? (double*)d_Phi : g->f64.Phi;
        launch_apply<double>(*g, g->f64, p, (const cpx<double>*)d_phi, (cpx<double>*)d_hphi, Phi, nullptr);
    } else {
        float* Phi = d_Phi ? (float*)d_Phi : g->f32.Phi;
        launch_apply<float>(*g, g->f32, p, (const cpx<float>*)d_phi, (cpx<float>*)d_hphi, Phi, nullptr);
    }
    if (d_mu) {
        hipError_t e = hipMemcpyAsync(d_mu, &g->st->mu, sizeof(double), hipMemcpyDeviceToDevice, g->stream);
        if (e != hipSuccess) return hip_fail(g, e, "mu copy");
    }
    return check_launch(g, "apply_H");
}

int bec_energy(bec_grid g, const bec_params* pp, const void* d_phi, bec_energies* out, int out_on_host) {
    int rc = check_grid(g);
    if (rc) return rc;
    Params p;
    if ((rc = validate_params(pp, p))) return rc;
    if (!d_phi || !out) return fail(BEC_EINVAL, "NULL pointer");
    if (p.lam != 0.0 && !g->have_symbol) return fail(BEC_EINVAL, "bec_atkm_symbol has not been called on this grid");
    launch_set_params(*g, p);
    if (g->precision == BEC_FP64)
        launch_apply<double>(*g, g->f64, p, (const cpx<double>*)d_phi, g->f64.hphi, g->f64.Phi, nullptr);
    else
        launch_apply<float>(*g, g->f32, p, (const cpx<float>*)d_phi, g->f32.hphi, g->f32.Phi, nullptr);
    if ((rc = check_launch(g, "energy"))) return rc;
    DevState hs;
    hipError_t e = hipMemcpyAsync(&hs, g->st, sizeof(DevState), hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "energy readback");
    bec_energies r;
    r.E = hs.E; r.Ekin = hs.Ekin; r.Epot = hs.Epot; r.Eint = hs.Eint; r.Edip = hs.Edip; r.Erot = hs.Erot;
    r.mu = hs.mu; r.mass = hs.mass;
    r.virial = 2 * hs.Ekin - 2 * hs.Epot + 3 * hs.Eint + 3 * hs.Edip;
    if (out_on_host) {
        *out = r;
    } else {
        e = hipMemcpyAsync(out, &r, sizeof(r), hipMemcpyHostToDevice, g->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) return hip_fail(g, e, "energy copy");
    }
    return BEC_OK;
}

int bec_fft3d(bec_grid g, const void* d_in, void* d_out, int dir) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!d_in || !d_out) return fail(BEC_EINVAL, "NULL field pointer");
    if (dir != -1 && dir != 1) return fail(BEC_EINVAL, "dir must be -1 or +1");
    if (g->precision == BEC_FP64)
        launch_fft3d<double>(*g, (const cpx<double>*)d_in, (cpx<double>*)d_out, dir);
    else
        launch_fft3d<float>(*g, (const cpx<float>*)d_in, (cpx<float>*)d_out, dir);
    return check_launch(g, "fft3d");
}

int bec_pcg_default_opts(bec_pcg_opts* o) {
    if (!o) return fail(BEC_EINVAL, "NULL opts");
    std::memset(o, 0, sizeof(*o));
    o->tol_res_inf = 1e-8;
    o->tol_step_inf = 0.0;
    o->max_iter = 20000;
    o->max_halvings = 30;
    o->t_default = 0.3;
    o->tau_E_ulps = 64.0;
    o->switch_res = 1e-5;
    o->check_every = 16;
    o->stall_window = 400;
    o->use_graph = 1;
    return BEC_OK;
}

int bec_pcg_solve(bec_grid g, const bec_params* pp, void* d_phi, const bec_pcg_opts* opts, bec_pcg_result* res) {
    int rc = check_grid(g);
    if (rc) return rc;
    Params p;
    if ((rc = validate_params(pp, p))) return rc;
    if (!d_phi || !res) return fail(BEC_EINVAL, "NULL pointer");
    bec_pcg_opts o;
    if (opts) o = *opts; else bec_pcg_default_opts(&o);
    if (!(o.tol_res_inf >= 0.0) || o.max_iter < 0 || o.max_halvings < 0 || o.check_every < 1)
        return fail(BEC_EINVAL, "bad options");
    if (p.lam != 0.0 && !g->have_symbol) return fail(BEC_EINVAL, "bec_atkm_symbol has not been called on this grid");
    return pcg_solve(*g, p, (cpx<double>*)d_phi, o, res);
}

int bec_time_stage(bec_grid g, const bec_params* pp, const void* d_phi, int which, int reps, double* avg_ms) {
    int rc = check_grid(g);
    if (rc) return rc;
    Params p;
    if ((rc = validate_params(pp, p))) return rc;
    if (!d_phi || !avg_ms || reps < 1 || which < 0 || which > 6) return fail(BEC_EINVAL, "bad arguments");
    if (which != 3 && which != 4 && !g->have_symbol) return fail(BEC_EINVAL, "bec_atkm_symbol has not been called on this grid");
    launch_set_params(*g, p);
    if (g->precision == BEC_FP64)
        *avg_ms = time_stage<double>(*g, g->f64, p, (const cpx<double>*)d_phi, which, reps);
    else
        *avg_ms = time_stage<float>(*g, g->f32, p, (const cpx<float>*)d_phi, which, reps);
    return check_launch(g, "time_stage");
}

}  // extern "C"
