// C ABI of the PCG-ATKM library: validation, workspace carving, FFT plans, entry points.
#include <hip/hip_runtime.h>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
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
    if (!std::isfinite(p->n[0]) || !std::isfinite(p->n[1]) || !std::isfinite(p->n[2]))
        return fail(BEC_EINVAL, "non-finite dipole axis");
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
    size_t state, params, stop, partials, uhat, symscr, tw64, tw32, f64, f32, total;
    long part_stride;
    size_t symscr_doubles;
};

// Row stride of the z half-spectrum buffers: Nz+1 entries padded to a multiple of 16, so that a
// tile of 8 (FP64) or 16 (FP32) consecutive kz columns starts on a 128-byte boundary.
int hs_ld(int nz) { return (nz + 1 + 15) / 16 * 16; }

// Tiles of an x pass over a half-spectrum buffer [Nx][nky][ld]: L consecutive ky at the Nyquist
// kz = nzq, then L consecutive kz < nzq at one ky.
void hs_tiles(Geo& g) {
    g.cpk = (g.nzq + g.L - 1) / g.L;
    g.nreg = g.nky * g.cpk;
    g.ntiles = g.nreg + (g.nky + g.L - 1) / g.L;
}

// Lines per block of the runtime-length (generic LDS) line kernels: a tile of at most kTileElems
// complex values (half that for two-field passes), divided by the grid's tile divisor for the axis.
static int lines_per_block(int nfft, int dual, int div) {
    int L = kTileElems / nfft;
    if (dual) L /= 2;
    L /= div;
    return L < 1 ? 1 : L;
}

Geo make_geo(int axis, int d0, int d1, int d2, int nfft, int dual, int div) {
    Geo g;
    std::memset(&g, 0, sizeof(g));
    g.axis = axis;
    int L = lines_per_block(nfft, dual, div);
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
        g.row = d2;
    } else {
        g.n_outer = 1;
        g.n_inner = d1 * d2;
        if (L > g.n_inner) L = g.n_inner;
        g.L = L;
        g.tpo = (g.n_inner + L - 1) / L;
        g.ntiles = g.tpo;
        g.dB = d2;
        g.row = g.n_inner;
    }
    return g;
}

// Padded y passes over the half-spectrum buffers: lines along y at (x, kz), kz <= nz, rows of ld.
// The Nyquist column kz = nz is tiled apart (L rows x per tile), as in the x passes, instead of
// filling one lane of a ninth L-column tile per x.
Geo make_geo_hs_y(int nx, int nz, int nfft, int div) {
    Geo g = make_geo(1, nx, 0, nz + 1, nfft, 0, div);
    g.row = hs_ld(nz);
    g.hs = 1;
    g.nky = nx;   // the tiled count (rows x)
    g.nzq = nz;
    g.ld = hs_ld(nz);
    hs_tiles(g);
    return g;
}

// Padded x passes over [Nx][nky][ld]: columns (ky, kz), the Nyquist column kz = nz tiled apart.
Geo make_geo_hs_x(int nky, int nz, int nfft, int dual, int div) {
    Geo g;
    std::memset(&g, 0, sizeof(g));
    g.axis = 0;
    g.L = lines_per_block(nfft, dual, div);
    g.n_outer = 1;
    g.n_inner = nky * (nz + 1);
    g.hs = 1;
    g.nky = nky;
    g.nzq = nz;
    g.ld = hs_ld(nz);
    g.row = (long)nky * g.ld;
    hs_tiles(g);
    return g;
}

constexpr int kMaxTileDiv = 16;

// Line-pass geometries from the grid size and the per-axis tile divisors. Only the generic
// (runtime-length) kernels read L from here; the register kernels fix it per length.
void plan_lines(Grid& g) {
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int* d = g.tile_div;
    g.gz = make_geo(2, nx, ny, nz, nz, 0, d[2]);
    g.gy = make_geo(1, nx, ny, nz, ny, 0, d[1]);
    g.gx = make_geo(0, nx, ny, nz, nx, 0, d[0]);
    g.g_ay = make_geo_hs_y(nx, nz, 2 * ny, d[1]);
    g.g_ax = make_geo_hs_x(2 * ny, nz, 2 * nx, 0, d[0]);
    g.g_ax2 = make_geo_hs_x(2 * ny, nz, 2 * nx, 1, d[0]);
    g.zf_L = lines_per_block(2 * nz, 0, d[2]);
}

// Does axis a run any pass on the generic kernels (whose tiles the divisors set)?
static bool axis_tunable(const Grid& g, int a) {
    return !g.use_rf || !rf_length(g.n[a]) || !rf_length(2 * g.n[a]);
}

Layout layout(const int n[3], int precision, int batch) {
    Layout L;
    const size_t N = (size_t)n[0] * n[1] * n[2];
    const size_t Nz1 = (size_t)n[0] * n[1] * hs_ld(n[2]);
    const size_t Ny2 = (size_t)n[0] * 2 * n[1] * hs_ld(n[2]);
    // partial sums of one reducing kernel: at most (blocks of the largest pass) x slots; the
    // register-FFT passes use fewer lines per block than the generic ones at small N, so bound
    // by one block per column as well
    size_t maxt = 0;
    maxt = std::max(maxt, (size_t)2 * n[1] * (n[2] + 1));          // padded x pass, >= 1 column per block
    maxt = std::max(maxt, (size_t)n[1] * n[2]);                    // N-grid x pass
    maxt = std::max(maxt, (size_t)n[0] * (n[2] + 1));              // y passes
    maxt = std::max(maxt, (size_t)n[0] * n[1]);                    // z passes
    maxt = std::max(maxt, (size_t)kRedBlocks);
    // room for the partial rows of every reduction finished by one k_fin launch (<= 18 slots
    // of at most maxt rows each, rounded per segment)
    L.part_stride = (long)(maxt * 24 + 64);
    const int ms = 651;
    size_t sd = 2 * ms;
    for (int d = 0; d < 3; ++d) sd += (size_t)ms * (n[d] + 1) + 2 * ((size_t)std::ceil(M_PI * n[d] / 2.0) + 80);
    L.symscr_doubles = sd;
    size_t tw = 0;
    for (int d = 0; d < 3; ++d) tw += al((size_t)n[d] * 16) + al((size_t)2 * n[d] * 16);
    const size_t B = (size_t)batch;
    size_t off = 0;
    L.state = off; off += al(B * sizeof(DevState));
    L.params = off; off += al(B * sizeof(Params));
    L.stop = off; off += al(B * sizeof(int));
    L.partials = off; off += al(B * L.part_stride * sizeof(double));
    L.uhat = off; off += al((size_t)(n[0] + 1) * (n[1] + 1) * (n[2] + 1) * sizeof(double));
    L.symscr = off; off += al(sd * sizeof(double));
    L.tw64 = off; off += tw;
    L.tw32 = off; off += precision ? tw : 0;
    auto fields_bytes = [&](size_t cs) {
        return 8 * al(B * N * 2 * cs) + 2 * al(B * N * cs) + 2 * al(B * Nz1 * 2 * cs) + 2 * al(B * Ny2 * 2 * cs);
    };
    L.f64 = off; off += fields_bytes(8);
    L.f32 = off; off += precision ? fields_bytes(4) : 0;
    L.total = off + 256;
    return L;
}

template <typename R> void carve_fields(Fields<R>& f, char*& p, const int n[3], int batch) {
    const size_t B = (size_t)batch;
    const size_t N = B * n[0] * n[1] * n[2];
    const size_t Nz1 = B * n[0] * n[1] * hs_ld(n[2]);
    const size_t Ny2 = B * n[0] * 2 * n[1] * hs_ld(n[2]);
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

// Validates `batch` parameter sets and uploads them to the device state of the grid.
int upload_params(Grid& g, const bec_params* pp) {
    if (!pp) return fail(BEC_EINVAL, "params is NULL");
    std::vector<Params> ps(g.batch);
    bool any = false;
    for (int b = 0; b < g.batch; ++b) {
        int rc = validate_params(pp + b, ps[b]);
        if (rc) return rc;
        any = any || ps[b].lam != 0.0;
    }
    if (any && !g.have_symbol) return fail(BEC_EINVAL, "bec_atkm_symbol has not been called on this grid");
    hipError_t e = hipMemcpyAsync(g.dparams, ps.data(), ps.size() * sizeof(Params), hipMemcpyHostToDevice, g.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g.stream);
    if (e != hipSuccess) return hip_fail(&g, e, "params upload");
    g.lam_any = any;
    launch_set_params(g);
    return check_launch(&g, "set params");
}

int read_states(Grid& g, std::vector<DevState>& hs) {
    hs.resize(g.batch);
    hipError_t e = hipMemcpyAsync(hs.data(), g.st, g.batch * sizeof(DevState), hipMemcpyDeviceToHost, g.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g.stream);
    if (e != hipSuccess) return hip_fail(&g, e, "state readback");
    return BEC_OK;
}

// The solver's auxiliary stream and fork/join events (parallel branches of the iteration).
int open_branches(Grid& g) {
    hipError_t e = hipStreamCreateWithFlags(&g.aux, hipStreamNonBlocking);
    for (int k = 0; k < kBranchEvents && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&g.ev[k], hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(&g, e, "branch stream");
    return BEC_OK;
}

void close_branches(Grid& g) {
    if (g.aux) {
        (void)hipStreamSynchronize(g.aux);
        (void)hipStreamDestroy(g.aux);
    }
    for (int k = 0; k < kBranchEvents; ++k)
        if (g.ev[k]) (void)hipEventDestroy(g.ev[k]);
    g.aux = nullptr;
    for (int k = 0; k < kBranchEvents; ++k) g.ev[k] = nullptr;
}

// ------------------------------------------------------------------ PCG driver
// Algorithm 1 for every solve of a batched grid with all scalar decisions on the device. The
// host enqueues iterations (eagerly for the first two of a phase, then as a captured
// two-iteration HIP graph) on a private non-blocking stream and reads the device states every
// check_every iterations; a phase ends when every solve is done. On BEC_FP32 grids the FP32 bulk
// phase also stops solves whose ||r||_inf has not dropped below 0.9x its best for stall_window
// iterations, then the FP64 polish runs from the renormalised FP32 states.
//
// The run is resumable: issue() enqueues the iterations up to the next check and returns at
// once; poll() waits for them, reads the states and moves on (stall stops, phase switch, end).
// One grid alternates the two; several grids (bec_pcg_solve_ragged) issue in turn and then poll
// in turn, so the grids' iterations run side by side on their own streams.
class Solve {
public:
    Solve(Grid& g, cpx<double>* phi, const bec_pcg_opts& o) : g_(g), phi_(phi), o_(o) {}

    int begin() {
        user_ = g_.stream;
        hipError_t e = hipStreamCreateWithFlags(&ps_, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(ev_, user_);
        if (e == hipSuccess) e = hipStreamWaitEvent(ps_, ev_, 0);
        if (e != hipSuccess) return rc_ = hip_fail(&g_, e, "solve stream");
        g_.stream = ps_;
        g_.step_rule = o_.tol_step_inf > 0.0;
        if (o_.branches && (rc_ = open_branches(g_))) return rc_;
        const size_t NB = (size_t)g_.n[0] * g_.n[1] * g_.n[2] * g_.batch;
        CtlOpts co;
        co.tol_res = o_.tol_res_inf; co.tol_step = o_.tol_step_inf; co.t_default = o_.t_default;
        co.tau_ulps = o_.tau_E_ulps; co.dbg_t = o_.debug_t; co.dbg_c2 = o_.debug_c2; co.max_iter = o_.max_iter;
        co.max_halv = o_.max_halvings; co.dbg_flags = o_.debug_flags; co.fp32 = 0;
        // clear the CG memory buffers and stop flags once (outside any captured graph)
        e = hipMemsetAsync(g_.dstop, 0, g_.batch * sizeof(int), g_.stream);
        if (e == hipSuccess) e = hipMemsetAsync(g_.f64.p, 0, NB * sizeof(cpx<double>), g_.stream);
        if (e == hipSuccess) e = hipMemsetAsync(g_.f64.r1, 0, NB * sizeof(cpx<double>), g_.stream);
        if (e != hipSuccess) return rc_ = hip_fail(&g_, e, "solve init");
        fp32_ = g_.precision == BEC_FP32;
        if (fp32_) {
            // FP32 bulk phase: stop at ||r||_inf <= switch_res (times |mu| if relative) or when the
            // residual stalls. The trial energies are FP64 polynomials of FP64 sums, so the energy
            // test keeps its FP64 slack (an FP32-sized slack accepts energy increases and the
            // phase never settles).
            co.tol_res = o_.switch_relative ? o_.switch_res : std::max(o_.switch_res, o_.tol_res_inf);
            co.tol_rel = o_.switch_relative ? 1 : 0;
            launch_ctl_init(g_, co);
            e = hipMemsetAsync(g_.f32.p, 0, NB * sizeof(cpx<float>), g_.stream);
            if (e == hipSuccess) e = hipMemsetAsync(g_.f32.r1, 0, NB * sizeof(cpx<float>), g_.stream);
            if (e != hipSuccess) return rc_ = hip_fail(&g_, e, "solve init");
            launch_to_f32(g_, phi_, g_.f32.phi);
        } else {
            launch_ctl_init(g_, co);
        }
        const char* prog = std::getenv("BEC_PROGRESS");
        prog_every_ = prog ? std::atof(prog) : 0.0;
        last_print_ = now();
        return rc_ = start_phase();
    }

    bool finished() const { return done_ || rc_ != BEC_OK; }
    int rc() const { return rc_; }

    int issue() {
        if (finished()) return rc_;
        return rc_ = fp32_ ? issue_t<float>(g_.f32.phi) : issue_t<double>(phi_);
    }

    int poll() {
        if (finished()) return rc_;
        if ((rc_ = read_states(g_, hs_))) return rc_;
        bool all = true, new_stop = false;
        double rmin = 1e300, rmax = 0.0;
        int ndone = 0;
        for (int b = 0; b < g_.batch; ++b) {
            const DevState& S = hs_[b];
            if (S.done) { ++ndone; continue; }
            all = false;
            rmin = std::min(rmin, S.res_inf);
            rmax = std::max(rmax, S.res_inf);
            if (fp32_) {
                if (S.res_inf < 0.9 * best_[b]) { best_[b] = S.res_inf; best_it_[b] = S.iter; }
                else if (S.iter - best_it_[b] >= o_.stall_window && !stop_[b]) { stop_[b] = 1; new_stop = true; }
            }
        }
        if (prog_every_ > 0 && now() - last_print_ >= prog_every_) {
            std::fprintf(stderr, "[bec] %dx%dx%d %s iter %d done %d/%d res %.3e..%.3e E0 %.15f\n", g_.n[0], g_.n[1],
                         g_.n[2], fp32_ ? "fp32" : "fp64", hs_[0].iter, ndone, g_.batch, rmin, rmax, hs_[0].E);
            std::fflush(stderr);
            last_print_ = now();
        }
        if (all) {
            drop_graph();
            if (!fp32_) {
                done_ = true;
                return rc_;
            }
            // FP32 phase over: reopen the solves first (the normalisation kernels skip solves
            // marked done), then the FP64 polish from the renormalised states
            fp32_ = false;
            launch_ctl_phase(g_, o_.tol_res_inf, o_.max_iter, o_.tau_E_ulps, 2.220446049250313e-16);
            launch_to_f64_normalized(g_, g_.f32.phi, phi_);
            if ((rc_ = check_launch(&g_, "phase switch"))) return rc_;
            return rc_ = start_phase();
        }
        if (new_stop) {
            hipError_t e = hipMemcpyAsync(g_.dstop, stop_.data(), g_.batch * sizeof(int), hipMemcpyHostToDevice, g_.stream);
            if (e == hipSuccess) e = hipStreamSynchronize(g_.stream);
            if (e != hipSuccess) return rc_ = hip_fail(&g_, e, "stop flags");
            launch_ctl_stop(g_);
        }
        return rc_;
    }

    // Tears down streams and graphs (also after an error) and fills `batch` results.
    int finish(bec_pcg_result* res) {
        drop_graph();
        if (ps_) (void)hipStreamSynchronize(ps_);
        close_branches(g_);
        if (user_ || ps_) g_.stream = user_;
        if (ev_) (void)hipEventDestroy(ev_);
        if (ps_) (void)hipStreamDestroy(ps_);
        ev_ = nullptr;
        ps_ = nullptr;
        if (rc_) return rc_;
        if ((rc_ = read_states(g_, hs_))) return rc_;
        int worst = BEC_OK;
        for (int b = 0; b < g_.batch; ++b) {
            const DevState& S = hs_[b];
            bec_pcg_result& r = res[b];
            r.status = S.status == 0 ? BEC_OK : S.status;
            r.iters = S.iter;
            r.halvings = S.halvings;
            r.psd_resets = S.resets;
            r.forced_accepts = S.forced;
            r.fp32_iters = g_.precision == BEC_FP32 ? S.fp32_iters : 0;
            r.res_inf = S.res_inf;
            r.step_inf = g_.step_rule || g_.precision == BEC_FP32 ? S.step_inf : 0.0;
            r.e.E = S.E; r.e.Ekin = S.Ekin; r.e.Epot = S.Epot; r.e.Eint = S.Eint;
            r.e.Edip = S.Edip; r.e.Erot = S.Erot; r.e.mu = S.mu; r.e.mass = S.mass;
            r.e.virial = 2 * S.Ekin - 2 * S.Epot + 3 * S.Eint + 3 * S.Edip;
            if (r.status == BEC_ENUMERIC || (r.status == BEC_ENOTCONV && worst == BEC_OK)) worst = r.status;
        }
        return worst;
    }

private:
    static double now() {
        return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
    }

    int start_phase() {
        it_ = 0;
        best_.assign(g_.batch, 1e300);
        best_it_.assign(g_.batch, 0);
        stop_.assign(g_.batch, 0);
        if (fp32_) launch_pcg_start<float>(g_, g_.f32.phi);
        else launch_pcg_start<double>(g_, phi_);
        return check_launch(&g_, "pcg start");
    }

    void drop_graph() {
        if (exec_) (void)hipGraphExecDestroy(exec_);
        if (graph_) (void)hipGraphDestroy(graph_);
        exec_ = nullptr;
        graph_ = nullptr;
    }

    // enqueue iterations up to the next check: after the first, then every check_every
    template <typename R> int issue_t(cpx<R>* phi) {
        const long every = o_.check_every;
        do {
            if (o_.use_graph && it_ >= 2 && (it_ & 1) == 0) {
                if (!exec_) {
                    hipError_t e = hipStreamBeginCapture(g_.stream, hipStreamCaptureModeThreadLocal);
                    if (e != hipSuccess) return hip_fail(&g_, e, "begin capture");
                    launch_pcg_iteration<R>(g_, phi, 0);
                    launch_pcg_iteration<R>(g_, phi, 1);
                    e = hipStreamEndCapture(g_.stream, &graph_);
                    if (e != hipSuccess) return hip_fail(&g_, e, "end capture");
                    e = hipGraphInstantiate(&exec_, graph_, nullptr, nullptr, 0);
                    if (e != hipSuccess) return hip_fail(&g_, e, "graph instantiate");
                }
                hipError_t e = hipGraphLaunch(exec_, g_.stream);
                if (e != hipSuccess) return hip_fail(&g_, e, "graph launch");
                it_ += 2;
            } else {
                launch_pcg_iteration<R>(g_, phi, (int)(it_ & 1));
                it_ += 1;
            }
            int rc = check_launch(&g_, "pcg iteration");
            if (rc) return rc;
        } while (!(it_ % every == 0 || it_ < 2));
        return BEC_OK;
    }

    Grid& g_;
    cpx<double>* phi_;
    bec_pcg_opts o_;
    hipStream_t user_ = nullptr, ps_ = nullptr;
    hipEvent_t ev_ = nullptr;
    bool fp32_ = false, done_ = false;
    int rc_ = BEC_OK;
    long it_ = 0;
    hipGraph_t graph_ = nullptr;
    hipGraphExec_t exec_ = nullptr;
    std::vector<double> best_;
    std::vector<long> best_it_;
    std::vector<int> stop_;
    std::vector<DevState> hs_;
    double prog_every_ = 0.0, last_print_ = 0.0;
};

int pcg_solve(Grid& g, cpx<double>* phi, const bec_pcg_opts& o, bec_pcg_result* res) {
    Solve s(g, phi, o);
    if (!s.begin())
        while (!s.finished()) {
            if (s.issue()) break;
            if (s.poll()) break;
        }
    const int rc = s.finish(res);
    if (rc != BEC_OK && rc != BEC_ENOTCONV && rc != BEC_ENUMERIC) return rc;
    if (rc != BEC_OK) g_last_error = bec_status_string(rc);
    return rc;
}

// Iterations of Algorithm 1 with every launch timed by its own events (see bec_pcg_profile).
// The stream drains after each iteration, when the pairs are read and the pool reused.
template <typename R>
int profile_phase(Grid& g, cpx<R>* phi, int iters, double* ms, int32_t* cnt) {
    launch_pcg_start<R>(g, phi);
    int rc = check_launch(&g, "profile start");
    if (rc) return rc;
    KProf kp;
    kp.ev.resize(2 * 128);   // at most 128 launches per iteration
    for (auto& e : kp.ev) {
        hipError_t he = hipEventCreate(&e);
        if (he != hipSuccess) { rc = hip_fail(&g, he, "profile events"); break; }
    }
    for (int it = 0; it < iters && !rc; ++it) {
        kp.sites.clear();
        g.kprof = &kp;
        launch_pcg_iteration<R>(g, phi, it & 1);
        g.kprof = nullptr;
        if ((rc = check_launch(&g, "profile iteration"))) break;
        hipError_t he = hipStreamSynchronize(g.stream);
        if (he != hipSuccess) { rc = hip_fail(&g, he, "profile sync"); break; }
        for (size_t k = 0; k < kp.sites.size(); ++k) {
            float t = 0.f;
            he = hipEventElapsedTime(&t, kp.ev[2 * k], kp.ev[2 * k + 1]);
            if (he != hipSuccess) { rc = hip_fail(&g, he, "profile elapsed"); break; }
            ms[kp.sites[k]] += t;
            cnt[kp.sites[k]] += 1;
        }
    }
    g.kprof = nullptr;
    for (auto& e : kp.ev)
        if (e) hipEventDestroy(e);
    return rc;
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

int bec_version(void) { return 2; }

int bec_workspace_bytes_batched(const bec_grid_desc* desc, int precision, int batch, size_t* bytes) {
    int rc = validate_desc(desc);
    if (rc) return rc;
    if (!bytes) return fail(BEC_EINVAL, "bytes is NULL");
    if (precision != BEC_FP64 && precision != BEC_FP32) return fail(BEC_EINVAL, "bad precision");
    if (batch < 1 || batch > 65535) return fail(BEC_EINVAL, "batch must be in [1, 65535]");
    *bytes = layout(desc->n, precision, batch).total;
    return BEC_OK;
}

int bec_workspace_bytes(const bec_grid_desc* desc, int precision, size_t* bytes) {
    return bec_workspace_bytes_batched(desc, precision, 1, bytes);
}

int bec_init_grid_batched(const bec_grid_desc* desc, int precision, int batch, void* d_ws, size_t ws_bytes,
                          void* stream, bec_grid* out) {
    int rc = validate_desc(desc);
    if (rc) return rc;
    if (!out || !d_ws) return fail(BEC_EINVAL, "NULL workspace or output handle");
    if (precision != BEC_FP64 && precision != BEC_FP32) return fail(BEC_EINVAL, "bad precision");
    if (batch < 1 || batch > 65535) return fail(BEC_EINVAL, "batch must be in [1, 65535]");
    if (((uintptr_t)d_ws) & 255) return fail(BEC_EINVAL, "workspace must be 256-byte aligned");
    Layout L = layout(desc->n, precision, batch);
    if (ws_bytes < L.total) return fail(BEC_ENOMEM, "workspace smaller than bec_workspace_bytes");
    bec_grid g = new bec_grid_s();
    for (int i = 0; i < 3; ++i) {
        g->n[i] = desc->n[i];
        g->a[i] = desc->a[i];
        g->h[i] = 2.0 * desc->a[i] / desc->n[i];
    }
    g->h3 = g->h[0] * g->h[1] * g->h[2];
    g->precision = precision;
    g->batch = batch;
    g->stream = (hipStream_t)stream;
    g->ws = (char*)d_ws;
    g->ws_bytes = ws_bytes;
    g->st = (DevState*)(g->ws + L.state);
    g->dparams = (Params*)(g->ws + L.params);
    g->dstop = (int*)(g->ws + L.stop);
    g->partials = (double*)(g->ws + L.partials);
    g->part_stride = L.part_stride;
    g->uhat = (double*)(g->ws + L.uhat);
    g->sym_scratch = (double*)(g->ws + L.symscr);
    g->sym_scratch_bytes = L.symscr_doubles * sizeof(double);
    char* p = g->ws + L.f64;
    carve_fields<double>(g->f64, p, g->n, batch);
    if (precision) {
        p = g->ws + L.f32;
        carve_fields<float>(g->f32, p, g->n, batch);
    }
    const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    plan_lines(*g);
    const long N = (long)nx * ny * nz;
    g->bt64 = Bat{N, (long)nx * ny * hs_ld(nz), (long)nx * 2 * ny * hs_ld(nz), L.part_stride};
    g->bt32 = g->bt64;
    if (const char* ev = std::getenv("BEC_GENERIC_FFT")) g->use_rf = std::atoi(ev) ? 0 : 1;
    if ((rc = make_plans<double>(*g, g->f64, g->ws + L.tw64))) { delete g; return rc; }
    if (precision && (rc = make_plans<float>(*g, g->f32, g->ws + L.tw32))) { delete g; return rc; }
    hipError_t e = hipMemsetAsync(g->st, 0, batch * sizeof(DevState), g->stream);
    if (e != hipSuccess) { int r2 = hip_fail(g, e, "init state"); delete g; return r2; }
    *out = g;
    return BEC_OK;
}

int bec_init_grid(const bec_grid_desc* desc, int precision, void* d_ws, size_t ws_bytes, void* stream, bec_grid* out) {
    return bec_init_grid_batched(desc, precision, 1, d_ws, ws_bytes, stream, out);
}

int bec_grid_batch(bec_grid g) { return g ? g->batch : 0; }

int bec_destroy_grid(bec_grid g) {
    if (!g) return BEC_OK;
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
        launch_symbol_out(*g, d_out);
        if ((rc = check_launch(g, "symbol copy"))) return rc;
    }
    return BEC_OK;
}

int bec_dipolar(bec_grid g, const bec_params* pp, const void* d_phi, void* d_Phi) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!d_phi || !d_Phi) return fail(BEC_EINVAL, "NULL field pointer");
    if (!g->have_symbol) return fail(BEC_EINVAL, "bec_atkm_symbol has not been called on this grid");
    if ((rc = upload_params(*g, pp))) return rc;
    if (g->precision == BEC_FP64)
        launch_atkm<double>(*g, (const cpx<double>*)d_phi, (double*)d_Phi);
    else
        launch_atkm<float>(*g, (const cpx<float>*)d_phi, (float*)d_Phi);
    return check_launch(g, "dipolar");
}

int bec_apply_H(bec_grid g, const bec_params* pp, const void* d_phi, void* d_hphi, void* d_Phi, double* d_mu) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!d_phi || !d_hphi) return fail(BEC_EINVAL, "NULL field pointer");
    if (d_phi == d_hphi) return fail(BEC_EINVAL, "d_hphi must not alias d_phi");
    if ((rc = upload_params(*g, pp))) return rc;
    if (g->precision == BEC_FP64) {
        double* Phi = d_Phi ? (double*)d_Phi : g->f64.Phi;
        launch_apply<double>(*g, (const cpx<double>*)d_phi, (cpx<double>*)d_hphi, Phi);
    } else {
        float* Phi = d_Phi ? (float*)d_Phi : g->f32.Phi;
        launch_apply<float>(*g, (const cpx<float>*)d_phi, (cpx<float>*)d_hphi, Phi);
    }
    if (d_mu) {
        for (int b = 0; b < g->batch; ++b) {
            hipError_t e = hipMemcpyAsync(d_mu + b, &g->st[b].mu, sizeof(double), hipMemcpyDeviceToDevice, g->stream);
            if (e != hipSuccess) return hip_fail(g, e, "mu copy");
        }
    }
    return check_launch(g, "apply_H");
}

int bec_energy(bec_grid g, const bec_params* pp, const void* d_phi, bec_energies* out, int out_on_host) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!d_phi || !out) return fail(BEC_EINVAL, "NULL pointer");
    if ((rc = upload_params(*g, pp))) return rc;
    if (g->precision == BEC_FP64)
        launch_apply<double>(*g, (const cpx<double>*)d_phi, g->f64.hphi, g->f64.Phi);
    else
        launch_apply<float>(*g, (const cpx<float>*)d_phi, g->f32.hphi, g->f32.Phi);
    if ((rc = check_launch(g, "energy"))) return rc;
    std::vector<DevState> hs;
    if ((rc = read_states(*g, hs))) return rc;
    std::vector<bec_energies> r(g->batch);
    for (int b = 0; b < g->batch; ++b) {
        const DevState& S = hs[b];
        r[b].E = S.E; r[b].Ekin = S.Ekin; r[b].Epot = S.Epot; r[b].Eint = S.Eint; r[b].Edip = S.Edip;
        r[b].Erot = S.Erot; r[b].mu = S.mu; r[b].mass = S.mass;
        r[b].virial = 2 * S.Ekin - 2 * S.Epot + 3 * S.Eint + 3 * S.Edip;
    }
    if (out_on_host) {
        std::memcpy(out, r.data(), r.size() * sizeof(bec_energies));
    } else {
        hipError_t e = hipMemcpyAsync(out, r.data(), r.size() * sizeof(bec_energies), hipMemcpyHostToDevice, g->stream);
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
    // the transform needs no parameters; run with the solves marked active
    hipError_t e = hipMemsetAsync(g->st, 0, g->batch * sizeof(DevState), g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "fft3d state");
    if (g->precision == BEC_FP64)
        launch_fft3d<double>(*g, (const cpx<double>*)d_in, (cpx<double>*)d_out, dir);
    else
        launch_fft3d<float>(*g, (const cpx<float>*)d_in, (cpx<float>*)d_out, dir);
    return check_launch(g, "fft3d");
}

int bec_interp_spectral(bec_grid src, bec_grid dst, const void* d_in, int in_precision, void* d_out,
                        int out_precision) {
    int rc = check_grid(src);
    if (!rc) rc = check_grid(dst);
    if (rc) return rc;
    if (!d_in || !d_out) return fail(BEC_EINVAL, "NULL field pointer");
    if ((in_precision != BEC_FP64 && in_precision != BEC_FP32) || (out_precision != BEC_FP64 && out_precision != BEC_FP32))
        return fail(BEC_EINVAL, "precision must be BEC_FP64 or BEC_FP32");
    if (src == dst) return fail(BEC_EINVAL, "src and dst must be different handles");
    if (src->batch != dst->batch) return fail(BEC_EINVAL, "src and dst batch sizes differ");
    for (int i = 0; i < 3; ++i)
        if (!(std::fabs(src->a[i] - dst->a[i]) <= 1e-12 * std::fabs(dst->a[i])))
            return fail(BEC_EINVAL, "src and dst boxes differ");
    hipStream_t dst_stream = dst->stream;
    dst->stream = src->stream;   // one stream orders the two grids' work
    hipError_t e = hipMemsetAsync(src->st, 0, src->batch * sizeof(DevState), src->stream);
    if (e == hipSuccess) e = hipMemsetAsync(dst->st, 0, dst->batch * sizeof(DevState), src->stream);
    if (e != hipSuccess) {
        dst->stream = dst_stream;
        return hip_fail(src, e, "interp state");
    }
    launch_interp(*src, *dst, d_in, in_precision == BEC_FP32, d_out, out_precision == BEC_FP32);
    rc = check_launch(src, "interp");
    if (!rc && dst_stream != src->stream) {
        e = hipStreamSynchronize(src->stream);
        if (e != hipSuccess) rc = hip_fail(src, e, "interp sync");
    }
    dst->stream = dst_stream;
    return rc;
}

int bec_normalize(bec_grid g, void* d_phi) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!d_phi) return fail(BEC_EINVAL, "NULL field pointer");
    launch_normalize(*g, (cpx<double>*)d_phi);
    return check_launch(g, "normalize");
}

int bec_rotate_z(bec_grid g, const void* d_in, void* d_out, double alpha) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!d_in || !d_out) return fail(BEC_EINVAL, "NULL field pointer");
    if (g->n[0] != g->n[1] || !(std::fabs(g->a[0] - g->a[1]) <= 1e-12 * g->a[0]))
        return fail(BEC_EINVAL, "rotation about z needs N_x = N_y and a_x = a_y");
    if (!std::isfinite(alpha) || std::fabs(alpha) > 8.0 * M_PI) return fail(BEC_EINVAL, "angle must be finite, |alpha| <= 8 pi");
    hipError_t e = hipMemsetAsync(g->st, 0, g->batch * sizeof(DevState), g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "rotate state");
    launch_rotate(*g, (const cpx<double>*)d_in, (cpx<double>*)d_out, alpha);
    return check_launch(g, "rotate");
}

int bec_gauge_fix(bec_grid g, const bec_params* pp, void* d_phi) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!d_phi || !pp) return fail(BEC_EINVAL, "NULL pointer");
    std::vector<Params> ps(g->batch);
    for (int b = 0; b < g->batch; ++b)
        if ((rc = validate_params(pp + b, ps[b]))) return rc;
    hipError_t e = hipMemcpyAsync(g->dparams, ps.data(), ps.size() * sizeof(Params), hipMemcpyHostToDevice, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "params upload");
    launch_gauge(*g, (cpx<double>*)d_phi);
    return check_launch(g, "gauge fix");
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
    o->switch_relative = 1;
    o->branches = 1;
    return BEC_OK;
}

int bec_pcg_solve_batched(bec_grid g, const bec_params* pp, void* d_phi, const bec_pcg_opts* opts,
                          bec_pcg_result* res) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!d_phi || !res) return fail(BEC_EINVAL, "NULL pointer");
    bec_pcg_opts o;
    if (opts) o = *opts; else bec_pcg_default_opts(&o);
    if (!(o.tol_res_inf >= 0.0) || o.max_iter < 0 || o.max_halvings < 0 || o.check_every < 1)
        return fail(BEC_EINVAL, "bad options");
    if ((rc = upload_params(*g, pp))) return rc;
    return pcg_solve(*g, (cpx<double>*)d_phi, o, res);
}

int bec_pcg_solve(bec_grid g, const bec_params* pp, void* d_phi, const bec_pcg_opts* opts, bec_pcg_result* res) {
    return bec_pcg_solve_batched(g, pp, d_phi, opts, res);
}

int bec_pcg_solve_ragged(bec_grid* grids, const bec_params* const* pp, void* const* d_phis, int ngrids,
                         const bec_pcg_opts* opts, bec_pcg_result* res) {
    if (!grids || !pp || !d_phis || !res) return fail(BEC_EINVAL, "NULL pointer");
    if (ngrids < 1 || ngrids > 64) return fail(BEC_EINVAL, "ngrids must be in [1, 64]");
    bec_pcg_opts o;
    if (opts) o = *opts; else bec_pcg_default_opts(&o);
    if (!(o.tol_res_inf >= 0.0) || o.max_iter < 0 || o.max_halvings < 0 || o.check_every < 1)
        return fail(BEC_EINVAL, "bad options");
    int rc;
    for (int k = 0; k < ngrids; ++k) {
        if ((rc = check_grid(grids[k]))) return rc;
        if (!d_phis[k] || !pp[k]) return fail(BEC_EINVAL, "NULL field or parameter array");
        for (int j = 0; j < k; ++j)
            if (grids[j] == grids[k]) return fail(BEC_EINVAL, "a grid handle appears twice");
    }
    for (int k = 0; k < ngrids; ++k)
        if ((rc = upload_params(*grids[k], pp[k]))) return rc;
    std::vector<Solve> runs;
    runs.reserve(ngrids);
    for (int k = 0; k < ngrids; ++k) runs.emplace_back(*grids[k], (cpx<double>*)d_phis[k], o);
    int err = BEC_OK;
    for (int k = 0; k < ngrids && !err; ++k) err = runs[k].begin();
    // issue every grid's iterations up to its next check, then wait for and read each grid in
    // turn: while one grid is read, the others' iterations keep running on their streams
    for (bool active = !err; active && !err;) {
        active = false;
        for (auto& r : runs)
            if (!r.finished() && (err = r.issue())) break;
        for (auto& r : runs) {
            if (err) break;
            if (!r.finished() && (err = r.poll())) break;
            active = active || !r.finished();
        }
    }
    int worst = BEC_OK;
    long off = 0;
    for (int k = 0; k < ngrids; ++k) {
        const int w = runs[k].finish(res + off);
        off += grids[k]->batch;
        if (w != BEC_OK && w != BEC_ENOTCONV && w != BEC_ENUMERIC) {
            if (!err) err = w;
        } else if (w == BEC_ENUMERIC || (w == BEC_ENOTCONV && worst == BEC_OK)) {
            worst = w;
        }
    }
    if (err) return err;
    if (worst != BEC_OK) g_last_error = bec_status_string(worst);
    return worst;
}

}  // extern "C"

namespace {

// The iterations of bec_pcg_profile on a grid whose parameters are uploaded.
int run_profile(bec_grid g, void* d_phi, int iters, int flags, double* site_ms, int32_t* site_launches) {
    int rc = BEC_OK;
    for (int i = 0; i < BEC_NSITES; ++i) { site_ms[i] = 0.0; site_launches[i] = 0; }
    bec_pcg_opts o;
    bec_pcg_default_opts(&o);
    CtlOpts co;
    co.tol_res = 0.0; co.tol_step = 0.0; co.t_default = o.t_default; co.tau_ulps = o.tau_E_ulps;
    co.dbg_t = 0.0; co.dbg_c2 = 0.0; co.max_iter = 0x7fffffff; co.max_halv = o.max_halvings;
    co.dbg_flags = 0; co.fp32 = 0;
    g->step_rule = false;
    const size_t NB = (size_t)g->n[0] * g->n[1] * g->n[2] * g->batch;
    hipError_t e = hipMemsetAsync(g->dstop, 0, g->batch * sizeof(int), g->stream);
    if (e == hipSuccess) e = hipMemsetAsync(g->f64.p, 0, NB * sizeof(cpx<double>), g->stream);
    if (e == hipSuccess) e = hipMemsetAsync(g->f64.r1, 0, NB * sizeof(cpx<double>), g->stream);
    if (e == hipSuccess && g->precision == BEC_FP32) e = hipMemsetAsync(g->f32.p, 0, NB * sizeof(cpx<float>), g->stream);
    if (e == hipSuccess && g->precision == BEC_FP32) e = hipMemsetAsync(g->f32.r1, 0, NB * sizeof(cpx<float>), g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "profile init");
    launch_ctl_init(*g, co);
    if ((flags & 1) && (rc = open_branches(*g))) {
        close_branches(*g);
        return rc;
    }
    cpx<double>* phi = (cpx<double>*)d_phi;
    if (g->precision == BEC_FP32) {
        launch_to_f32(*g, phi, g->f32.phi);
        rc = profile_phase<float>(*g, g->f32.phi, iters, site_ms, site_launches);
        if (!rc) {
            launch_ctl_phase(*g, o.tol_res_inf, o.max_iter, o.tau_E_ulps, 2.220446049250313e-16);
            launch_to_f64_normalized(*g, g->f32.phi, phi);
            rc = check_launch(g, "profile convert");
        }
    } else {
        rc = profile_phase<double>(*g, phi, iters, site_ms, site_launches);
    }
    close_branches(*g);
    g->step_rule = false;
    if (rc) return rc;
    e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "profile sync");
    return BEC_OK;
}

}  // namespace

extern "C" {

int bec_pcg_profile(bec_grid g, const bec_params* pp, void* d_phi, int iters, int flags, double* site_ms,
                    int32_t* site_launches) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!d_phi || !site_ms || !site_launches || iters < 1) return fail(BEC_EINVAL, "bad arguments");
    if ((rc = upload_params(*g, pp))) return rc;
    return run_profile(g, d_phi, iters, flags, site_ms, site_launches);
}

static_assert(bec::kKernelVariants == BEC_KERNEL_VARIANTS, "variant count of the header and the kernels");
int bec_set_kernel_variants(bec_grid g, const int32_t* variants) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!variants) return fail(BEC_EINVAL, "variants is NULL");
    for (int s = 0; s < BEC_NSITES; ++s)
        if (variants[s] < 0 || variants[s] >= kKernelVariants) return fail(BEC_EINVAL, "kernel variant out of range");
    for (int s = 0; s < BEC_NSITES; ++s) g->variant[s] = variants[s];
    return BEC_OK;
}

int bec_get_kernel_variants(bec_grid g, int32_t* variants) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!variants) return fail(BEC_EINVAL, "variants is NULL");
    for (int s = 0; s < BEC_NSITES; ++s) variants[s] = g->variant[s];
    return BEC_OK;
}

// Every variant is profiled on every site at once (the sites are different kernels), `iters`
// iterations each, one stream; each site keeps its fastest variant.
int bec_autotune_kernels(bec_grid g, const bec_params* pp, void* d_phi, int iters, int32_t* variants_out,
                         double* ms_default, double* ms_best) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!d_phi || iters < 1) return fail(BEC_EINVAL, "bad arguments");
    if (!g->have_symbol) return fail(BEC_EINVAL, "bec_atkm_symbol has not been called on this grid");
    if ((rc = upload_params(*g, pp))) return rc;
    double ms[kKernelVariants][BEC_NSITES];
    int32_t cnt[BEC_NSITES];
    for (int v = 0; v < kKernelVariants && !rc; ++v) {
        for (int s = 0; s < BEC_NSITES; ++s) g->variant[s] = v;
        rc = run_profile(g, d_phi, iters, 0, ms[v], cnt);
    }
    for (int s = 0; s < BEC_NSITES; ++s) {
        // a variant replaces the default only when it is faster by more than the run-to-run spread
        int best = 0;
        if (!rc && site_has_variants(*g, s))
            for (int v = 1; v < kKernelVariants; ++v)
                if (site_variant_distinct(*g, s, v) && ms[v][s] < 0.98 * ms[0][s] && ms[v][s] < ms[best][s]) best = v;
        g->variant[s] = best;
        if (variants_out) variants_out[s] = best;
        if (ms_default) ms_default[s] = rc ? 0.0 : ms[0][s] / iters;
        if (ms_best) ms_best[s] = rc ? 0.0 : ms[best][s] / iters;
    }
    return rc;
}

int bec_time_stage(bec_grid g, const bec_params* pp, const void* d_phi, int which, int reps, double* avg_ms) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!d_phi || !avg_ms || reps < 1 || which < 0 || which > 6) return fail(BEC_EINVAL, "bad arguments");
    if (which != 3 && which != 4 && !g->have_symbol) return fail(BEC_EINVAL, "bec_atkm_symbol has not been called on this grid");
    if ((rc = upload_params(*g, pp))) return rc;
    if (g->precision == BEC_FP64)
        *avg_ms = time_stage<double>(*g, (const cpx<double>*)d_phi, which, reps);
    else
        *avg_ms = time_stage<float>(*g, (const cpx<float>*)d_phi, which, reps);
    return check_launch(g, "time_stage");
}

int bec_set_line_tiles(bec_grid g, const int32_t div[3]) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!div) return fail(BEC_EINVAL, "div is NULL");
    for (int a = 0; a < 3; ++a)
        if (div[a] < 1 || div[a] > kMaxTileDiv || (div[a] & (div[a] - 1)))
            return fail(BEC_EINVAL, "tile divisors must be powers of two in [1, 16]");
    for (int a = 0; a < 3; ++a) g->tile_div[a] = div[a];
    plan_lines(*g);
    return BEC_OK;
}

int bec_get_line_tiles(bec_grid g, int32_t div[3], int32_t tunable[3]) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!div) return fail(BEC_EINVAL, "div is NULL");
    for (int a = 0; a < 3; ++a) {
        div[a] = g->tile_div[a];
        if (tunable) tunable[a] = axis_tunable(*g, a) ? 1 : 0;
    }
    return BEC_OK;
}

// Coordinate search over the per-axis divisors 1, 2, 4, ..., kMaxTileDiv (z, then y, then x):
// each candidate is timed as one H apply plus one two-density Parseval pass (every line pass of
// the iteration on every axis), `reps` times after one warm-up, with HIP events on the grid
// stream. Axes whose passes all use the register kernels are skipped.
int bec_autotune_line_tiles(bec_grid g, const bec_params* pp, const void* d_phi, int reps, int32_t div_out[3],
                            double* ms_out) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!d_phi || reps < 1) return fail(BEC_EINVAL, "bad arguments");
    if (!g->have_symbol) return fail(BEC_EINVAL, "bec_atkm_symbol has not been called on this grid");
    if ((rc = upload_params(*g, pp))) return rc;
    auto measure = [&]() {
        if (g->precision == BEC_FP64)
            return time_stage<double>(*g, (const cpx<double>*)d_phi, 2, reps) +
                   time_stage<double>(*g, (const cpx<double>*)d_phi, 6, reps);
        return time_stage<float>(*g, (const cpx<float>*)d_phi, 2, reps) +
               time_stage<float>(*g, (const cpx<float>*)d_phi, 6, reps);
    };
    double best = measure();
    if ((rc = check_launch(g, "autotune"))) return rc;
    for (int a = 2; a >= 0; --a) {
        if (!axis_tunable(*g, a)) continue;
        const int keep = g->tile_div[a];
        int pick = keep;
        for (int d = 1; d <= kMaxTileDiv; d *= 2) {
            if (d == keep) continue;
            g->tile_div[a] = d;
            plan_lines(*g);
            const double t = measure();
            if ((rc = check_launch(g, "autotune"))) {
                g->tile_div[a] = pick;   // leave the best set found so far
                plan_lines(*g);
                return rc;
            }
            if (t < best) {
                best = t;
                pick = d;
            }
        }
        g->tile_div[a] = pick;
        plan_lines(*g);
    }
    if (div_out)
        for (int a = 0; a < 3; ++a) div_out[a] = g->tile_div[a];
    if (ms_out) *ms_out = best;
    return BEC_OK;
}

}  // extern "C"

#include "static_apply.inc"
