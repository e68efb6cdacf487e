// Host-side grid context shared by the launch wrappers and the C ABI.
#pragma once
#include <string>
#include <vector>
#include "../../include/bec.h"
#include "common.h"
#include "kernels.h"

namespace bec {

// physical parameters of one solve (validated copy of bec_params, dipole axis normalised)
struct Params {
    double gamma[3], beta, lam, nd[3], omega;
};

// Device buffers of one precision, carved from the caller's workspace. Every field holds the
// whole batch: solve b starts at b * (its per-solve size).
template <typename R> struct Fields {
    cpx<R>* hphi = nullptr;   // H phi
    cpx<R>* acc = nullptr;    // line-operator accumulator
    cpx<R>* r0 = nullptr;     // residual (current / previous alternate)
    cpx<R>* r1 = nullptr;
    cpx<R>* pr = nullptr;     // preconditioned residual
    cpx<R>* p = nullptr;      // search direction
    cpx<R>* w = nullptr;      // 3-D FFT scratch (N grid)
    cpx<R>* phi = nullptr;    // iterate (FP32 phase / staging)
    cpx<R>* z1 = nullptr;     // [Nx][Ny][Nz+1]
    cpx<R>* z2 = nullptr;
    cpx<R>* y1 = nullptr;     // [Nx][2Ny][Nz+1]
    cpx<R>* y2 = nullptr;
    R* Phi = nullptr;         // dipolar potential (real)
    R* Phi_aux = nullptr;
    FftPlan pz, py, px, pzp, pyp, pxp;   // twiddle tables in this precision
};

constexpr int kBranchEvents = 8;   // fork/join events per iteration (distinct points)

struct Grid {
    int n[3];
    double a[3], h[3], h3;
    int precision;            // 0: FP64 only; 1: FP64 + FP32 fields
    int batch;                // number of same-grid solves held by the workspace
    hipStream_t stream;
    char* ws;
    size_t ws_bytes;
    Fields<double> f64;
    Fields<float> f32;
    double* uhat = nullptr;   // symbol octant in the working layout [Ny+1][Nz+1][Nx+1], shared by the batch
    bool have_symbol = false;
    DevState* st = nullptr;   // device scalar state, one per solve
    Params* dparams = nullptr;   // device copy of the per-solve parameters
    int* dstop = nullptr;     // host-set stop flags, one per solve
    double* partials = nullptr;
    long part_stride = 0;     // doubles of partial sums per solve
    double* sym_scratch = nullptr;
    size_t sym_scratch_bytes = 0;
    int poisoned = 0;
    int use_rf = 1;           // power-of-two register-FFT fast paths (0: generic LDS kernels)
    bool lam_any = false;     // some solve of the batch has lambda != 0
    // geometries
    Geo gz, gy, gx;           // N grid line passes (z: Nz, y: Ny, x: Nx)
    Geo g_ay, g_ax, g_ax2;    // padded passes (y forward/inverse, x, two-field x)
    int zf_L;                 // packed lines per block of the runtime-length z pair kernels
    int tile_div[3] = {1, 1, 1};   // per-axis divisor of the generic kernels' lines per block
    // when set, the next line pass (or two-density Parseval pass) is launched with these events
    // recording its own start and end (stage timing)
    hipEvent_t tev0 = nullptr, tev1 = nullptr;
    Bat bt64, bt32;           // per-solve strides of the FP64 / FP32 buffers
    // in-iteration profile: when kprof is set, every launch takes a pair of events from its pool
    // and is recorded under the launch site in `site` (see bec_pcg_profile)
    int site = 0;
    struct KProf* kprof = nullptr;
    // second stream and fork/join events of the solver (null outside bec_pcg_solve / profile):
    // passes that do not depend on each other run as parallel branches of the iteration
    hipStream_t aux = nullptr;
    hipEvent_t ev[kBranchEvents] = {};
    // the solve uses the paper's step rule ||phi_{n+1} - phi_n||_inf <= tol (FP64 iterations
    // compute the step's sums only then)
    bool step_rule = false;
    // launch-shape variant of the register kernels per launch site (0: default; see
    // bec_autotune_kernels); lengths without variants ignore it
    int variant[BEC_NSITES] = {};
};

// Event pool of an in-iteration profile: pairs are handed out in launch order and harvested
// (elapsed time per site) after the stream has drained.
struct KProf {
    std::vector<hipEvent_t> ev;   // 2 * capacity events
    std::vector<int> sites;       // site of each pair handed out
    bool take(int site, hipEvent_t& a, hipEvent_t& b) {
        const size_t k = sites.size();
        if (2 * k + 1 >= ev.size()) return false;   // pool exhausted: the launch goes untimed
        a = ev[2 * k];
        b = ev[2 * k + 1];
        sites.push_back(site);
        return true;
    }
};

template <typename R> inline Fields<R>& fields(Grid& g);
template <> inline Fields<double>& fields<double>(Grid& g) { return g.f64; }
template <> inline Fields<float>& fields<float>(Grid& g) { return g.f32; }
template <typename R> inline const Bat& bat(const Grid& g) { return sizeof(R) == 8 ? g.bt64 : g.bt32; }

// launch wrappers (kernels.hip). Parameters are read on the device from DevState[b].
template <typename R> void launch_fft3d(Grid& g, const cpx<R>* in, cpx<R>* out, int dir);
template <typename R> void launch_atkm(Grid& g, const cpx<R>* phi, R* Phi);
// P_ret: the FP64 iteration's direction, for the retraction fused into the first ATKM pass
template <typename R> void launch_apply(Grid& g, const cpx<R>* phi, cpx<R>* hphi, R* Phi, const cpx<R>* P_ret = nullptr);
void launch_symbol(Grid& g, std::vector<double>& tables_host_scratch);
void launch_symbol_out(Grid& g, double* out);   // octant layout [Nx+1][Ny+1][Nz+1]
void launch_set_params(Grid& g);   // copies g.dparams[b] into st[b] (already uploaded)

struct CtlOpts {
    double tol_res, tol_step, t_default, tau_ulps, dbg_t, dbg_c2;
    int max_iter, max_halv, dbg_flags, fp32;
    int tol_rel = 0;   // stop at ||r||_inf <= tol_res |mu| (the FP32 phase's switch)
};
template <typename R> void launch_pcg_iteration(Grid& g, cpx<R>* phi, int parity);
template <typename R> void launch_pcg_start(Grid& g, cpx<R>* phi);
void launch_ctl_init(Grid& g, const CtlOpts& o);
void launch_ctl_phase(Grid& g, double tol, int max_iter, double tau_ulps, double eps_E);
void launch_ctl_stop(Grid& g);
template <typename R> double time_stage(Grid& g, const cpx<R>* phi, int which, int reps);
void launch_to_f32(Grid& g, const cpx<double>* a, cpx<float>* b);
void launch_to_f64_normalized(Grid& g, const cpx<float>* a, cpx<double>* b);
// field utilities (gridops); `st` must be cleared (solves active) by the caller
void launch_interp(Grid& src, Grid& dst, const void* in, int in_fp32, void* out, int out_fp32);
void launch_normalize(Grid& g, cpx<double>* phi);
void launch_gauge(Grid& g, cpx<double>* phi);
void launch_rotate(Grid& g, const cpx<double>* in, cpx<double>* out, double alpha);
bool site_has_variants(const Grid& g, int site);   // launch-shape variants exist for this site
bool site_variant_distinct(const Grid& g, int site, int v);   // v launches kernels no u < v does

}  // namespace bec
