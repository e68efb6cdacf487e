// Host-side grid context shared by the launch wrappers and the C ABI.
#pragma once
#include <string>
#include <vector>
#include "common.h"
#include "kernels.h"

namespace bec {

struct Params {
    double gamma[3], beta, lam, nd[3], omega;
};

// Device buffers of one precision, carved from the caller's workspace.
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

struct Grid {
    int n[3];
    double a[3], h[3], h3;
    int precision;            // 0: FP64 only; 1: FP64 + FP32 fields
    hipStream_t stream;
    char* ws;
    size_t ws_bytes;
    size_t ws_used;
    Fields<double> f64;
    Fields<float> f32;
    double* uhat = nullptr;   // octant [Nx+1][Ny+1][Nz+1]
    bool have_symbol = false;
    DevState* st = nullptr;   // device scalar state
    int* done_flag = nullptr; // points into st (done)
    double* partials = nullptr;
    size_t partials_cap = 0;
    size_t partials_off = 0;
    double* sym_scratch = nullptr;
    size_t sym_scratch_bytes = 0;
    int poisoned = 0;
    int use_rf = 1;           // power-of-two register-FFT fast paths (0: generic LDS kernels)
    // geometries
    Geo gz, gy, gx;           // N grid line passes (z: Nz, y: Ny, x: Nx)
    Geo g_ay, g_ax, g_ax2, g_ayi;   // padded passes
    int zf_L, zf2_L, zi_L;
    hipGraphExec_t graph = nullptr;
    int graph_prec = -1;
};

// workspace layout
size_t workspace_bytes(const int n[3], int precision);
int carve(Grid& g);

// launch wrappers (kernels.hip)
template <typename R> void launch_fft3d(Grid& g, const cpx<R>* in, cpx<R>* out, int dir);
template <typename R> void launch_atkm(Grid& g, Fields<R>& f, const Params& p, const cpx<R>* phi, R* Phi, const int* done);
template <typename R> void launch_apply(Grid& g, Fields<R>& f, const Params& p, const cpx<R>* phi, cpx<R>* hphi,
                                        R* Phi, const int* done);
void launch_symbol(Grid& g, std::vector<double>& tables_host_scratch);
void launch_set_params(Grid& g, const Params& p);

struct CtlOpts {
    double tol_res, tol_step, t_default, tau_ulps, dbg_t, dbg_c2;
    int max_iter, max_halv, dbg_flags, fp32;
};
template <typename R> void launch_pcg_iteration(Grid& g, Fields<R>& f, const Params& p, cpx<R>* phi, int parity);
template <typename R> void launch_pcg_start(Grid& g, Fields<R>& f, const Params& p, cpx<R>* phi);
void launch_ctl_init(Grid& g, const CtlOpts& o);
void launch_ctl_phase(Grid& g, double tol, int max_iter);
template <typename R> double time_stage(Grid& g, Fields<R>& f, const Params& p, const cpx<R>* phi, int which, int reps);
void launch_to_f32(Grid& g, const cpx<double>* a, cpx<float>* b);
void launch_to_f64_normalized(Grid& g, const cpx<float>* a, cpx<double>* b);

}  // namespace bec
