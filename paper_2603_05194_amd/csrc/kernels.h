// Kernel argument structs and host-side launch wrappers (implemented in kernels.hip).
#pragma once
#include "common.h"

// kernels.hip is compiled twice so that the two halves build in parallel: once for the FP64
// instantiations and everything shared, once (kernels_f32.hip, BEC_UNIT_F32) for the FP32
// instantiations alone. In the FP32 unit the non-template kernels get internal linkage
// (BEC_SHARED) and the non-template host functions are left out.
#ifdef BEC_UNIT_F32
#define BEC_SHARED static
#else
#define BEC_SHARED
#endif

namespace bec {

// Geometry of one line pass: lines run along `axis` of a C-order 3-D array.
//  axis 2: a line is `outer` in [0, n_outer) (= i0*d1 + i1), element j at outer*na + j.
//  axis 0/1: a line is (outer, inner); element j at outer*na*n_inner + j*n_inner + inner.
//   axis 1: outer = i0, inner = i2; axis 0: outer = 0, inner = i1*d2 + i2.
struct Geo {
    int axis;
    int n_outer, n_inner;
    int L;            // lines per block
    int tpo;          // tiles per outer (axes 0/1)
    int ntiles;
    int dA, dB;       // axis 2: dA = d1 (to split outer); axis 0: dB = d2 (to split inner)
    long row;         // axes 0/1: elements between consecutive points of a line
    // axis 0 over a half-spectrum buffer [Nx][nky][ld] (hs = 1): tiles of L columns ky at the
    // Nyquist kz = nzq, then tiles of L columns kz < nzq at one ky (cpk per ky, nreg in all).
    // axis 1 over [Nx][ny][ld] (hs = 1): the same with rows x in place of columns ky (nky = Nx).
    int hs, nky, nzq, ld, cpk, nreg;
};

// Scalars shared between field kernels and the single-thread control kernels (FP64 always).
struct DevState {
    // physical parameters and grid constants
    double gamma[3], beta, lam, nd[3], omega;
    double h3;
    // energy parts of the current iterate
    double Ekin, Epot, Eint, Edip, Erot, E, mu, mass;
    double res_inf, step_inf, alpha;
    // preconditioned CG memory and step coefficients
    double den_prev;
    double cPr, cPhi, cP;          // p <- cPr * Pr + cPhi * phi + cP * p
    double cRet, sRet;             // phi <- cRet * phi + sRet * p
    double t, c2, d1, beta_cg, pnorm;
    double tau_E, eps_E;
    // options
    double tol_res, tol_step, t_default, tau_ulps;
    int tol_rel;                   // 1: tol_res is relative to |mu|
    double dbg_t, dbg_c2;
    int max_iter, max_halv, dbg_flags;
    // counters and flags
    int iter, halvings, resets, forced, restart, done, status, accepted_last;
    int fp32_iters;
    // reduction landing area (filled by finalize kernels)
    double red[4][kMaxRed];
};

enum RedSlot { RS_APPLY = 0, RS_PREC = 1, RS_DIR = 2, RS_AUX = 3 };

// Partial-sum segments finished by one k_fin launch (offsets in doubles within a solve's region)
constexpr int kFinQ = 10;     // slots per segment at most
constexpr int kFinSeg = 6;    // segments per launch at most
struct FinSeg {
    long off;
    int nb, nq;
    unsigned maxmask;
    int row, q0;
};
struct FinList {
    int n;
    FinSeg s[kFinSeg];
};
enum FinCtl { FC_NONE = 0, FC_RES = 1, FC_DIR = 2, FC_STEP = 3, FC_POST = 4, FC_APPLY = 5 };

// Element strides between the solves of a batch (blockIdx.y selects the solve): complex N-grid
// fields, real N-grid fields, the [Nx][Ny][Nz+1] and [Nx][2Ny][Nz+1] padded buffers, and the
// per-solve partial-sum region.
struct Bat {
    long n, z, y, part;
};

template <typename R> struct Tables {
    FftPlan plan_z, plan_y, plan_x;          // N-grid lengths
    FftPlan plan_zp, plan_yp, plan_xp;       // padded lengths 2N
};

struct GridConst {
    int nx, ny, nz;
    double ax, ay, az;
    double hx, hy, hz, h3;
};

}  // namespace bec
