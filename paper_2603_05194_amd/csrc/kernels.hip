// Field kernels of the PCG-ATKM hot path for gfx950.
//
// Line passes (a block holds L lines of one axis; FFT in registers or LDS; written back):
//   ATKM forward  z: rho -> pad 2Nz -> R2C (two real lines packed in one complex FFT)
//                 y: pad 2Ny -> C2C;  x: pad 2Nx -> C2C -> x S' -> inverse -> crop
//   ATKM inverse  y: inverse -> crop;  z: C2R (two real lines per complex FFT) -> crop
//   line operators: per axis, FFT -> x (nu^2/2 +- Omega coord nu) -> inverse (kinetic and
//                 rotation terms are sums of one-axis operators), fused H assembly on x
//   preconditioner: 3-D FFT with P_V^{1/2} scaling on the z passes, shift division on x
// Every kernel serves a batch of same-grid solves: blockIdx.y is the solve; per-solve
// parameters and flags live in DevState[b]. Reductions are FP64 per block (wave shuffles +
// LDS), finished by a fixed-order tree, so results are deterministic.
#include "lines.h"
#include "impl.h"
#include "regfft.h"

namespace bec {

// ------------------------------------------------------------------ geometry helpers
struct SymArgs {
    const double* uhat;   // octant values in the working layout [ny+1][nz+1][nx+1]
    int nx, ny, nz;       // N grid (padded axes have 2N points)
    double px, py, pz;    // pi / (2 a): padded frequency step
    double scale;         // 1 / (8 N)
};

// S'_k = (3 (n.nu_k)^2 U_k - 1) / (8N) at padded frequency (kx, ky) in FFT order and kz in
// [0, Nz] (R2C half; kz = Nz is the Nyquist plane). Cross terms vanish on Nyquist planes.
__device__ __forceinline__ double sym_prime(const SymArgs& s, const double* nd, int kx, int ky, int kz) {
    const int sx = kx < s.nx ? kx : kx - 2 * s.nx;
    const int sy = ky < s.ny ? ky : ky - 2 * s.ny;
    const int sz = kz < s.nz ? kz : -s.nz;
    const bool qx = kx == s.nx, qy = ky == s.ny, qz = kz == s.nz;
    const double vx = sx * s.px, vy = sy * s.py, vz = sz * s.pz;
    double nn = nd[0] * nd[0] * vx * vx + nd[1] * nd[1] * vy * vy + nd[2] * nd[2] * vz * vz;
    if (!(qx || qy)) nn += 2.0 * nd[0] * nd[1] * vx * vy;
    if (!(qx || qz)) nn += 2.0 * nd[0] * nd[2] * vx * vz;
    if (!(qy || qz)) nn += 2.0 * nd[1] * nd[2] * vy * vz;
    const int ax = sx < 0 ? -sx : sx, ay = sy < 0 ? -sy : sy;
    const double u = s.uhat[((long)ay * (s.nz + 1) + kz) * (s.nx + 1) + ax];
    return (3.0 * nn * u - 1.0) * s.scale;
}

// S'_k along one padded x line (fixed ky, kz), with the line constants hoisted:
//   (n.nu)^2 = a sx^2 + b sx + c  (b = 0 on the kx Nyquist plane), sx the signed kx index,
// and the contiguous symbol row U[|sy|][kz][.]. Equal to sym_prime up to rounding order.
struct SymLine {
    const double* row;
    double a, b, c, scale;
    int nx;
};

__device__ __forceinline__ SymLine sym_line(const SymArgs& s, const double* nd, int ky, int kz) {
    const int sy = ky < s.ny ? ky : ky - 2 * s.ny;
    const int sz = kz < s.nz ? kz : -s.nz;
    const bool qy = ky == s.ny, qz = kz == s.nz;
    const double vy = sy * s.py, vz = sz * s.pz;
    SymLine L;
    L.a = nd[0] * nd[0] * s.px * s.px;
    L.b = 2.0 * nd[0] * s.px * ((qy ? 0.0 : nd[1] * vy) + (qz ? 0.0 : nd[2] * vz));
    L.c = nd[1] * nd[1] * vy * vy + nd[2] * nd[2] * vz * vz + ((qy || qz) ? 0.0 : 2.0 * nd[1] * nd[2] * vy * vz);
    const int ay = sy < 0 ? -sy : sy;
    L.row = s.uhat + ((long)ay * (s.nz + 1) + kz) * (s.nx + 1);
    L.scale = s.scale;
    L.nx = s.nx;
    return L;
}

__device__ __forceinline__ double sym_eval(const SymLine& L, int kx) {
    const int sx = kx < L.nx ? kx : kx - 2 * L.nx;
    const double v = (double)sx;
    const double nn = (L.a * v + (kx == L.nx ? 0.0 : L.b)) * v + L.c;
    const double u = L.row[sx < 0 ? -sx : sx];
    return (3.0 * nn * u - 1.0) * L.scale;
}

__device__ __forceinline__ int fft_signed(int k, int n) { return k < n / 2 ? k : k - n; }

template <typename R> __device__ __forceinline__ R rho_of(cpx<R> a) { return a.x * a.x + a.y * a.y; }

struct LineOpArgs {
    int nx, ny, nz;
    double ax, ay, az, hx, hy, hz;
    double nu_step;       // pi / a of this axis
};

struct PrecArgs {
    int nx, ny, nz;
    double ax, ay, az, hx, hy, hz;
    double nux, nuy, nuz;     // pi / a per axis
};

__device__ __forceinline__ double trap_at(const PrecArgs& p, const double* g2, int i, int j, int k) {
    const double x = -p.ax + i * p.hx, y = -p.ay + j * p.hy, z = -p.az + k * p.hz;
    return 0.5 * (g2[0] * x * x + g2[1] * y * y + g2[2] * z * z);
}

// Launch shape of the register line kernels. Variant V (chosen per launch site, see
// bec_autotune_kernels); bits 0 and 1 keep the L lines per block, hence the tiles and partial-sum rows:
//  bit 0: half the points per thread in blocks of twice the threads (power-of-two lengths with
//         at least 16 points per thread);
//  bit 1: whole complex values through LDS even where the split exchange would be used.
//  bit 2: twice the lines per block in blocks of twice the threads (lengths 256 and 512; the
//         LDS tile of 1024 would not fit): 256-byte column segments in FP64, half the tiles.
template <typename R, int N> constexpr bool rf_wide_ok() { return odd_part(N) == 1 && N >= 256 && N <= 512; }
template <typename R, int N, int V = 0> struct RFK {
    static constexpr int E0 = rf_points<R>(N);
    static constexpr bool HALF = (V & 1) != 0 && odd_part(N) == 1 && E0 >= 16;
    static constexpr bool WIDE = (V & 4) != 0 && rf_wide_ok<R, N>();
    static constexpr int E = HALF ? E0 / 2 : E0;
    static constexpr int NT = kThreads * (E0 / E) * (WIDE ? 2 : 1);
    using T = RF<R, N, E, NT, (V & 2) != 0>;
    static constexpr int L = T::L;
    static_assert(T::lds_line_bytes <= 160 * 1024, "line tile beyond the LDS of a CU");
};

// The variant that V amounts to for length N (bits that change nothing are cleared).
template <typename R, int N> constexpr int rf_variant(int v) {
    const int e0 = rf_points<R>(N);
    const bool half_ok = odd_part(N) == 1 && e0 >= 16;
    const bool split_default = RF<R, N, e0>::SPLIT || RF<R, N, e0 / (half_ok ? 2 : 1), half_ok ? 2 * kThreads : kThreads>::SPLIT;
    return (half_ok ? (v & 1) : 0) | (split_default ? (v & 2) : 0) | (rf_wide_ok<R, N>() ? (v & 4) : 0);
}

// Two-density Parseval pass: both spectra live in registers. For power-of-two lengths with at
// least 16 points per thread it takes half of them in blocks of twice the threads: the same L
// lines per block (128-byte column segments, the same tiles and partial rows as RFK) with
// registers low enough for four waves per SIMD.
template <typename R, int N> struct RFK2 {
    static constexpr int E1 = rf_points<R>(N);
    static constexpr int E = (odd_part(N) > 1 || E1 < 16) ? E1 : E1 / 2;
    static constexpr int NT = kThreads * (E1 / E);
    using T = RF<R, N, E, NT, true>;   // whole complex values through LDS
    static constexpr int L = T::L;
    static_assert(L == RFK<R, N>::L, "same tiles as the line kernels");
};

#include "ops.inc"
#include "special.inc"

// ------------------------------------------------------------------ finalize + apply energies
// One block per solve: sums partials[b][nb][nq] over blocks in a fixed order (max for slots in
// maxmask) into st[b].red[row][q0 + q].
BEC_SHARED __global__ __launch_bounds__(kThreads) void k_finalize(const double* __restrict__ partials, long part_stride, int nb,
                                                       int nq, unsigned maxmask, DevState* __restrict__ st, int row,
                                                       int q0) {
    const int b = blockIdx.x;
    if (st[b].done) return;
    partials += b * part_stride;
    __shared__ double sh[kThreads];
    for (int q = 0; q < nq; ++q) {
        const bool mx = (maxmask >> q) & 1u;
        double x = 0.0;
        for (int i = threadIdx.x; i < nb; i += kThreads) {
            const double y = partials[(long)i * nq + q];
            x = mx ? fmax(x, y) : x + y;
        }
        sh[threadIdx.x] = x;
        __syncthreads();
        for (int s = kThreads / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) sh[threadIdx.x] = mx ? fmax(sh[threadIdx.x], sh[threadIdx.x + s]) : sh[threadIdx.x] + sh[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) st[b].red[row][q0 + q] = sh[0];
        __syncthreads();
    }
}

// Energy parts from the apply reductions (row RS_APPLY):
//   [0..1] z (kin, rot), [2..3] y (kin, rot), [4..10] x (kin, rot, V rho, rho^2, Phi rho, rho, mu)
__device__ void apply_finish(DevState& S) {
    if (S.done) return;
    const double* r = S.red[RS_APPLY];
    const double h3 = S.h3;
    S.Ekin = h3 * (r[0] + r[2] + r[4]);
    S.Erot = h3 * (r[1] + r[3] + r[5]);
    S.Epot = h3 * r[6];
    S.Eint = 0.5 * S.beta * h3 * r[7];
    S.Edip = 0.5 * S.lam * h3 * r[8];
    S.mass = h3 * r[9];
    S.mu = h3 * r[10];
    S.E = S.Ekin + S.Epot + S.Eint + S.Edip + S.Erot;
    // what the next iteration of Algorithm 1 needs from these parts: the shift alpha
    // (alpha_Lap = alpha_V, without the rotation term) and the energy-test slack
    S.alpha = S.Ekin + S.Epot + 2.0 * S.Eint + fabs(2.0 * S.Edip);
    S.tau_E = S.tau_ulps * S.eps_E * (fabs(S.Ekin) + fabs(S.Epot) + fabs(S.Eint) + fabs(S.Edip) + fabs(S.Erot));
}

BEC_SHARED __global__ void k_apply_finish(DevState* st, int nbatch) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbatch) return;
    apply_finish(st[b]);
}

// ------------------------------------------------------------------ symbol
// Per-axis tables T[m][k] = I(s_m; nu_k, b) = int_{-b}^{b} exp(-s^2 y^2) cos(nu y) dy,
// nu_k = pi k / (2a) for k = 0..N (octant of the padded axis), b = 2a; closed form when s b > 6.5,
// else Gauss-Legendre with the nodes/weights given for [-b, b].
BEC_SHARED __global__ void k_sym_tables(const double* __restrict__ s_nodes, int ms, int nk, double nu_step, double b,
                             const double* __restrict__ gy, const double* __restrict__ gw, int nq,
                             double* __restrict__ T) {
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long)ms * nk) return;
    const int m = (int)(id / nk), k = (int)(id - (long)m * nk);
    const double s = s_nodes[m];
    const double nu = k * nu_step;
    double val;
    if (s * b > 6.5) {
        val = 1.7724538509055160272981674833411452 / s * exp(-nu * nu / (4.0 * s * s));
    } else {
        double acc = 0.0, comp = 0.0;
        for (int q = 0; q < nq; ++q) {
            const double y = gy[q];
            const double t = gw[q] * exp(-s * s * y * y) * cos(nu * y) - comp;
            const double u = acc + t;
            comp = (u - acc) - t;
            acc = u;
        }
        val = acc;
    }
    T[(long)m * nk + k] = val;
}

// U = sum_m c_m Tx[m][kx] Ty[m][ky] Tz[m][kz] (compensated summation over m), stored in the
// working layout [ky][kz][kx] (kx fastest): the x passes then read, for each of their columns
// (ky, kz), one contiguous row over kx.
BEC_SHARED __global__ void k_sym_contract(const double* __restrict__ c, int ms, const double* __restrict__ Tx,
                               const double* __restrict__ Ty, const double* __restrict__ Tz, int nkx, int nky, int nkz,
                               double* __restrict__ U) {
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long tot = (long)nkx * nky * nkz;
    if (id >= tot) return;
    const int kx = (int)(id % nkx);
    const int kz = (int)((id / nkx) % nkz);
    const int ky = (int)(id / ((long)nkx * nkz));
    double acc = 0.0, comp = 0.0;
    for (int m = 0; m < ms; ++m) {
        const double t = c[m] * Tx[(long)m * nkx + kx] * Ty[(long)m * nky + ky] * Tz[(long)m * nkz + kz] - comp;
        const double u = acc + t;
        comp = (u - acc) - t;
        acc = u;
    }
    U[id] = acc;
}

// working layout [ky][kz][kx] -> octant layout [kx][ky][kz] (the documented output)
BEC_SHARED __global__ void k_sym_to_octant(const double* __restrict__ U, int nkx, int nky, int nkz, double* __restrict__ out) {
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long tot = (long)nkx * nky * nkz;
    if (id >= tot) return;
    const int kz = (int)(id % nkz);
    const int ky = (int)((id / nkz) % nky);
    const int kx = (int)(id / ((long)nkz * nky));
    out[id] = U[((long)ky * nkz + kz) * nkx + kx];
}

#include "pcg.inc"

// ------------------------------------------------------------------ fused finalize + control
// One block per solve (or per segment and solve, see gridDim.y). Each segment holds nb per-block
// partial rows of nq slots at offset `off`
// of the solve's partial region; every thread sums its rows in order, waves reduce by shuffles,
// the four wave results are combined in a fixed order into st[b].red[row][q0 + q]. Then one
// thread runs the control step that consumes the sums (CTL), replacing separate finalize and
// control launches.
template <int CTL>
__global__ __launch_bounds__(kThreads) void k_fin(const double* __restrict__ partials, long part_stride, FinList L,
                                                  DevState* __restrict__ st) {
    const int b = blockIdx.x;
    if (st[b].done) return;
    __shared__ double sh[kThreads / 64][kFinQ];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // gridDim.y > 1: the segments are shared out over the blocks of a solve (CTL is then FC_NONE)
    for (int si = blockIdx.y; si < L.n; si += gridDim.y) {
        const FinSeg sg = L.s[si];
        const double* p = partials + b * part_stride + sg.off;
        double acc[kFinQ];
#pragma unroll
        for (int q = 0; q < kFinQ; ++q) acc[q] = 0.0;
        // four rows per thread per round, all loads issued before any is used
        constexpr int U = 4;
        for (int i0 = threadIdx.x; i0 < sg.nb; i0 += U * kThreads) {
            double y[U][kFinQ];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * kThreads;
#pragma unroll
                for (int q = 0; q < kFinQ; ++q) y[u][q] = (q < sg.nq && i < sg.nb) ? p[(long)i * sg.nq + q] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int q = 0; q < kFinQ; ++q)
                    if (q < sg.nq) acc[q] = ((sg.maxmask >> q) & 1u) ? fmax(acc[q], y[u][q]) : acc[q] + y[u][q];
            }
        }
#pragma unroll
        for (int q = 0; q < kFinQ; ++q) {
            if (q < sg.nq) {
                const bool mx = (sg.maxmask >> q) & 1u;
                double x = acc[q];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    const double y = __shfl_xor(x, off, 64);
                    x = mx ? fmax(x, y) : x + y;
                }
                if (lane == 0) sh[wave][q] = x;
            }
        }
        __syncthreads();
        if (threadIdx.x < sg.nq) {
            const int q = threadIdx.x;
            const bool mx = (sg.maxmask >> q) & 1u;
            double x = sh[0][q];
            for (int w = 1; w < kThreads / 64; ++w) x = mx ? fmax(x, sh[w][q]) : x + sh[w][q];
            st[b].red[sg.row][sg.q0 + q] = x;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        DevState& S = st[b];
        if constexpr (CTL == FC_RES) ctl_res(S);
        else if constexpr (CTL == FC_DIR) { ctl_res(S); ctl_dir(S); }
        else if constexpr (CTL == FC_STEP) ctl_step(S);
        else if constexpr (CTL == FC_POST) ctl_post(S);
        else if constexpr (CTL == FC_APPLY) apply_finish(S);
    }
}
#include "gridops.inc"

}  // namespace bec

#include "launch.inc"
