// Field kernels of the PCG-ATKM hot path for gfx950.
//
// Line passes (one block = L lines of one axis staged in LDS, FFT'd in LDS, written back):
//   ATKM forward  z: rho -> pad 2Nz -> R2C (two real lines packed in one complex FFT)
//                 y: pad 2Ny -> C2C;  x: pad 2Nx -> C2C -> x S' -> inverse -> crop
//   ATKM inverse  y: inverse -> crop;  z: C2R (two real lines per complex FFT) -> crop
//   line operators: per axis, FFT -> x (nu^2/2 +- Omega coord nu) -> inverse (kinetic and
//                 rotation terms are sums of one-axis operators), fused H assembly on x
//   preconditioner: 3-D FFT with P_V^{1/2} scaling on the z passes, shift division on x
// Reductions are FP64 per block (wave shuffles + LDS), finished by a fixed-order tree.
#include "lines.h"
#include "impl.h"
#include "regfft.h"

namespace bec {

// ------------------------------------------------------------------ symbol helpers
struct SymArgs {
    const double* uhat;   // octant [nx+1][ny+1][nz+1]
    int nx, ny, nz;       // N grid (padded axes have 2N points)
    double px, py, pz;    // pi / (2 a): padded frequency step
    double nd[3];
    double scale;         // 1 / (8 N)
};

// S'_k = (3 (n.nu_k)^2 U_k - 1) / (8N) at padded frequency (kx, ky) in FFT order and kz in
// [0, Nz] (R2C half; kz = Nz is the Nyquist plane). Cross terms vanish on Nyquist planes.
__device__ __forceinline__ double sym_prime(const SymArgs& s, int kx, int ky, int kz) {
    const int sx = kx < s.nx ? kx : kx - 2 * s.nx;
    const int sy = ky < s.ny ? ky : ky - 2 * s.ny;
    const int sz = kz < s.nz ? kz : -s.nz;
    const bool qx = kx == s.nx, qy = ky == s.ny, qz = kz == s.nz;
    const double vx = sx * s.px, vy = sy * s.py, vz = sz * s.pz;
    double nn = s.nd[0] * s.nd[0] * vx * vx + s.nd[1] * s.nd[1] * vy * vy + s.nd[2] * s.nd[2] * vz * vz;
    if (!(qx || qy)) nn += 2.0 * s.nd[0] * s.nd[1] * vx * vy;
    if (!(qx || qz)) nn += 2.0 * s.nd[0] * s.nd[2] * vx * vz;
    if (!(qy || qz)) nn += 2.0 * s.nd[1] * s.nd[2] * vy * vz;
    const int ax = sx < 0 ? -sx : sx, ay = sy < 0 ? -sy : sy;
    const double u = s.uhat[((long)ax * (s.ny + 1) + ay) * (s.nz + 1) + kz];
    return (3.0 * nn * u - 1.0) * s.scale;
}

__device__ __forceinline__ int fft_signed(int k, int n) { return k < n / 2 ? k : k - n; }

template <typename R> __device__ __forceinline__ R rho_of(cpx<R> a) { return a.x * a.x + a.y * a.y; }

// ------------------------------------------------------------------ generic C2C line pass
template <typename R, int DIR>
__global__ __launch_bounds__(kThreads) void k_c2c(const cpx<R>* in, cpx<R>* out,
                                                  Geo g, FftPlan plan, const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem);
    const int n = plan.n, ldl = n + 1;
    const Tile ti = tile_of(g, blockIdx.x);
    load_tile(lds, ldl, g, ti, n, n, [&](long a, int, int) { return in[a]; });
    __syncthreads();
    lds_fft<DIR>(lds, plan, g.L, ldl);
    visit_tile(lds, ldl, g, ti, n, [&](long a, int, int, cpx<R> v) { out[a] = v; });
}

// ATKM y forward: lines of na_in points, zero-padded to plan.n, full spectrum out.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_pad_fwd(const cpx<R>* __restrict__ in, cpx<R>* __restrict__ out,
                                                      Geo g, FftPlan plan, int na_in, const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem);
    const int n = plan.n, ldl = n + 1;
    const Tile ti = tile_of(g, blockIdx.x);
    load_tile(lds, ldl, g, ti, na_in, n, [&](long a, int, int) { return in[a]; });
    __syncthreads();
    lds_fft<-1>(lds, plan, g.L, ldl);
    visit_tile(lds, ldl, g, ti, n, [&](long a, int, int, cpx<R> v) { out[a] = v; });
}

// ATKM y inverse: full lines of plan.n points, inverse, first na_out points out.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_inv_crop(const cpx<R>* __restrict__ in, cpx<R>* __restrict__ out,
                                                       Geo g, FftPlan plan, int na_out, const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem);
    const int n = plan.n, ldl = n + 1;
    const Tile ti = tile_of(g, blockIdx.x);
    load_tile(lds, ldl, g, ti, n, n, [&](long a, int, int) { return in[a]; });
    __syncthreads();
    lds_fft<+1>(lds, plan, g.L, ldl);
    visit_tile(lds, ldl, g, ti, na_out, [&](long a, int, int, cpx<R> v) { out[a] = v; });
}

// ATKM x pass, in place on the [Nx][2Ny][Nz+1] buffer: pad 2Nx, forward, x S', inverse, crop.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_atkm_x(cpx<R>* __restrict__ buf, Geo g, FftPlan plan, SymArgs s,
                                                     const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem);
    const int n = plan.n, ldl = n + 1, na = s.nx;
    const Tile ti = tile_of(g, blockIdx.x);
    load_tile(lds, ldl, g, ti, na, n, [&](long a, int, int) { return buf[a]; });
    __syncthreads();
    lds_fft<-1>(lds, plan, g.L, ldl);
    visit_lds(lds, ldl, g.L, n, [&](int l, int k, cpx<R>& v) {
        if (!line_ok(g, ti, l)) return;
        int ky, kz;
        line_coords(g, ti, l, ky, kz);
        v = (R)sym_prime(s, k, ky, kz) * v;
    });
    __syncthreads();
    lds_fft<+1>(lds, plan, g.L, ldl);
    visit_tile(lds, ldl, g, ti, na, [&](long a, int, int, cpx<R> v) { buf[a] = v; });
}

// ATKM x pass, forward only, Parseval sums against S' (h^3 applied by the caller):
//   single: q0 = sum S' w |Y1|^2;  dual: q0 = sum S' w |Y1|^2, q1 = sum S' w Re(Y1 conj Y2),
//   q2 = sum S' w |Y2|^2, with w = 1 on the kz = 0, Nz planes and 2 elsewhere (R2C half).
template <typename R, int DUAL>
__global__ __launch_bounds__(kThreads) void k_atkm_x_pars(const cpx<R>* __restrict__ b1, const cpx<R>* __restrict__ b2,
                                                          Geo g, FftPlan plan, SymArgs s, double* __restrict__ partials,
                                                          const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem);
    const int n = plan.n, ldl = n + 1, na = s.nx;
    const Tile ti = tile_of(g, blockIdx.x);
    load_tile(lds, ldl, g, ti, na, n, [&](long a, int, int) { return b1[a]; });
    if (DUAL) load_tile(lds + g.L * ldl, ldl, g, ti, na, n, [&](long a, int, int) { return b2[a]; });
    __syncthreads();
    lds_fft<-1>(lds, plan, DUAL ? 2 * g.L : g.L, ldl);
    constexpr int NQ = DUAL ? 3 : 1;
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    const int M = g.L * n;
    for (int e = threadIdx.x; e < M; e += kThreads) {
        const int l = e / n, k = e - l * n;
        if (!line_ok(g, ti, l)) continue;
        int ky, kz;
        line_coords(g, ti, l, ky, kz);
        const double w = sym_prime(s, k, ky, kz) * ((kz == 0 || kz == s.nz) ? 1.0 : 2.0);
        const cpx<R> a = lds[l * ldl + k];
        acc[0] += w * ((double)a.x * a.x + (double)a.y * a.y);
        if constexpr (DUAL != 0) {
            const cpx<R> b = lds[(g.L + l) * ldl + k];
            acc[1] += w * ((double)a.x * b.x + (double)a.y * b.y);
            acc[2] += w * ((double)b.x * b.x + (double)b.y * b.y);
        }
    }
    block_reduce<NQ, 0u>(acc, partials);
}

// ATKM z forward. Two real lines u, v are packed as u + i v, zero-padded to 2Nz and
// transformed once; U[k] = (Z[k] + conj Z[-k]) / 2, V[k] = (Z[k] - conj Z[-k]) / (2i), k <= Nz.
//  MODE 0: u, v = |phi|^2 of lines 2p, 2p+1 -> Z1 lines 2p, 2p+1.
//  MODE 1: u = Re(conj(phi) p), v = |p|^2 of line p -> Z1, Z2 line p.
template <typename R, int MODE>
__global__ __launch_bounds__(kThreads) void k_atkm_zf(const cpx<R>* __restrict__ phi, const cpx<R>* __restrict__ pp,
                                                      cpx<R>* __restrict__ z1, cpx<R>* __restrict__ z2,
                                                      int nlines_out, int nz, int L, FftPlan plan,
                                                      const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem);
    const int n = plan.n, ldl = n + 1;       // n = 2 nz
    const int p0 = blockIdx.x * L;
    // load
    if constexpr (MODE == 0) {
        const int M = L * 2 * nz;
        for (int e = threadIdx.x; e < M; e += kThreads) {
            const int l = e / (2 * nz), q = e - l * 2 * nz;
            if (p0 + l >= nlines_out) continue;
            const R r = rho_of(phi[(long)(2 * (p0 + l)) * nz + q]);
            R* dst = reinterpret_cast<R*>(&lds[l * ldl + (q < nz ? q : q - nz)]);
            dst[q < nz ? 0 : 1] = r;
        }
    } else {
        const int M = L * nz;
        for (int e = threadIdx.x; e < M; e += kThreads) {
            const int l = e / nz, j = e - l * nz;
            if (p0 + l >= nlines_out) continue;
            const long a = (long)(p0 + l) * nz + j;
            const cpx<R> f = phi[a], q = pp[a];
            lds[l * ldl + j] = mk<R>(f.x * q.x + f.y * q.y, rho_of(q));
        }
    }
    for (int e = threadIdx.x; e < L * nz; e += kThreads) {
        const int l = e / nz, j = nz + e - l * nz;
        lds[l * ldl + j] = mk<R>(0, 0);
    }
    __syncthreads();
    lds_fft<-1>(lds, plan, L, ldl);
    const int M = L * (nz + 1);
    for (int e = threadIdx.x; e < M; e += kThreads) {
        const int l = e / (nz + 1), k = e - l * (nz + 1);
        if (p0 + l >= nlines_out) continue;
        const cpx<R> U = lds[l * ldl + k];
        const cpx<R> V = conj(lds[l * ldl + (k == 0 ? 0 : n - k)]);
        const cpx<R> A = (R)0.5 * (U + V);
        const cpx<R> B = mul_i<-1>((R)0.5 * (U - V));
        if constexpr (MODE == 0) {
            z1[(long)(2 * (p0 + l)) * (nz + 1) + k] = A;
            z1[(long)(2 * (p0 + l) + 1) * (nz + 1) + k] = B;
        } else {
            z1[(long)(p0 + l) * (nz + 1) + k] = A;
            z2[(long)(p0 + l) * (nz + 1) + k] = B;
        }
    }
}

// ATKM z inverse (C2R) for pairs of lines 2p, 2p+1 of the [lines][Nz+1] half spectrum:
// full spectrum A~ + i B~ (Hermitian extension, imaginary parts of DC/Nyquist dropped),
// inverse of length 2Nz, real part -> line 2p, imaginary part -> line 2p+1, first Nz points.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_atkm_zi(const cpx<R>* __restrict__ zb, R* __restrict__ Phi,
                                                      int npairs, int nz, int L, FftPlan plan,
                                                      const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem);
    const int n = plan.n, ldl = n + 1;
    const int p0 = blockIdx.x * L;
    const int M = L * n;
    for (int e = threadIdx.x; e < M; e += kThreads) {
        const int l = e / n, k = e - l * n;
        if (p0 + l >= npairs) continue;
        const long ra = (long)(2 * (p0 + l)) * (nz + 1), rb = ra + (nz + 1);
        cpx<R> A, B;
        if (k <= nz) { A = zb[ra + k]; B = zb[rb + k]; }
        else { A = conj(zb[ra + n - k]); B = conj(zb[rb + n - k]); }
        if (k == 0 || k == nz) { A.y = 0; B.y = 0; }
        lds[l * ldl + k] = mk<R>(A.x - B.y, A.y + B.x);
    }
    __syncthreads();
    lds_fft<+1>(lds, plan, L, ldl);
    const int Mo = L * 2 * nz;
    for (int e = threadIdx.x; e < Mo; e += kThreads) {
        const int l = e / (2 * nz), q = e - l * 2 * nz;
        if (p0 + l >= npairs) continue;
        const cpx<R> v = lds[l * ldl + (q < nz ? q : q - nz)];
        Phi[(long)(2 * (p0 + l)) * nz + q] = q < nz ? v.x : v.y;
    }
}

// ------------------------------------------------------------------ line operators
struct LineOpArgs {
    int nx, ny, nz;
    double ax, ay, az, hx, hy;
    double nu_step;       // pi / a of this axis
    double omega;
    double gamma[3], beta, lam;
};

// Kinetic + rotation line operator along axis AX (FFT order k):
//   z: nu^2/2;  y: nu^2/2 - Omega x nu;  x: nu^2/2 + Omega y nu.
// MODE 0: acc = op(phi); 1: acc += op(phi); 2: H phi = acc + op(phi) + (V + beta rho + lambda Phi) phi
// with sums (kin, rot, V rho, rho^2, Phi rho, rho, Re(H phi conj phi));
// MODE 3: Parseval sums (kin, rot) only.
// The kin/rot sums are over sum_k m |phi_hat_k|^2 / n of each line (h^3 applied later).
template <typename R, int AX, int MODE>
__global__ __launch_bounds__(kThreads) void k_lineop(const cpx<R>* __restrict__ phi, cpx<R>* __restrict__ acc,
                                                     const R* __restrict__ Phi, cpx<R>* __restrict__ hphi,
                                                     Geo g, FftPlan plan, LineOpArgs o, double* __restrict__ partials,
                                                     const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem);
    const int n = plan.n, ldl = n + 1;
    const Tile ti = tile_of(g, blockIdx.x);
    load_tile(lds, ldl, g, ti, n, n, [&](long a, int, int) { return phi[a]; });
    __syncthreads();
    lds_fft<-1>(lds, plan, g.L, ldl);
    constexpr int NQ = MODE == 2 ? 7 : 2;
    double red[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) red[q] = 0.0;
    const double inv_n = 1.0 / n;
    visit_lds(lds, ldl, g.L, n, [&](int l, int k, cpx<R>& v) {
        if (!line_ok(g, ti, l)) return;
        int c0, c1;
        line_coords(g, ti, l, c0, c1);
        const double nu = fft_signed(k, n) * o.nu_step;
        const double kin = 0.5 * nu * nu;
        double rot = 0.0;
        if (AX == 1) rot = -o.omega * (-o.ax + c0 * o.hx) * nu;     // c0 = i0 (x index)
        if (AX == 0) rot = o.omega * (-o.ay + c0 * o.hy) * nu;      // c0 = i1 (y index)
        const double p2 = ((double)v.x * v.x + (double)v.y * v.y) * inv_n;
        red[0] += kin * p2;
        red[1] += rot * p2;
        if (MODE != 3) v = (R)((kin + rot) * inv_n) * v;
    });
    if constexpr (MODE != 3) {
        __syncthreads();
        lds_fft<+1>(lds, plan, g.L, ldl);
        if constexpr (MODE == 0) {
            visit_tile(lds, ldl, g, ti, n, [&](long a, int, int, cpx<R> v) { acc[a] = v; });
        } else if constexpr (MODE == 1) {
            visit_tile(lds, ldl, g, ti, n, [&](long a, int, int, cpx<R> v) { acc[a] = acc[a] + v; });
        } else if constexpr (MODE == 2) {
            visit_tile(lds, ldl, g, ti, n, [&](long a, int l, int j, cpx<R> v) {
                int i1, i2;
                line_coords(g, ti, l, i1, i2);
                const double x = -o.ax + j * o.hx, y = -o.ay + i1 * o.hy, z = -o.az + i2 * (2.0 * o.az / o.nz);
                const double V = 0.5 * (o.gamma[0] * o.gamma[0] * x * x + o.gamma[1] * o.gamma[1] * y * y +
                                        o.gamma[2] * o.gamma[2] * z * z);
                const cpx<R> f = phi[a];
                const double r = (double)f.x * f.x + (double)f.y * f.y;
                const double ph = Phi ? (double)Phi[a] : 0.0;
                const R pot = (R)(V + o.beta * r + o.lam * ph);
                const cpx<R> h = acc[a] + v + pot * f;
                hphi[a] = h;
                red[2] += V * r;
                red[3] += r * r;
                red[4] += ph * r;
                red[5] += r;
                red[6] += (double)h.x * f.x + (double)h.y * f.y;
            });
        }
    }
    block_reduce<NQ, 0u>(red, partials);
}

// ------------------------------------------------------------------ preconditioner
struct PrecArgs {
    int nx, ny, nz;
    double ax, ay, az, hx, hy, hz;
    double gamma[3], beta, lam;
    double nux, nuy, nuz;     // pi / a per axis
};

__device__ __forceinline__ double trap_at(const PrecArgs& p, int i, int j, int k) {
    const double x = -p.ax + i * p.hx, y = -p.ay + j * p.hy, z = -p.az + k * p.hz;
    return 0.5 * (p.gamma[0] * p.gamma[0] * x * x + p.gamma[1] * p.gamma[1] * y * y + p.gamma[2] * p.gamma[2] * z * z);
}

// sqrt(P_V) at grid point (i, j, k): P_V = 1 / (alpha + V + beta |phi|^2 + |lambda| max(Phi, 0)).
template <typename R>
__device__ __forceinline__ double sqrt_pv(const PrecArgs& p, double alpha, int i, int j, int k, cpx<R> f, R ph) {
    const double r = (double)f.x * f.x + (double)f.y * f.y;
    const double d = alpha + trap_at(p, i, j, k) + p.beta * r + fabs(p.lam) * fmax((double)ph, 0.0);
    return 1.0 / sqrt(d);
}

// z pass 1: r = H phi - mu phi (written to rbuf), s = sqrt(P_V) r, forward z FFT -> W.
// Reduction: ||r||_inf (max).
template <typename R>
__global__ __launch_bounds__(kThreads) void k_prec_z(const cpx<R>* __restrict__ hphi, const cpx<R>* __restrict__ phi,
                                                     const R* __restrict__ Phi, cpx<R>* __restrict__ rbuf,
                                                     cpx<R>* __restrict__ W, Geo g, FftPlan plan, PrecArgs pa,
                                                     const DevState* __restrict__ st, double* __restrict__ partials,
                                                     const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem);
    const int n = plan.n, ldl = n + 1;
    const Tile ti = tile_of(g, blockIdx.x);
    const double mu = st->mu, alpha = st->alpha;
    double red[1] = {0.0};
    load_tile(lds, ldl, g, ti, n, n, [&](long a, int l, int j) {
        const cpx<R> f = phi[a], h = hphi[a];
        const cpx<R> r = mk<R>((R)(h.x - mu * f.x), (R)(h.y - mu * f.y));
        rbuf[a] = r;
        red[0] = fmax(red[0], sqrt((double)r.x * r.x + (double)r.y * r.y));
        int i0, i1;
        line_coords(g, ti, l, i0, i1);
        return (R)sqrt_pv(pa, alpha, i0, i1, j, f, Phi ? Phi[a] : (R)0) * r;
    });
    __syncthreads();
    lds_fft<-1>(lds, plan, g.L, ldl);
    visit_tile(lds, ldl, g, ti, n, [&](long a, int, int, cpx<R> v) { W[a] = v; });
    block_reduce<1, 1u>(red, partials);
}

// x pass: forward, divide by (alpha + |nu|^2 / 2) N, inverse (in place on W).
template <typename R>
__global__ __launch_bounds__(kThreads) void k_prec_x(cpx<R>* __restrict__ W, Geo g, FftPlan plan, PrecArgs pa,
                                                     const DevState* __restrict__ st, const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem);
    const int n = plan.n, ldl = n + 1;
    const Tile ti = tile_of(g, blockIdx.x);
    const double alpha = st->alpha;
    const double invN = 1.0 / ((double)pa.nx * pa.ny * pa.nz);
    load_tile(lds, ldl, g, ti, n, n, [&](long a, int, int) { return W[a]; });
    __syncthreads();
    lds_fft<-1>(lds, plan, g.L, ldl);
    visit_lds(lds, ldl, g.L, n, [&](int l, int k, cpx<R>& v) {
        int ky, kz;
        line_coords(g, ti, l, ky, kz);
        const double vx = fft_signed(k, pa.nx) * pa.nux, vy = fft_signed(ky, pa.ny) * pa.nuy,
                     vz = fft_signed(kz, pa.nz) * pa.nuz;
        v = (R)(invN / (alpha + 0.5 * (vx * vx + vy * vy + vz * vz))) * v;
    });
    __syncthreads();
    lds_fft<+1>(lds, plan, g.L, ldl);
    visit_tile(lds, ldl, g, ti, n, [&](long a, int, int, cpx<R> v) { W[a] = v; });
}

// z pass 2: inverse z FFT of W, Pr = sqrt(P_V) (.)
template <typename R>
__global__ __launch_bounds__(kThreads) void k_prec_zi(const cpx<R>* __restrict__ W, const cpx<R>* __restrict__ phi,
                                                      const R* __restrict__ Phi, cpx<R>* __restrict__ Pr, Geo g,
                                                      FftPlan plan, PrecArgs pa, const DevState* __restrict__ st,
                                                      const int* __restrict__ done) {
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem);
    const int n = plan.n, ldl = n + 1;
    const Tile ti = tile_of(g, blockIdx.x);
    const double alpha = st->alpha;
    load_tile(lds, ldl, g, ti, n, n, [&](long a, int, int) { return W[a]; });
    __syncthreads();
    lds_fft<+1>(lds, plan, g.L, ldl);
    visit_tile(lds, ldl, g, ti, n, [&](long a, int l, int j, cpx<R> v) {
        int i0, i1;
        line_coords(g, ti, l, i0, i1);
        Pr[a] = (R)sqrt_pv(pa, alpha, i0, i1, j, phi[a], Phi ? Phi[a] : (R)0) * v;
    });
}

// ------------------------------------------------------------------ finalize + control
// Sums partials[nb][nq] over blocks in a fixed order; max for slots in maxmask.
__global__ __launch_bounds__(kThreads) void k_finalize(const double* __restrict__ partials, int nb, int nq,
                                                       unsigned maxmask, double* __restrict__ out,
                                                       const int* __restrict__ done) {
    if (done && *done) return;
    __shared__ double sh[kThreads];
    for (int q = 0; q < nq; ++q) {
        const bool mx = (maxmask >> q) & 1u;
        double x = 0.0;
        for (int b = threadIdx.x; b < nb; b += kThreads) {
            const double y = partials[(long)b * nq + q];
            x = mx ? fmax(x, y) : x + y;
        }
        sh[threadIdx.x] = x;
        __syncthreads();
        for (int s = kThreads / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) sh[threadIdx.x] = mx ? fmax(sh[threadIdx.x], sh[threadIdx.x + s]) : sh[threadIdx.x] + sh[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[q] = sh[0];
        __syncthreads();
    }
}

// Energy parts from the apply reductions (slot RS_APPLY):
//   [0..1] z (kin, rot), [2..3] y (kin, rot), [4..10] x (kin, rot, V rho, rho^2, Phi rho, rho, mu)
__global__ void k_apply_finish(DevState* st, const int* __restrict__ done) {
    if (done && *done) return;
    const double* r = st->red[RS_APPLY];
    const double h3 = st->h3;
    st->Ekin = h3 * (r[0] + r[2] + r[4]);
    st->Erot = h3 * (r[1] + r[3] + r[5]);
    st->Epot = h3 * r[6];
    st->Eint = 0.5 * st->beta * h3 * r[7];
    st->Edip = 0.5 * st->lam * h3 * r[8];
    st->mass = h3 * r[9];
    st->mu = h3 * r[10];
    st->E = st->Ekin + st->Epot + st->Eint + st->Edip + st->Erot;
}

// ------------------------------------------------------------------ symbol
// Per-axis tables T[m][k] = I(s_m; nu_k, b) = int_{-b}^{b} exp(-s^2 y^2) cos(nu y) dy,
// nu_k = pi k / (2a) for k = 0..N (octant of the padded axis), b = 2a; closed form when s b > 6.5,
// else Gauss-Legendre with the nodes/weights given for [-b, b].
__global__ void k_sym_tables(const double* __restrict__ s_nodes, int ms, int nk, double nu_step, double b,
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

// U[kx][ky][kz] = sum_m c_m Tx[m][kx] Ty[m][ky] Tz[m][kz] (compensated summation over m).
__global__ void k_sym_contract(const double* __restrict__ c, int ms, const double* __restrict__ Tx,
                               const double* __restrict__ Ty, const double* __restrict__ Tz, int nkx, int nky, int nkz,
                               double* __restrict__ U) {
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long tot = (long)nkx * nky * nkz;
    if (id >= tot) return;
    const int kz = (int)(id % nkz);
    const int ky = (int)((id / nkz) % nky);
    const int kx = (int)(id / ((long)nkz * nky));
    double acc = 0.0, comp = 0.0;
    for (int m = 0; m < ms; ++m) {
        const double t = c[m] * Tx[(long)m * nkx + kx] * Ty[(long)m * nky + ky] * Tz[(long)m * nkz + kz] - comp;
        const double u = acc + t;
        comp = (u - acc) - t;
        acc = u;
    }
    U[id] = acc;
}

// ------------------------------------------------------------------ misc pointwise
template <typename R>
__global__ void k_copy_state_scalar(const DevState* st, int which, double* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = which == 0 ? st->mu : st->E;
}

#include "pcg.inc"
#include "rfkern.inc"

}  // namespace bec

#include "launch.inc"
