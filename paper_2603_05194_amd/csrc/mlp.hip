// Learned initial guess: dense tanh network, BF16 matrix-core GEMMs (gfx950 MFMA 32x32x16),
// FP32 accumulation, Adam on FP32 master weights. Every buffer is caller-owned.
//
// All GEMMs run in one "NT" form, C[m][n] = sum_k A[m][k] B[n][k], with both operands
// K-contiguous BF16. The forward pass needs no transposes (weights are stored [out][in]);
// the backward pass keeps transposed BF16 copies of the activations, output gradients and of
// W2, W3, written by the kernels that produce them, so every product streams contiguous K.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <algorithm>
#include <cmath>
#include <string>

#include "bec.h"
#include "bec_mlp.h"

namespace bec_mlp_impl {

constexpr int kT = 256;  // threads per block
constexpr int GBM = 128, GBN = 128, GBK = 64, GPAD = 8;
constexpr int kSK = GBK / 8;                // threads per staged row (8 BF16 each)
constexpr int kSR = kT / kSK;               // rows staged per pass
constexpr int kSP = GBM / kSR;              // passes per operand tile
constexpr int kMaxGroups = 64;     // row groups of the batch reductions

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// FP32 -> BF16, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ------------------------------------------------------------------ GEMM (matrix cores)
// 8 BF16 of row min(r, rows - 1) at column kc (an in-range address for any r).
__device__ __forceinline__ uint4 ld_row(const uint16_t* __restrict__ p, int ld, int r, int rows, int kc) {
    return *(const uint4*)(p + (size_t)min(r, rows - 1) * ld + kc);
}

// Block tile 128 x 128, K step 32; four waves in a 2 x 2 layout, each owning a 64 x 64 sub-tile
// of 2 x 2 MFMA 32x32 accumulators. MFMA 32x32x16 bf16 operand layout: lane l supplies row
// (l mod 32) of A (resp. column of B) and k = 8 (l div 32) + 0..7; accumulator register r of
// lane l holds C[8 (r div 4) + 4 (l div 32) + (r mod 4)][l mod 32].
// blockIdx.z selects a K slice [z kper, (z+1) kper); its result goes to C + z * zstride.
__global__ __launch_bounds__(kT) void k_gemm_nt(int M, int N, int K, int kper, const uint16_t* __restrict__ A, int lda,
                                                const uint16_t* __restrict__ B, int ldb, float* __restrict__ C, int ldc,
                                                long zstride, const float* __restrict__ bias) {
    __shared__ __attribute__((aligned(16))) uint16_t As[GBM][GBK + GPAD];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[GBN][GBK + GPAD];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
    const int kb = blockIdx.z * kper;
    const int ke = min(K, kb + kper);
    const int wm = (w >> 1) * 64, wn = (w & 1) * 64;
    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    // Thread tid stages rows tid/kSK + p kSR (p < kSP) of each operand tile at k offset
    // 8 (tid mod kSK); the next K step is loaded into registers while this one is multiplied.
    // Out-of-range rows and k are loaded from a clamped in-range address and zeroed by a mask
    // when written to LDS, so every load is unconditional and the stage stays in registers.
    const int srow = tid / kSK, sk = (tid % kSK) * 8;
    uint4 ra[kSP], rb[kSP];
    auto gload = [&](int k0) {
        const int kc = min(k0 + sk, ke - 8);
#pragma unroll
        for (int p = 0; p < kSP; ++p) {
            ra[p] = ld_row(A, lda, m0 + p * kSR + srow, M, kc);
            rb[p] = ld_row(B, ldb, n0 + p * kSR + srow, N, kc);
        }
    };
    if (kb < ke) gload(kb);
    for (int k0 = kb; k0 < ke; k0 += GBK) {
        __syncthreads();
        const bool kok = k0 + sk < ke;
#pragma unroll
        for (int p = 0; p < kSP; ++p) {
            const uint32_t ma = (kok && m0 + p * kSR + srow < M) ? 0xffffffffu : 0u;
            const uint32_t mb = (kok && n0 + p * kSR + srow < N) ? 0xffffffffu : 0u;
            *(uint4*)&As[p * kSR + srow][sk] = make_uint4(ra[p].x & ma, ra[p].y & ma, ra[p].z & ma, ra[p].w & ma);
            *(uint4*)&Bs[p * kSR + srow][sk] = make_uint4(rb[p].x & mb, rb[p].y & mb, rb[p].z & mb, rb[p].w & mb);
        }
        __syncthreads();
        if (k0 + GBK < ke) gload(k0 + GBK);
#pragma unroll
        for (int kk = 0; kk < GBK; kk += 16) {
            bf16x8 a[2], b[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                a[t] = __builtin_bit_cast(bf16x8, *(const uint4*)&As[wm + t * 32 + (lane & 31)][kk + 8 * (lane >> 5)]);
                b[t] = __builtin_bit_cast(bf16x8, *(const uint4*)&Bs[wn + t * 32 + (lane & 31)][kk + 8 * (lane >> 5)]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
    C += blockIdx.z * zstride;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn + j * 32 + (lane & 31);
            if (n >= N) continue;
            const float bv = bias ? bias[n] : 0.0f;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = m0 + wm + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (m < M) C[(size_t)m * ldc + n] = acc[i][j][r] + bv;
            }
        }
}

// C[m][n] = sum_z part[z][m][n] + bias[n]. A block covers 64 consecutive elements; its four
// waves sum consecutive quarters of the z range, which are then added in order (deterministic).
__global__ __launch_bounds__(kT) void k_split_sum(const float* __restrict__ part, int S, int M, int N,
                                                  float* __restrict__ C, int ldc, const float* __restrict__ bias) {
    __shared__ float q[4][64];
    const long MN = (long)M * N;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int zq = (S + 3) / 4, z0 = w * zq, z1 = min(S, z0 + zq);
    for (long base = (long)blockIdx.x * 64; base < MN; base += (long)gridDim.x * 64) {
        const long i = base + lane;
        float s = 0.0f;
        if (i < MN)
            for (int z = z0; z < z1; ++z) s += part[z * MN + i];
        q[w][lane] = s;
        __syncthreads();
        if (w == 0 && i < MN) {
            const float v = ((q[0][lane] + q[1][lane]) + q[2][lane]) + q[3][lane];
            const int n = (int)(i % N), m = (int)(i / N);
            C[(size_t)m * ldc + n] = v + (bias ? bias[n] : 0.0f);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ elementwise kernels
// dst[c][r] = src[r][c] for r < R, zero for R <= r < Rp (c < Cn); 64 x 64 tiles through LDS.
// blockIdx.x runs along the longer of the two dimensions (rows if x_rows), so that blocks in
// flight together read and write neighbouring addresses rather than one column of rows a large
// power of two apart.
__global__ __launch_bounds__(kT) void k_transpose_bf16(const uint16_t* __restrict__ src, int R, int Cn, int lds_,
                                                       uint16_t* __restrict__ dst, int Rp, int ldd, int x_rows) {
    __shared__ uint16_t t[64][65];
    const int r0 = (x_rows ? blockIdx.x : blockIdx.y) * 64, c0 = (x_rows ? blockIdx.y : blockIdx.x) * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += kT) {
        const int r = e >> 6, c = e & 63;
        const int gr = r0 + r, gc = c0 + c;
        t[r][c] = (gr < R && gc < Cn) ? src[(size_t)gr * lds_ + gc] : (uint16_t)0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += kT) {
        const int c = e >> 6, r = e & 63;
        const int gr = r0 + r, gc = c0 + c;
        if (gc < Cn && gr < Rp) dst[(size_t)gc * ldd + gr] = t[r][c];
    }
}

// p -> BF16 copy
__global__ __launch_bounds__(kT) void k_to_bf16(const float* __restrict__ p, uint16_t* __restrict__ q, long n) {
    for (long i = (long)blockIdx.x * kT + threadIdx.x; i < n; i += (long)gridDim.x * kT) q[i] = f2bf(p[i]);
}

// Layer 1 (d_in inputs, FP32): t = tanh(W1 x + b1) with BF16 W1; writes t and its BF16 copy.
__global__ __launch_bounds__(kT) void k_layer1(int batch, int din, int dh, const float* __restrict__ x,
                                               const int32_t* __restrict__ idx, const uint16_t* __restrict__ w1b,
                                               const float* __restrict__ b1, float* __restrict__ t,
                                               uint16_t* __restrict__ hb) {
    const long tot = (long)batch * dh;
    for (long e = (long)blockIdx.x * kT + threadIdx.x; e < tot; e += (long)gridDim.x * kT) {
        const int o = (int)(e % dh), b = (int)(e / dh);
        const long row = idx ? idx[b] : b;
        float s = 0.0f;
        for (int i = 0; i < din; ++i) s += bf2f(w1b[(size_t)o * din + i]) * x[row * din + i];
        const float v = tanhf(s + b1[o]);
        t[e] = v;
        hb[e] = f2bf(v);
    }
}

// t = tanh(t) in place (t already holds W h + b); BF16 copy to hb.
__global__ __launch_bounds__(kT) void k_tanh(float* __restrict__ t, uint16_t* __restrict__ hb, long n) {
    for (long i = (long)blockIdx.x * kT + threadIdx.x; i < n; i += (long)gridDim.x * kT) {
        const float v = tanhf(t[i]);
        t[i] = v;
        hb[i] = f2bf(v);
    }
}

// Column reductions over the batch are done in two passes: a grid of (column chunk, row group)
// blocks, one thread per column summing its rows in order into part[group][column] (FP64), then
// k_col_finish adding the groups in order. Both passes are deterministic.

// Block sum of one double per thread (fixed tree); the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[kT / 64];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kT / 64; ++i) r += red[i];
    return r;
}

// Output layer, rows [g rpg, (g+1) rpg) of column o: dY = s (y - target[idx[b]]) as BF16,
// colpart[g][o] = sum_b (y - target) and per-block sums of (y - target)^2 into sqpart.
__global__ __launch_bounds__(kT) void k_out_grad(int batch, int dout, int rpg, const float* __restrict__ y,
                                                 const float* __restrict__ tg, const int32_t* __restrict__ idx, float s,
                                                 uint16_t* __restrict__ dyb, double* __restrict__ colpart,
                                                 double* __restrict__ sqpart) {
    const int o = blockIdx.x * kT + threadIdx.x, g = blockIdx.y;
    const int b0 = g * rpg, b1 = min(batch, b0 + rpg);
    double sq = 0.0;
    if (o < dout) {
        double cs = 0.0;
#pragma unroll 4
        for (int b = b0; b < b1; ++b) {
            const long row = idx ? idx[b] : b;
            const float d = y[(size_t)b * dout + o] - tg[row * dout + o];
            cs += (double)d;
            sq += (double)d * d;
            dyb[(size_t)b * dout + o] = f2bf(s * d);
        }
        colpart[(size_t)g * dout + o] = cs;
    }
    const double t = block_sum(sq);
    if (threadIdx.x == 0) sqpart[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
}

// Hidden layer 2, rows [g rpg, (g+1) rpg) of column o: d = g (1 - t^2) in place, BF16 copy to db,
// colpart[g][o] = sum_b d.
__global__ __launch_bounds__(kT) void k_dtanh_cols(int batch, int n, int rpg, float* __restrict__ gr,
                                                   const float* __restrict__ t, uint16_t* __restrict__ db,
                                                   double* __restrict__ colpart) {
    const int o = blockIdx.x * kT + threadIdx.x, g = blockIdx.y;
    if (o >= n) return;
    const int b0 = g * rpg, b1 = min(batch, b0 + rpg);
    double cs = 0.0;
#pragma unroll 4
    for (int b = b0; b < b1; ++b) {
        const size_t e = (size_t)b * n + o;
        const float tv = t[e];
        const float v = gr[e] * (1.0f - tv * tv);
        gr[e] = v;
        db[e] = f2bf(v);
        cs += (double)v;
    }
    colpart[(size_t)g * n + o] = cs;
}

// Hidden layer 1, rows [g rpg, (g+1) rpg) of unit o: d1 = g (1 - t^2) (FP32),
// colpart[g][o] = sum_b d1 and wpart[g][o][i] = sum_b d1 x[idx[b]][i], inputs in chunks of 8.
__global__ __launch_bounds__(kT) void k_d1_cols(int batch, int din, int dh, int rpg, const float* __restrict__ gr,
                                                const float* __restrict__ t, const float* __restrict__ x,
                                                const int32_t* __restrict__ idx, double* __restrict__ colpart,
                                                double* __restrict__ wpart) {
    const int o = blockIdx.x * kT + threadIdx.x, g = blockIdx.y;
    if (o >= dh) return;
    const int b0 = g * rpg, b1 = min(batch, b0 + rpg);
    double cs = 0.0;
    for (int c0 = 0; c0 < din; c0 += 8) {
        double acc[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = 0.0;
        for (int b = b0; b < b1; ++b) {
            const size_t e = (size_t)b * dh + o;
            const float tv = t[e];
            const float v = gr[e] * (1.0f - tv * tv);
            if (c0 == 0) cs += (double)v;
            const float* xr = x + (size_t)(idx ? idx[b] : b) * din + c0;
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (c0 + j < din) acc[j] += (double)v * xr[j];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (c0 + j < din) wpart[((size_t)g * dh + o) * din + c0 + j] = acc[j];
    }
    colpart[(size_t)g * dh + o] = cs;
}

// out[o] = scale * sum_g part[g][o]. A block covers 64 columns; its four waves sum consecutive
// quarters of the groups, which are then added in order (deterministic).
__global__ __launch_bounds__(kT) void k_col_finish(int n, int groups, const double* __restrict__ part, double scale,
                                                   float* __restrict__ out) {
    __shared__ double q[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int o = blockIdx.x * 64 + lane;
    const int gq = (groups + 3) / 4, g0 = w * gq, g1 = min(groups, g0 + gq);
    double v = 0.0;
    if (o < n)
#pragma unroll 4
        for (int g = g0; g < g1; ++g) v += part[(size_t)g * n + o];
    q[w][lane] = v;
    __syncthreads();
    if (w == 0 && o < n) out[o] = (float)(scale * (((q[0][lane] + q[1][lane]) + q[2][lane]) + q[3][lane]));
}

// *out = scale * sum_i part[i]: one block, strided per-thread sums then a fixed tree.
__global__ __launch_bounds__(kT) void k_loss_final(const double* __restrict__ part, int n, double scale,
                                                   double* __restrict__ out) {
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += kT) v += part[i];
    const double t = block_sum(v);
    if (threadIdx.x == 0) *out = t * scale;
}

// Adam (FP32). Every coefficient comes from the host, rounded once from FP64:
// b1, 1-b1, b2, 1-b2, c1 = 1/(1-b1^t), c2 = 1/(1-b2^t).
__global__ __launch_bounds__(kT) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                             float* __restrict__ v, uint16_t* __restrict__ pb, long n, float lr, float b1,
                                             float omb1, float b2, float omb2, float eps, float c1, float c2) {
    for (long i = (long)blockIdx.x * kT + threadIdx.x; i < n; i += (long)gridDim.x * kT) {
        const float gi = g[i];
        const float mi = b1 * m[i] + omb1 * gi;
        const float vi = b2 * v[i] + omb2 * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
        p[i] = pi;
        pb[i] = f2bf(pi);
    }
}

// ------------------------------------------------------------------ host side
thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int grid1(long n) {
    long b = (n + kT * 4 - 1) / (kT * 4);
    if (b > 4096) b = 4096;
    return (int)(b < 1 ? 1 : b);
}

// Upper bound of row_groups(B, cols), non-decreasing in B: scratch is sized by it.
int group_cap(int B, int cols) {
    const int cb = (cols + kT - 1) / kT;
    return std::min(B, std::min(kMaxGroups, (1024 + cb - 1) / cb));
}

// Row groups for a batch reduction over `cols` columns: about 1024 blocks in all, at most
// kMaxGroups groups and none empty. *rpg receives the rows per group.
int row_groups(int B, int cols, int* rpg) {
    const int G = group_cap(B, cols);
    const int r = (B + G - 1) / G;
    *rpg = r;
    return (B + r - 1) / r;
}

struct Offs {
    size_t w1, b1, w2, b2, w3, b3, total;
};

Offs offsets(int din, int dh, int dout) {
    Offs o;
    o.w1 = 0;
    o.b1 = o.w1 + (size_t)dh * din;
    o.w2 = o.b1 + dh;
    o.b2 = o.w2 + (size_t)dh * dh;
    o.w3 = o.b2 + dh;
    o.b3 = o.w3 + (size_t)dout * dh;
    o.total = o.b3 + dout;
    return o;
}

// K split of an M x N x K product: enough blocks to fill the chip (>= 512), K slices of at
// least 256 (a multiple of the K step).
int plan_splits(int M, int N, int K, int* kper) {
    const long tiles = (long)((M + GBM - 1) / GBM) * ((N + GBN - 1) / GBN);
    int S = (int)((512 + tiles - 1) / tiles);
    const int smax = (K + 255) / 256;
    if (S > smax) S = smax;
    if (S < 1) S = 1;
    int kp = (K + S - 1) / S;
    kp = (kp + GBK - 1) / GBK * GBK;
    S = (K + kp - 1) / kp;
    if (S < 1) S = 1;
    *kper = kp;
    return S;
}

void gemm(hipStream_t s, int M, int N, int K, const uint16_t* A, int lda, const uint16_t* B, int ldb, float* C, int ldc,
          const float* bias, int S, int kper, float* part) {
    dim3 grid((N + GBN - 1) / GBN, (M + GBM - 1) / GBM, S);
    if (S == 1) {
        hipLaunchKernelGGL(k_gemm_nt, grid, dim3(kT), 0, s, M, N, K, kper, A, lda, B, ldb, C, ldc, 0L, bias);
    } else {
        hipLaunchKernelGGL(k_gemm_nt, grid, dim3(kT), 0, s, M, N, K, kper, A, lda, B, ldb, part, N, (long)M * N,
                           (const float*)nullptr);
        const long blocks = std::min(((long)M * N + 63) / 64, 65536L);
        hipLaunchKernelGGL(k_split_sum, dim3((unsigned)blocks), dim3(kT), 0, s, (const float*)part, S, M, N, C, ldc, bias);
    }
}

void gemm_auto(hipStream_t s, int M, int N, int K, const uint16_t* A, int lda, const uint16_t* B, int ldb, float* C,
               int ldc, const float* bias, float* part) {
    int kper = 0;
    const int S = plan_splits(M, N, K, &kper);
    gemm(s, M, N, K, A, lda, B, ldb, C, ldc, bias, S, kper, part);
}

size_t part_elems(int M, int N, int K) {
    int kper = 0;
    const int S = plan_splits(M, N, K, &kper);
    return S > 1 ? (size_t)S * M * N : 0;
}

int check_net(const bec_mlp* n) {
    if (!n) return fail(BEC_EINVAL, "network descriptor is NULL");
    if (n->d_in < 1 || n->d_h < 8 || n->d_out < 8 || n->d_h % 8 || n->d_out % 8)
        return fail(BEC_EINVAL, "d_in must be >= 1 and d_h, d_out positive multiples of 8");
    if (!n->params || !n->params_bf16 || !n->w2t_bf16 || !n->w3t_bf16)
        return fail(BEC_EINVAL, "NULL parameter buffer");
    return BEC_OK;
}

size_t al(size_t x) { return (x + 255) / 256 * 256; }

struct Scratch {
    float *t1, *t2, *z, *y, *part, *d2;
    uint16_t *h1b, *h1bT, *h2b, *h2bT, *dyb, *dybT, *d2b, *d2bT;
    double *colp, *wp, *lossp;
    size_t bytes;
};

Scratch carve(const bec_mlp* n, int B, char* base) {
    const int dh = n->d_h, D = n->d_out, Bp = (B + 7) / 8 * 8;
    size_t off = 0;
    Scratch s;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += al(bytes);
        return p;
    };
    s.t1 = (float*)take(sizeof(float) * B * dh);
    s.t2 = (float*)take(sizeof(float) * B * dh);
    s.z = (float*)take(sizeof(float) * B * dh);
    s.d2 = (float*)take(sizeof(float) * B * dh);
    s.y = (float*)take(sizeof(float) * (size_t)B * D);
    size_t pe = part_elems(B, dh, dh);
    pe = std::max(pe, part_elems(B, D, dh));
    pe = std::max(pe, part_elems(D, dh, Bp));
    pe = std::max(pe, part_elems(B, dh, D));
    pe = std::max(pe, part_elems(dh, dh, Bp));
    s.part = (float*)take(sizeof(float) * pe);
    s.h1b = (uint16_t*)take(2 * (size_t)B * dh);
    s.h1bT = (uint16_t*)take(2 * (size_t)dh * Bp);
    s.h2b = (uint16_t*)take(2 * (size_t)B * dh);
    s.h2bT = (uint16_t*)take(2 * (size_t)dh * Bp);
    s.dyb = (uint16_t*)take(2 * (size_t)B * D);
    s.dybT = (uint16_t*)take(2 * (size_t)D * Bp);
    s.d2b = (uint16_t*)take(2 * (size_t)B * dh);
    s.d2bT = (uint16_t*)take(2 * (size_t)dh * Bp);
    const int Gd = group_cap(B, D), Gh = group_cap(B, dh);
    s.colp = (double*)take(sizeof(double) * std::max((size_t)Gd * D, (size_t)Gh * dh));
    s.wp = (double*)take(sizeof(double) * (size_t)Gh * dh * n->d_in);
    s.lossp = (double*)take(sizeof(double) * (size_t)Gd * ((D + kT - 1) / kT));
    s.bytes = off;
    return s;
}

void transpose(hipStream_t st, const uint16_t* src, int R, int Cn, int lds_, uint16_t* dst, int Rp, int ldd) {
    const int cb = (Cn + 63) / 64, rb = (Rp + 63) / 64, x_rows = rb > cb;
    dim3 grid(x_rows ? rb : cb, x_rows ? cb : rb);
    hipLaunchKernelGGL(k_transpose_bf16, grid, dim3(kT), 0, st, src, R, Cn, lds_, dst, Rp, ldd, x_rows);
}

void refresh_transposes(const bec_mlp* n, hipStream_t st) {
    const Offs o = offsets(n->d_in, n->d_h, n->d_out);
    transpose(st, n->params_bf16 + o.w2, n->d_h, n->d_h, n->d_h, n->w2t_bf16, n->d_h, n->d_h);
    transpose(st, n->params_bf16 + o.w3, n->d_out, n->d_h, n->d_h, n->w3t_bf16, n->d_out, n->d_out);
}

// Forward pass into scratch: t1/h1b, t2/h2b, y (FP32, bias included).
void forward(const bec_mlp* n, int B, const float* x, const int32_t* idx, float* y, const Scratch& s, hipStream_t st) {
    const Offs o = offsets(n->d_in, n->d_h, n->d_out);
    const int dh = n->d_h, D = n->d_out;
    hipLaunchKernelGGL(k_layer1, dim3(grid1((long)B * dh)), dim3(kT), 0, st, B, n->d_in, dh, x, idx,
                       (const uint16_t*)(n->params_bf16 + o.w1), (const float*)(n->params + o.b1), s.t1, s.h1b);
    gemm_auto(st, B, dh, dh, s.h1b, dh, n->params_bf16 + o.w2, dh, s.t2, dh, n->params + o.b2, s.part);
    hipLaunchKernelGGL(k_tanh, dim3(grid1((long)B * dh)), dim3(kT), 0, st, s.t2, s.h2b, (long)B * dh);
    gemm_auto(st, B, D, dh, s.h2b, dh, n->params_bf16 + o.w3, dh, y, D, n->params + o.b3, s.part);
}

int launch_status(const char* where) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(BEC_EHIP, std::string(where) + ": " + hipGetErrorString(e));
    return BEC_OK;
}

}  // namespace bec_mlp_impl

using namespace bec_mlp_impl;

extern "C" {

const char* bec_mlp_last_error(void) { return g_err.c_str(); }

size_t bec_mlp_param_count(int d_in, int d_h, int d_out) {
    if (d_in < 1 || d_h < 1 || d_out < 1) return 0;
    return offsets(d_in, d_h, d_out).total;
}

int bec_mlp_scratch_bytes(const bec_mlp* net, int batch, size_t* bytes) {
    int rc = check_net(net);
    if (rc) return rc;
    if (batch < 1 || !bytes) return fail(BEC_EINVAL, "batch must be >= 1 and bytes non-NULL");
    *bytes = carve(net, batch, nullptr).bytes;
    return BEC_OK;
}

int bec_mlp_sync(const bec_mlp* net, void* stream) {
    int rc = check_net(net);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const long P = (long)offsets(net->d_in, net->d_h, net->d_out).total;
    hipLaunchKernelGGL(k_to_bf16, dim3(grid1(P)), dim3(kT), 0, st, (const float*)net->params, net->params_bf16, P);
    refresh_transposes(net, st);
    return launch_status("mlp sync");
}

int bec_mlp_forward(const bec_mlp* net, int batch, const float* d_x, const int32_t* d_idx, float* d_y, void* d_scratch,
                    size_t scratch_bytes, void* stream) {
    int rc = check_net(net);
    if (rc) return rc;
    if (batch < 1) return fail(BEC_EINVAL, "batch must be >= 1");
    if (!d_x || !d_y || !d_scratch) return fail(BEC_EINVAL, "NULL pointer");
    Scratch s = carve(net, batch, (char*)d_scratch);
    if (scratch_bytes < s.bytes) return fail(BEC_ENOMEM, "scratch buffer too small");
    forward(net, batch, d_x, d_idx, d_y, s, (hipStream_t)stream);
    return launch_status("mlp forward");
}

int bec_mlp_loss_grad(const bec_mlp* net, int batch, const float* d_x, const float* d_target, const int32_t* d_idx,
                      float* d_y, double* d_loss, void* d_scratch, size_t scratch_bytes, void* stream) {
    int rc = check_net(net);
    if (rc) return rc;
    if (batch < 1) return fail(BEC_EINVAL, "batch must be >= 1");
    if (!d_x || !d_target || !d_loss || !d_scratch || !net->grads) return fail(BEC_EINVAL, "NULL pointer");
    Scratch s = carve(net, batch, (char*)d_scratch);
    if (scratch_bytes < s.bytes) return fail(BEC_ENOMEM, "scratch buffer too small");
    hipStream_t st = (hipStream_t)stream;
    const Offs o = offsets(net->d_in, net->d_h, net->d_out);
    const int B = batch, Bp = (B + 7) / 8 * 8, dh = net->d_h, D = net->d_out, din = net->d_in;
    float* y = d_y ? d_y : s.y;
    float* g = net->grads;
    forward(net, B, d_x, d_idx, y, s, st);
    const float sc = (float)(2.0 / ((double)B * D));
    // output layer: dY (BF16), loss, bias gradient, weight gradient gW3 = dY^T h2
    int rd = 0, rh = 0;
    const int Gd = row_groups(B, D, &rd), Gh = row_groups(B, dh, &rh);
    const int cbd = (D + kT - 1) / kT, cbh = (dh + kT - 1) / kT;
    hipLaunchKernelGGL(k_out_grad, dim3(cbd, Gd), dim3(kT), 0, st, B, D, rd, (const float*)y, d_target, d_idx, sc, s.dyb,
                       s.colp, s.lossp);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kT), 0, st, (const double*)s.lossp, cbd * Gd, 1.0 / ((double)B * D),
                       d_loss);
    hipLaunchKernelGGL(k_col_finish, dim3((D + 63) / 64), dim3(kT), 0, st, D, Gd, (const double*)s.colp, (double)sc, g + o.b3);
    transpose(st, s.dyb, B, D, D, s.dybT, Bp, Bp);
    transpose(st, s.h2b, B, dh, dh, s.h2bT, Bp, Bp);
    transpose(st, s.h1b, B, dh, dh, s.h1bT, Bp, Bp);
    gemm_auto(st, D, dh, Bp, s.dybT, Bp, s.h2bT, Bp, g + o.w3, dh, nullptr, s.part);
    // hidden layer 2: dH2 = dY W3, dA2 = dH2 (1 - t2^2)
    gemm_auto(st, B, dh, D, s.dyb, D, net->w3t_bf16, D, s.z, dh, nullptr, s.part);
    hipLaunchKernelGGL(k_dtanh_cols, dim3(cbh, Gh), dim3(kT), 0, st, B, dh, rh, s.z, (const float*)s.t2, s.d2b, s.colp);
    hipLaunchKernelGGL(k_col_finish, dim3((dh + 63) / 64), dim3(kT), 0, st, dh, Gh, (const double*)s.colp, 1.0, g + o.b2);
    transpose(st, s.d2b, B, dh, dh, s.d2bT, Bp, Bp);
    gemm_auto(st, dh, dh, Bp, s.d2bT, Bp, s.h1bT, Bp, g + o.w2, dh, nullptr, s.part);
    // hidden layer 1: dH1 = dA2 W2, dA1 = dH1 (1 - t1^2) (FP32), gW1 = dA1^T x
    gemm_auto(st, B, dh, dh, s.d2b, dh, net->w2t_bf16, dh, s.d2, dh, nullptr, s.part);
    hipLaunchKernelGGL(k_d1_cols, dim3(cbh, Gh), dim3(kT), 0, st, B, din, dh, rh, (const float*)s.d2, (const float*)s.t1,
                       d_x, d_idx, s.colp, s.wp);
    hipLaunchKernelGGL(k_col_finish, dim3((dh + 63) / 64), dim3(kT), 0, st, dh, Gh, (const double*)s.colp, 1.0, g + o.b1);
    hipLaunchKernelGGL(k_col_finish, dim3((dh * din + 63) / 64), dim3(kT), 0, st, dh * din, Gh, (const double*)s.wp, 1.0,
                       g + o.w1);
    return launch_status("mlp loss_grad");
}

int bec_mlp_adam_step(const bec_mlp* net, double lr, double beta1, double beta2, double eps, int32_t t, void* stream) {
    int rc = check_net(net);
    if (rc) return rc;
    if (!net->grads || !net->adam_m || !net->adam_v) return fail(BEC_EINVAL, "NULL gradient or moment buffer");
    if (t < 1 || !(lr >= 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
        return fail(BEC_EINVAL, "bad Adam hyper-parameters");
    hipStream_t st = (hipStream_t)stream;
    const long P = (long)offsets(net->d_in, net->d_h, net->d_out).total;
    const double c1 = 1.0 / (1.0 - std::pow(beta1, (double)t)), c2 = 1.0 / (1.0 - std::pow(beta2, (double)t));
    hipLaunchKernelGGL(k_adam, dim3(grid1(P)), dim3(kT), 0, st, net->params, (const float*)net->grads, net->adam_m,
                       net->adam_v, net->params_bf16, P, (float)lr, (float)beta1, (float)(1.0 - beta1), (float)beta2,
                       (float)(1.0 - beta2), (float)eps, (float)c1, (float)c2);
    refresh_transposes(net, st);
    return launch_status("mlp adam");
}

int bec_gemm_bf16_nt(int M, int N, int K, const uint16_t* A, int lda, const uint16_t* B, int ldb, float* C, int ldc,
                     const float* bias, int splits, float* part, void* stream) {
    if (M < 1 || N < 1 || K < 8 || K % 8 || lda < K || ldb < K || ldc < N || lda % 8 || ldb % 8)
        return fail(BEC_EINVAL, "bad GEMM dimensions (K, lda, ldb must be multiples of 8)");
    if (!A || !B || !C) return fail(BEC_EINVAL, "NULL matrix pointer");
    if (((uintptr_t)A | (uintptr_t)B) & 15) return fail(BEC_EINVAL, "A and B must be 16-byte aligned");
    if (splits < 1) return fail(BEC_EINVAL, "splits must be >= 1");
    int kper = (K + splits - 1) / splits;
    kper = (kper + GBK - 1) / GBK * GBK;
    const int S = (K + kper - 1) / kper;
    if (S > 1 && !part) return fail(BEC_EINVAL, "splits > 1 needs a partial-sum buffer");
    gemm((hipStream_t)stream, M, N, K, A, lda, B, ldb, C, ldc, bias, S, kper, part);
    return launch_status("gemm");
}

}  // extern "C"
