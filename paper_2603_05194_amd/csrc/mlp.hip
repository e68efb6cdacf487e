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
constexpr int GBM = 128, GBN = 128, GBK = 32, GPAD = 8;
constexpr int kLossBlocks = 1024;

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

    uint4 ra[2], rb[2];
    auto gload = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int c = tid + kT * i;
            const int row = c >> 2, k = k0 + (c & 3) * 8;
            const uint4 z = make_uint4(0u, 0u, 0u, 0u);
            ra[i] = (m0 + row < M && k < ke) ? *(const uint4*)(A + (size_t)(m0 + row) * lda + k) : z;
            rb[i] = (n0 + row < N && k < ke) ? *(const uint4*)(B + (size_t)(n0 + row) * ldb + k) : z;
        }
    };
    if (kb < ke) gload(kb);
    for (int k0 = kb; k0 < ke; k0 += GBK) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int c = tid + kT * i;
            const int row = c >> 2, kc = (c & 3) * 8;
            *(uint4*)&As[row][kc] = ra[i];
            *(uint4*)&Bs[row][kc] = rb[i];
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

// C[m][n] = sum_z part[z][m][n] (fixed order) + bias[n]
__global__ __launch_bounds__(kT) void k_split_sum(const float* __restrict__ part, int S, int M, int N,
                                                  float* __restrict__ C, int ldc, const float* __restrict__ bias) {
    const long MN = (long)M * N;
    for (long i = (long)blockIdx.x * kT + threadIdx.x; i < MN; i += (long)gridDim.x * kT) {
        float s = 0.0f;
        for (int z = 0; z < S; ++z) s += part[z * MN + i];
        const int n = (int)(i % N), m = (int)(i / N);
        C[(size_t)m * ldc + n] = s + (bias ? bias[n] : 0.0f);
    }
}

// ------------------------------------------------------------------ elementwise kernels
// dst[c][r] = src[r][c] for r < R, zero for R <= r < Rp (c < Cn); 64 x 64 tiles through LDS.
__global__ __launch_bounds__(kT) void k_transpose_bf16(const uint16_t* __restrict__ src, int R, int Cn, int lds_,
                                                       uint16_t* __restrict__ dst, int Rp, int ldd) {
    __shared__ uint16_t t[64][65];
    const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
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

// d = g * (1 - t^2) (tanh derivative), in place on g; BF16 copy to db (nullable).
__global__ __launch_bounds__(kT) void k_dtanh(float* __restrict__ g, const float* __restrict__ t, uint16_t* __restrict__ db,
                                              long n) {
    for (long i = (long)blockIdx.x * kT + threadIdx.x; i < n; i += (long)gridDim.x * kT) {
        const float v = g[i] * (1.0f - t[i] * t[i]);
        g[i] = v;
        if (db) db[i] = f2bf(v);
    }
}

// dY = s (y - target[idx[b]]) as BF16; per-block FP64 sums of (y - target)^2.
__global__ __launch_bounds__(kT) void k_mse(int batch, int dout, const float* __restrict__ y, const float* __restrict__ tg,
                                            const int32_t* __restrict__ idx, float s, uint16_t* __restrict__ dyb,
                                            double* __restrict__ part) {
    const long tot = (long)batch * dout;
    double acc = 0.0;
    for (long e = (long)blockIdx.x * kT + threadIdx.x; e < tot; e += (long)gridDim.x * kT) {
        const int o = (int)(e % dout), b = (int)(e / dout);
        const long row = idx ? idx[b] : b;
        const float d = y[e] - tg[row * dout + o];
        acc += (double)d * d;
        dyb[e] = f2bf(s * d);
    }
    __shared__ double red[kT / 64];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int i = 0; i < kT / 64; ++i) v += red[i];
        part[blockIdx.x] = v;
    }
}

__global__ void k_loss_final(const double* __restrict__ part, int n, double scale, double* __restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double v = 0.0;
        for (int i = 0; i < n; ++i) v += part[i];
        *out = v * scale;
    }
}

// gb[o] = s * sum_b (y[b][o] - target[idx[b]][o])  (bias gradient of the output layer)
__global__ __launch_bounds__(kT) void k_colsum_out(int batch, int dout, const float* __restrict__ y,
                                                   const float* __restrict__ tg, const int32_t* __restrict__ idx, float s,
                                                   float* __restrict__ gb) {
    const int o = blockIdx.x * kT + threadIdx.x;
    if (o >= dout) return;
    double acc = 0.0;
    for (int b = 0; b < batch; ++b) {
        const long row = idx ? idx[b] : b;
        acc += (double)(y[(size_t)b * dout + o] - tg[row * dout + o]);
    }
    gb[o] = (float)(s * acc);
}

// gb[o] = sum_b d[b][o]
__global__ __launch_bounds__(kT) void k_colsum(int batch, int n, const float* __restrict__ d, float* __restrict__ gb) {
    const int o = blockIdx.x * kT + threadIdx.x;
    if (o >= n) return;
    double acc = 0.0;
    for (int b = 0; b < batch; ++b) acc += d[(size_t)b * n + o];
    gb[o] = (float)acc;
}

// gW1[o][i] = sum_b d1[b][o] x[idx[b]][i]
__global__ __launch_bounds__(kT) void k_gw1(int batch, int din, int dh, const float* __restrict__ d1,
                                            const float* __restrict__ x, const int32_t* __restrict__ idx,
                                            float* __restrict__ gw) {
    const int e = blockIdx.x * kT + threadIdx.x;
    if (e >= dh * din) return;
    const int o = e / din, i = e % din;
    double acc = 0.0;
    for (int b = 0; b < batch; ++b) {
        const long row = idx ? idx[b] : b;
        acc += (double)d1[(size_t)b * dh + o] * x[row * din + i];
    }
    gw[e] = (float)acc;
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
        hipLaunchKernelGGL(k_split_sum, dim3(grid1((long)M * N)), dim3(kT), 0, s, (const float*)part, S, M, N, C, ldc, bias);
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
    double* lossp;
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
    s.lossp = (double*)take(sizeof(double) * kLossBlocks);
    s.bytes = off;
    return s;
}

void transpose(hipStream_t st, const uint16_t* src, int R, int Cn, int lds_, uint16_t* dst, int Rp, int ldd) {
    dim3 grid((Cn + 63) / 64, (Rp + 63) / 64);
    hipLaunchKernelGGL(k_transpose_bf16, grid, dim3(kT), 0, st, src, R, Cn, lds_, dst, Rp, ldd);
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
    hipLaunchKernelGGL(k_mse, dim3(kLossBlocks), dim3(kT), 0, st, B, D, (const float*)y, d_target, d_idx, sc, s.dyb, s.lossp);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, st, (const double*)s.lossp, kLossBlocks, 1.0 / ((double)B * D),
                       d_loss);
    hipLaunchKernelGGL(k_colsum_out, dim3((D + kT - 1) / kT), dim3(kT), 0, st, B, D, (const float*)y, d_target, d_idx, sc,
                       g + o.b3);
    transpose(st, s.dyb, B, D, D, s.dybT, Bp, Bp);
    transpose(st, s.h2b, B, dh, dh, s.h2bT, Bp, Bp);
    transpose(st, s.h1b, B, dh, dh, s.h1bT, Bp, Bp);
    gemm_auto(st, D, dh, Bp, s.dybT, Bp, s.h2bT, Bp, g + o.w3, dh, nullptr, s.part);
    // hidden layer 2: dH2 = dY W3, dA2 = dH2 (1 - t2^2)
    gemm_auto(st, B, dh, D, s.dyb, D, net->w3t_bf16, D, s.z, dh, nullptr, s.part);
    hipLaunchKernelGGL(k_dtanh, dim3(grid1((long)B * dh)), dim3(kT), 0, st, s.z, (const float*)s.t2, s.d2b, (long)B * dh);
    hipLaunchKernelGGL(k_colsum, dim3((dh + kT - 1) / kT), dim3(kT), 0, st, B, dh, (const float*)s.z, g + o.b2);
    transpose(st, s.d2b, B, dh, dh, s.d2bT, Bp, Bp);
    gemm_auto(st, dh, dh, Bp, s.d2bT, Bp, s.h1bT, Bp, g + o.w2, dh, nullptr, s.part);
    // hidden layer 1: dH1 = dA2 W2, dA1 = dH1 (1 - t1^2) (FP32), gW1 = dA1^T x
    gemm_auto(st, B, dh, dh, s.d2b, dh, net->w2t_bf16, dh, s.d2, dh, nullptr, s.part);
    hipLaunchKernelGGL(k_dtanh, dim3(grid1((long)B * dh)), dim3(kT), 0, st, s.d2, (const float*)s.t1, (uint16_t*)nullptr,
                       (long)B * dh);
    hipLaunchKernelGGL(k_colsum, dim3((dh + kT - 1) / kT), dim3(kT), 0, st, B, dh, (const float*)s.d2, g + o.b1);
    hipLaunchKernelGGL(k_gw1, dim3((dh * din + kT - 1) / kT), dim3(kT), 0, st, B, din, dh, (const float*)s.d2, d_x, d_idx,
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
