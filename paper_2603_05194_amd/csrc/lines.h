// Tile addressing, LDS staging and block reductions shared by the line-pass kernels.
#pragma once
#include "common.h"
#include "fft.h"
#include "kernels.h"

namespace bec {

constexpr int kLoadIters = kTileElems / kThreads;   // 16 elements per thread per tile

struct Tile {
    int outer;    // axis 2: first line index; axes 0/1: outer index
    int inner0;   // axes 0/1: first inner index
};

__device__ __forceinline__ Tile tile_of(const Geo& g, int t) {
    Tile ti;
    if (g.axis == 2) { ti.outer = t * g.L; ti.inner0 = 0; }
    else { ti.outer = t / g.tpo; ti.inner0 = (t - ti.outer * g.tpo) * g.L; }
    return ti;
}

__device__ __forceinline__ bool line_ok(const Geo& g, const Tile& ti, int l) {
    return g.axis == 2 ? (ti.outer + l < g.n_outer) : (ti.inner0 + l < g.n_inner);
}

// Address of element j of tile line l in an array whose extent along the axis is na.
__device__ __forceinline__ long line_addr(const Geo& g, const Tile& ti, int l, int j, int na) {
    if (g.axis == 2) return (long)(ti.outer + l) * na + j;
    return ((long)ti.outer * na + j) * g.n_inner + ti.inner0 + l;
}

// The two coordinates of a line besides its axis: (i0,i1) for axis 2, (i0,i2) for axis 1,
// (i1,i2) for axis 0.
__device__ __forceinline__ void line_coords(const Geo& g, const Tile& ti, int l, int& c0, int& c1) {
    if (g.axis == 2) { int line = ti.outer + l; c0 = line / g.dA; c1 = line - c0 * g.dA; }
    else if (g.axis == 1) { c0 = ti.outer; c1 = ti.inner0 + l; }
    else { int inner = ti.inner0 + l; c0 = inner / g.dB; c1 = inner - c0 * g.dB; }
}

// Map flat element e of an (L x na) tile to (l, j) so that consecutive threads touch
// consecutive global addresses: j fastest for contiguous (axis 2) lines, l fastest otherwise.
__device__ __forceinline__ void tile_lj(const Geo& g, int e, int na, int& l, int& j) {
    if (g.axis == 2) { l = e / na; j = e - l * na; }
    else { j = e / g.L; l = e - j * g.L; }
}

// Load na elements of each tile line into LDS (fetch(addr, l, j) -> cpx<R>) and zero
// j in [na, nfft). Loads are issued before the LDS writes.
template <typename R, typename F>
__device__ __forceinline__ void load_tile(cpx<R>* lds, int ldl, const Geo& g, const Tile& ti,
                                          int na, int nfft, F fetch) {
    const int M = g.L * na;
    cpx<R> v[kLoadIters];
#pragma unroll
    for (int it = 0; it < kLoadIters; ++it) {
        const int e = threadIdx.x + it * kThreads;
        v[it] = mk<R>(0, 0);
        if (e < M) {
            int l, j;
            tile_lj(g, e, na, l, j);
            if (line_ok(g, ti, l)) v[it] = fetch(line_addr(g, ti, l, j, na), l, j);
        }
    }
#pragma unroll
    for (int it = 0; it < kLoadIters; ++it) {
        const int e = threadIdx.x + it * kThreads;
        if (e < M) {
            int l, j;
            tile_lj(g, e, na, l, j);
            lds[l * ldl + j] = v[it];
        }
    }
    if (nfft > na) {
        const int P = g.L * (nfft - na);
        for (int e = threadIdx.x; e < P; e += kThreads) {
            const int l = e / (nfft - na);
            const int j = na + e - l * (nfft - na);
            lds[l * ldl + j] = mk<R>(0, 0);
        }
    }
}

// Visit the first na elements of each valid tile line: f(addr, l, j, value_in_lds).
template <typename R, typename F>
__device__ __forceinline__ void visit_tile(cpx<R>* lds, int ldl, const Geo& g, const Tile& ti, int na, F f) {
    const int M = g.L * na;
    for (int e = threadIdx.x; e < M; e += kThreads) {
        int l, j;
        tile_lj(g, e, na, l, j);
        if (line_ok(g, ti, l)) f(line_addr(g, ti, l, j, na), l, j, lds[l * ldl + j]);
    }
}

// Visit LDS entries of all tile lines in j-fastest order (for spectral multipliers).
template <typename R, typename F>
__device__ __forceinline__ void visit_lds(cpx<R>* lds, int ldl, int L, int n, F f) {
    const int M = L * n;
    for (int e = threadIdx.x; e < M; e += kThreads) {
        const int l = e / n;
        const int k = e - l * n;
        f(l, k, lds[l * ldl + k]);
    }
}

// Block reduction of NQ doubles over NT threads; slot q is a max-reduction if bit q of MAXMASK
// is set. Writes partials[blockIdx.x * NQ + q].
template <int NQ, unsigned MAXMASK, int NT = kThreads>
__device__ __forceinline__ void block_reduce(double (&v)[NQ], double* __restrict__ partials) {
    __shared__ double red[NT / 64][NQ > 0 ? NQ : 1];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double x = v[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double y = __shfl_xor(x, off, 64);
            x = ((MAXMASK >> q) & 1u) ? fmax(x, y) : x + y;
        }
        if (lane == 0) red[wave][q] = x;
    }
    __syncthreads();
    if (threadIdx.x < NQ) {
        const int q = threadIdx.x;
        double x = red[0][q];
        for (int w = 1; w < NT / 64; ++w) x = ((MAXMASK >> q) & 1u) ? fmax(x, red[w][q]) : x + red[w][q];
        partials[(long)blockIdx.x * NQ + q] = x;
    }
}

}  // namespace bec
