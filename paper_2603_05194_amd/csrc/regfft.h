// Register-resident batched FFT for line lengths known at compile time: powers of two, and
// c 2^p with c = 3 or 5.
//
// A block of 256 threads transforms L lines of N points; each thread keeps E points of one
// line in registers. Stage s of radix R_s applies the Stockham step
//   v_k = x[j + k N/R] * w^(k (j mod Ns)),  v = DFT_R(v),  y[(j - j mod Ns) R + j mod Ns + k Ns] = v_k
// to the E/R butterflies j = jb + (N/E) b of the thread; between stages the points go through
// LDS once (write outputs, barrier, read the next stage's inputs, barrier). Radices, forward
// order: for N = 2^p, radix 2 or 4 first when p is not a multiple of 3, then radix 8; for
// N = c 2^p, radix c, then radix 2 when p is odd, then radix 4, so that E = 4c points per
// thread is a multiple of every radix and N / E stays a power of two.
//
// Register layouts: on entry v[b R_first + k] = x[jb + (N/E) b + k N/R_first]; on exit
// v[b R_last + k] = X[jb + (N/E) b + k N/R_last] (natural-order frequency index). The inverse
// transform runs the stages in reverse order, so an inverse started from a forward's exit
// layout ends in the forward's entry layout: forward -> pointwise multiply -> inverse needs no
// extra data movement.
#pragma once
#include <type_traits>

#include "common.h"
#include "fft.h"

namespace bec {

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

constexpr int odd_part(int n) { return n % 2 ? n : odd_part(n / 2); }

template <int N> struct RfPlan {
    static constexpr int c = odd_part(N);         // 1, 3 or 5
    static constexpr int p = ilog2(N / c);
    static_assert(c == 1 || c == 3 || c == 5, "register FFT lengths are 2^p, 3 2^p or 5 2^p");
    static constexpr int rem = c == 1 ? p % 3 : p % 2;
    static constexpr int ns = c == 1 ? p / 3 + (rem ? 1 : 0) : 1 + p / 2 + rem;
    // forward order: the odd radix, then the small power-of-two radix, then the large ones
    static constexpr int fwd(int s) {
        return c == 1 ? ((rem && s == 0) ? (1 << rem) : 8) : (s == 0 ? c : ((rem && s == 1) ? 2 : 4));
    }
    static constexpr int inv(int s) { return fwd(ns - 1 - s); }
    template <int DIR> static constexpr int radix(int s) { return DIR < 0 ? fwd(s) : inv(s); }
    template <int DIR> static constexpr int span(int s) {   // product of the radices before s
        return s == 0 ? 1 : span<DIR>(s - 1) * radix<DIR>(s - 1);
    }
};

// points per thread. Powers of two: enough lines per block for 128-byte column segments, at
// least 8. c 2^p: 4c, the least multiple of every radix of the plan.
template <typename R> constexpr int rf_points(int N) {
    if (odd_part(N) > 1) return 4 * odd_part(N);
    const int per_seg = 128 / (int)sizeof(cpx<R>);          // complex values per 128 B
    int e = per_seg * N / kThreads;
    if (e < 8) e = 8;
    if (e > 32) e = 32;
    if (e > N) e = N;
    return e;
}

template <typename R, int N, int E, int NT = kThreads, bool NOSPLIT = false> struct RF {
    static constexpr int TPL = N / E;          // threads per line
    static constexpr int L = NT / TPL;         // lines per block of NT threads
    static constexpr int LD = N + 1;           // LDS line stride (odd: spreads banks)
    static constexpr size_t lds_bytes = (size_t)L * LD * sizeof(cpx<R>);
    // Line kernels whose complex tile exceeds 48 KB exchange one component at a time through a
    // real tile of half the size (two barriers more per stage), so that LDS admits twice the
    // blocks per CU (FP64 N = 512: 64 KB -> 32 KB, four blocks instead of two), unless NOSPLIT.
    static constexpr bool SPLIT = !NOSPLIT && lds_bytes > 48 * 1024;
    static constexpr size_t lds_line_bytes = SPLIT ? (size_t)L * LD * sizeof(R) : lds_bytes;
};

// LP is the LDS element type: cpx<R> (whole complex values) or R (one component at a time).
template <typename R, int N, int E, int DIR, int S, typename LP>
__device__ __forceinline__ void rf_run(cpx<R> (&v)[E], LP* __restrict__ line, int jb,
                                       const cpx<R>* __restrict__ tw) {
    using P = RfPlan<N>;
    constexpr int RD = P::template radix<DIR>(S);
    constexpr int Ns = P::template span<DIR>(S);
    constexpr int TPL = N / E;
    constexpr int BPT = E / RD;
    static_assert(E % RD == 0, "points per thread must be a multiple of every radix");
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
        const int j = jb + TPL * b;
        if constexpr (Ns > 1) {
            // one table read per butterfly; the other twiddles are its powers (at most three
            // products deep: w2 = w1 w1, w3 = w2 w1, w4 = w2 w2, w5 = w4 w1, w6 = w3 w3, w7 = w4 w3)
            const int jm = j % Ns;
            cpx<R> w[RD];
            w[1] = tw[jm * (N / (Ns * RD))];
            if constexpr (DIR > 0) w[1] = conj(w[1]);
            if constexpr (RD > 2) w[2] = cmul(w[1], w[1]);
            if constexpr (RD > 3) w[3] = cmul(w[2], w[1]);
            if constexpr (RD > 4) w[4] = cmul(w[2], w[2]);
            if constexpr (RD > 5) {
                w[5] = cmul(w[4], w[1]);
                w[6] = cmul(w[3], w[3]);
                w[7] = cmul(w[4], w[3]);
            }
#pragma unroll
            for (int k = 1; k < RD; ++k) v[b * RD + k] = cmul(v[b * RD + k], w[k]);
        }
        dft_small<RD, DIR>(&v[b * RD]);
    }
    if constexpr (S + 1 < P::ns) {
        constexpr int RN = P::template radix<DIR>(S + 1);
        constexpr int BN = E / RN;
        if constexpr (sizeof(LP) == sizeof(cpx<R>)) {
#pragma unroll
            for (int b = 0; b < BPT; ++b) {
                const int j = jb + TPL * b;
                const int jm = j % Ns;
                LP* o = line + (j - jm) * RD + jm;
#pragma unroll
                for (int k = 0; k < RD; ++k) o[k * Ns] = v[b * RD + k];
            }
            __syncthreads();
#pragma unroll
            for (int b = 0; b < BN; ++b) {
                const int j = jb + TPL * b;
#pragma unroll
                for (int k = 0; k < RN; ++k) v[b * RN + k] = line[j + k * (N / RN)];
            }
            __syncthreads();
        } else {
            // real parts out, new real parts in, then the same for the imaginary parts: the
            // imaginary registers still hold the old layout while the real ones are exchanged
#pragma unroll
            for (int c = 0; c < 2; ++c) {
#pragma unroll
                for (int b = 0; b < BPT; ++b) {
                    const int j = jb + TPL * b;
                    const int jm = j % Ns;
                    LP* o = line + (j - jm) * RD + jm;
#pragma unroll
                    for (int k = 0; k < RD; ++k) o[k * Ns] = c ? v[b * RD + k].y : v[b * RD + k].x;
                }
                __syncthreads();
#pragma unroll
                for (int b = 0; b < BN; ++b) {
                    const int j = jb + TPL * b;
#pragma unroll
                    for (int k = 0; k < RN; ++k) {
                        if (c) v[b * RN + k].y = line[j + k * (N / RN)];
                        else v[b * RN + k].x = line[j + k * (N / RN)];
                    }
                }
                __syncthreads();
            }
        }
        rf_run<R, N, E, DIR, S + 1>(v, line, jb, tw);
    }
}

// Twiddles of stage S for butterfly j: w[k] = w1^k, k = 1..RD-1, from one table read.
template <typename R, int N, int E, int DIR, int S>
__device__ __forceinline__ void rf_twiddles(cpx<R> (&w)[8], int j, const cpx<R>* __restrict__ tw) {
    using P = RfPlan<N>;
    constexpr int RD = P::template radix<DIR>(S);
    constexpr int Ns = P::template span<DIR>(S);
    const int jm = j % Ns;
    w[1] = tw[jm * (N / (Ns * RD))];
    if constexpr (DIR > 0) w[1] = conj(w[1]);
    if constexpr (RD > 2) w[2] = cmul(w[1], w[1]);
    if constexpr (RD > 3) w[3] = cmul(w[2], w[1]);
    if constexpr (RD > 4) w[4] = cmul(w[2], w[2]);
    if constexpr (RD > 5) {
        w[5] = cmul(w[4], w[1]);
        w[6] = cmul(w[3], w[3]);
        w[7] = cmul(w[4], w[3]);
    }
}

// One LDS exchange between stage S and S+1 of the register layout (whole complex values).
template <typename R, int N, int E, int DIR, int S>
__device__ __forceinline__ void rf_exchange_cpx(cpx<R> (&v)[E], cpx<R>* __restrict__ line, int jb) {
    using P = RfPlan<N>;
    constexpr int RD = P::template radix<DIR>(S);
    constexpr int Ns = P::template span<DIR>(S);
    constexpr int TPL = N / E;
    constexpr int BPT = E / RD;
    constexpr int RN = P::template radix<DIR>(S + 1);
    constexpr int BN = E / RN;
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
        const int j = jb + TPL * b;
        const int jm = j % Ns;
        cpx<R>* o = line + (j - jm) * RD + jm;
#pragma unroll
        for (int k = 0; k < RD; ++k) o[k * Ns] = v[b * RD + k];
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BN; ++b) {
        const int j = jb + TPL * b;
#pragma unroll
        for (int k = 0; k < RN; ++k) v[b * RN + k] = line[j + k * (N / RN)];
    }
    __syncthreads();
}

// Two transforms of the same length and direction side by side (two fields on the same lines):
// each butterfly's twiddles are formed once and serve both, and the two register sets go
// through the LDS line one after the other at each stage boundary.
template <typename R, int N, int E, int DIR, int S>
__device__ __forceinline__ void rf_run2(cpx<R> (&v)[E], cpx<R> (&u)[E], cpx<R>* __restrict__ line, int jb,
                                        const cpx<R>* __restrict__ tw) {
    using P = RfPlan<N>;
    constexpr int RD = P::template radix<DIR>(S);
    constexpr int Ns = P::template span<DIR>(S);
    constexpr int TPL = N / E;
    constexpr int BPT = E / RD;
    static_assert(E % RD == 0, "points per thread must be a multiple of every radix");
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
        if constexpr (Ns > 1) {
            cpx<R> w[8];
            rf_twiddles<R, N, E, DIR, S>(w, jb + TPL * b, tw);
#pragma unroll
            for (int k = 1; k < RD; ++k) {
                v[b * RD + k] = cmul(v[b * RD + k], w[k]);
                u[b * RD + k] = cmul(u[b * RD + k], w[k]);
            }
        }
        dft_small<RD, DIR>(&v[b * RD]);
        dft_small<RD, DIR>(&u[b * RD]);
    }
    if constexpr (S + 1 < P::ns) {
        rf_exchange_cpx<R, N, E, DIR, S>(v, line, jb);
        rf_exchange_cpx<R, N, E, DIR, S>(u, line, jb);
        rf_run2<R, N, E, DIR, S + 1>(v, u, line, jb, tw);
    }
}

template <typename R, int N, int E, int DIR>
__device__ __forceinline__ void rf_fft2(cpx<R> (&v)[E], cpx<R> (&u)[E], cpx<R>* line, int jb, const cpx<R>* tw) {
    rf_run2<R, N, E, DIR, 0>(v, u, line, jb, tw);
}

// Full transform; `line` is this thread's line in LDS (lds + l * LD elements of type LP).
template <typename R, int N, int E, int DIR, typename LP>
__device__ __forceinline__ void rf_fft(cpx<R> (&v)[E], LP* line, int jb, const cpx<R>* tw) {
    rf_run<R, N, E, DIR, 0, LP>(v, line, jb, tw);
}

// Index (within the line) of register slot i for the entry layout of direction DIR
// (i.e. the layout rf_fft<DIR> expects on entry).
template <int N, int E, int DIR> __device__ __forceinline__ int rf_in_index(int jb, int i) {
    using P = RfPlan<N>;
    constexpr int RD = P::template radix<DIR>(0);
    return jb + (N / E) * (i / RD) + (i % RD) * (N / RD);
}

// Zero padding and cropping at compile time. In the entry layout of direction DIR, slot i holds
// position jb + (N/E)(i/R) + (i%R)(N/R) with R the first radix and jb + (N/E)(i/R) < N/R, so
// for even R the position lies in the first half of the line iff i % R < R/2; the same holds
// for the exit layout with R the last radix. A transform whose input is zero beyond N/2 (or
// whose output is needed only below N/2) can then drop those slots as compile-time zeros (dead
// values), and the first (last) butterfly stage simplifies.
template <int N, int E, int DIR> constexpr bool rf_in_low_half(int i) {
    constexpr int RD = RfPlan<N>::template radix<DIR>(0);
    return RD % 2 != 0 || i % RD < RD / 2;
}
template <int N, int E, int DIR> constexpr bool rf_out_low_half(int i) {
    constexpr int RD = RfPlan<N>::template radix<DIR>(RfPlan<N>::ns - 1);
    return RD % 2 != 0 || i % RD < RD / 2;
}
// true when the slot test above decides the half exactly (even first / last radix)
template <int N, int DIR> constexpr bool rf_in_half_exact() { return RfPlan<N>::template radix<DIR>(0) % 2 == 0; }
template <int N, int DIR> constexpr bool rf_out_half_exact() {
    return RfPlan<N>::template radix<DIR>(RfPlan<N>::ns - 1) % 2 == 0;
}

// Index of register slot i for the exit layout of direction DIR.
template <int N, int E, int DIR> __device__ __forceinline__ int rf_out_index(int jb, int i) {
    using P = RfPlan<N>;
    constexpr int RD = P::template radix<DIR>(P::ns - 1);
    return jb + (N / E) * (i / RD) + (i % RD) * (N / RD);
}

}  // namespace bec
