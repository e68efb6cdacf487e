// In-LDS batched 1-D FFT (Stockham autosort, radices 2/3/4/5/8) used by every line pass.
//
// A block holds L lines of length n in LDS, line-major with a padded line stride ldl
// (element j of line l at lds[l*ldl + j]). Each stage of radix R does, for every butterfly
// j in [0, n/R) of every line:
//   v_k = x[j + k n/R],  v_k *= w^(k (j mod Ns)) (w = exp(-2 pi i / (Ns R)), none when Ns = 1),
//   v = DFT_R(v),        y[(j - j mod Ns) R + j mod Ns + k Ns] = v_k,
// with Ns the product of the radices already applied; the output is in natural order.
// Reads of a stage complete (barrier) before its writes, so one LDS buffer suffices.
#pragma once
#include "common.h"

namespace bec {

// DIR = -1: forward exp(-2 pi i jk / R); DIR = +1: inverse exp(+2 pi i jk / R).
template <int DIR, typename R> __device__ __forceinline__ void dft2(cpx<R>* v) {
    cpx<R> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
}

template <int DIR, typename R> __device__ __forceinline__ void dft4(cpx<R>& a0, cpx<R>& a1, cpx<R>& a2, cpx<R>& a3) {
    cpx<R> s02 = a0 + a2, d02 = a0 - a2, s13 = a1 + a3, d13 = a1 - a3;
    // forward: y1 = d02 - i d13, y3 = d02 + i d13
    cpx<R> t = mul_i<DIR>(d13);
    a0 = s02 + s13;
    a2 = s02 - s13;
    a1 = d02 + t;
    a3 = d02 - t;
}

template <int DIR, typename R> __device__ __forceinline__ void dft8(cpx<R>* v) {
    const R r = (R)0.70710678118654752440084436210484904;
    cpx<R> b0 = v[0] + v[4], b4 = v[0] - v[4];
    cpx<R> b1 = v[1] + v[5], b5 = v[1] - v[5];
    cpx<R> b2 = v[2] + v[6], b6 = v[2] - v[6];
    cpx<R> b3 = v[3] + v[7], b7 = v[3] - v[7];
    // twiddles w8^1, w8^2, w8^3 on the odd half; forward w8 = (1 - i)/sqrt2
    if (DIR < 0) {
        b5 = mk(r * (b5.x + b5.y), r * (b5.y - b5.x));
        b6 = mul_i<-1>(b6);
        b7 = mk(r * (b7.y - b7.x), -r * (b7.x + b7.y));
    } else {
        b5 = mk(r * (b5.x - b5.y), r * (b5.x + b5.y));
        b6 = mul_i<+1>(b6);
        b7 = mk(-r * (b7.x + b7.y), r * (b7.x - b7.y));
    }
    dft4<DIR>(b0, b1, b2, b3);
    dft4<DIR>(b4, b5, b6, b7);
    v[0] = b0; v[2] = b1; v[4] = b2; v[6] = b3;
    v[1] = b4; v[3] = b5; v[5] = b6; v[7] = b7;
}

template <int DIR, typename R> __device__ __forceinline__ void dft3(cpx<R>* v) {
    const R s3 = (R)0.86602540378443864676372317075293618;  // sin(2 pi / 3)
    cpx<R> t = v[1] + v[2];
    cpx<R> d = v[1] - v[2];
    cpx<R> m = v[0] - (R)0.5 * t;
    // forward: y1 = m - i s3 d, y2 = m + i s3 d
    cpx<R> u = mul_i<DIR>(s3 * d);
    v[0] = v[0] + t;
    v[1] = m + u;
    v[2] = m - u;
}

template <int DIR, typename R> __device__ __forceinline__ void dft5(cpx<R>* v) {
    const R c1 = (R)0.30901699437494742410229341718281906;   // cos(2 pi / 5)
    const R c2 = (R)-0.80901699437494742410229341718281906;  // cos(4 pi / 5)
    const R s1 = (R)0.95105651629515357211643933337938214;   // sin(2 pi / 5)
    const R s2 = (R)0.58778525229247312916870595463907277;   // sin(4 pi / 5)
    cpx<R> t1 = v[1] + v[4], t2 = v[2] + v[3], t3 = v[1] - v[4], t4 = v[2] - v[3];
    cpx<R> a = v[0] + c1 * t1 + c2 * t2;
    cpx<R> b = v[0] + c2 * t1 + c1 * t2;
    cpx<R> u = mul_i<DIR>(s1 * t3 + s2 * t4);   // forward: y1 = a - i(...), y4 = a + i(...)
    cpx<R> w = mul_i<DIR>(s2 * t3 - s1 * t4);   // forward: y2 = b - i(...), y3 = b + i(...)
    v[0] = v[0] + t1 + t2;
    v[1] = a + u;
    v[4] = a - u;
    v[2] = b + w;
    v[3] = b - w;
}

template <int RD, int DIR, typename R> __device__ __forceinline__ void dft_small(cpx<R>* v) {
    if constexpr (RD == 2) dft2<DIR>(v);
    else if constexpr (RD == 3) dft3<DIR>(v);
    else if constexpr (RD == 4) dft4<DIR>(v[0], v[1], v[2], v[3]);
    else if constexpr (RD == 5) dft5<DIR>(v);
    else dft8<DIR>(v);
}

template <int RD, int DIR, typename R>
__device__ __forceinline__ void fft_stage(cpx<R>* lds, int n, int L, int ldl, int Ns,
                                          const cpx<R>* __restrict__ tw) {
    constexpr int NB = ((kTileElems / RD) + kThreads - 1) / kThreads;
    const int nbf = n / RD;
    const int total = nbf * L;
    const int tid = threadIdx.x;
    cpx<R> v[NB][RD];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int idx = tid + b * kThreads;
        if (idx < total) {
            const int l = idx / nbf;
            const int j = idx - l * nbf;
            const cpx<R>* src = lds + l * ldl + j;
#pragma unroll
            for (int k = 0; k < RD; ++k) v[b][k] = src[k * nbf];
        }
    }
    __syncthreads();
    const int span = n / (Ns * RD);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int idx = tid + b * kThreads;
        if (idx < total) {
            const int l = idx / nbf;
            const int j = idx - l * nbf;
            const int jm = j % Ns;
            if (Ns > 1) {
#pragma unroll
                for (int k = 1; k < RD; ++k) {
                    cpx<R> w = tw[jm * k * span];
                    if (DIR > 0) w = conj(w);
                    v[b][k] = cmul(v[b][k], w);
                }
            }
            dft_small<RD, DIR>(v[b]);
            cpx<R>* o = lds + l * ldl + (j - jm) * RD + jm;
#pragma unroll
            for (int k = 0; k < RD; ++k) o[k * Ns] = v[b][k];
        }
    }
    __syncthreads();
}

// Full transform of the L lines held in LDS. `plan.tw` points at the n-entry table
// exp(-2 pi i t / n) in the precision R.
template <int DIR, typename R>
__device__ void lds_fft(cpx<R>* lds, const FftPlan& plan, int L, int ldl) {
    const cpx<R>* tw = reinterpret_cast<const cpx<R>*>(plan.tw);
    int Ns = 1;
    for (int s = 0; s < plan.nst; ++s) {
        const int rd = plan.radix[s];
        switch (rd) {
            case 8: fft_stage<8, DIR>(lds, plan.n, L, ldl, Ns, tw); break;
            case 4: fft_stage<4, DIR>(lds, plan.n, L, ldl, Ns, tw); break;
            case 2: fft_stage<2, DIR>(lds, plan.n, L, ldl, Ns, tw); break;
            case 3: fft_stage<3, DIR>(lds, plan.n, L, ldl, Ns, tw); break;
            default: fft_stage<5, DIR>(lds, plan.n, L, ldl, Ns, tw); break;
        }
        Ns *= rd;
    }
}

}  // namespace bec
