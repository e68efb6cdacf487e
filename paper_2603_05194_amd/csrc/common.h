// Shared device/host definitions: complex type, launch constants, reduction slots.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bec {

template <typename R> struct alignas(2 * sizeof(R)) cpx { R x, y; };

template <typename R> __host__ __device__ __forceinline__ cpx<R> mk(R a, R b) { cpx<R> c; c.x = a; c.y = b; return c; }
template <typename R> __host__ __device__ __forceinline__ cpx<R> operator+(cpx<R> a, cpx<R> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename R> __host__ __device__ __forceinline__ cpx<R> operator-(cpx<R> a, cpx<R> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename R> __host__ __device__ __forceinline__ cpx<R> operator*(R s, cpx<R> a) { return mk(s * a.x, s * a.y); }
template <typename R> __host__ __device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
    return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename R> __host__ __device__ __forceinline__ cpx<R> cmulc(cpx<R> a, cpx<R> b) {  // a * conj(b)
    return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename R> __host__ __device__ __forceinline__ cpx<R> conj(cpx<R> a) { return mk(a.x, -a.y); }
// multiply by -i (s = -1) or +i (s = +1)
template <int S, typename R> __host__ __device__ __forceinline__ cpx<R> mul_i(cpx<R> a) {
    return S > 0 ? mk(-a.y, a.x) : mk(a.y, -a.x);
}

// Streaming (nontemporal) store of a field value, for outputs that the pass right after does
// not read: they then bypass the caches instead of displacing the inputs of the next pass. Used
// where it measured faster (the padded y forward's output, the retraction, the preconditioned
// residual, the direction, r and H phi); outputs that the next pass reads keep plain stores.
// Streaming loads likewise for inputs read once: the padded x passes' spectra (the symbol rows,
// which the +ky and -ky columns share, stay cached), the last preconditioner pass's W, r_prev
// and p_prev, the direction pass's P r and p_prev, and the x operator's partial sum.
template <typename R> __device__ __forceinline__ void st_stream(cpx<R>* p, cpx<R> v) {
    typedef R V2 __attribute__((ext_vector_type(2)));
    V2 t = {v.x, v.y};
    __builtin_nontemporal_store(t, reinterpret_cast<V2*>(p));
}

template <typename R> __device__ __forceinline__ cpx<R> ld_stream(const cpx<R>* p) {
    typedef R V2 __attribute__((ext_vector_type(2)));
    const V2 t = __builtin_nontemporal_load(reinterpret_cast<const V2*>(p));
    return mk<R>(t.x, t.y);
}

constexpr int kThreads = 256;         // threads per block of every field kernel
constexpr int kTileElems = 4096;      // complex elements held in LDS by one line-FFT block
constexpr int kMaxStages = 12;
constexpr int kMaxRed = 32;           // reduction slots per kernel
constexpr int kRedBlocks = 1024;      // blocks of the grid-stride pointwise reductions
constexpr int kKernelVariants = 8;    // launch-shape variants of the register kernels (BEC_KERNEL_VARIANTS)

// Line lengths with register-resident FFT kernels: powers of two 32..1024 and 3 or 5 times a
// power of two (48..384, 160, 320). Every other length runs on the runtime-length LDS kernels.
__host__ __device__ inline bool rf_length(int n) {
    switch (n) {
        case 32: case 64: case 128: case 256: case 512: case 1024:
        case 48: case 96: case 192: case 384: case 160: case 320: return true;
        default: return false;
    }
}

// Per-size FFT plan (device-visible, passed by value).
struct FftPlan {
    int n;
    int nst;
    int radix[kMaxStages];
    const void* tw;                   // n twiddles exp(-2 pi i t / n), element type cpx<R>
};

}  // namespace bec
