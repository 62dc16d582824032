// Device helpers: complex arithmetic, the 3-point kernel weights, radix
// butterflies and the in-LDS Stockham line transform, block reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "mb_internal.h"

namespace mb {

constexpr int WAVE = 64;

template <typename T>
struct __align__(2 * sizeof(T)) cplx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) {
    return {a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) {
    return {a.x - b.x, a.y - b.y};
}
template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) {
    return {a.x, -a.y};
}
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cplx<T> mul_mi(cplx<T> a) {
    return INV ? cplx<T>{-a.y, a.x} : cplx<T>{a.y, -a.x};
}

// 1/sqrt(x) for a normal float64 x > 0: the hardware estimate refined by
// two Newton steps y <- y + y (1/2 - x y^2 / 2) for the root of 1/y^2 - x,
// each of which squares the relative error (an estimate good to 2^-14
// ends below the float64 rounding).
template <int NEWTON = 2>
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int i = 0; i < NEWTON; ++i) {
        const double r = fma(-(x * y), 0.5 * y, 0.5);
        y = fma(y, r, y);
    }
    return y;
}

// Weights of the 3-point kernel at the nodes i0-1, i0, i0+1 of a point at
// offset t in [-1/2, 1/2] from node i0 (t = x/h - i0).  With s = sqrt(1-3t^2):
// Phi(t) = (1+s)/3 and Phi(1 -+ t) = (2 +- 3t - s)/6.
// sqrt(x) for the kernel weights, x in [1/4, 1]: the hardware square root
// for float32 (within an ulp; the correctly rounded sequence costs ~16
// instructions), x (1/sqrt x) with the Newton-refined reciprocal square root
// for float64.
__device__ __forceinline__ float weight_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double weight_sqrt(double x) { return x * rsqrt_nr(x); }

// 1/x: the hardware reciprocal for float32 (within an ulp), the division
// for float64.
__device__ __forceinline__ float field_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double field_rcp(double x) { return 1.0 / x; }

template <typename T>
__device__ __forceinline__ void kernel_weights(T t, T w[3]) {
    const T s = weight_sqrt(T(1) - T(3) * t * t);
    const T sixth = T(1) / T(6);
    w[1] = (T(1) + s) * (T(1) / T(3));
    w[2] = (T(2) + T(3) * t - s) * sixth;
    w[0] = (T(2) - T(3) * t - s) * sixth;
}

// The weights and their derivatives with respect to t: d/dt Phi(t) =
// -t/s, d/dt Phi(1 -+ t) = +-1/2 + t/(2s) (Phi is C^1, s >= 1/2 on
// [-1/2, 1/2]).
template <typename T>
__device__ __forceinline__ void kernel_weights_deriv(T t, T w[3], T dw[3]) {
    const T s = sqrt(T(1) - T(3) * t * t);
    const T sixth = T(1) / T(6);
    w[1] = (T(1) + s) * (T(1) / T(3));
    w[2] = (T(2) + T(3) * t - s) * sixth;
    w[0] = (T(2) - T(3) * t - s) * sixth;
    const T r = t / (T(2) * s);
    dw[1] = -T(2) * r;
    dw[2] = T(0.5) + r;
    dw[0] = -T(0.5) + r;
}

// ---------------------------------------------------------------------------
// Radix-R DFT of R values in registers: y_k = sum_r v_r W_R^{rk} with
// W_R = exp(-2 pi i / R) (forward) or its conjugate (inverse).
template <typename T, bool INV>
__device__ __forceinline__ void dft2(cplx<T>* v) {
    cplx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cplx<T>& a0, cplx<T>& a1, cplx<T>& a2,
                                     cplx<T>& a3) {
    cplx<T> s02 = cadd(a0, a2), d02 = csub(a0, a2);
    cplx<T> s13 = cadd(a1, a3), d13 = mul_mi<T, INV>(csub(a1, a3));
    a0 = cadd(s02, s13);
    a2 = csub(s02, s13);
    a1 = cadd(d02, d13);
    a3 = csub(d02, d13);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4v(cplx<T>* v) {
    dft4<T, INV>(v[0], v[1], v[2], v[3]);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(cplx<T>* v) {
    // even / odd halves, then combine with W_8^k
    cplx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cplx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<T, INV>(e0, e1, e2, e3);
    dft4<T, INV>(o0, o1, o2, o3);
    const T r = T(0.70710678118654752440084436210484903928);
    // W_8^1 = r(1 - i) forward, r(1 + i) inverse
    cplx<T> t1 = INV ? cplx<T>{r * (o1.x - o1.y), r * (o1.x + o1.y)}
                     : cplx<T>{r * (o1.x + o1.y), r * (o1.y - o1.x)};
    cplx<T> t2 = mul_mi<T, INV>(o2);
    // W_8^3 = -r(1 + i) forward, -r(1 - i) inverse
    cplx<T> t3 = INV ? cplx<T>{-r * (o3.x + o3.y), r * (o3.x - o3.y)}
                     : cplx<T>{r * (o3.y - o3.x), -r * (o3.x + o3.y)};
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, t1);
    v[5] = csub(e1, t1);
    v[2] = cadd(e2, t2);
    v[6] = csub(e2, t2);
    v[3] = cadd(e3, t3);
    v[7] = csub(e3, t3);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft3(cplx<T>* v) {
    const T c = T(0.86602540378443864676372317075293618347);  // sqrt(3)/2
    cplx<T> s = cadd(v[1], v[2]);
    cplx<T> d = csub(v[1], v[2]);
    cplx<T> t = {v[0].x - T(0.5) * s.x, v[0].y - T(0.5) * s.y};
    // W_3 = -1/2 - i c (forward): y1 = t - i c d, y2 = t + i c d
    cplx<T> icd = {-c * d.y, c * d.x};
    v[0] = cadd(v[0], s);
    if (INV) {
        v[1] = cadd(t, icd);
        v[2] = csub(t, icd);
    } else {
        v[1] = csub(t, icd);
        v[2] = cadd(t, icd);
    }
}

// W_16^m (m = 1, 2, 3, 6, 9) applied to a: forward W = cos(pi m/8) -
// i sin(pi m/8), inverse its conjugate.
template <typename T, bool INV, int M>
__device__ __forceinline__ cplx<T> w16(cplx<T> a) {
    constexpr double C[10] = {1.0, 0.92387953251128675613, 0.70710678118654752440,
                              0.38268343236508977173, 0.0, -0.38268343236508977173,
                              -0.70710678118654752440, -0.92387953251128675613, -1.0,
                              -0.92387953251128675613};
    constexpr double S[10] = {0.0, 0.38268343236508977173, 0.70710678118654752440,
                              0.92387953251128675613, 1.0, 0.92387953251128675613,
                              0.70710678118654752440, 0.38268343236508977173, 0.0,
                              -0.38268343236508977173};
    const T c = (T)C[M];
    const T s = INV ? (T)S[M] : -(T)S[M];  // W = c + i s
    return cplx<T>{a.x * c - a.y * s, a.x * s + a.y * c};
}

// 16-point DFT as 4 x 4: DFTs of the four decimated sequences v[4 n1 + n2]
// (over n1), twiddles W_16^{n2 k1}, then DFTs over n2; output k1 + 4 k2.
template <typename T, bool INV>
__device__ __forceinline__ void dft16(cplx<T>* v) {
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4<T, INV>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
    // v[4 k1 + n2] now holds Y[n2][k1]
    v[4 + 1] = w16<T, INV, 1>(v[4 + 1]);
    v[4 + 2] = w16<T, INV, 2>(v[4 + 2]);
    v[4 + 3] = w16<T, INV, 3>(v[4 + 3]);
    v[8 + 1] = w16<T, INV, 2>(v[8 + 1]);
    v[8 + 2] = mul_mi<T, INV>(v[8 + 2]);  // W_16^4 = -i (forward)
    v[8 + 3] = w16<T, INV, 6>(v[8 + 3]);
    v[12 + 1] = w16<T, INV, 3>(v[12 + 1]);
    v[12 + 2] = w16<T, INV, 6>(v[12 + 2]);
    v[12 + 3] = w16<T, INV, 9>(v[12 + 3]);
    cplx<T> o[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cplx<T> a0 = v[4 * k1], a1 = v[4 * k1 + 1], a2 = v[4 * k1 + 2], a3 = v[4 * k1 + 3];
        dft4<T, INV>(a0, a1, a2, a3);
        o[k1] = a0;
        o[k1 + 4] = a1;
        o[k1 + 8] = a2;
        o[k1 + 12] = a3;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = o[k];
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dftR(cplx<T>* v) {
    if constexpr (R == 2) dft2<T, INV>(v);
    else if constexpr (R == 3) dft3<T, INV>(v);
    else if constexpr (R == 4) dft4v<T, INV>(v);
    else if constexpr (R == 8) dft8<T, INV>(v);
    else dft16<T, INV>(v);
}

// ---------------------------------------------------------------------------
// Block reductions (blockDim.x a multiple of 64, at most 1024).
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}

// Sum (or max) of one value per thread; the result is valid in every
// thread.  `scratch` holds at least 16 doubles.  Contains barriers.
template <bool MAX>
__device__ double block_reduce(double v, double* scratch) {
    const int lane = threadIdx.x % WAVE;
    const int wid = threadIdx.x / WAVE;
    const int nw = (blockDim.x + WAVE - 1) / WAVE;
    v = MAX ? wave_max(v) : wave_sum(v);
    __syncthreads();
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    double r = MAX ? 0.0 : 0.0;
    if (MAX) {
        r = scratch[0];
        for (int i = 1; i < nw; ++i) r = fmax(r, scratch[i]);
    } else {
        for (int i = 0; i < nw; ++i) r += scratch[i];
    }
    __syncthreads();
    return r;
}

// Sums of three doubles over the block, returned to every thread (scratch:
// 3 * 16 doubles).
__device__ __forceinline__ void block_reduce3(double v[3], double* scratch) {
    const int lane = threadIdx.x % WAVE;
    const int wid = threadIdx.x / WAVE;
    const int nw = (blockDim.x + WAVE - 1) / WAVE;
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = wave_sum(v[c]);
    if (lane == 0) {
        scratch[3 * wid] = v[0];
        scratch[3 * wid + 1] = v[1];
        scratch[3 * wid + 2] = v[2];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double r = 0.0;
        for (int i = 0; i < nw; ++i) r += scratch[3 * i + c];
        v[c] = r;
    }
    __syncthreads();
}

// Exclusive prefix sum of one int per thread over the block; returns the
// thread's exclusive prefix and writes the block total to *total.
__device__ __forceinline__ int block_exclusive_scan(int v, int* scratch,
                                                    int* total) {
    const int lane = threadIdx.x % WAVE;
    const int wid = threadIdx.x / WAVE;
    const int nw = (blockDim.x + WAVE - 1) / WAVE;
    int x = v;
    for (int o = 1; o < WAVE; o <<= 1) {
        int y = __shfl_up(x, o, WAVE);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == WAVE - 1) scratch[wid] = x;
    __syncthreads();
    int before = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        if (i < wid) before += scratch[i];
        tot += scratch[i];
    }
    __syncthreads();
    *total = tot;
    return before + x - v;
}

// Block index -> work index such that each of the 8 XCDs (which receive
// blocks round-robin) works on one contiguous range of work items.
// Element `i` of an array from its (wave-uniform) base with a 32-bit
// unsigned byte offset, so the load takes the base from scalar registers and
// one offset register, with no 64-bit address arithmetic per load (every
// array the kernels index this way is below 4 GiB).
template <typename T>
__device__ __forceinline__ T ld32(const T* __restrict__ base, unsigned i) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) +
                                       i * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st32(T* __restrict__ base, unsigned i, const T& x) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (unsigned)sizeof(T)) = x;
}

// A hook that does nothing (default of the "after the loads are issued"
// callbacks).
struct NoOp {
    __device__ void operator()() const {}
};

__device__ __forceinline__ int xcd_remap(int b, int n) {
    const int per = n / 8;
    return (b % 8) * per + b / 8;
}

}  // namespace mb
