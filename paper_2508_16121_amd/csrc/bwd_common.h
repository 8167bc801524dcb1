// Helpers shared by the backward kernels: fixed-point LDS accumulation with a per-workgroup
// power-of-two scale, float atomics to global memory, block-wide maxima.
#pragma once

#include "lut_common.h"

#include <cfloat>

namespace svdlut {

__device__ __forceinline__ void lds_addi(int* p, int v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void gbl_add(float* p, float v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int fix(float v) { return __float2int_rn(v); }

// round(a * b) to the nearest integer (ties to even) for |a * b| < 2^22, in two instructions:
// one fma adds 1.5 * 2^23, whose ulp is 1, so the exact product is rounded once and lands in
// the low mantissa bits, which an integer subtraction takes out.  The scales from fix_scale
// keep every accumulated term below 2^22.
__device__ __forceinline__ int fix_mul(float a, float b) {
    return __float_as_int(fmaf(a, b, 12582912.0f)) - 0x4B400000;
}

// Largest power of two 2^e with n * m1 * m2 * 2^e < 2^30 (1 when a factor is 0); sets
// `bad` when the bound does not fit the float exponent range.  n counts as at least 1024, so
// a single term (or a sum of up to four terms merged in registers) stays below 2^22, the
// range of fix_mul.
__device__ inline float fix_scale(float n, float m1, float m2, bool& bad) {
    if (!(n > 0.f) || !(m1 > 0.f) || !(m2 > 0.f)) return 1.f;
    int en, e1, e2;
    frexpf(fmaxf(n, 1024.f), &en);
    frexpf(m1, &e1);
    frexpf(m2, &e2);
    const int e = 30 - (en + e1 + e2);   // each factor f < 2^ef
    if (e < -126) { bad = true; return 1.f; }
    return ldexpf(1.f, min(e, 126));
}

// Rounding of one term to the accumulator's integer grid for any |a * b| < 2^31 (three
// instructions): used when a workgroup's scale lets single terms exceed fix_mul's range.
__device__ __forceinline__ int fix_exact(float a, float b) { return __float2int_rn(a * b); }

// Fixed-point scale of one accumulator family from the workgroup's own bounds: the largest
// power of two 2^e with sum * m2 * 2^e < 2^30, where `sum` bounds the sum of |dy| over the
// pixels that can feed one entry and m2 the other factor of a term (|S| or |phi|; the
// interpolation weights are <= 1 and each pixel adds at most one term to an entry), so no
// partial sum can reach 2^30.  `one` bounds a single pixel's |dy|: while one * m2 * 2^e <
// 2^20 single terms (and sums of four merged in registers) stay in fix_mul's range;
// otherwise `exact` is set and the terms must be rounded with fix_exact.  A bound taken from
// the sum rather than from (pixels x largest |dy|) keeps one large |dy| (an outlier of the
// loss gradient) from coarsening the grid of every other term.  Returns 1 when a factor is
// 0; sets `bad` when the bound does not fit the float exponent range.
__device__ inline float fix_scale_sum(float sum, float one, float m2, bool& exact, bool& bad) {
    if (!(sum > 0.f) || !(one > 0.f) || !(m2 > 0.f)) return 1.f;
    int es, eo, e2;
    frexpf(sum, &es);
    frexpf(one, &eo);
    frexpf(m2, &e2);
    const int e_sum = 30 - (es + e2);    // each factor f < 2^ef
    const int e_one = 20 - (eo + e2);
    if (e_sum > e_one) exact = true;
    if (e_sum < -126) { bad = true; return 1.f; }
    return ldexpf(1.f, min(e_sum, 126));
}

// sum over the block of one value per thread in a fixed order (every thread gets the result)
__device__ inline float block_sum(float v, float* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int nw = blockDim.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    float m = red[0];
    for (int i = 1; i < nw; ++i) m += red[i];
    __syncthreads();
    return m;
}

// max over the block of one value per thread (every thread gets the result); `red` holds
// one float per wave and is free again when the function returns
__device__ inline float block_max(float v, float* red) {
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    const int nw = blockDim.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    float m = red[0];
    for (int i = 1; i < nw; ++i) m = fmaxf(m, red[i]);
    __syncthreads();
    return m;
}

__device__ __forceinline__ void absmax_acc(float v, float& m, bool& bad) {
    v = fabsf(v);
    bad |= !(v <= FLT_MAX);
    m = fmaxf(m, v);
}

// max |p[i]| over [0, n) by the whole block: 4-element vector loads (eight per thread in
// flight) when p is aligned to 4 elements, element loads for the rest
template <typename T>
__device__ inline void absmax_range(const T* p, int64_t n, float& m, bool& bad) {
    int64_t i0 = 0;
    if ((reinterpret_cast<uintptr_t>(p) & (4 * sizeof(T) - 1)) == 0) {
        const int64_t n4 = n / 4, step = blockDim.x;
        int64_t v = threadIdx.x;
        for (; v + 7 * step < n4; v += 8 * step) {
            float q[8][4];
#pragma unroll
            for (int u = 0; u < 8; ++u) ld4<T>(p + 4 * (v + u * step), q[u]);
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int e = 0; e < 4; ++e) absmax_acc(q[u][e], m, bad);
        }
        for (; v < n4; v += step) {
            float q[4];
            ld4<T>(p + 4 * v, q);
#pragma unroll
            for (int e = 0; e < 4; ++e) absmax_acc(q[e], m, bad);
        }
        i0 = n4 * 4;
    }
    for (int64_t i = i0 + threadIdx.x; i < n; i += blockDim.x) absmax_acc(ldf<T>(p + i), m, bad);
}

__device__ __forceinline__ void abssum_acc(float v, float& s, float& m, bool& bad) {
    v = fabsf(v);
    bad |= !(v <= FLT_MAX);
    s += v;
    m = fmaxf(m, v);
}

// sum and max of |p[i]| over [0, n) by the whole block (this thread's share: a fixed-order
// partial sum), 4-element vector loads when p is aligned to 4 elements
template <typename T>
__device__ inline void abssum_range(const T* p, int64_t n, float& s, float& m, bool& bad) {
    int64_t i0 = 0;
    if ((reinterpret_cast<uintptr_t>(p) & (4 * sizeof(T) - 1)) == 0) {
        const int64_t n4 = n / 4, step = blockDim.x;
        int64_t v = threadIdx.x;
        for (; v + 7 * step < n4; v += 8 * step) {
            float q[8][4];
#pragma unroll
            for (int u = 0; u < 8; ++u) ld4<T>(p + 4 * (v + u * step), q[u]);
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int e = 0; e < 4; ++e) abssum_acc(q[u][e], s, m, bad);
        }
        for (; v < n4; v += step) {
            float q[4];
            ld4<T>(p + 4 * v, q);
#pragma unroll
            for (int e = 0; e < 4; ++e) abssum_acc(q[e], s, m, bad);
        }
        i0 = n4 * 4;
    }
    for (int64_t i = i0 + threadIdx.x; i < n; i += blockDim.x) abssum_acc(ldf<T>(p + i), s, m, bad);
}

}  // namespace svdlut
