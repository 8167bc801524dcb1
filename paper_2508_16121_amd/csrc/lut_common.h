// Device helpers shared by the LUT kernels: typed loads/stores, LUT staging in LDS,
// spatial-map row staging and workgroup -> tile mapping.
#pragma once

#include "internal.h"

namespace svdlut {

// ---------------------------------------------------------------- typed element access
template <typename T> __device__ __forceinline__ float ldf(const T* p);
template <> __device__ __forceinline__ float ldf<float>(const float* p) { return *p; }
template <> __device__ __forceinline__ float ldf<__half>(const __half* p) { return __half2float(*p); }

template <typename T> __device__ __forceinline__ void stf(T* p, float v);
template <> __device__ __forceinline__ void stf<float>(float* p, float v) { *p = v; }
template <> __device__ __forceinline__ void stf<__half>(__half* p, float v) { *p = __float2half_rn(v); }

// Four consecutive elements; p must be aligned to 4 elements.  Image planes are streamed:
// read once and written once per launch, so their vector accesses carry the nontemporal
// hint, which keeps them from displacing the LUT factors and the spatial map (read by every
// workgroup) in the caches (4K apply 55 -> 52.5 us).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <typename T> __device__ __forceinline__ void ld4(const T* p, float (&o)[4]);
template <> __device__ __forceinline__ void ld4<float>(const float* p, float (&o)[4]) {
    const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
template <> __device__ __forceinline__ void ld4<__half>(const __half* p, float (&o)[4]) {
    const u32x2 v = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p));
    const uint32_t vx = v.x, vy = v.y;
    const __half2 a = *reinterpret_cast<const __half2*>(&vx);
    const __half2 b = *reinterpret_cast<const __half2*>(&vy);
    const float2 fa = __half22float2(a), fb = __half22float2(b);
    o[0] = fa.x; o[1] = fa.y; o[2] = fb.x; o[3] = fb.y;
}

template <typename T> __device__ __forceinline__ void st4(T* p, const float (&o)[4]);
template <> __device__ __forceinline__ void st4<float>(float* p, const float (&o)[4]) {
    const f32x4 v = {o[0], o[1], o[2], o[3]};
    __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(p));
}
template <> __device__ __forceinline__ void st4<__half>(__half* p, const float (&o)[4]) {
    __half2 a = __floats2half2_rn(o[0], o[1]);
    __half2 b = __floats2half2_rn(o[2], o[3]);
    const u32x2 v = {*reinterpret_cast<uint32_t*>(&a), *reinterpret_cast<uint32_t*>(&b)};
    __builtin_nontemporal_store(v, reinterpret_cast<u32x2*>(p));
}

// The lane's 4 pixels [x0, x0+4) of one row, x0 < n.  VEC: one aligned vector access
// (the caller guarantees alignment and x0 + 4 <= n).  Otherwise element accesses with the
// index clamped to n-1; the clamped duplicate stores write the value that belongs there.
template <typename T, bool VEC>
__device__ __forceinline__ void load_px4(const T* row, int x0, int n, float (&o)[4]) {
    if (VEC) {
        ld4<T>(row + x0, o);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k] = ldf<T>(row + min(x0 + k, n - 1));
    }
}

template <typename T, bool VEC>
__device__ __forceinline__ void store_px4(T* row, int x0, int n, const float (&o)[4]) {
    if (VEC) {
        st4<T>(row + x0, o);
    } else {
        const int cnt = n - x0;
        const float v1 = cnt > 1 ? o[1] : o[0];
        const float v2 = cnt > 2 ? o[2] : v1;
        const float v3 = cnt > 3 ? o[3] : v2;
        stf<T>(row + x0, o[0]);
        stf<T>(row + x0 + min(1, cnt - 1), v1);
        stf<T>(row + x0 + min(2, cnt - 1), v2);
        stf<T>(row + x0 + min(3, cnt - 1), v3);
    }
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- LUT colour decode
// p = min(max(x, 0), 1) (NaN -> 0), q = p*(D-1) in float32, i = min(floor q, D-2), d = q - i.
__device__ __forceinline__ void decode(float xv, float Dm1, int Dm2, int& i, float& d) {
    const float p = fminf(fmaxf(xv, 0.f), 1.f);
    const float q = p * Dm1;
    const int ii = min(static_cast<int>(q), Dm2);
    i = ii;
    d = q - static_cast<float>(ii);
}

// ---------------------------------------------------------------- LUT staging in LDS
// Layout of the staged LUTs ("pair-major, channel-minor"): for pair p, vertex (i, j) and
// output channel c the value T_{3c+p}[i][j] sits at p*D*RS + i*RS + 3*j + c.  The four
// corners of one cell for all three output channels are then reached from one base
// address with constant offsets (0..5 and RS..RS+5, within a ds_read2 offset field).
// RS (the row stride) is 3*D padded to 14 (mod 32): the 3x3 neighbourhood of a cell then maps
// to nine distinct LDS banks whether the LDS is viewed as 32 or 64 banks, which matters
// because per-pixel noise scatters neighbouring pixels over adjacent cells.  Measured on the
// 4K apply at D = 33: 14 (mod 32) 55.7 us, 18: 56.0, 12: 56.4, 10 or 22: 56.5, 20: 56.9,
// 16: 69.2, unpadded (3 mod 32): 81.4.
constexpr int kNode = 3;   // floats per LUT vertex (the three output channels)

__host__ __device__ inline int lut_row_stride(int D) {
    // kNode*D rounded up to the next value that is 14 modulo 32
    const int rs = kNode * D;
    return rs + ((14 - rs) & 31);
}
__host__ __device__ inline int lut_pair_stride(int D) { return D * lut_row_stride(D); }
__host__ __device__ inline int lut_floats(int D) { return (3 * lut_pair_stride(D) + 3) & ~3; }

__device__ __forceinline__ int lut_slot(int p, int i, int j, int c, int D) {
    return p * lut_pair_stride(D) + i * lut_row_stride(D) + kNode * j + c;
}

// Exact unsigned division num / d for num < 2^32 by a reciprocal multiply and at most two
// corrections (m = floor((2^32-1)/d) underestimates the quotient by less than 2).
struct Div {
    uint32_t d, m;
};
__device__ __forceinline__ Div make_div(uint32_t d) {
    Div v;
    v.d = d;
    v.m = 0xFFFFFFFFu / d;
    return v;
}
__device__ __forceinline__ void divmod(const Div& v, uint32_t num, uint32_t& q, uint32_t& r) {
    q = __umulhi(num, v.m);
    r = num - q * v.d;
    if (r >= v.d) { ++q; r -= v.d; }
    if (r >= v.d) { ++q; r -= v.d; }
}

// Rebuild the nine LUTs of one image (T_l = U_l diag(s_l) V_l^T) into Tl.
// scratch must hold 2 * 9 * D * 8 floats.  The rank is processed 8 columns at a time
// (missing columns are zero-padded so the inner loop is always 8 fused multiply-adds);
// partial sums accumulate in Tl.  Work item (l, j, half) keeps V_l[j][k0..k0+7] in
// registers and walks half of the rows i, reading U_l[i] (times s_l) as two 16-byte
// broadcast loads.  Starts and ends with a barrier.
__device__ inline void stage_luts(float* Tl, float* scratch, const float* U, const float* s,
                                  const float* V, int D, int R, int /*kc*/) {
    constexpr int KC = 8;
    const int nthr = blockDim.x;
    const int tid = threadIdx.x;
    const int nrows = 9 * D;
    const int RS = lut_row_stride(D);
    const int PS = lut_pair_stride(D);
    float* Us = scratch;                 // [9*D][8]  (U * s)
    float* Vs = scratch + nrows * KC;    // [9*D][8]
    const int half = (D + 1) / 2;
    for (int k0 = 0; k0 < R; k0 += KC) {
        const int kn = min(KC, R - k0);
        __syncthreads();
        for (int e = tid; e < nrows * KC; e += nthr) {
            const int r = e >> 3, k = e & 7;
            const int l = r / D;
            float u = 0.f, v = 0.f;
            if (k < kn) {
                const int src = r * R + k0 + k;
                u = U[src] * s[l * R + k0 + k];
                v = V[src];
            }
            Us[e] = u;
            Vs[e] = v;
        }
        __syncthreads();
        for (int item = tid; item < nrows * 2; item += nthr) {
            const int lj = item >> 1;            // l * D + j
            const int hf = item & 1;
            const int l = lj / D;
            const int j = lj - l * D;
            const float4 va = *reinterpret_cast<const float4*>(Vs + lj * KC);
            const float4 vb = *reinterpret_cast<const float4*>(Vs + lj * KC + 4);
            const int c = l / 3, p = l - 3 * c;
            const int i0 = hf ? half : 0;
            const int i1 = hf ? D : half;
            float* out = Tl + p * PS + i0 * RS + kNode * j + c;
            const float* urow = Us + (l * D + i0) * KC;
            for (int i = i0; i < i1; ++i, out += RS, urow += KC) {
                const float4 ua = *reinterpret_cast<const float4*>(urow);
                const float4 ub = *reinterpret_cast<const float4*>(urow + 4);
                float acc = ua.x * va.x;
                acc = fmaf(ua.y, va.y, acc);
                acc = fmaf(ua.z, va.z, acc);
                acc = fmaf(ua.w, va.w, acc);
                acc = fmaf(ub.x, vb.x, acc);
                acc = fmaf(ub.y, vb.y, acc);
                acc = fmaf(ub.z, vb.z, acc);
                acc = fmaf(ub.w, vb.w, acc);
                *out = (k0 == 0) ? acc : *out + acc;
            }
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------- spatial-map geometry
// Corner-aligned source coordinate of output position x on an n_out axis for an n_in grid:
// u = x*(n_in-1)/(n_out-1).  Returned as the left index (clamped to n_in-2) and the
// integer remainder num - idx*(n_out-1), so the fractional weight is rem/(n_out-1) exactly.
struct AxisMap {
    Div div;             // by max(n_out - 1, 1)
    uint32_t num_step;   // n_in - 1
    int32_t last;        // max(n_in - 2, 0)
    float inv;           // 1/(n_out - 1), or 0 when n_out == 1
};

__device__ __forceinline__ AxisMap make_axis(int n_out, int n_in) {
    AxisMap a;
    a.num_step = static_cast<uint32_t>(n_in - 1);
    a.div = make_div(static_cast<uint32_t>(n_out > 1 ? n_out - 1 : 1));
    a.last = n_in >= 2 ? n_in - 2 : 0;
    a.inv = n_out > 1 ? 1.f / static_cast<float>(n_out - 1) : 0.f;
    return a;
}

// left index (clamped) and remainder relative to it (may equal den at the clamped edge)
__device__ __forceinline__ void axis_left(const AxisMap& a, int x, int& idx, uint32_t& rem) {
    const uint32_t num = static_cast<uint32_t>(x) * a.num_step;
    uint32_t q, r;
    divmod(a.div, num, q, r);
    if (static_cast<int>(q) > a.last) {      // only at the last position (or a size-1 grid)
        r += (q - a.last) * a.div.d;
        q = a.last;
    }
    idx = static_cast<int>(q);
    rem = r;
}

// XCD-aware workgroup order: workgroups are dispatched round-robin over the 8 XCDs, so
// give each XCD a contiguous run of logical chunks (neighbouring rows then share the map
// rows and the factors in that XCD's L2).
__device__ __forceinline__ int logical_block(int bid, int G) {
    const int q = G >> 3, r = G & 7;
    const int x = bid & 7;
    return x * q + min(x, r) + (bid >> 3);
}

}  // namespace svdlut
