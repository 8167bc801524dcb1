// Loss (mean L1 / mean squared error with their gradients) and the Adam update.
#include "internal.h"

#include <cmath>

namespace svdlut {

namespace {

constexpr int kLossThreads = 256;
constexpr int kLossMaxBlocks = 1024;

template <typename T> __device__ __forceinline__ float tof(T v);
template <> __device__ __forceinline__ float tof<float>(float v) { return v; }
template <> __device__ __forceinline__ float tof<__half>(__half v) { return __half2float(v); }
template <typename T> __device__ __forceinline__ T fromf(float v);
template <> __device__ __forceinline__ float fromf<float>(float v) { return v; }
template <> __device__ __forceinline__ __half fromf<__half>(float v) { return __float2half_rn(v); }

// Four consecutive elements as floats (vector access: float4 for fp32, 8 bytes for fp16).
__device__ __forceinline__ void ld4(const float* p, float (&o)[4]) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void ld4(const __half* p, float (&o)[4]) {
    const uint2 v = *reinterpret_cast<const uint2*>(p);
    const __half2 a = *reinterpret_cast<const __half2*>(&v.x), b = *reinterpret_cast<const __half2*>(&v.y);
    o[0] = __low2float(a); o[1] = __high2float(a); o[2] = __low2float(b); o[3] = __high2float(b);
}
__device__ __forceinline__ void st4(float* p, const float (&o)[4]) {
    *reinterpret_cast<float4*>(p) = make_float4(o[0], o[1], o[2], o[3]);
}
__device__ __forceinline__ void st4(__half* p, const float (&o)[4]) {
    const __half2 a = __floats2half2_rn(o[0], o[1]), b = __floats2half2_rn(o[2], o[3]);
    uint2 v;
    v.x = *reinterpret_cast<const uint32_t*>(&a);
    v.y = *reinterpret_cast<const uint32_t*>(&b);
    *reinterpret_cast<uint2*>(p) = v;
}

__device__ __forceinline__ float loss_term(float d, int kind, float invn, float& g) {
    if (kind == SVDLUT_LOSS_L1) {
        g = d > 0.f ? invn : (d < 0.f ? -invn : 0.f);
        return fabsf(d);
    }
    g = 2.f * d * invn;
    return d * d;
}

// Stage 1: per-block partial sums (fixed grid-stride order over groups of four elements,
// vector loads when the buffers allow) and the gradient.
template <typename T>
__global__ void __launch_bounds__(kLossThreads) loss_partial_kernel(const T* __restrict__ y,
                                                                     const T* __restrict__ t, int64_t n,
                                                                     int kind, T* __restrict__ dy,
                                                                     float* __restrict__ partial) {
    __shared__ float red[kLossThreads / 64];
    const float invn = 1.f / static_cast<float>(n);
    constexpr uintptr_t kAlign = 4 * sizeof(T) - 1;
    const bool vec = ((reinterpret_cast<uintptr_t>(y) | reinterpret_cast<uintptr_t>(t) |
                       reinterpret_cast<uintptr_t>(dy)) & kAlign) == 0;
    const int64_t n4 = n / 4;
    const int64_t tid = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    float acc = 0.f;
    for (int64_t q = tid; q < n4; q += stride) {
        const int64_t i = 4 * q;
        float a[4], b[4], g[4];
        if (vec) {
            ld4(y + i, a);
            ld4(t + i, b);
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) { a[k] = tof<T>(y[i + k]); b[k] = tof<T>(t[i + k]); }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) acc += loss_term(a[k] - b[k], kind, invn, g[k]);
        if (dy) {
            if (vec) st4(dy + i, g);
            else
#pragma unroll
                for (int k = 0; k < 4; ++k) dy[i + k] = fromf<T>(g[k]);
        }
    }
    if (tid < n - 4 * n4) {               // the last n mod 4 elements
        const int64_t i = 4 * n4 + tid;
        float g;
        acc += loss_term(tof<T>(y[i]) - tof<T>(t[i]), kind, invn, g);
        if (dy) dy[i] = fromf<T>(g);
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int i = 0; i < kLossThreads / 64; ++i) s += red[i];
        partial[blockIdx.x] = s;
    }
}

// Stage 2: one wave sums the partials in a fixed order.
__global__ void loss_final_kernel(const float* __restrict__ partial, int nb, int64_t n, float* __restrict__ out) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += 64) acc += partial[i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (threadIdx.x == 0) out[0] = static_cast<float>(acc / static_cast<double>(n));
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float b1, float b2, float eps,
                            float step_size, float inv_sqrt_bc2) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const float gi = g[i];
        const float mi = fmaf(b1, m[i], (1.f - b1) * gi);
        const float vi = fmaf(b2, v[i], (1.f - b2) * gi * gi);
        m[i] = mi;
        v[i] = vi;
        p[i] -= step_size * mi / (sqrtf(vi) * inv_sqrt_bc2 + eps);
    }
}

}  // namespace

int loss_blocks(int64_t n) {
    const int64_t b = (n + kLossThreads * 8 - 1) / (kLossThreads * 8);
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(b, kLossMaxBlocks)));
}

svdlut_status launch_loss(const void* y, const void* t, svdlut_dtype io, int64_t n, int kind, float* loss,
                          void* dy, float* partial, int nb, hipStream_t st) {
    if (io == SVDLUT_F32)
        hipLaunchKernelGGL(loss_partial_kernel<float>, dim3(nb), dim3(kLossThreads), 0, st,
                           static_cast<const float*>(y), static_cast<const float*>(t), n, kind,
                           static_cast<float*>(dy), partial);
    else
        hipLaunchKernelGGL(loss_partial_kernel<__half>, dim3(nb), dim3(kLossThreads), 0, st,
                           static_cast<const __half*>(y), static_cast<const __half*>(t), n, kind,
                           static_cast<__half*>(dy), partial);
    hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(64), 0, st, partial, nb, n, loss);
    return check_launch("loss");
}

}  // namespace svdlut

using namespace svdlut;

extern "C" {

size_t svdlut_loss_workspace_size(int64_t n) {
    if (n < 1) return 0;
    return sizeof(float) * static_cast<size_t>(loss_blocks(n));
}

svdlut_status svdlut_loss(const void* y, const void* target, svdlut_dtype io, int64_t n, svdlut_loss_kind kind,
                          float* loss, void* dy, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!y || !target || !loss || !ws) return fail(SVDLUT_EINVAL, "loss: null pointer");
    if (n < 1) return fail(SVDLUT_EINVAL, "loss: n must be >= 1");
    if (io != SVDLUT_F32 && io != SVDLUT_F16) return fail(SVDLUT_EUNSUPPORTED, "loss: dtype");
    if (kind != SVDLUT_LOSS_L1 && kind != SVDLUT_LOSS_MSE) return fail(SVDLUT_EINVAL, "loss: kind");
    const int nb = loss_blocks(n);
    if (ws_bytes < sizeof(float) * static_cast<size_t>(nb))
        return fail(SVDLUT_EINVAL, "loss: workspace smaller than svdlut_loss_workspace_size()");
    return launch_loss(y, target, io, n, kind, loss, dy, static_cast<float*>(ws), nb, stream);
}

svdlut_status svdlut_adam_step(float* params, const float* grads, float* m, float* v, int64_t n, float lr,
                               float b1, float b2, float eps, int32_t step, hipStream_t stream) {
    if (!params || !grads || !m || !v) return fail(SVDLUT_EINVAL, "adam: null pointer");
    if (n < 1 || step < 1) return fail(SVDLUT_EINVAL, "adam: n and step must be >= 1");
    if (!(lr >= 0.f) || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) || !(eps > 0.f))
        return fail(SVDLUT_EINVAL, "adam: hyper-parameters out of range");
    const double bc1 = 1.0 - std::pow(static_cast<double>(b1), step);
    const double bc2 = 1.0 - std::pow(static_cast<double>(b2), step);
    const float step_size = static_cast<float>(lr / bc1);
    const float inv_sqrt_bc2 = static_cast<float>(1.0 / std::sqrt(bc2));
    const int64_t nb = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(adam_kernel, dim3(static_cast<unsigned>(nb)), dim3(256), 0, stream, params, grads, m, v, n,
                       b1, b2, eps, step_size, inv_sqrt_bc2);
    return check_launch("adam");
}

}  // extern "C"
