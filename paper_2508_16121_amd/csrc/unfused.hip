// The unfused "original structure" the paper starts from (Sec. "Preliminary"): slicing of the
// bilateral grids into K spatial-feature planes f_s written to HBM (Eq. slicing), a 1x1
// convolution of concat(X, f_s) into the fused image X_bar written to HBM (Eq. fusion), and a
// 3D-LUT transform of X_bar by trilinear interpolation (Eq. coloren).  A baseline: it
// measures on this GPU what the intermediate planes cost against the fused pass.
//
// Three kernels, each a streaming pass over the pixels with 4 consecutive pixels per thread
// (float4 planes when the rows allow it):
//   slice_fs_kernel  reads X (12 B/px), writes f_s (4K B/px); the K grids' planes in LDS
//   fuse_kernel      reads X and f_s, writes X_bar (12 B/px)
//   lut3d_kernel     reads X_bar, writes Y; the 3D LUTs packed as one float4 per vertex
//                    (the three output channels and a pad) in the workspace, read through L2.
//
// The same file holds the other LUT dimensions the paper weighs the 2D decomposition against
// (Sec. "Preliminary", the LUT-dimension analysis): a standalone 3D-LUT transform of X
// (lut3d_kernel on the input) and a per-channel 1D-LUT transform (lut1d_kernel, the three
// curves in LDS).
#include "internal.h"
#include "lut_common.h"

#include <algorithm>

namespace svdlut {

namespace {

constexpr int kUfBlock = 256;

// Pixels [p0, p0+4) of a plane of n pixels: vector access when the plane base is 16-byte
// aligned and all four are inside, element accesses otherwise.
__device__ __forceinline__ void uf_load4(const float* pl, int64_t p0, int64_t n, bool vec, float (&o)[4]) {
    if (vec && p0 + 4 <= n) {
        const float4 v = *reinterpret_cast<const float4*>(pl + p0);
        o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k] = pl[min(p0 + k, n - 1)];
    }
}
__device__ __forceinline__ void uf_store4(float* pl, int64_t p0, int64_t n, bool vec, const float (&o)[4]) {
    if (vec && p0 + 4 <= n) {
        *reinterpret_cast<float4*>(pl + p0) = make_float4(o[0], o[1], o[2], o[3]);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (p0 + k < n) pl[p0 + k] = o[k];
    }
}

// Left vertex (float) and weight of the LUT decode with n vertices.
__device__ __forceinline__ void uf_decode(float v, float nm1, float nm2, float& f, float& d) {
    const float q = fminf(fmaxf(v, 0.f), 1.f) * nm1;
    f = fminf(floorf(q), nm2);
    d = q - f;
}

// f_s of image blockIdx.y: Psi^k = w_xy psi_xy + w_xc psi_xc + w_yc psi_yc + b^k per pixel.
__global__ void __launch_bounds__(kUfBlock) slice_fs_kernel(const float* __restrict__ x, float* __restrict__ fs,
                                                            const float* __restrict__ grids,
                                                            const float* __restrict__ gw,
                                                            const float* __restrict__ gb, int H, int W, int K,
                                                            int Ds) {
    extern __shared__ float gl[];              // [K][3][Ds][Dsp]
    const int b = blockIdx.y;
    const int Dsp = grid_plane_stride(Ds), PL = Ds * Dsp;
    const float* gsrc = grids + static_cast<size_t>(b) * K * 3 * Ds * Ds;
    for (int e = threadIdx.x; e < K * 3 * Ds * Ds; e += blockDim.x) {
        const int kp = e / (Ds * Ds), r = e - kp * (Ds * Ds);
        const int i = r / Ds, j = r - i * Ds;
        gl[kp * PL + i * Dsp + j] = gsrc[e];
    }
    __syncthreads();
    const int64_t n = static_cast<int64_t>(H) * W;
    const float* xb = x + static_cast<int64_t>(b) * 3 * n;
    float* fb = fs + static_cast<int64_t>(b) * K * n;
    const bool vec = (W & 3) == 0 && ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(fs)) & 15) == 0;
    const float Dsm1 = static_cast<float>(Ds - 1), Dsm2 = static_cast<float>(Ds - 2);
    const AxisMap gax = make_axis(W, Ds), gay = make_axis(H, Ds);
    const float* wb = gw + static_cast<size_t>(b) * K * 3;
    const float* bb = gb + static_cast<size_t>(b) * K;
    for (int64_t p0 = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) * 4; p0 < n;
         p0 += static_cast<int64_t>(gridDim.x) * blockDim.x * 4) {
        float px[3][4];
#pragma unroll
        for (int c = 0; c < 3; ++c) uf_load4(xb + c * n, p0, n, vec, px[c]);
        float fx[4], dx[4], fy[4], dy[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t p = min(p0 + k, n - 1);
            const int yy = static_cast<int>(p / W), xx = static_cast<int>(p - static_cast<int64_t>(yy) * W);
            int i; uint32_t r;
            axis_left(gax, xx, i, r);
            fx[k] = static_cast<float>(i); dx[k] = static_cast<float>(r) * gax.inv;
            axis_left(gay, yy, i, r);
            fy[k] = static_cast<float>(i); dy[k] = static_cast<float>(r) * gay.inv;
        }
        for (int kk = 0; kk < K; ++kk) {
            const int c = kk % 3;
            const float* G = gl + kk * 3 * PL;
            const float w0 = wb[3 * kk], w1 = wb[3 * kk + 1], w2 = wb[3 * kk + 2], bias = bb[kk];
            float o[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float fc, dc;
                uf_decode(px[c][k], Dsm1, Dsm2, fc, dc);
                const int ix = static_cast<int>(fx[k]), iy = static_cast<int>(fy[k]), ic = static_cast<int>(fc);
                auto bil = [&](const float* t, float a, float bw) {
                    return (1.f - a) * (1.f - bw) * t[0] + a * (1.f - bw) * t[Dsp] + (1.f - a) * bw * t[1] +
                           a * bw * t[Dsp + 1];
                };
                const float vxy = bil(G + ix * Dsp + iy, dx[k], dy[k]);
                const float vxc = bil(G + PL + ix * Dsp + ic, dx[k], dc);
                const float vyc = bil(G + 2 * PL + iy * Dsp + ic, dy[k], dc);
                o[k] = fmaf(w0, vxy, fmaf(w1, vxc, fmaf(w2, vyc, bias)));
            }
            uf_store4(fb + kk * n, p0, n, vec, o);
        }
    }
}

// X_bar_c = sum_j Wf[c][j] in_j + bf[c], in = (r, g, b, f_0 .. f_{K-1}).
__global__ void __launch_bounds__(kUfBlock) fuse_kernel(const float* __restrict__ x, const float* __restrict__ fs,
                                                        float* __restrict__ xbar, const float* __restrict__ Wf,
                                                        const float* __restrict__ bf, int64_t n, int K) {
    const int b = blockIdx.y;
    const float* xb = x + static_cast<int64_t>(b) * 3 * n;
    const float* fb = fs + static_cast<int64_t>(b) * K * n;
    float* ob = xbar + static_cast<int64_t>(b) * 3 * n;
    const float* wb = Wf + static_cast<size_t>(b) * 3 * (K + 3);
    const bool vec = (n & 3) == 0 && ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(fs) |
                                       reinterpret_cast<uintptr_t>(xbar)) & 15) == 0;
    for (int64_t p0 = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) * 4; p0 < n;
         p0 += static_cast<int64_t>(gridDim.x) * blockDim.x * 4) {
        float acc[3][4];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[c][k] = bf[3 * b + c];
        for (int j = 0; j < K + 3; ++j) {
            float v[4];
            uf_load4(j < 3 ? xb + j * n : fb + (j - 3) * n, p0, n, vec, v);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int k = 0; k < 4; ++k) acc[c][k] = fmaf(wb[c * (K + 3) + j], v[k], acc[c][k]);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) uf_store4(ob + c * n, p0, n, vec, acc[c]);
    }
}

// T3 [B][3][D][D][D] -> packed [B][D][D][D] float4 (t^0, t^1, t^2, 0).
__global__ void pack_lut3d_kernel(const float* __restrict__ T3, float4* __restrict__ packed, int B, int D) {
    const int64_t nv = static_cast<int64_t>(D) * D * D;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < B * nv;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t b = e / nv, v = e - b * nv;
        const float* t = T3 + b * 3 * nv;
        packed[e] = make_float4(t[v], t[nv + v], t[2 * nv + v], 0.f);
    }
}

// Y_c = trilinear lookup of t^c at X_bar (all three output channels per vertex read).
__global__ void __launch_bounds__(kUfBlock) lut3d_kernel(const float* __restrict__ xbar, float* __restrict__ y,
                                                         const float4* __restrict__ packed, int64_t n, int D) {
    const int b = blockIdx.y;
    const float* xb = xbar + static_cast<int64_t>(b) * 3 * n;
    float* yb = y + static_cast<int64_t>(b) * 3 * n;
    const float4* T = packed + static_cast<int64_t>(b) * D * D * D;
    const bool vec = (n & 3) == 0 && ((reinterpret_cast<uintptr_t>(xbar) | reinterpret_cast<uintptr_t>(y)) & 15) == 0;
    const float Dm1 = static_cast<float>(D - 1), Dm2 = static_cast<float>(D - 2);
    for (int64_t p0 = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) * 4; p0 < n;
         p0 += static_cast<int64_t>(gridDim.x) * blockDim.x * 4) {
        float px[3][4], out[3][4];
#pragma unroll
        for (int c = 0; c < 3; ++c) uf_load4(xb + c * n, p0, n, vec, px[c]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float f[3], d[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) uf_decode(px[c][k], Dm1, Dm2, f[c], d[c]);
            const int base = (static_cast<int>(f[0]) * D + static_cast<int>(f[1])) * D + static_cast<int>(f[2]);
            float acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int bb = 0; bb < 2; ++bb)
#pragma unroll
                    for (int cc = 0; cc < 2; ++cc) {
                        const float w = (a ? d[0] : 1.f - d[0]) * (bb ? d[1] : 1.f - d[1]) * (cc ? d[2] : 1.f - d[2]);
                        const float4 t = T[base + (a * D + bb) * D + cc];
                        acc[0] = fmaf(w, t.x, acc[0]);
                        acc[1] = fmaf(w, t.y, acc[1]);
                        acc[2] = fmaf(w, t.z, acc[2]);
                    }
#pragma unroll
            for (int c = 0; c < 3; ++c) out[c][k] = acc[c];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) uf_store4(yb + c * n, p0, n, vec, out[c]);
    }
}

// Y_c = linear interpolation of the 1D LUT t_c (D vertices) at X_c, per pixel.
__global__ void __launch_bounds__(kUfBlock) lut1d_kernel(const float* __restrict__ x, float* __restrict__ y,
                                                         const float* __restrict__ T1, int64_t n, int D) {
    __shared__ float t[3 * (kMaxD + 1)];
    const int b = blockIdx.y;
    for (int i = threadIdx.x; i < 3 * D; i += blockDim.x) t[(i / D) * (kMaxD + 1) + i % D] = T1[b * 3 * D + i];
    __syncthreads();
    const float* xb = x + static_cast<int64_t>(b) * 3 * n;
    float* yb = y + static_cast<int64_t>(b) * 3 * n;
    const bool vec = (n & 3) == 0 && ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 15) == 0;
    const float Dm1 = static_cast<float>(D - 1), Dm2 = static_cast<float>(D - 2);
    for (int64_t p0 = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) * 4; p0 < n;
         p0 += static_cast<int64_t>(gridDim.x) * blockDim.x * 4) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float px[4], out[4];
            uf_load4(xb + c * n, p0, n, vec, px);
            const float* tc = t + c * (kMaxD + 1);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float f, d;
                uf_decode(px[k], Dm1, Dm2, f, d);
                const int i = static_cast<int>(f);
                out[k] = fmaf(d, tc[i + 1] - tc[i], tc[i]);
            }
            uf_store4(yb + c * n, p0, n, vec, out);
        }
    }
}

int stream_blocks(int64_t n, int B) {
    const DeviceInfo& di = device_info();
    const int64_t quads = (n + 3) / 4;
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(
        (quads + kUfBlock - 1) / kUfBlock, static_cast<int64_t>(di.cus) * 8 / std::max(B, 1) + 1)));
}

}  // namespace

size_t lut3d_workspace_bytes(int B, int D) { return sizeof(float4) * static_cast<size_t>(B) * D * D * D; }

svdlut_status launch_lut3d(const float* x, float* y, const float* T3, int B, int H, int W, int D, void* ws,
                           hipStream_t st) {
    const int64_t n = static_cast<int64_t>(H) * W;
    float4* packed = static_cast<float4*>(ws);
    hipLaunchKernelGGL(pack_lut3d_kernel, dim3(64), dim3(256), 0, st, T3, packed, B, D);
    hipLaunchKernelGGL(lut3d_kernel, dim3(stream_blocks(n, B), B), dim3(kUfBlock), 0, st, x, y, packed, n, D);
    return check_launch("lut3d_apply");
}

svdlut_status launch_lut1d(const float* x, float* y, const float* T1, int B, int H, int W, int D, hipStream_t st) {
    const int64_t n = static_cast<int64_t>(H) * W;
    hipLaunchKernelGGL(lut1d_kernel, dim3(stream_blocks(n, B), B), dim3(kUfBlock), 0, st, x, y, T1, n, D);
    return check_launch("lut1d_apply");
}

size_t unfused_workspace_bytes(int B, int H, int W, int K, int D) {
    const size_t n = static_cast<size_t>(H) * W;
    const size_t fs = static_cast<size_t>(B) * K * n, xb = static_cast<size_t>(B) * 3 * n;
    const size_t lut = static_cast<size_t>(B) * D * D * D * 4;
    return sizeof(float) * (((fs + 63) & ~static_cast<size_t>(63)) + ((xb + 63) & ~static_cast<size_t>(63)) + lut);
}

svdlut_status launch_unfused(const UnfusedLaunch& a, hipStream_t st) {
    const size_t n = static_cast<size_t>(a.H) * a.W;
    float* fs = static_cast<float*>(a.ws);
    float* xbar = fs + ((static_cast<size_t>(a.B) * a.K * n + 63) & ~static_cast<size_t>(63));
    float4* packed = reinterpret_cast<float4*>(xbar + ((static_cast<size_t>(a.B) * 3 * n + 63) & ~static_cast<size_t>(63)));
    const DeviceInfo& di = device_info();
    const int64_t quads = (static_cast<int64_t>(n) + 3) / 4;
    const int bx = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(
        (quads + kUfBlock - 1) / kUfBlock, static_cast<int64_t>(di.cus) * 8 / std::max(a.B, 1) + 1)));
    const size_t lds = sizeof(float) * a.K * 3 * a.Ds * grid_plane_stride(a.Ds);
    hipLaunchKernelGGL(slice_fs_kernel, dim3(bx, a.B), dim3(kUfBlock), lds, st, a.x, fs, a.grids, a.gw, a.gb,
                       a.H, a.W, a.K, a.Ds);
    hipLaunchKernelGGL(fuse_kernel, dim3(bx, a.B), dim3(kUfBlock), 0, st, a.x, fs, xbar, a.Wf, a.bf,
                       static_cast<int64_t>(n), a.K);
    hipLaunchKernelGGL(pack_lut3d_kernel, dim3(64), dim3(256), 0, st, a.T3, packed, a.B, a.D);
    hipLaunchKernelGGL(lut3d_kernel, dim3(bx, a.B), dim3(kUfBlock), 0, st, xbar, a.y, packed,
                       static_cast<int64_t>(n), a.D);
    return check_launch("unfused");
}

}  // namespace svdlut
