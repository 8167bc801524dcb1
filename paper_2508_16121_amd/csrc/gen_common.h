// Shared pieces of the generator networks: bf16 helpers, convolution geometry, implicit-GEMM
// operand loaders for the forward, input-gradient and weight-gradient products, the bf16
// matrix-core GEMM, the bilinear downsample and small reduction kernels.  Convolutions are
// 3x3 with zero padding 1 on NHWC activations; weights are [Cout][3][3][Cin] fp32, rounded
// to bf16 when gathered into the MFMA operand registers.
#pragma once

#include "internal.h"

#include <algorithm>

namespace svdlut {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kNet = 256;            // network input resolution

// ---------------------------------------------------------------- bf16 helpers
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);      // round to nearest, ties to even
    return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }
__device__ __forceinline__ bool bf_pos(uint16_t h) { return h != 0 && !(h & 0x8000u); }

__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
    bf16x4 r;
    r[0] = static_cast<short>(f2bf(a));
    r[1] = static_cast<short>(f2bf(b));
    r[2] = static_cast<short>(f2bf(c));
    r[3] = static_cast<short>(f2bf(d));
    return r;
}

// ---------------------------------------------------------------- geometry
struct ConvGeo {
    int N, Hi, Wi, Ci, Cs;   // input: batch, size, real channels, channel stride in memory
    int Ho, Wo, Co, Cos;     // output: size, real channels, channel stride (multiple of 4)
    int stride;
};


// ---------------------------------------------------------------- operand loaders
// Each loader returns, for one GEMM row (or column) index and a k that is a multiple of 4,
// the four bf16 values at k..k+3 in the lane order the MFMA expects.

// Forward A: im2col of the NHWC input; row = output pixel, k = tap*Cs + ci.
struct FwdA {
    const uint16_t* in;
    ConvGeo g;
    struct Row { int64_t base; int y0, x0; bool valid; };
    __device__ Row row(int m) const {
        Row r;
        r.valid = m < g.N * g.Ho * g.Wo;
        const int mm = r.valid ? m : 0;
        const int n = mm / (g.Ho * g.Wo);
        const int p = mm - n * g.Ho * g.Wo;
        const int yo = p / g.Wo, xo = p - (p / g.Wo) * g.Wo;
        r.y0 = yo * g.stride - 1;
        r.x0 = xo * g.stride - 1;
        r.base = static_cast<int64_t>(n) * g.Hi * g.Wi;
        return r;
    }
    __device__ bf16x4 load(const Row& r, int k) const {
        const int tap = k / g.Cs, ci = k - tap * g.Cs;
        const int ky = tap / 3, kx = tap - 3 * (tap / 3);
        const int y = r.y0 + ky, x = r.x0 + kx;
        bf16x4 v = {0, 0, 0, 0};
        if (r.valid && tap < 9 && y >= 0 && y < g.Hi && x >= 0 && x < g.Wi) {
            const uint2 raw = *reinterpret_cast<const uint2*>(in + (r.base + static_cast<int64_t>(y) * g.Wi + x) * g.Cs + ci);
            v = *reinterpret_cast<const bf16x4*>(&raw);
        }
        return v;
    }
};

// Forward B: weights [Co][3][3][Ci] fp32 -> bf16; column = co, k = tap*Cs + ci.
struct FwdB {
    const float* w;
    ConvGeo g;
    struct Col { int co; };
    __device__ Col col(int n) const { return Col{n}; }
    __device__ bf16x4 load(const Col& c, int k) const {
        const int tap = k / g.Cs, ci = k - tap * g.Cs;
        float v[4] = {0.f, 0.f, 0.f, 0.f};
        if (c.co < g.Co && tap < 9) {
            const float* src = w + (static_cast<int64_t>(c.co) * 9 + tap) * g.Ci;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (ci + j < g.Ci) v[j] = src[ci + j];
        }
        return pack4(v[0], v[1], v[2], v[3]);
    }
};

// Input-gradient A: row = input pixel (n, yi, xi), k = tap*Cos + co; the output pixel that
// reaches (yi, xi) through tap (ky, kx) is yo = (yi + 1 - ky) / stride when divisible.
template <class DZ>
struct DgradA {
    DZ dz;
    ConvGeo g;
    struct Row { int n, yi, xi; bool valid; };
    __device__ Row row(int m) const {
        Row r;
        r.valid = m < g.N * g.Hi * g.Wi;
        const int mm = r.valid ? m : 0;
        r.n = mm / (g.Hi * g.Wi);
        const int p = mm - r.n * g.Hi * g.Wi;
        r.yi = p / g.Wi;
        r.xi = p - r.yi * g.Wi;
        return r;
    }
    __device__ bf16x4 load(const Row& r, int k) const {
        const int tap = k / g.Cos, co = k - tap * g.Cos;
        const int ky = tap / 3, kx = tap - 3 * (tap / 3);
        const int ty = r.yi + 1 - ky, tx = r.xi + 1 - kx;
        float v[4] = {0.f, 0.f, 0.f, 0.f};
        if (r.valid && tap < 9 && ty >= 0 && tx >= 0 && ty % g.stride == 0 && tx % g.stride == 0) {
            const int yo = ty / g.stride, xo = tx / g.stride;
            if (yo < g.Ho && xo < g.Wo) {
                const int mo = (r.n * g.Ho + yo) * g.Wo + xo;
#pragma unroll
                for (int j = 0; j < 4; ++j) v[j] = dz(mo, co + j);
            }
        }
        return pack4(v[0], v[1], v[2], v[3]);
    }
};

// Input-gradient B: weights as [(tap, co)][ci]; column = ci.
struct DgradB {
    const float* w;
    ConvGeo g;
    struct Col { int ci; };
    __device__ Col col(int n) const { return Col{n}; }
    __device__ bf16x4 load(const Col& c, int k) const {
        const int tap = k / g.Cos, co = k - tap * g.Cos;
        float v[4] = {0.f, 0.f, 0.f, 0.f};
        if (c.ci < g.Ci && tap < 9) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (co + j < g.Co) v[j] = w[(static_cast<int64_t>(co + j) * 9 + tap) * g.Ci + c.ci];
        }
        return pack4(v[0], v[1], v[2], v[3]);
    }
};

// Weight-gradient A: row = co, k = output pixel m.
template <class DZ>
struct WgradA {
    DZ dz;
    ConvGeo g;
    struct Row { int co; };
    __device__ Row row(int m) const { return Row{m}; }
    __device__ bf16x4 load(const Row& r, int k) const {
        const int M = g.N * g.Ho * g.Wo;
        float v[4] = {0.f, 0.f, 0.f, 0.f};
        if (r.co < g.Co) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (k + j < M) v[j] = dz(k + j, r.co);
        }
        return pack4(v[0], v[1], v[2], v[3]);
    }
};

// Weight-gradient B: row k = output pixel m, column = tap*Cs + ci (the im2col value).
struct WgradB {
    const uint16_t* in;
    ConvGeo g;
    struct Col { int tap, ci; bool valid; };
    __device__ Col col(int n) const {
        Col c;
        c.tap = n / g.Cs;
        c.ci = n - c.tap * g.Cs;
        c.valid = c.tap < 9 && c.ci < g.Ci;
        return c;
    }
    __device__ bf16x4 load(const Col& c, int k) const {
        const int M = g.N * g.Ho * g.Wo;
        bf16x4 v = {0, 0, 0, 0};
        if (!c.valid || k >= M) return v;
        const int ky = c.tap / 3, kx = c.tap - 3 * (c.tap / 3);
        if ((g.Wo & 3) == 0) {
            // k is a multiple of 4 and Wo of 4: the four pixels k..k+3 lie in one output row
            const int HoWo = g.Ho * g.Wo;
            const int n = k / HoWo;
            const int p = k - n * HoWo;
            const int yo = p / g.Wo, xo = p - (p / g.Wo) * g.Wo;
            const int y = yo * g.stride - 1 + ky;
            if (y < 0 || y >= g.Hi) return v;
            const int64_t row = (static_cast<int64_t>(n) * g.Hi + y) * g.Wi;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int x = (xo + j) * g.stride - 1 + kx;
                if (k + j < M && x >= 0 && x < g.Wi) v[j] = static_cast<short>(in[(row + x) * g.Cs + c.ci]);
            }
            return v;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = k + j;
            if (m < M) {
                const int n = m / (g.Ho * g.Wo);
                const int p = m - n * g.Ho * g.Wo;
                const int yo = p / g.Wo, xo = p - (p / g.Wo) * g.Wo;
                const int y = yo * g.stride - 1 + ky, x = xo * g.stride - 1 + kx;
                if (y >= 0 && y < g.Hi && x >= 0 && x < g.Wi)
                    v[j] = static_cast<short>(in[((static_cast<int64_t>(n) * g.Hi + y) * g.Wi + x) * g.Cs + c.ci]);
            }
        }
        return v;
    }
};

// ---------------------------------------------------------------- epilogues
struct EpiStore {        // plain fp32 store (or accumulate) of an NHWC gradient
    float* out;
    int M, C, accumulate;
    __device__ void operator()(int m, int c, float v) const {
        if (m < M && c < C) {
            float* p = out + static_cast<int64_t>(m) * C + c;
            *p = accumulate ? *p + v : v;
        }
    }
};

// ---------------------------------------------------------------- the MFMA GEMM
// C[M][N] = sum_k A[m][k] B[k][n].  Workgroup = 4 waves; wave w owns rows
// blockIdx.x*64 + 16w .. +15 and columns blockIdx.y*16*NT .. +16*NT-1 (NT 16x16 tiles),
// over the k range [blockIdx.z*kchunk, +kchunk).  Per 16-wide k step each lane loads its
// four A values (row lane%16, k lane/16*4..+3) and, per tile, four B values (column
// lane%16, same k) and issues one v_mfma_f32_16x16x16_bf16; accumulator element i of lane
// l is C[4*(l/16)+i][l%16].
template <int NT, class AL, class BL, class EP>
__global__ void __launch_bounds__(256) mfma_gemm_kernel(AL al, BL bl, EP ep, int K, int kchunk) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m0 = blockIdx.x * 64 + wave * 16;
    const int n0 = blockIdx.y * 16 * NT;
    const int kb = blockIdx.z * kchunk;
    const int ke = min(K, kb + kchunk);
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const typename AL::Row ar = al.row(m0 + (lane & 15));
    typename BL::Col bc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) bc[t] = bl.col(n0 + 16 * t + (lane & 15));
    const int kl = 4 * (lane >> 4);
    // operands of step k + 16 are gathered while the matrix cores work on step k
    bf16x4 a = al.load(ar, kb + kl);
    bf16x4 b[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) b[t] = bl.load(bc[t], kb + kl);
    for (int k = kb; k < ke; k += 16) {
        bf16x4 an = {0, 0, 0, 0};
        bf16x4 bn[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) bn[t] = bf16x4{0, 0, 0, 0};
        if (k + 16 < ke) {
            an = al.load(ar, k + 16 + kl);
#pragma unroll
            for (int t = 0; t < NT; ++t) bn[t] = bl.load(bc[t], k + 16 + kl);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[t], acc[t], 0, 0, 0);
        a = an;
#pragma unroll
        for (int t = 0; t < NT; ++t) b[t] = bn[t];
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) ep(m0 + 4 * (lane >> 4) + i, n0 + 16 * t + (lane & 15), acc[t][i]);
}

// k range per workgroup and number of k slices for a requested split of a K-long reduction
inline int gemm_kchunk(int K, int splitk) {
    const int Kp = (K + 15) / 16 * 16;
    return ((Kp + splitk - 1) / splitk + 15) / 16 * 16;
}
inline int gemm_slices(int K, int splitk) {
    const int Kp = (K + 15) / 16 * 16;
    const int kc = gemm_kchunk(K, splitk);
    return (Kp + kc - 1) / kc;
}

template <int NT, class AL, class BL, class EP>
void gemm(AL al, BL bl, EP ep, int M, int N, int K, int splitk, hipStream_t st) {
    const int Kp = (K + 15) / 16 * 16;
    const int kchunk = gemm_kchunk(K, splitk);
    const int gz = gemm_slices(K, splitk);
    dim3 grid((M + 63) / 64, (N + 16 * NT - 1) / (16 * NT), gz);
    hipLaunchKernelGGL((mfma_gemm_kernel<NT, AL, BL, EP>), grid, dim3(256), 0, st, al, bl, ep, Kp, kchunk);
}

// ---------------------------------------------------------------- other kernels
// Bilinear resize (half-pixel centres, no antialias) of planar [B][3][H][W] to NHWC bf16
// [B][256][256][4] (channel 3 = 0).  Source index and weight come from integers:
// src*2O = (2*dst + 1)*N - O, clamped at 0, so they are exact.
template <typename IO>
__global__ void downsample_kernel(const IO* __restrict__ x, uint16_t* __restrict__ out, int B, int H, int W) {
    const int64_t total = static_cast<int64_t>(B) * kNet * kNet;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int b = static_cast<int>(i / (kNet * kNet));
        const int p = static_cast<int>(i - static_cast<int64_t>(b) * kNet * kNet);
        const int oy = p / kNet, ox = p - (p / kNet) * kNet;
        const int64_t ny = std::max<int64_t>(0, static_cast<int64_t>(2 * oy + 1) * H - kNet);
        const int64_t nx = std::max<int64_t>(0, static_cast<int64_t>(2 * ox + 1) * W - kNet);
        const int y0 = min(static_cast<int>(ny / (2 * kNet)), H - 1);
        const int x0 = min(static_cast<int>(nx / (2 * kNet)), W - 1);
        const float ly = static_cast<float>(ny - static_cast<int64_t>(y0) * 2 * kNet) * (1.f / (2 * kNet));
        const float lx = static_cast<float>(nx - static_cast<int64_t>(x0) * 2 * kNet) * (1.f / (2 * kNet));
        const int y1 = min(y0 + 1, H - 1), x1 = min(x0 + 1, W - 1);
        uint16_t o[4] = {0, 0, 0, 0};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const IO* pl = x + (static_cast<int64_t>(b) * 3 + c) * H * W;
            auto at = [&](int yy, int xx) {
                const IO v = pl[static_cast<int64_t>(yy) * W + xx];
                return static_cast<float>(v);
            };
            const float top = at(y0, x0) * (1.f - lx) + at(y0, x1) * lx;
            const float bot = at(y1, x0) * (1.f - lx) + at(y1, x1) * lx;
            o[c] = f2bf(top * (1.f - ly) + bot * ly);
        }
        uint2 v;
        v.x = o[0] | (static_cast<uint32_t>(o[1]) << 16);
        v.y = o[2] | (static_cast<uint32_t>(o[3]) << 16);
        *reinterpret_cast<uint2*>(out + i * 4) = v;
    }
}

// Bias gradient db[co] = sum of dz(m, co) over the output pixels, in a fixed order.  256
// threads: thread t takes channel t % Co and pixel lane t / Co (256 / Co lanes, 16 pixels
// each); workgroup g takes chunks g, g + G, ... of nl * 16 pixels, adds its lanes in LDS and
// stores one partial per channel; bias_sum_kernel adds the G partials in workgroup order.
constexpr int kBiasPx = 16;
constexpr int kBiasGroups = 1024;

inline int bias_lanes(int Co) { return std::max(1, 256 / Co); }

template <class DZ>
__global__ void __launch_bounds__(256) bias_grad_kernel(DZ dz, float* __restrict__ part, int M, int Co) {
    __shared__ float red[256];
    const int t = threadIdx.x, nl = max(1, 256 / Co);
    const int co = t % Co, lane = t / Co;
    const int chunk = nl * kBiasPx;
    float acc = 0.f;
    if (lane < nl && t < Co * nl)
        for (int m0 = blockIdx.x * chunk; m0 < M; m0 += gridDim.x * chunk) {
            // the chunk's kBiasPx pixels of this lane: all loads in flight, then added in order
            float v[kBiasPx];
#pragma unroll
            for (int q = 0; q < kBiasPx; ++q) {
                const int m = m0 + lane + q * nl;
                v[q] = m < M ? dz(m, co) : 0.f;
            }
#pragma unroll
            for (int q = 0; q < kBiasPx; ++q) acc += v[q];
        }
    red[t] = acc;
    __syncthreads();
    if (t < Co) {
        float s = 0.f;
        for (int l = 0; l < nl; ++l) s += red[l * Co + t];
        part[static_cast<int64_t>(blockIdx.x) * Co + t] = s;
    }
}

// db[c] = sum over g of part[g][c] (Co <= 256, one workgroup of 256 threads): thread (c, l)
// adds rows l, l + L, ... in order (L = 256 / Co lanes per channel, loads issued eight at a
// time), then the L lane sums of each channel are added in lane order.
__global__ void __launch_bounds__(256) bias_sum_kernel(const float* __restrict__ part, int groups, int Co,
                                                       float* __restrict__ db) {
    __shared__ float red[256];
    const int t = threadIdx.x, L = max(1, 256 / Co), c = t % Co, l = t / Co;
    float s = 0.f;
    if (l < L)
#pragma unroll 8
        for (int g = l; g < groups; g += L) s += part[static_cast<int64_t>(g) * Co + c];
    red[t] = s;
    __syncthreads();
    if (t < Co) {
        float v = 0.f;
        for (int i = 0; i < L; ++i) v += red[i * Co + t];
        db[t] = v;
    }
}

// dW[co][tap][ci] = sum over the split-K slices of part[z][co][tap * Cs + ci]: one wave per
// output element, lane l adds slices l, l + 64, ... and a fixed butterfly adds the lanes, so
// the result does not depend on scheduling.
__global__ void __launch_bounds__(256) wgrad_reduce_kernel(const float* __restrict__ part, int slices,
                                                           float* __restrict__ dw, int Co, int Ci, int Cs) {
    const int N = 9 * Cs;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= Co * N) return;          // wave-uniform
    const int64_t stride = static_cast<int64_t>(Co) * N;
    float acc = 0.f;
    for (int z = lane; z < slices; z += 64) acc += part[z * stride + i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    const int co = i / N, n = i - co * N;
    const int tap = n / Cs, ci = n - tap * Cs;
    if (lane == 0 && ci < Ci) dw[(static_cast<int64_t>(co) * 9 + tap) * Ci + ci] = acc;
}

// The same sums for split-K partials of up to kWgradColumnsMax slices: a workgroup of 64 x nw
// threads takes 64 consecutive entries (consecutive addresses in every slice), wave w adds
// the slices [w S / nw, (w + 1) S / nw) of its lane's entry in order with eight loads in
// flight, and the waves' sums are added in wave order.
constexpr int kWgradColumnsMax = 512;
__global__ void __launch_bounds__(1024) wgrad_reduce_cols_kernel(const float* __restrict__ part, int slices,
                                                                float* __restrict__ dw, int Co, int Ci, int Cs) {
    __shared__ float red[16][kWave];
    const int N = 9 * Cs;
    const int64_t total = static_cast<int64_t>(Co) * N;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kWave + lane;
    const int z0 = static_cast<int>(static_cast<int64_t>(slices) * wave / nw);
    const int z1 = static_cast<int>(static_cast<int64_t>(slices) * (wave + 1) / nw);
    float acc = 0.f;
    if (i < total) {
        int z = z0;
        for (; z + 8 <= z1; z += 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = part[(z + u) * total + i];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += v[u];
        }
        for (; z < z1; ++z) acc += part[z * total + i];
    }
    red[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && i < total) {
        float sum = red[0][lane];
        for (int w = 1; w < nw; ++w) sum += red[w][lane];
        const int co = static_cast<int>(i / N), n = static_cast<int>(i - static_cast<int64_t>(co) * N);
        const int tap = n / Cs, ci = n - tap * Cs;
        if (ci < Ci) dw[(static_cast<int64_t>(co) * 9 + tap) * Ci + ci] = sum;
    }
}

__global__ void zero_f32_kernel(float* p, int64_t n) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = 0.f;
}

template <class AL, class BL, class EP>
void gemm_nt(int ncols, AL al, BL bl, EP ep, int M, int K, int splitk, hipStream_t st) {
    if (ncols <= 16) gemm<1>(al, bl, ep, M, ncols, K, splitk, st);
    else if (ncols <= 32) gemm<2>(al, bl, ep, M, ncols, K, splitk, st);
    else gemm<4>(al, bl, ep, M, ncols, K, splitk, st);
}

// Split-K.  A launch with few workgroups cannot hide its operand gathers, and each of its
// waves walks the whole reduction.  An M x N x K product whose plain launch (gemm_nt's tile
// width) has fewer than kNoSplitWgs workgroups and a reduction of at least 16 k steps is
// split into slices of at least four k steps, run with 16-column tiles, until about
// kSplitTarget workgroups run.  Each slice writes its partial product to part[slice][m][n];
// a second kernel sums the slices in fixed order.  Returns the split (1 = none).
constexpr int kNoSplitWgs = 512;
constexpr int kSplitTarget = 1024;

inline int gemm_nt_tiles(int ncols) { return ncols <= 16 ? 1 : (ncols <= 32 ? 2 : 4); }

inline int long_k_splits(int M, int N, int K) {
    const int ksteps = (K + 15) / 16;
    const int wgs16 = ((M + 63) / 64) * ((N + 15) / 16);
    const int nt = gemm_nt_tiles(N);
    const int wgs_nt = ((M + 63) / 64) * ((N + 16 * nt - 1) / (16 * nt));
    if (wgs_nt >= kNoSplitWgs || ksteps < 16) return 1;
    return std::max(1, std::min(ksteps / 4, (kSplitTarget + wgs16 - 1) / wgs16));
}

// Forward convolutions: layers with very few output tiles (fewer than 128 16-column tiles)
// split into slices of at least two k steps until about 256 workgroups run (the partials are
// then summed with the bias and the activation); the others follow long_k_splits.
inline int fwd_splits(int M, int N, int K) {
    const int ksteps = (K + 15) / 16;
    const int wgs = ((M + 63) / 64) * ((N + 15) / 16);
    if (wgs < 128) return std::max(1, std::min(ksteps / 2, (256 + wgs - 1) / wgs));
    return long_k_splits(M, N, K);
}

struct EpiPartial {
    float* part;
    int M, N;
    __device__ void operator()(int m, int n, float v) const {
        if (m < M && n < N) part[(static_cast<int64_t>(blockIdx.z) * M + m) * N + n] = v;
    }
};

size_t align256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

// Weight gradient split: the Co x 9Cs product reduces over all output pixels, so it is split
// into slices (at least four k steps each) until about 2048 workgroups run; each slice stores
// its partial product and wgrad_reduce_kernel adds them in fixed order.
inline int wgrad_splits(const ConvGeo& g) {
    const int Mo = g.N * g.Ho * g.Wo;
    const int wgs = ((g.Co + 63) / 64) * ((9 * g.Cs + 63) / 64);
    const int ksteps = (Mo + 15) / 16;
    return std::max(1, std::min(ksteps / 4, (2048 + wgs - 1) / wgs));
}

// floats of split-K partials the weight gradient of layer g needs
inline size_t wgrad_part_floats(const ConvGeo& g) {
    const int Mo = g.N * g.Ho * g.Wo;
    return static_cast<size_t>(gemm_slices(Mo, wgrad_splits(g))) * g.Co * 9 * g.Cs;
}

// Input gradient of layer g (an Mi x Ci x 9Cos product): its split, and the floats of its
// partials ([slice][Mi][Cs]; 0 without a split)
inline int dgrad_splits(const ConvGeo& g) { return long_k_splits(g.N * g.Hi * g.Wi, g.Ci, 9 * g.Cos); }
inline size_t dgrad_part_floats(const ConvGeo& g) {
    const int sk = dgrad_splits(g);
    if (sk <= 1) return 0;
    return static_cast<size_t>(gemm_slices(9 * g.Cos, sk)) * g.N * g.Hi * g.Wi * g.Cs;
}

// scratch a layer's backward needs for its split-K partials (weight and input gradients,
// used one after the other)
inline size_t bwd_part_floats(const ConvGeo& g) { return std::max(wgrad_part_floats(g), dgrad_part_floats(g)); }

// out[i] (= or +=) sum over the slices of part[z][i], in slice order, for the M x C input
// gradient of a split convolution
__global__ void __launch_bounds__(256) dgrad_reduce_kernel(const float* __restrict__ part, int slices,
                                                           float* __restrict__ out, int64_t n, int accumulate) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    float v = 0.f;
    for (int z = 0; z < slices; ++z) v += part[z * n + i];
    out[i] = accumulate ? out[i] + v : v;
}

// wpart: scratch of at least bwd_part_floats(g) floats.
template <class DZ>
void conv_backward(const ConvGeo& g, DZ dz, const uint16_t* in, const float* w, float* dw, float* db,
                   float* da_in, int accumulate_da, float* wpart, hipStream_t st) {
    const int Mo = g.N * g.Ho * g.Wo;
    const int N = 9 * g.Cs;
    const int sk = wgrad_splits(g);
    gemm<4>(WgradA<DZ>{dz, g}, WgradB{in, g}, EpiPartial{wpart, g.Co, N}, g.Co, N, Mo, sk, st);
    const int slices = gemm_slices(Mo, sk);
    if (slices <= kWgradColumnsMax) {   // one lane per weight, waves over the slices
        const int nw = std::min(16, std::max(1, (slices + 31) / 32));
        hipLaunchKernelGGL(wgrad_reduce_cols_kernel, dim3((g.Co * N + kWave - 1) / kWave), dim3(kWave * nw), 0, st,
                           wpart, slices, dw, g.Co, g.Ci, g.Cs);
    } else {                            // one wave per weight, lanes over the slices
        hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((g.Co * N + 3) / 4), dim3(256), 0, st, wpart, slices, dw, g.Co,
                           g.Ci, g.Cs);
    }
    // the weight-gradient partials are consumed by now: wpart takes the bias partials
    const int px_per_wg = bias_lanes(g.Co) * kBiasPx;
    const int groups = static_cast<int>(std::max<size_t>(
        1, std::min<size_t>({static_cast<size_t>((Mo + px_per_wg - 1) / px_per_wg), static_cast<size_t>(kBiasGroups),
                             wgrad_part_floats(g) / g.Co})));
    hipLaunchKernelGGL(bias_grad_kernel<DZ>, dim3(groups), dim3(256), 0, st, dz, wpart, Mo, g.Co);
    hipLaunchKernelGGL(bias_sum_kernel, dim3(1), dim3(256), 0, st, wpart, groups, g.Co, db);
    if (da_in) {
        const int Mi = g.N * g.Hi * g.Wi;
        const int skd = dgrad_splits(g);
        if (skd > 1) {   // wpart is free again once the bias partials are summed
            gemm<1>(DgradA<DZ>{dz, g}, DgradB{w, g}, EpiPartial{wpart, Mi, g.Cs}, Mi, g.Ci, 9 * g.Cos, skd, st);
            const int64_t n = static_cast<int64_t>(Mi) * g.Cs;
            hipLaunchKernelGGL(dgrad_reduce_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st,
                               wpart, gemm_slices(9 * g.Cos, skd), da_in, n, accumulate_da);
        } else {
            gemm_nt(g.Ci, DgradA<DZ>{dz, g}, DgradB{w, g}, EpiStore{da_in, Mi, g.Cs, accumulate_da}, Mi,
                    9 * g.Cos, 1, st);
        }
    }
}

}  // namespace

}  // namespace svdlut
