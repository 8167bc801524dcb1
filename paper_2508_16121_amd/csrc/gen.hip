// Learned generator of the factors and the spatial map: bilinear downsample, five stride-2
// 3x3 convolutions with ReLU, a 3x3 map head, global average pooling and a fully connected
// factor head; forward and backward.  Convolutions (forward, input gradient and weight
// gradient) are implicit GEMMs on bf16 matrix cores (v_mfma_f32_16x16x16_bf16, fp32
// accumulation); operands are gathered straight from NHWC activations into the MFMA
// register layout.  Activations are stored as bf16; pooling, FC, biases, gradients of the
// activations and all parameter gradients are fp32.
#include "internal.h"

#include <algorithm>
#include <cstring>

namespace svdlut {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kNet = 256;            // network input resolution
constexpr int kConvs = 5;
constexpr int kCh[kConvs + 1] = {3, 16, 32, 64, 128, 128};
constexpr int kHeadIn = 64;          // the map head reads the third conv layer's output
constexpr int kMapC = 9;
constexpr int kMapHW = 32;
constexpr int kGap = 128;

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

// ---------------------------------------------------------------- gradient sources
// dz(m, co): gradient of the loss w.r.t. the conv layer's pre-activation output at output
// pixel m (NHWC order n, y, x) and channel co.
struct DzMasked {           // dz = da * (act > 0), da fp32 NHWC, act bf16 NHWC (post-ReLU)
    const float* da;
    const uint16_t* act;
    int C;
    __device__ float operator()(int m, int co) const {
        const int64_t o = static_cast<int64_t>(m) * C + co;
        return bf_pos(act[o]) ? da[o] : 0.f;
    }
};
struct DzGap {              // dz = g[n][co] / (Ho*Wo) * (act > 0): through global average pooling
    const float* dg;
    const uint16_t* act;
    int C, HW;
    float inv;
    __device__ float operator()(int m, int co) const {
        const int64_t o = static_cast<int64_t>(m) * C + co;
        return bf_pos(act[o]) ? dg[(m / HW) * C + co] * inv : 0.f;
    }
};
struct DzMap {              // dz = dL/dmap, planar [n][9][32][32], linear head
    const float* dmap;
    int C, HW;
    __device__ float operator()(int m, int co) const {
        if (co >= C) return 0.f;
        const int n = m / HW, p = m - (m / HW) * HW;
        return dmap[(static_cast<int64_t>(n) * C + co) * HW + p];
    }
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
        if (!c.valid) return v;
        const int ky = c.tap / 3, kx = c.tap - 3 * (c.tap / 3);
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
struct EpiAct {          // bf16(relu(acc + bias)) into NHWC, channel stride Cos
    uint16_t* out;
    const float* bias;
    int M, Co, Cos;
    __device__ void operator()(int m, int co, float v) const {
        if (m < M && co < Cos) out[static_cast<int64_t>(m) * Cos + co] = co < Co ? f2bf(fmaxf(v + bias[co], 0.f)) : 0;
    }
};
struct EpiMap {          // acc + bias into the planar [n][9][32][32] map (linear head)
    float* out;
    const float* bias;
    int M, C, HW;
    __device__ void operator()(int m, int co, float v) const {
        if (m < M && co < C) {
            const int n = m / HW, p = m - (m / HW) * HW;
            out[(static_cast<int64_t>(n) * C + co) * HW + p] = v + bias[co];
        }
    }
};
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
struct EpiWgrad {        // split-K partial of dW[co][tap][ci] (fp32 atomics)
    float* dw;
    int Co, Ci, Cs;
    __device__ void operator()(int co, int n, float v) const {
        const int tap = n / Cs, ci = n - (n / Cs) * Cs;
        if (co < Co && tap < 9 && ci < Ci)
            __hip_atomic_fetch_add(dw + (static_cast<int64_t>(co) * 9 + tap) * Ci + ci, v, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
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
    for (int k = kb; k < ke; k += 16) {
        const bf16x4 a = al.load(ar, k + kl);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const bf16x4 b = bl.load(bc[t], k + kl);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) ep(m0 + 4 * (lane >> 4) + i, n0 + 16 * t + (lane & 15), acc[t][i]);
}

template <int NT, class AL, class BL, class EP>
void gemm(AL al, BL bl, EP ep, int M, int N, int K, int splitk, hipStream_t st) {
    const int Kp = (K + 15) / 16 * 16;
    int kchunk = (Kp + splitk - 1) / splitk;
    kchunk = (kchunk + 15) / 16 * 16;
    const int gz = (Kp + kchunk - 1) / kchunk;
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

// Global average pool of the last activation: g[n][c] = mean over 8x8 (fp32).
__global__ void gap_kernel(const uint16_t* __restrict__ a, float* __restrict__ g, int B, int HW, int C) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * C) return;
    const int n = i / C, c = i - (i / C) * C;
    float s = 0.f;
    for (int p = 0; p < HW; ++p) s += bf2f(a[(static_cast<int64_t>(n) * HW + p) * C + c]);
    g[i] = s / static_cast<float>(HW);
}

// FC head: o[n][j] = sum_c g[n][c] W[j][c] + b[j], scattered to U, s, V.
__global__ void fc_fwd_kernel(const float* __restrict__ g, const float* __restrict__ Wt,
                              const float* __restrict__ bias, float* __restrict__ U, float* __restrict__ s,
                              float* __restrict__ V, int B, int D, int R) {
    const int nout = 9 * (2 * D * R + R);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * nout) return;
    const int n = i / nout, j = i - (i / nout) * nout;
    const float* gr = g + n * kGap;
    const float* wr = Wt + static_cast<int64_t>(j) * kGap;
    float acc = bias[j];
    for (int c = 0; c < kGap; ++c) acc = fmaf(gr[c], wr[c], acc);
    const int blk = 2 * D * R + R;
    const int l = j / blk, r = j - l * blk;
    if (r < D * R) U[(static_cast<int64_t>(n) * 9 + l) * D * R + r] = acc;
    else if (r < D * R + R) s[(static_cast<int64_t>(n) * 9 + l) * R + (r - D * R)] = acc;
    else V[(static_cast<int64_t>(n) * 9 + l) * D * R + (r - D * R - R)] = acc;
}

// dL/d(FC output) gathered from dU, ds, dV.
__global__ void fc_gather_kernel(const float* __restrict__ dU, const float* __restrict__ ds,
                                 const float* __restrict__ dV, float* __restrict__ dout, int B, int D, int R) {
    const int blk = 2 * D * R + R;
    const int nout = 9 * blk;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * nout) return;
    const int n = i / nout, j = i - (i / nout) * nout;
    const int l = j / blk, r = j - l * blk;
    float v;
    if (r < D * R) v = dU[(static_cast<int64_t>(n) * 9 + l) * D * R + r];
    else if (r < D * R + R) v = ds[(static_cast<int64_t>(n) * 9 + l) * R + (r - D * R)];
    else v = dV[(static_cast<int64_t>(n) * 9 + l) * D * R + (r - D * R - R)];
    dout[i] = v;
}

// dW[j][c] = sum_n dout[n][j] g[n][c];  db[j] = sum_n dout[n][j].
__global__ void fc_wgrad_kernel(const float* __restrict__ dout, const float* __restrict__ g,
                                float* __restrict__ dW, float* __restrict__ db, int B, int nout) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i >= static_cast<int64_t>(nout) * (kGap + 1)) return;
    const int j = static_cast<int>(i / (kGap + 1));
    const int c = static_cast<int>(i - static_cast<int64_t>(j) * (kGap + 1));
    float acc = 0.f;
    for (int n = 0; n < B; ++n) acc = fmaf(dout[static_cast<int64_t>(n) * nout + j], c < kGap ? g[n * kGap + c] : 1.f, acc);
    if (c < kGap) dW[static_cast<int64_t>(j) * kGap + c] = acc;
    else db[j] = acc;
}

// dg[n][c] = sum_j dout[n][j] W[j][c]: one workgroup per n, one thread per c.
__global__ void fc_dgrad_kernel(const float* __restrict__ dout, const float* __restrict__ Wt,
                                float* __restrict__ dg, int nout) {
    const int n = blockIdx.x, c = threadIdx.x;
    const float* d = dout + static_cast<int64_t>(n) * nout;
    float acc = 0.f;
    for (int j = 0; j < nout; ++j) acc = fmaf(d[j], Wt[static_cast<int64_t>(j) * kGap + c], acc);
    dg[n * kGap + c] = acc;
}

// Bias gradient: db[co] += sum over a chunk of 64 output pixels of dz(m, co).
template <class DZ>
__global__ void bias_grad_kernel(DZ dz, float* __restrict__ db, int M, int Co) {
    const int co = threadIdx.x;
    if (co >= Co) return;
    const int m0 = blockIdx.x * 64;
    float acc = 0.f;
    for (int m = m0; m < min(M, m0 + 64); ++m) acc += dz(m, co);
    __hip_atomic_fetch_add(db + co, acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void zero_f32_kernel(float* p, int64_t n) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = 0.f;
}

// ---------------------------------------------------------------- parameter / workspace layout
struct Params {
    const float* w[kConvs];
    const float* b[kConvs];
    const float* hw;
    const float* hb;
    const float* fw;
    const float* fb;
};

template <typename P>
P* carve_params(P* base, int D, int R, P* w[kConvs], P* b[kConvs], P** hw, P** hb, P** fw, P** fb) {
    P* p = base;
    for (int i = 0; i < kConvs; ++i) {
        w[i] = p; p += static_cast<size_t>(kCh[i + 1]) * 9 * kCh[i];
        b[i] = p; p += kCh[i + 1];
    }
    *hw = p; p += static_cast<size_t>(kMapC) * 9 * kHeadIn;
    *hb = p; p += kMapC;
    const size_t nfc = static_cast<size_t>(9) * (2 * D * R + R);
    *fw = p; p += nfc * kGap;
    *fb = p; p += nfc;
    return p;
}

int act_c(int i) { return i == 0 ? 4 : kCh[i]; }      // channel stride of activation i
int act_hw(int i) { return kNet >> i; }

struct WS {
    uint16_t* a[kConvs + 1];     // activations a0..a5 (bf16 NHWC)
    float* g;                    // [B][128]
    float* dout;                 // [B][nfc]
    float* dg;                   // [B][128]
    float* da[kConvs];           // da[i] = gradient w.r.t. activation i (i = 1..4), fp32 NHWC
};

size_t align256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

size_t carve_ws(char* base, int B, int D, int R, WS* w) {
    size_t off = 0;
    for (int i = 0; i <= kConvs; ++i) {
        const size_t n = static_cast<size_t>(B) * act_hw(i) * act_hw(i) * act_c(i);
        if (w) w->a[i] = reinterpret_cast<uint16_t*>(base + off);
        off = align256(off + n * 2);
    }
    const size_t nfc = static_cast<size_t>(9) * (2 * D * R + R);
    if (w) w->g = reinterpret_cast<float*>(base + off);
    off = align256(off + sizeof(float) * B * kGap);
    if (w) w->dout = reinterpret_cast<float*>(base + off);
    off = align256(off + sizeof(float) * B * nfc);
    if (w) w->dg = reinterpret_cast<float*>(base + off);
    off = align256(off + sizeof(float) * B * kGap);
    for (int i = 1; i < kConvs; ++i) {
        const size_t n = static_cast<size_t>(B) * act_hw(i) * act_hw(i) * act_c(i);
        if (w) w->da[i] = reinterpret_cast<float*>(base + off);
        off = align256(off + sizeof(float) * n);
    }
    return off;
}

ConvGeo conv_geo(int i, int B) {       // conv layer i (0..4): activation i -> activation i+1
    ConvGeo g;
    g.N = B;
    g.Hi = g.Wi = act_hw(i);
    g.Ci = kCh[i];
    g.Cs = act_c(i);
    g.Ho = g.Wo = act_hw(i + 1);
    g.Co = kCh[i + 1];
    g.Cos = act_c(i + 1);
    g.stride = 2;
    return g;
}

ConvGeo head_geo(int B) {
    ConvGeo g;
    g.N = B;
    g.Hi = g.Wi = kMapHW;
    g.Ci = kHeadIn;
    g.Cs = kHeadIn;
    g.Ho = g.Wo = kMapHW;
    g.Co = kMapC;
    g.Cos = 16;
    g.stride = 1;
    return g;
}

template <class AL, class BL, class EP>
void gemm_nt(int ncols, AL al, BL bl, EP ep, int M, int K, int splitk, hipStream_t st) {
    if (ncols <= 16) gemm<1>(al, bl, ep, M, ncols, K, splitk, st);
    else if (ncols <= 32) gemm<2>(al, bl, ep, M, ncols, K, splitk, st);
    else gemm<4>(al, bl, ep, M, ncols, K, splitk, st);
}

int wgrad_split(int M) { return std::max(1, std::min(256, M / 512)); }

template <class DZ>
void conv_backward(const ConvGeo& g, DZ dz, const uint16_t* in, const float* w, float* dw, float* db,
                   float* da_in, int accumulate_da, hipStream_t st) {
    const int Mo = g.N * g.Ho * g.Wo;
    // weight gradient: [Co] x [9*Cs] over the Mo output pixels (split over workgroups)
    gemm_nt(9 * g.Cs, WgradA<DZ>{dz, g}, WgradB{in, g}, EpiWgrad{dw, g.Co, g.Ci, g.Cs}, g.Co, Mo,
            wgrad_split(Mo), st);
    hipLaunchKernelGGL(bias_grad_kernel<DZ>, dim3((Mo + 63) / 64), dim3(128), 0, st, dz, db, Mo, g.Co);
    if (da_in) {
        const int Mi = g.N * g.Hi * g.Wi;
        gemm_nt(g.Ci, DgradA<DZ>{dz, g}, DgradB{w, g}, EpiStore{da_in, Mi, g.Cs, accumulate_da}, Mi,
                9 * g.Cos, 1, st);
    }
}

}  // namespace

size_t generator_param_count(int D, int R) {
    size_t n = 0;
    for (int i = 0; i < kConvs; ++i) n += static_cast<size_t>(kCh[i + 1]) * 9 * kCh[i] + kCh[i + 1];
    n += static_cast<size_t>(kMapC) * 9 * kHeadIn + kMapC;
    const size_t nfc = static_cast<size_t>(9) * (2 * D * R + R);
    return n + nfc * kGap + nfc;
}

size_t generator_ws_bytes(int B, int D, int R) { return carve_ws(nullptr, B, D, R, nullptr); }

svdlut_status generator_forward(const float* params, const void* x, svdlut_dtype io, int B, int H, int W, int D,
                                int R, float* U, float* s, float* V, float* map, void* ws, hipStream_t st) {
    float *w[kConvs], *b[kConvs], *hw, *hb, *fw, *fb;
    carve_params(const_cast<float*>(params), D, R, w, b, &hw, &hb, &fw, &fb);
    WS k;
    carve_ws(static_cast<char*>(ws), B, D, R, &k);
    const int64_t npx = static_cast<int64_t>(B) * kNet * kNet;
    const int blocks = static_cast<int>(std::min<int64_t>((npx + 255) / 256, 4096));
    if (io == SVDLUT_F32)
        hipLaunchKernelGGL(downsample_kernel<float>, dim3(blocks), dim3(256), 0, st, static_cast<const float*>(x),
                           k.a[0], B, H, W);
    else
        hipLaunchKernelGGL(downsample_kernel<__half>, dim3(blocks), dim3(256), 0, st, static_cast<const __half*>(x),
                           k.a[0], B, H, W);
    for (int i = 0; i < kConvs; ++i) {
        const ConvGeo g = conv_geo(i, B);
        const int M = B * g.Ho * g.Wo;
        gemm_nt(g.Cos, FwdA{k.a[i], g}, FwdB{w[i], g}, EpiAct{k.a[i + 1], b[i], M, g.Co, g.Cos}, M, 9 * g.Cs, 1, st);
        if (i == 2) {
            const ConvGeo hg = head_geo(B);
            const int Mh = B * kMapHW * kMapHW;
            gemm_nt(16, FwdA{k.a[3], hg}, FwdB{hw, hg}, EpiMap{map, hb, Mh, kMapC, kMapHW * kMapHW}, Mh, 9 * hg.Cs, 1, st);
        }
    }
    hipLaunchKernelGGL(gap_kernel, dim3((B * kGap + 127) / 128), dim3(128), 0, st, k.a[kConvs], k.g, B,
                       act_hw(kConvs) * act_hw(kConvs), kGap);
    const int nout = 9 * (2 * D * R + R);
    hipLaunchKernelGGL(fc_fwd_kernel, dim3((B * nout + 255) / 256), dim3(256), 0, st, k.g, fw, fb, U, s, V, B, D, R);
    return check_launch("generator_fwd");
}

svdlut_status generator_backward(const float* params, const float* dU, const float* ds, const float* dV,
                                 const float* dmap, float* grads, int B, int D, int R, void* ws, hipStream_t st) {
    float *w[kConvs], *b[kConvs], *hw, *hb, *fw, *fb;
    carve_params(const_cast<float*>(params), D, R, w, b, &hw, &hb, &fw, &fb);
    float *gw[kConvs], *gb[kConvs], *ghw, *ghb, *gfw, *gfb;
    carve_params(grads, D, R, gw, gb, &ghw, &ghb, &gfw, &gfb);
    WS k;
    carve_ws(static_cast<char*>(ws), B, D, R, &k);
    const int64_t np = static_cast<int64_t>(generator_param_count(D, R));
    hipLaunchKernelGGL(zero_f32_kernel, dim3(1024), dim3(256), 0, st, grads, np);
    const int nout = 9 * (2 * D * R + R);
    hipLaunchKernelGGL(fc_gather_kernel, dim3((B * nout + 255) / 256), dim3(256), 0, st, dU, ds, dV, k.dout, B, D, R);
    const int64_t nfw = static_cast<int64_t>(nout) * (kGap + 1);
    hipLaunchKernelGGL(fc_wgrad_kernel, dim3(static_cast<unsigned>((nfw + 255) / 256)), dim3(256), 0, st, k.dout, k.g,
                       gfw, gfb, B, nout);
    hipLaunchKernelGGL(fc_dgrad_kernel, dim3(B), dim3(kGap), 0, st, k.dout, fw, k.dg, nout);
    // conv5: through the average pool
    {
        const ConvGeo g = conv_geo(4, B);
        DzGap dz{k.dg, k.a[5], kGap, g.Ho * g.Wo, 1.f / static_cast<float>(g.Ho * g.Wo)};
        conv_backward(g, dz, k.a[4], w[4], gw[4], gb[4], k.da[4], 0, st);
    }
    // conv4 -> gradient of the third activation, then the map head adds its part
    {
        const ConvGeo g = conv_geo(3, B);
        conv_backward(g, DzMasked{k.da[4], k.a[4], g.Cos}, k.a[3], w[3], gw[3], gb[3], k.da[3], 0, st);
        const ConvGeo hg = head_geo(B);
        conv_backward(hg, DzMap{dmap, kMapC, kMapHW * kMapHW}, k.a[3], hw, ghw, ghb, k.da[3], 1, st);
    }
    for (int i = 2; i >= 0; --i) {
        const ConvGeo g = conv_geo(i, B);
        conv_backward(g, DzMasked{k.da[i + 1], k.a[i + 1], g.Cos}, k.a[i], w[i], gw[i], gb[i],
                      i > 0 ? k.da[i] : nullptr, 0, st);
    }
    return check_launch("generator_bwd");
}

}  // namespace svdlut

using namespace svdlut;

extern "C" {

size_t svdlut_generator_param_count(int32_t D, int32_t R) {
    if (D < 2 || D > kMaxD || R < 1 || R > kMaxR) return 0;
    return generator_param_count(D, R);
}

size_t svdlut_generator_workspace_size(int32_t B, int32_t D, int32_t R) {
    if (B < 1 || D < 2 || D > kMaxD || R < 1 || R > kMaxR) return 0;
    return generator_ws_bytes(B, D, R);
}

svdlut_status svdlut_generator_fwd(const float* params, const void* x, svdlut_dtype io, int32_t B, int32_t H,
                                   int32_t W, int32_t D, int32_t R, float* U, float* s, float* V, float* map,
                                   void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!params || !x || !U || !s || !V || !map || !ws) return fail(SVDLUT_EINVAL, "generator_fwd: null pointer");
    if (io != SVDLUT_F32 && io != SVDLUT_F16) return fail(SVDLUT_EUNSUPPORTED, "generator_fwd: dtype");
    if (B < 1 || H < 1 || W < 1 || H > kMaxDim || W > kMaxDim)
        return fail(SVDLUT_EINVAL, "generator_fwd: B, H, W out of range");
    if (D < 2 || D > kMaxD || R < 1 || R > kMaxR) return fail(SVDLUT_EINVAL, "generator_fwd: D or R out of range");
    if (ws_bytes < generator_ws_bytes(B, D, R))
        return fail(SVDLUT_EINVAL, "generator_fwd: workspace smaller than svdlut_generator_workspace_size()");
    return generator_forward(params, x, io, B, H, W, D, R, U, s, V, map, ws, stream);
}

svdlut_status svdlut_generator_bwd(const float* params, const float* dU, const float* ds, const float* dV,
                                   const float* dmap, float* grads, int32_t B, int32_t D, int32_t R, void* ws,
                                   size_t ws_bytes, hipStream_t stream) {
    if (!params || !dU || !ds || !dV || !dmap || !grads || !ws)
        return fail(SVDLUT_EINVAL, "generator_bwd: null pointer");
    if (B < 1) return fail(SVDLUT_EINVAL, "generator_bwd: B must be >= 1");
    if (D < 2 || D > kMaxD || R < 1 || R > kMaxR) return fail(SVDLUT_EINVAL, "generator_bwd: D or R out of range");
    if (ws_bytes < generator_ws_bytes(B, D, R))
        return fail(SVDLUT_EINVAL, "generator_bwd: workspace smaller than svdlut_generator_workspace_size()");
    return generator_backward(params, dU, ds, dV, dmap, grads, B, D, R, ws, stream);
}

}  // extern "C"
