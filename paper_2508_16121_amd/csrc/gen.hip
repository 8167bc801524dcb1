// Learned generator of the factors and the spatial map: bilinear downsample, five stride-2
// 3x3 convolutions with ReLU, a 3x3 map head, global average pooling and a fully connected
// factor head; forward and backward.  Convolutions (forward, input gradient and weight
// gradient) are implicit GEMMs on bf16 matrix cores (v_mfma_f32_16x16x16_bf16, fp32
// accumulation); operands are gathered straight from NHWC activations into the MFMA
// register layout.  Activations are stored as bf16; pooling, FC, biases, gradients of the
// activations and all parameter gradients are fp32.
#include "gen_common.h"

#include <algorithm>
#include <cstring>

namespace svdlut {

namespace {

constexpr int kConvs = 5;
constexpr int kCh[kConvs + 1] = {3, 16, 32, 64, 128, 128};
constexpr int kHeadIn = 64;          // the map head reads the third conv layer's output
constexpr int kMapC = 9;
constexpr int kMapHW = 32;
constexpr int kGap = 128;

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

// ---------------------------------------------------------------- epilogues
struct EpiAct {          // bf16(relu(acc + bias)) into NHWC, channel stride Cos
    uint16_t* out;
    const float* bias;
    int M, Co, Cos;
    __device__ void operator()(int m, int co, float v) const {
        if (m < M && co < Cos) out[static_cast<int64_t>(m) * Cos + co] = co < Co ? f2bf(fmaxf(v + bias[co], 0.f)) : 0;
    }
};
// sum of the split-K slices in fixed order + bias -> ReLU -> bf16 NHWC (channel stride Cos,
// padding channels zero)
__global__ void splitk_relu_kernel(const float* __restrict__ part, int splits, const float* __restrict__ bias,
                                   uint16_t* __restrict__ out, int M, int Co, int Cos) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    const int64_t MN = static_cast<int64_t>(M) * Cos;
    if (i >= MN) return;
    const int co = static_cast<int>(i % Cos);
    if (co >= Co) {
        out[i] = 0;
        return;
    }
    float z = bias[co];
    for (int k = 0; k < splits; ++k) z += part[k * MN + i];
    out[i] = f2bf(fmaxf(z, 0.f));
}

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
// Global average pool of the last activation: g[n][c] = mean over 8x8 (fp32).
__global__ void gap_kernel(const uint16_t* __restrict__ a, float* __restrict__ g, int B, int HW, int C) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * C) return;
    const int n = i / C, c = i - (i / C) * C;
    const uint16_t* src = a + static_cast<int64_t>(n) * HW * C + c;
    float s = 0.f;
    int p = 0;
    for (; p + 8 <= HW; p += 8) {      // eight loads in flight, added in pixel order
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = bf2f(src[static_cast<int64_t>(p + u) * C]);
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; p < HW; ++p) s += bf2f(src[static_cast<int64_t>(p) * C]);
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

// dg[n][c] = sum_j dout[n][j] W[j][c].  The j range is cut into chunks of kDgChunk rows, one
// workgroup (one thread per c) per (n, chunk), partial sums to part[n][chunk][c]; a second
// kernel adds the chunks in order.
constexpr int kDgChunk = 64;

__global__ void fc_dgrad_kernel(const float* __restrict__ dout, const float* __restrict__ Wt,
                                float* __restrict__ part, int nout) {
    const int n = blockIdx.x, ch = blockIdx.y, c = threadIdx.x;
    const int j0 = ch * kDgChunk, j1 = min(nout, j0 + kDgChunk);
    const float* d = dout + static_cast<int64_t>(n) * nout;
    float acc = 0.f;
#pragma unroll 8
    for (int j = j0; j < j1; ++j) acc = fmaf(d[j], Wt[static_cast<int64_t>(j) * kGap + c], acc);
    part[(static_cast<int64_t>(n) * gridDim.y + ch) * kGap + c] = acc;
}

__global__ void fc_dgrad_reduce_kernel(const float* __restrict__ part, float* __restrict__ dg, int nch) {
    const int n = blockIdx.x, c = threadIdx.x;
    const float* src = part + static_cast<int64_t>(n) * nch * kGap + c;
    float acc = 0.f;
    int k = 0;
    for (; k + 8 <= nch; k += 8) {     // eight loads in flight, added in chunk order
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = src[static_cast<int64_t>(k + u) * kGap];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; k < nch; ++k) acc += src[static_cast<int64_t>(k) * kGap];
    dg[n * kGap + c] = acc;
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
    float* skp;                  // split-K partial products of the small forward convolutions
    float* wpart;                // split-K partial products of the weight gradients
    uint16_t* a[kConvs + 1];     // activations a0..a5 (bf16 NHWC)
    float* g;                    // [B][128]
    float* dout;                 // [B][nfc]
    float* dg;                   // [B][128]
    float* dgp;                  // [B][chunks][128] partial sums of dg
    float* da[kConvs];           // da[i] = gradient w.r.t. activation i (i = 1..4), fp32 NHWC
};

ConvGeo conv_geo(int i, int B);
ConvGeo head_geo(int B);

int fwd_splits(const ConvGeo& g) { return fwd_splits(g.N * g.Ho * g.Wo, g.Cos, 9 * g.Cs); }

size_t carve_ws(char* base, int B, int D, int R, WS* w) {
    size_t off = 0;
    size_t nsk = 0;
    for (int i = 0; i < kConvs; ++i) {
        const ConvGeo g = conv_geo(i, B);
        const int sk = fwd_splits(g);
        if (sk > 1)
            nsk = std::max<size_t>(nsk, static_cast<size_t>(gemm_slices(9 * g.Cs, sk)) * g.N * g.Ho * g.Wo * g.Cos);
    }
    if (w) w->skp = reinterpret_cast<float*>(base + off);
    off = align256(off + sizeof(float) * nsk);
    size_t nwp = bwd_part_floats(head_geo(B));
    for (int i = 0; i < kConvs; ++i) nwp = std::max(nwp, bwd_part_floats(conv_geo(i, B)));
    if (w) w->wpart = reinterpret_cast<float*>(base + off);
    off = align256(off + sizeof(float) * nwp);
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
    if (w) w->dgp = reinterpret_cast<float*>(base + off);
    off = align256(off + sizeof(float) * B * kGap * ((nfc + kDgChunk - 1) / kDgChunk));
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
        const int sk = fwd_splits(g);
        if (sk > 1) {
            gemm<1>(FwdA{k.a[i], g}, FwdB{w[i], g}, EpiPartial{k.skp, M, g.Cos}, M, g.Cos, 9 * g.Cs, sk, st);
            const int64_t n = static_cast<int64_t>(M) * g.Cos;
            hipLaunchKernelGGL(splitk_relu_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st,
                               k.skp, gemm_slices(9 * g.Cs, sk), b[i], k.a[i + 1], M, g.Co, g.Cos);
        } else {
            gemm_nt(g.Cos, FwdA{k.a[i], g}, FwdB{w[i], g}, EpiAct{k.a[i + 1], b[i], M, g.Co, g.Cos}, M, 9 * g.Cs, 1,
                    st);
        }
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
    const int nch = (nout + kDgChunk - 1) / kDgChunk;
    hipLaunchKernelGGL(fc_dgrad_kernel, dim3(B, nch), dim3(kGap), 0, st, k.dout, fw, k.dgp, nout);
    hipLaunchKernelGGL(fc_dgrad_reduce_kernel, dim3(B), dim3(kGap), 0, st, k.dgp, k.dg, nch);
    // conv5: through the average pool
    {
        const ConvGeo g = conv_geo(4, B);
        DzGap dz{k.dg, k.a[5], kGap, g.Ho * g.Wo, 1.f / static_cast<float>(g.Ho * g.Wo)};
        conv_backward(g, dz, k.a[4], w[4], gw[4], gb[4], k.da[4], 0, k.wpart, st);
    }
    // conv4 -> gradient of the third activation, then the map head adds its part
    {
        const ConvGeo g = conv_geo(3, B);
        conv_backward(g, DzMasked{k.da[4], k.a[4], g.Cos}, k.a[3], w[3], gw[3], gb[3], k.da[3], 0, k.wpart, st);
        const ConvGeo hg = head_geo(B);
        conv_backward(hg, DzMap{dmap, kMapC, kMapHW * kMapHW}, k.a[3], hw, ghw, ghb, k.da[3], 1, k.wpart, st);
    }
    for (int i = 2; i >= 0; --i) {
        const ConvGeo g = conv_geo(i, B);
        conv_backward(g, DzMasked{k.da[i + 1], k.a[i + 1], g.Cos}, k.a[i], w[i], gw[i], gb[i],
                      i > 0 ? k.da[i] : nullptr, 0, k.wpart, st);
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
    if (B < 1 || B > kMaxGenBatch || D < 2 || D > kMaxD || R < 1 || R > kMaxR) return 0;
    return generator_ws_bytes(B, D, R);
}

svdlut_status svdlut_generator_fwd(const float* params, const void* x, svdlut_dtype io, int32_t B, int32_t H,
                                   int32_t W, int32_t D, int32_t R, float* U, float* s, float* V, float* map,
                                   void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!params || !x || !U || !s || !V || !map || !ws) return fail(SVDLUT_EINVAL, "generator_fwd: null pointer");
    if (io != SVDLUT_F32 && io != SVDLUT_F16) return fail(SVDLUT_EUNSUPPORTED, "generator_fwd: dtype");
    if (B < 1 || B > kMaxGenBatch || H < 1 || W < 1 || H > kMaxDim || W > kMaxDim)
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
    if (B < 1 || B > kMaxGenBatch) return fail(SVDLUT_EINVAL, "generator_bwd: B must be in [1, 4096]");
    if (D < 2 || D > kMaxD || R < 1 || R > kMaxR) return fail(SVDLUT_EINVAL, "generator_bwd: D or R out of range");
    if (ws_bytes < generator_ws_bytes(B, D, R))
        return fail(SVDLUT_EINVAL, "generator_bwd: workspace smaller than svdlut_generator_workspace_size()");
    return generator_backward(params, dU, ds, dV, dmap, grads, B, D, R, ws, stream);
}

}  // extern "C"
