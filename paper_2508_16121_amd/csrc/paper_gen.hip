// The paper's own generator network (supplementary Sec. "Details of Network Structure"):
// bilinear downsample to 256x256, five conv3x3 stride-2 blocks with m = 8 channels
// (3 -> 8 -> 16 -> 32 -> 64 -> 64), each conv + bias -> LeakyReLU(0.2) -> instance norm with
// learned scale and shift (the fifth block without the norm), dropout 0.5 from a caller keep
// mask, 4x4 average pooling to 2x2 and 256 features, then four two-layer FC generators
// (256 -> 8 -> n, no activation between): H_t (the U, S, V factors of the nine 2D LUTs),
// H_tw (per output channel three LUT weights and a bias), H_s (K grids of three 17x17 planes)
// and H_sw (per grid three plane weights and a bias).  Forward and backward.
//
// Convolutions (forward, input and weight gradients) run on the bf16 matrix-core implicit
// GEMM of gen_common.h with fp32 accumulation; the LeakyReLU output of every block is kept in
// fp32 for the norm statistics and the backward, the normalised activation that feeds the next
// convolution is stored as bf16.  Norm statistics, pooling, the FC generators and all
// gradients other than the bf16 matrix products are fp32.
#include "gen_common.h"

namespace svdlut {

namespace {

constexpr int kBlocks = 5;
constexpr int kPCh[kBlocks + 1] = {3, 8, 16, 32, 64, 64};
constexpr int kHid = 8;              // hidden width of every FC generator
constexpr int kFeat = 256;           // 8m channels x 2 x 2 pooled
constexpr float kSlope = 0.2f;
constexpr float kEps = 1e-5f;
constexpr int kHeads = 4;            // t, tw, s, sw

int blk_hw(int j) { return kNet >> j; }            // spatial size of activation j (0..5)
int blk_cs(int j) { return j == 0 ? 4 : kPCh[j]; } // channel stride of the bf16 activation j

// ---------------------------------------------------------------- heads
struct Heads {
    int n;                       // 2 (LUT only) or 4
    int width[kHeads];
    int off[kHeads];             // offset of each head in the concatenated output
    int total;
    const float* w1[kHeads];     // [8][256]
    const float* b1[kHeads];     // [8]
    const float* w2[kHeads];     // [width][8]
    const float* b2[kHeads];     // [width]
};

struct HeadGrads {               // gradient destinations of the FC generators
    float* w1[kHeads];
    float* b1[kHeads];
    float* w2[kHeads];
    float* b2[kHeads];
};

struct Outs {                    // the generator outputs (or their gradients)
    float *U, *s, *V, *lw, *lb, *grids, *gw, *gb;
    int D, R, K, Ds;
};

// ---------------------------------------------------------------- epilogue / gradient source
struct EpiLrelu {                // h = LeakyReLU(acc + bias), fp32 NHWC [M][Co]
    float* out;
    const float* bias;
    int M, Co;
    __device__ void operator()(int m, int co, float v) const {
        if (m < M && co < Co) {
            const float z = v + bias[co];
            out[static_cast<int64_t>(m) * Co + co] = z > 0.f ? z : kSlope * z;
        }
    }
};
struct DzArr {                   // precomputed dL/dz, fp32 NHWC [M][C]
    const float* dz;
    int C;
    __device__ float operator()(int m, int co) const { return dz[static_cast<int64_t>(m) * C + co]; }
};

// ---------------------------------------------------------------- instance norm
// Each image's H x W pixels are cut into chunks of 4096 / C pixels (16 values per thread);
// one workgroup of kNormThreads threads per (image, chunk).  Thread t owns channel t % C and
// every (kNormThreads / C)-th pixel of the chunk from t / C, so each pass reads the NHWC block
// coalesced.  The statistics kernel writes each chunk's per-channel sums; the kernel that
// applies the norm (or its gradient) merges the chunks of its image with a fixed-order tree,
// so the result does not depend on scheduling.  Every layer has exactly 256 chunk x channel
// partials per image (chunks = HW C / 4096).  Forward sums (x and x^2) are accumulated in
// fp64 so the variance E[x^2] - mean^2 does not cancel.
constexpr int kNormThreads = 256;
constexpr int kNormPer = 16;                       // values per thread per chunk

__host__ __device__ inline int norm_chunk_px(int C) { return kNormThreads * kNormPer / C; }
__host__ __device__ inline int norm_chunks(int HW, int C) { return (HW + norm_chunk_px(C) - 1) / norm_chunk_px(C); }

template <typename T>
__device__ void pair_tree(T* r0, T* r1, int t, int stop) {
    for (int s = kNormThreads / 2; s >= stop; s >>= 1) {
        __syncthreads();
        if (t < s) {
            r0[t] += r0[t + s];
            r1[t] += r1[t + s];
        }
    }
    __syncthreads();
}

// Merge the nch x C partials of image b into per-channel totals: thread t takes partial
// index t (chunk t / C, channel t % C) and a tree over the chunks leaves channel c's totals
// in slot c.  nch * C <= kNormThreads.
template <typename T, typename P>
__device__ void merge_partials(const P* part, int b, int nch, int C, T* r0, T* r1) {
    const int t = threadIdx.x;
    T v0 = 0, v1 = 0;
    if (t < nch * C) {
        const P v = part[static_cast<int64_t>(b) * nch * C + t];
        v0 = v.x;
        v1 = v.y;
    }
    r0[t] = v0;
    r1[t] = v1;
    pair_tree(r0, r1, t, C);
}

// part[(b * nch + chunk) * C + c] = (sum x, sum x^2) over the chunk, fp64
__global__ void __launch_bounds__(kNormThreads) norm_stats_kernel(const float* __restrict__ h,
                                                                    double2* __restrict__ part, int HW, int C) {
    __shared__ double r0[kNormThreads], r1[kNormThreads];
    const int nch = norm_chunks(HW, C), cpx = norm_chunk_px(C);
    const int b = blockIdx.x / nch, ch = blockIdx.x - b * nch;
    const int p0 = ch * cpx, p1 = min(HW, p0 + cpx);
    const int t = threadIdx.x, c = t % C, pstep = kNormThreads / C;
    const float* hb = h + static_cast<int64_t>(b) * HW * C;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll 4
    for (int p = p0 + t / C; p < p1; p += pstep) {
        const double v = hb[static_cast<int64_t>(p) * C + c];
        s0 += v;
        s1 = fma(v, v, s1);
    }
    r0[t] = s0;
    r1[t] = s1;
    pair_tree(r0, r1, t, C);
    if (t < C) part[static_cast<int64_t>(blockIdx.x) * C + c] = make_double2(r0[c], r1[c]);
}

// a = bf16(scale * (h - mean) * rstd + shift) over this workgroup's chunk; chunk 0 of each
// image also stores the image's mean and rstd for the backward.
__global__ void __launch_bounds__(kNormThreads) norm_apply_kernel(const float* __restrict__ h,
                                                                    const double2* __restrict__ part,
                                                                    uint16_t* __restrict__ a, float* __restrict__ mu,
                                                                    float* __restrict__ rs,
                                                                    const float* __restrict__ gamma,
                                                                    const float* __restrict__ beta, int HW, int C) {
    __shared__ double r0[kNormThreads], r1[kNormThreads];
    __shared__ float coef[2][64];
    const int nch = norm_chunks(HW, C), cpx = norm_chunk_px(C);
    const int b = blockIdx.x / nch, ch = blockIdx.x - b * nch;
    const int t = threadIdx.x;
    merge_partials(part, b, nch, C, r0, r1);
    if (t < C) {
        const double m = r0[t] / HW;
        const double var = fmax(r1[t] / HW - m * m, 0.0);
        const float mean = static_cast<float>(m);
        const float rstd = 1.f / sqrtf(static_cast<float>(var) + kEps);
        if (ch == 0) {
            mu[b * C + t] = mean;
            rs[b * C + t] = rstd;
        }
        const float g = gamma[t] * rstd;
        coef[0][t] = g;
        coef[1][t] = beta[t] - g * mean;
    }
    __syncthreads();
    const int p0 = ch * cpx, p1 = min(HW, p0 + cpx);
    const int c = t % C, pstep = kNormThreads / C;
    const float g = coef[0][c], sh = coef[1][c];
    const int64_t base = static_cast<int64_t>(b) * HW * C;
#pragma unroll 4
    for (int p = p0 + t / C; p < p1; p += pstep) {
        const int64_t o = base + static_cast<int64_t>(p) * C + c;
        a[o] = f2bf(fmaf(g, h[o], sh));
    }
}

// Backward statistics: per chunk, sum of da and sum of da * xhat (xhat from the image's
// forward mean and rstd), fp32.
__global__ void __launch_bounds__(kNormThreads) norm_bwd_stats_kernel(const float* __restrict__ h,
                                                                        const float* __restrict__ da,
                                                                        const float* __restrict__ mu,
                                                                        const float* __restrict__ rs,
                                                                        float2* __restrict__ part, int HW, int C) {
    __shared__ float r0[kNormThreads], r1[kNormThreads];
    const int nch = norm_chunks(HW, C), cpx = norm_chunk_px(C);
    const int b = blockIdx.x / nch, ch = blockIdx.x - b * nch;
    const int p0 = ch * cpx, p1 = min(HW, p0 + cpx);
    const int t = threadIdx.x, c = t % C, pstep = kNormThreads / C;
    const float mean = mu[b * C + c], rstd = rs[b * C + c];
    const int64_t base = static_cast<int64_t>(b) * HW * C;
    float s0 = 0.f, s1 = 0.f;
#pragma unroll 4
    for (int p = p0 + t / C; p < p1; p += pstep) {
        const int64_t o = base + static_cast<int64_t>(p) * C + c;
        const float g = da[o];
        s0 += g;
        s1 = fmaf(g, (h[o] - mean) * rstd, s1);
    }
    r0[t] = s0;
    r1[t] = s1;
    pair_tree(r0, r1, t, C);
    if (t < C) part[static_cast<int64_t>(blockIdx.x) * C + c] = make_float2(r0[c], r1[c]);
}

// Scale and shift gradients of one norm: per channel, the sums of da * xhat and of da over
// the whole batch from the chunk partials (C <= 64, one workgroup of 256 threads): thread
// (c, l) adds partials l, l + L, ... in order (L = 256 / C), then the lane sums of each
// channel are added in lane order.
__global__ void __launch_bounds__(256) norm_param_grad_kernel(const float2* __restrict__ part, int nparts, int C,
                                                              float* __restrict__ dgamma, float* __restrict__ dbeta) {
    __shared__ float r0[256], r1[256];
    const int t = threadIdx.x, L = max(1, 256 / C), c = t % C, l = t / C;
    float s0 = 0.f, s1 = 0.f;
    if (l < L)
#pragma unroll 8
        for (int i = l; i < nparts; i += L) {
            const float2 v = part[static_cast<int64_t>(i) * C + c];
            s0 += v.x;
            s1 += v.y;
        }
    r0[t] = s0;
    r1[t] = s1;
    __syncthreads();
    if (t < C) {
        float v0 = 0.f, v1 = 0.f;
        for (int i = 0; i < L; ++i) {
            v0 += r0[i * C + t];
            v1 += r1[i * C + t];
        }
        dbeta[t] = v0;
        dgamma[t] = v1;
    }
}

// dz = dL/d(conv output before LeakyReLU) over this chunk.
__global__ void __launch_bounds__(kNormThreads) norm_bwd_apply_kernel(const float* __restrict__ h,
                                                                        const float* __restrict__ da,
                                                                        const float2* __restrict__ part,
                                                                        const float* __restrict__ mu,
                                                                        const float* __restrict__ rs,
                                                                        const float* __restrict__ gamma,
                                                                        float* __restrict__ dz, int HW, int C) {
    __shared__ float r0[kNormThreads], r1[kNormThreads];
    __shared__ float coef[2][64];
    const int nch = norm_chunks(HW, C), cpx = norm_chunk_px(C);
    const int b = blockIdx.x / nch, ch = blockIdx.x - b * nch;
    const int t = threadIdx.x;
    merge_partials(part, b, nch, C, r0, r1);
    if (t < C) {
        const float s0 = r0[t], s1 = r1[t];
        const float inv = 1.f / static_cast<float>(HW);
        coef[0][t] = gamma[t] * s0 * inv;
        coef[1][t] = gamma[t] * s1 * inv;
    }
    __syncthreads();
    const int p0 = ch * cpx, p1 = min(HW, p0 + cpx);
    const int c = t % C, pstep = kNormThreads / C;
    const float m1 = coef[0][c], m2 = coef[1][c];
    const float mean = mu[b * C + c], rstd = rs[b * C + c], gm = gamma[c];
    const int64_t base = static_cast<int64_t>(b) * HW * C;
#pragma unroll 4
    for (int p = p0 + t / C; p < p1; p += pstep) {
        const int64_t o = base + static_cast<int64_t>(p) * C + c;
        const float hv = h[o];
        const float xh = (hv - mean) * rstd;
        const float d = rstd * (gm * da[o] - m1 - xh * m2);
        dz[o] = hv > 0.f ? d : kSlope * d;
    }
}

// ---------------------------------------------------------------- split-K forward convolution
// sum of the split-K slices in fixed order + bias -> LeakyReLU (fp32 NHWC)
__global__ void splitk_lrelu_kernel(const float* __restrict__ part, int splits, const float* __restrict__ bias,
                                    float* __restrict__ out, int M, int N) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    const int64_t MN = static_cast<int64_t>(M) * N;
    if (i >= MN) return;
    float z = bias[static_cast<int>(i % N)];
    for (int k = 0; k < splits; ++k) z += part[k * MN + i];
    out[i] = z > 0.f ? z : kSlope * z;
}

// ---------------------------------------------------------------- dropout + pooling
// f[b][4c + 2py + px] = mean over the 4x4 window (py, px) of h5 * keep, keep = 2 mask or 1.
__global__ void pool_fwd_kernel(const float* __restrict__ h5, const uint8_t* __restrict__ mask,
                                float* __restrict__ f, int B) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * kFeat) return;
    const int b = i / kFeat, j = i - b * kFeat;
    const int c = j >> 2, py = (j >> 1) & 1, px = j & 1;
    const int C = kPCh[5];
    float acc = 0.f;
    for (int y = 4 * py; y < 4 * py + 4; ++y)
        for (int x = 4 * px; x < 4 * px + 4; ++x) {
            float v = h5[(static_cast<int64_t>(b) * 64 + y * 8 + x) * C + c];
            if (mask) v *= mask[((static_cast<int64_t>(b) * C + c) * 8 + y) * 8 + x] ? 2.f : 0.f;
            acc += v;
        }
    f[i] = acc * (1.f / 16.f);
}

// dz5 = df / 16 * keep * LeakyReLU'(h5), NHWC [B][64][64].
__global__ void pool_bwd_kernel(const float* __restrict__ df, const float* __restrict__ h5,
                                const uint8_t* __restrict__ mask, float* __restrict__ dz, int B) {
    const int C = kPCh[5];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * 64 * C) return;
    const int b = i / (64 * C), r = i - b * 64 * C;
    const int p = r / C, c = r - (r / C) * C;
    const int y = p >> 3, x = p & 7;
    float g = df[b * kFeat + 4 * c + 2 * (y >> 2) + (x >> 2)] * (1.f / 16.f);
    if (mask) g *= mask[((static_cast<int64_t>(b) * C + c) * 8 + y) * 8 + x] ? 2.f : 0.f;
    dz[i] = h5[i] > 0.f ? g : kSlope * g;
}

// ---------------------------------------------------------------- FC generators
__device__ __forceinline__ int head_of(const Heads& hs, int J) {
    int h = 0;
    while (h + 1 < hs.n && J >= hs.off[h + 1]) ++h;
    return h;
}

__global__ void hid_fwd_kernel(const float* __restrict__ f, Heads hs, float* __restrict__ hid, int B) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * hs.n * kHid) return;
    const int b = i / (hs.n * kHid), r = i - b * hs.n * kHid;
    const int h = r / kHid, k = r - h * kHid;
    const float* w = hs.w1[h] + k * kFeat;
    const float* fb = f + b * kFeat;
    float acc = hs.b1[h][k];
#pragma unroll 16
    for (int c = 0; c < kFeat; ++c) acc = fmaf(fb[c], w[c], acc);
    hid[b * kHeads * kHid + h * kHid + k] = acc;
}

__global__ void out_fwd_kernel(const float* __restrict__ hid, Heads hs, Outs o, int B) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i >= static_cast<int64_t>(B) * hs.total) return;
    const int b = static_cast<int>(i / hs.total), J = static_cast<int>(i - static_cast<int64_t>(b) * hs.total);
    const int h = head_of(hs, J), j = J - hs.off[h];
    const float* w = hs.w2[h] + j * kHid;
    const float* hb = hid + b * kHeads * kHid + h * kHid;
    float v = hs.b2[h][j];
#pragma unroll
    for (int k = 0; k < kHid; ++k) v = fmaf(hb[k], w[k], v);
    if (h == 0) {
        const int nU = 9 * o.D * o.R, nS = 9 * o.R;
        if (j < nU) o.U[static_cast<int64_t>(b) * nU + j] = v;
        else if (j < nU + nS) o.s[static_cast<int64_t>(b) * nS + (j - nU)] = v;
        else o.V[static_cast<int64_t>(b) * nU + (j - nU - nS)] = v;
    } else if (h == 1) {
        const int c = j >> 2, t = j & 3;
        if (t < 3) o.lw[b * 9 + 3 * c + t] = v;
        else o.lb[b * 3 + c] = v;
    } else if (h == 2) {
        o.grids[static_cast<int64_t>(b) * hs.width[2] + j] = v;
    } else {
        const int k = j >> 2, t = j & 3;
        if (t < 3) o.gw[(b * o.K + k) * 3 + t] = v;
        else o.gb[b * o.K + k] = v;
    }
}

// Concatenated upstream gradient dO[b][J] (a null input counts as zero).
__global__ void out_gather_kernel(Outs g, Heads hs, float* __restrict__ dO, int B) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i >= static_cast<int64_t>(B) * hs.total) return;
    const int b = static_cast<int>(i / hs.total), J = static_cast<int>(i - static_cast<int64_t>(b) * hs.total);
    const int h = head_of(hs, J), j = J - hs.off[h];
    const float* src = nullptr;
    int64_t o = 0;
    if (h == 0) {
        const int nU = 9 * g.D * g.R, nS = 9 * g.R;
        if (j < nU) { src = g.U; o = static_cast<int64_t>(b) * nU + j; }
        else if (j < nU + nS) { src = g.s; o = static_cast<int64_t>(b) * nS + (j - nU); }
        else { src = g.V; o = static_cast<int64_t>(b) * nU + (j - nU - nS); }
    } else if (h == 1) {
        const int c = j >> 2, t = j & 3;
        if (t < 3) { src = g.lw; o = b * 9 + 3 * c + t; }
        else { src = g.lb; o = b * 3 + c; }
    } else if (h == 2) {
        src = g.grids; o = static_cast<int64_t>(b) * hs.width[2] + j;
    } else {
        const int k = j >> 2, t = j & 3;
        if (t < 3) { src = g.gw; o = (b * g.K + k) * 3 + t; }
        else { src = g.gb; o = b * g.K + k; }
    }
    dO[i] = src ? src[o] : 0.f;
}

// dW2[J][k] = sum_b dO[b][J] hid[b][h][k] (k < 8); db2[J] = sum_b dO[b][J] (k == 8).
__global__ void fc2_grad_kernel(const float* __restrict__ dO, const float* __restrict__ hid, Heads hs,
                                HeadGrads gr, int B) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i >= static_cast<int64_t>(hs.total) * (kHid + 1)) return;
    const int J = static_cast<int>(i / (kHid + 1)), k = static_cast<int>(i - static_cast<int64_t>(J) * (kHid + 1));
    const int h = head_of(hs, J), j = J - hs.off[h];
    float acc = 0.f;
    for (int b = 0; b < B; ++b)
        acc = fmaf(dO[static_cast<int64_t>(b) * hs.total + J], k < kHid ? hid[b * kHeads * kHid + h * kHid + k] : 1.f, acc);
    if (k < kHid) gr.w2[h][j * kHid + k] = acc;
    else gr.b2[h][j] = acc;
}

// dhid[b][h][k] = sum_j dO[b][off_h + j] W2_h[j][k]: one workgroup of 256 per (b, h).
__global__ void __launch_bounds__(256) dhid_kernel(const float* __restrict__ dO, Heads hs,
                                                   float* __restrict__ dhid) {
    __shared__ float red[kHid][256];
    const int b = blockIdx.x / hs.n, h = blockIdx.x - b * hs.n;
    const int t = threadIdx.x;
    const float* d = dO + static_cast<int64_t>(b) * hs.total + hs.off[h];
    const float* w = hs.w2[h];
    float acc[kHid] = {};
    for (int j = t; j < hs.width[h]; j += 256) {
        const float g = d[j];
#pragma unroll
        for (int k = 0; k < kHid; ++k) acc[k] = fmaf(g, w[j * kHid + k], acc[k]);
    }
#pragma unroll
    for (int k = 0; k < kHid; ++k) red[k][t] = acc[k];
    for (int s = 128; s > 0; s >>= 1) {
        __syncthreads();
        if (t < s)
#pragma unroll
            for (int k = 0; k < kHid; ++k) red[k][t] += red[k][t + s];
    }
    __syncthreads();
    if (t < kHid) dhid[b * kHeads * kHid + h * kHid + t] = red[t][0];
}

// dW1[k][c] = sum_b dhid[b][h][k] f[b][c] (c < 256); db1[k] = sum_b dhid[b][h][k] (c == 256).
__global__ void fc1_grad_kernel(const float* __restrict__ dhid, const float* __restrict__ f, Heads hs,
                                HeadGrads gr, int B) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= hs.n * kHid * (kFeat + 1)) return;
    const int hk = i / (kFeat + 1), c = i - hk * (kFeat + 1);
    const int h = hk / kHid, k = hk - h * kHid;
    float acc = 0.f;
    for (int b = 0; b < B; ++b)
        acc = fmaf(dhid[b * kHeads * kHid + h * kHid + k], c < kFeat ? f[b * kFeat + c] : 1.f, acc);
    if (c < kFeat) gr.w1[h][k * kFeat + c] = acc;
    else gr.b1[h][k] = acc;
}

// df[b][c] = sum_h sum_k dhid[b][h][k] W1_h[k][c].
__global__ void df_kernel(const float* __restrict__ dhid, Heads hs, float* __restrict__ df, int B) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * kFeat) return;
    const int b = i / kFeat, c = i - b * kFeat;
    float acc = 0.f;
    for (int h = 0; h < hs.n; ++h)
        for (int k = 0; k < kHid; ++k) acc = fmaf(dhid[b * kHeads * kHid + h * kHid + k], hs.w1[h][k * kFeat + c], acc);
    df[i] = acc;
}

// ---------------------------------------------------------------- parameter / workspace layout
int head_count(int K) { return K > 0 ? 4 : 2; }

int head_width(int h, int D, int R, int K, int Ds) {
    switch (h) {
        case 0: return 9 * (2 * D * R + R);
        case 1: return 12;
        case 2: return K * 3 * Ds * Ds;
        default: return 4 * K;
    }
}

struct PParams {
    float* cw[kBlocks];
    float* cb[kBlocks];
    float* ng[kBlocks - 1];
    float* nb[kBlocks - 1];
    float* w1[kHeads];
    float* b1[kHeads];
    float* w2[kHeads];
    float* b2[kHeads];
};

size_t carve_pparams(float* base, int D, int R, int K, int Ds, PParams* P) {
    size_t off = 0;
    auto take = [&](size_t n) { float* p = base ? base + off : nullptr; off += n; return p; };
    for (int i = 0; i < kBlocks; ++i) {
        P->cw[i] = take(static_cast<size_t>(kPCh[i + 1]) * 9 * kPCh[i]);
        P->cb[i] = take(kPCh[i + 1]);
        if (i < kBlocks - 1) {
            P->ng[i] = take(kPCh[i + 1]);
            P->nb[i] = take(kPCh[i + 1]);
        }
    }
    for (int h = 0; h < kHeads; ++h) P->w1[h] = P->b1[h] = P->w2[h] = P->b2[h] = nullptr;
    for (int h = 0; h < head_count(K); ++h) {
        const size_t n = head_width(h, D, R, K, Ds);
        P->w1[h] = take(static_cast<size_t>(kHid) * kFeat);
        P->b1[h] = take(kHid);
        P->w2[h] = take(n * kHid);
        P->b2[h] = take(n);
    }
    return off;
}

Heads make_heads(const PParams& P, int D, int R, int K, int Ds) {
    Heads hs{};
    hs.n = head_count(K);
    int off = 0;
    for (int h = 0; h < hs.n; ++h) {
        hs.width[h] = head_width(h, D, R, K, Ds);
        hs.off[h] = off;
        off += hs.width[h];
        hs.w1[h] = P.w1[h];
        hs.b1[h] = P.b1[h];
        hs.w2[h] = P.w2[h];
        hs.b2[h] = P.b2[h];
    }
    hs.total = off;
    return hs;
}

struct PWS {
    uint16_t* a[kBlocks];        // bf16 activations 0..4 (input of each conv)
    float* h[kBlocks];           // fp32 LeakyReLU outputs of blocks 1..5 (index j - 1)
    float* mu[kBlocks - 1];
    float* rs[kBlocks - 1];
    float* f;                    // [B][256]
    float* hid;                  // [B][4][8]
    float* dO;                   // [B][total]
    float* dhid;                 // [B][4][8]
    float* df;                   // [B][256]
    float* dz[kBlocks];          // dL/d(conv output) of blocks 1..5 (index j - 1)
    float* da[kBlocks];          // dL/d(bf16 activation j), j = 1..4
    double2* part;               // per-chunk norm statistics [B][chunks x C = 256]
    float* skp;                  // split-K partial products of the small forward convolutions
    float* wpart;                // split-K partial products of the weight gradients
};

ConvGeo pconv_geo(int i, int B) {      // block i (0..4): activation i -> LeakyReLU output i + 1
    ConvGeo g;
    g.N = B;
    g.Hi = g.Wi = blk_hw(i);
    g.Ci = kPCh[i];
    g.Cs = blk_cs(i);
    g.Ho = g.Wo = blk_hw(i + 1);
    g.Co = kPCh[i + 1];
    g.Cos = kPCh[i + 1];
    g.stride = 2;
    return g;
}

int fwd_splits(const ConvGeo& g) { return fwd_splits(g.N * g.Ho * g.Wo, g.Co, 9 * g.Cs); }

size_t carve_pws(char* base, int B, int total, PWS* w) {
    size_t off = 0;
    auto take = [&](size_t bytes) { char* p = base ? base + off : nullptr; off = align256(off + bytes); return p; };
    for (int j = 0; j < kBlocks; ++j)
        w->a[j] = reinterpret_cast<uint16_t*>(take(2 * static_cast<size_t>(B) * blk_hw(j) * blk_hw(j) * blk_cs(j)));
    for (int j = 1; j <= kBlocks; ++j) {
        const size_t n = static_cast<size_t>(B) * blk_hw(j) * blk_hw(j) * kPCh[j];
        w->h[j - 1] = reinterpret_cast<float*>(take(4 * n));
        w->dz[j - 1] = reinterpret_cast<float*>(take(4 * n));
        w->da[j - 1] = j < kBlocks ? reinterpret_cast<float*>(take(4 * n)) : nullptr;
    }
    for (int j = 0; j < kBlocks - 1; ++j) {
        w->mu[j] = reinterpret_cast<float*>(take(4 * static_cast<size_t>(B) * kPCh[j + 1]));
        w->rs[j] = reinterpret_cast<float*>(take(4 * static_cast<size_t>(B) * kPCh[j + 1]));
    }
    w->f = reinterpret_cast<float*>(take(4 * static_cast<size_t>(B) * kFeat));
    w->hid = reinterpret_cast<float*>(take(4 * static_cast<size_t>(B) * kHeads * kHid));
    w->dO = reinterpret_cast<float*>(take(4 * static_cast<size_t>(B) * total));
    w->dhid = reinterpret_cast<float*>(take(4 * static_cast<size_t>(B) * kHeads * kHid));
    w->df = reinterpret_cast<float*>(take(4 * static_cast<size_t>(B) * kFeat));
    w->part = reinterpret_cast<double2*>(take(sizeof(double2) * static_cast<size_t>(B) * kNormThreads));
    size_t nsk = 0;
    for (int i = 0; i < kBlocks; ++i) {
        const ConvGeo g = pconv_geo(i, B);
        const int sk = fwd_splits(g);
        if (sk > 1)
            nsk = std::max<size_t>(nsk, static_cast<size_t>(gemm_slices(9 * g.Cs, sk)) * g.N * g.Ho * g.Wo * g.Co);
    }
    w->skp = reinterpret_cast<float*>(take(sizeof(float) * nsk));
    size_t nwp = 0;
    for (int i = 0; i < kBlocks; ++i) nwp = std::max(nwp, bwd_part_floats(pconv_geo(i, B)));
    w->wpart = reinterpret_cast<float*>(take(sizeof(float) * nwp));
    return off;
}

int grid1d(int64_t n, int t = 256) { return static_cast<int>((n + t - 1) / t); }

}  // namespace

size_t paper_generator_param_count(int D, int R, int K, int Ds) {
    PParams P;
    return carve_pparams(nullptr, D, R, K, Ds, &P);
}

size_t paper_generator_ws_bytes(int B, int D, int R, int K, int Ds) {
    int total = 0;
    for (int h = 0; h < head_count(K); ++h) total += head_width(h, D, R, K, Ds);
    PWS w;
    return carve_pws(nullptr, B, total, &w);
}

svdlut_status paper_generator_forward(const float* params, const void* x, svdlut_dtype io, int B, int H, int W,
                                      int D, int R, int K, int Ds, const uint8_t* mask, float* U, float* s,
                                      float* V, float* lw, float* lb, float* grids, float* gw, float* gb, void* ws,
                                      hipStream_t st) {
    PParams P;
    carve_pparams(const_cast<float*>(params), D, R, K, Ds, &P);
    const Heads hs = make_heads(P, D, R, K, Ds);
    PWS k;
    carve_pws(static_cast<char*>(ws), B, hs.total, &k);
    const int64_t npx = static_cast<int64_t>(B) * kNet * kNet;
    const int blocks = static_cast<int>(std::min<int64_t>((npx + 255) / 256, 4096));
    if (io == SVDLUT_F32)
        hipLaunchKernelGGL(downsample_kernel<float>, dim3(blocks), dim3(256), 0, st, static_cast<const float*>(x),
                           k.a[0], B, H, W);
    else
        hipLaunchKernelGGL(downsample_kernel<__half>, dim3(blocks), dim3(256), 0, st, static_cast<const __half*>(x),
                           k.a[0], B, H, W);
    for (int i = 0; i < kBlocks; ++i) {
        const ConvGeo g = pconv_geo(i, B);
        const int M = B * g.Ho * g.Wo;
        const int sk = fwd_splits(g);
        if (sk > 1) {
            gemm<1>(FwdA{k.a[i], g}, FwdB{P.cw[i], g}, EpiPartial{k.skp, M, g.Co}, M, g.Co, 9 * g.Cs, sk, st);
            hipLaunchKernelGGL(splitk_lrelu_kernel, dim3(grid1d(static_cast<int64_t>(M) * g.Co)), dim3(256), 0, st,
                               k.skp, gemm_slices(9 * g.Cs, sk), P.cb[i], k.h[i], M, g.Co);
        } else {
            gemm_nt(g.Co, FwdA{k.a[i], g}, FwdB{P.cw[i], g}, EpiLrelu{k.h[i], P.cb[i], M, g.Co}, M, 9 * g.Cs, 1, st);
        }
        if (i < kBlocks - 1) {
            const int HW = g.Ho * g.Wo;
            const dim3 grid(B * norm_chunks(HW, g.Co));
            hipLaunchKernelGGL(norm_stats_kernel, grid, dim3(kNormThreads), 0, st, k.h[i], k.part, HW, g.Co);
            hipLaunchKernelGGL(norm_apply_kernel, grid, dim3(kNormThreads), 0, st, k.h[i], k.part, k.a[i + 1], k.mu[i],
                               k.rs[i], P.ng[i], P.nb[i], HW, g.Co);
        }
    }
    hipLaunchKernelGGL(pool_fwd_kernel, dim3(grid1d(B * kFeat)), dim3(256), 0, st, k.h[kBlocks - 1], mask, k.f, B);
    hipLaunchKernelGGL(hid_fwd_kernel, dim3(grid1d(B * hs.n * kHid)), dim3(256), 0, st, k.f, hs, k.hid, B);
    const Outs o{U, s, V, lw, lb, grids, gw, gb, D, R, K, Ds};
    hipLaunchKernelGGL(out_fwd_kernel, dim3(grid1d(static_cast<int64_t>(B) * hs.total)), dim3(256), 0, st, k.hid, hs,
                       o, B);
    return check_launch("paper_generator_fwd");
}

svdlut_status paper_generator_backward(const float* params, const uint8_t* mask, const float* dU, const float* ds,
                                       const float* dV, const float* dlw, const float* dlb, const float* dgrids,
                                       const float* dgw, const float* dgb, float* grads, int B, int D, int R, int K,
                                       int Ds, void* ws, hipStream_t st) {
    PParams P, G;
    const size_t np = carve_pparams(const_cast<float*>(params), D, R, K, Ds, &P);
    carve_pparams(grads, D, R, K, Ds, &G);
    const Heads hs = make_heads(P, D, R, K, Ds);
    PWS k;
    carve_pws(static_cast<char*>(ws), B, hs.total, &k);
    hipLaunchKernelGGL(zero_f32_kernel, dim3(256), dim3(256), 0, st, grads, static_cast<int64_t>(np));
    HeadGrads gr;
    for (int h = 0; h < kHeads; ++h) {
        gr.w1[h] = G.w1[h];
        gr.b1[h] = G.b1[h];
        gr.w2[h] = G.w2[h];
        gr.b2[h] = G.b2[h];
    }
    const Outs g{const_cast<float*>(dU), const_cast<float*>(ds), const_cast<float*>(dV), const_cast<float*>(dlw),
                 const_cast<float*>(dlb), const_cast<float*>(dgrids), const_cast<float*>(dgw),
                 const_cast<float*>(dgb), D, R, K, Ds};
    const int64_t nO = static_cast<int64_t>(B) * hs.total;
    hipLaunchKernelGGL(out_gather_kernel, dim3(grid1d(nO)), dim3(256), 0, st, g, hs, k.dO, B);
    hipLaunchKernelGGL(fc2_grad_kernel, dim3(grid1d(static_cast<int64_t>(hs.total) * (kHid + 1))), dim3(256), 0, st,
                       k.dO, k.hid, hs, gr, B);
    hipLaunchKernelGGL(dhid_kernel, dim3(B * hs.n), dim3(256), 0, st, k.dO, hs, k.dhid);
    hipLaunchKernelGGL(fc1_grad_kernel, dim3(grid1d(hs.n * kHid * (kFeat + 1))), dim3(256), 0, st, k.dhid, k.f, hs,
                       gr, B);
    hipLaunchKernelGGL(df_kernel, dim3(grid1d(B * kFeat)), dim3(256), 0, st, k.dhid, hs, k.df, B);
    hipLaunchKernelGGL(pool_bwd_kernel, dim3(grid1d(B * 64 * kPCh[5])), dim3(256), 0, st, k.df, k.h[kBlocks - 1], mask,
                       k.dz[kBlocks - 1], B);
    for (int i = kBlocks - 1; i >= 0; --i) {
        const ConvGeo cg = pconv_geo(i, B);
        conv_backward(cg, DzArr{k.dz[i], cg.Co}, k.a[i], P.cw[i], G.cw[i], G.cb[i], i > 0 ? k.da[i - 1] : nullptr, 0,
                      k.wpart, st);
        if (i == 0) break;
        // norm of block i (its output is activation i): da[i - 1] -> dz[i - 1]
        const int HW = blk_hw(i) * blk_hw(i), C = kPCh[i];
        const dim3 grid(B * norm_chunks(HW, C));
        float2* bpart = reinterpret_cast<float2*>(k.part);
        hipLaunchKernelGGL(norm_bwd_stats_kernel, grid, dim3(kNormThreads), 0, st, k.h[i - 1], k.da[i - 1],
                           k.mu[i - 1], k.rs[i - 1], bpart, HW, C);
        hipLaunchKernelGGL(norm_param_grad_kernel, dim3(1), dim3(256), 0, st, bpart, static_cast<int>(grid.x), C,
                           G.ng[i - 1], G.nb[i - 1]);
        hipLaunchKernelGGL(norm_bwd_apply_kernel, grid, dim3(kNormThreads), 0, st, k.h[i - 1], k.da[i - 1], bpart,
                           k.mu[i - 1], k.rs[i - 1], P.ng[i - 1], k.dz[i - 1], HW, C);
    }
    return check_launch("paper_generator_bwd");
}

}  // namespace svdlut

using namespace svdlut;

namespace {

bool pgen_dims_ok(int D, int R, int K, int Ds) {
    return D >= 2 && D <= kMaxD && R >= 1 && R <= kMaxR && K >= 0 && K <= kMaxGrids &&
           (K == 0 || (Ds >= 2 && Ds <= kMaxDs));
}

}  // namespace

extern "C" {

size_t svdlut_paper_generator_param_count(int32_t D, int32_t R, int32_t K, int32_t Ds) {
    if (!pgen_dims_ok(D, R, K, Ds)) return 0;
    return paper_generator_param_count(D, R, K, Ds);
}

size_t svdlut_paper_generator_workspace_size(int32_t B, int32_t D, int32_t R, int32_t K, int32_t Ds) {
    if (B < 1 || B > kMaxGenBatch || !pgen_dims_ok(D, R, K, Ds)) return 0;
    return paper_generator_ws_bytes(B, D, R, K, Ds);
}

svdlut_status svdlut_paper_generator_fwd(const float* params, const void* x, svdlut_dtype io, int32_t B, int32_t H,
                                         int32_t W, int32_t D, int32_t R, int32_t K, int32_t Ds,
                                         const uint8_t* keep_mask, float* U, float* s, float* V, float* lut_w,
                                         float* lut_b, float* grids, float* gw, float* gb, void* ws,
                                         size_t ws_bytes, hipStream_t stream) {
    if (!params || !x || !U || !s || !V || !lut_w || !lut_b || !ws)
        return fail(SVDLUT_EINVAL, "paper_generator_fwd: null pointer");
    if (io != SVDLUT_F32 && io != SVDLUT_F16) return fail(SVDLUT_EUNSUPPORTED, "paper_generator_fwd: dtype");
    if (B < 1 || B > kMaxGenBatch || H < 1 || W < 1 || H > kMaxDim || W > kMaxDim)
        return fail(SVDLUT_EINVAL, "paper_generator_fwd: B, H, W out of range");
    if (!pgen_dims_ok(D, R, K, Ds)) return fail(SVDLUT_EINVAL, "paper_generator_fwd: D, R, K or Ds out of range");
    if (K > 0 && (!grids || !gw || !gb)) return fail(SVDLUT_EINVAL, "paper_generator_fwd: null grid output");
    if (ws_bytes < paper_generator_ws_bytes(B, D, R, K, Ds))
        return fail(SVDLUT_EINVAL, "paper_generator_fwd: workspace smaller than svdlut_paper_generator_workspace_size()");
    return paper_generator_forward(params, x, io, B, H, W, D, R, K, Ds, keep_mask, U, s, V, lut_w, lut_b, grids, gw,
                                   gb, ws, stream);
}

svdlut_status svdlut_paper_generator_bwd(const float* params, const uint8_t* keep_mask, const float* dU,
                                         const float* ds, const float* dV, const float* dlut_w, const float* dlut_b,
                                         const float* dgrids, const float* dgw, const float* dgb, float* grads,
                                         int32_t B, int32_t D, int32_t R, int32_t K, int32_t Ds, void* ws,
                                         size_t ws_bytes, hipStream_t stream) {
    if (!params || !grads || !ws) return fail(SVDLUT_EINVAL, "paper_generator_bwd: null pointer");
    if (B < 1 || B > kMaxGenBatch) return fail(SVDLUT_EINVAL, "paper_generator_bwd: B must be in [1, 4096]");
    if (!pgen_dims_ok(D, R, K, Ds)) return fail(SVDLUT_EINVAL, "paper_generator_bwd: D, R, K or Ds out of range");
    if (ws_bytes < paper_generator_ws_bytes(B, D, R, K, Ds))
        return fail(SVDLUT_EINVAL, "paper_generator_bwd: workspace smaller than svdlut_paper_generator_workspace_size()");
    return paper_generator_backward(params, keep_mask, dU, ds, dV, dlut_w, dlut_b, dgrids, dgw, dgb, grads, B, D, R,
                                    K, Ds, ws, stream);
}

}  // extern "C"
