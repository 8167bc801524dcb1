// Backward of the fused 2D-LUT transform: dL/dT (-> dU, ds, dV), dL/dmap, dL/dx, dL/dbias.
//
// Decomposition.  Each image gets `gpi` workgroups; workgroup j of image b processes a
// contiguous band of row segments.  It rebuilds T into LDS, accumulates its share of dT
// in a second LDS array, and writes that array to its own slot of a partial buffer (plain
// stores).  A second kernel sums the gpi partials of each LUT in a fixed order and applies
// the chain rule of T = U diag(s) V^T.  dmap contributions go first to per-wave staged map
// columns, then to a workgroup copy of the map rows its band touches, then to global
// memory (one atomic per touched map element per workgroup).  dx is written directly.
//
// Fixed-point LDS accumulation.  On gfx950 an LDS float atomic add costs about 200 cycles
// per wave instruction whatever the addresses, an LDS integer add about 17 (measured), so
// the LDS accumulators hold signed 32-bit fixed-point values.  Each workgroup first bounds
// its contributions: every dT term is dy * S * w with |S| <= max|map| (S interpolates the
// map) and 0 <= w <= 1, every dmap term is dy * phi * w with |phi| <= max|T|, an entry of LUT
// or map channel l only receives terms of output channel c = l / 3, and each pixel adds at
// most one term to an entry.  So no entry (and no partial sum of it) exceeds
// Sigma_c * max|map| (dT) or Sigma_c * max|T| (dmap), where Sigma_c is the band's sum of
// |dy_c|, and the scale is the largest power of two 2^e keeping max_c Sigma_c * max|.| * 2^e
// below 2^30: no accumulator can overflow, every term is rounded once to within 2^-(e+1) of
// its value, and the power-of-two scale makes the conversions exact apart from that one
// rounding.  A bound from the sum (rather than pixels x largest |dy|) keeps a few large |dy|
// from coarsening the grid of all other terms.  Terms below 2^22 take a two-instruction
// rounding; when the scale lets one pixel's term exceed it (a |dy| holding more than about
// 1/1024 of its band's sum) the workgroup uses the exact conversion instead.  Integer sums
// are independent of the order of the atomics.  Non-finite dy, map or T values (or bounds
// beyond the float range) make the workgroup report NaN for its dT and dmap contributions.
#include "bwd_common.h"

#include <algorithm>
#include <cfloat>

namespace svdlut {

namespace {

constexpr int kBwdStride = 9;   // values per staged map column in the backward
// floats per raw map column (nine top values at 0, nine row differences at 12); odd, like
// kBwdStride, so the ~32 columns a wave touches at once fall on distinct LDS banks
constexpr int kBwdRawStride = 21;

struct BwdDev {
    BwdLaunch a;
    int gpi;            // workgroups per image
    int64_t per;        // tiles per workgroup
    int ncol_max;       // staged columns per wave
    int mrows;          // map rows held per workgroup (0: flush dmap straight to global)
    int fast_map;
    int want_dT, want_dmap, want_dx, want_db;
    // fused loss (svdlut_apply_loss_bwd): a.dy holds the target and dy = dL/dy is formed per
    // pixel from the recomputed output
    const float* bias;  // forward bias [B][3] (nullable)
    float inv_n;        // 1 / (B * 3 * H * W)
    float* lpart;       // per-workgroup loss partial sums [B * gpi]
    // deterministic mode (rowlo non-null): each workgroup stores its first map row, its dbias
    // partial and its map-row accumulator as floats; det_reduce_kernel adds them up in
    // workgroup order instead of float atomics
    int* rowlo;         // [B * gpi]
    float* dbpart;      // [B * gpi][3]
    float* mpart;       // [B * gpi][9][mrows][w]
};

// Geometry shared by all tiles of a workgroup.
struct BwdGeo {
    AxisMap ax, ay;
    int nseg;
    int64_t plane, mplane;
};

// One tile (row y, 256-pixel segment seg) of the backward.  The staged raw map rows (the
// nine channels of rows iv and iv+1 for the segment's columns) are kept per wave and only
// reloaded when the wave moves to another segment or another pair of map rows.
// Term -> accumulator integer: the two-instruction rounding while terms stay below 2^22,
// the exact conversion when the workgroup's scale allows larger ones.
template <bool EXACT>
__device__ __forceinline__ int fixc(float a, float b) { return EXACT ? fix_exact(a, b) : fix_mul(a, b); }

template <typename IO, typename MT, bool FASTMAP, bool VEC, int LOSS, bool EXACT>
__device__ __forceinline__ void bwd_tile(const BwdDev& P, const BwdGeo& G, int b, int y, int seg,
                                         const float* Tl, int* dTl, int* macc, int row_lo,
                                         float* raw, float* stage, int* dstage, int& st_seg, int& st_iv,
                                         float sT, float sM, float iM, float (&dbsum)[3],
                                         const float (&bias3)[3], float& lacc) {
    const BwdLaunch& a = P.a;
    const int lane = threadIdx.x & (kWave - 1);
    const int H = a.H, W = a.W, h = a.h, w = a.w, D = a.D;
    (void)H;
    const int xs = seg * kSeg;
    // lane -> 4-pixel block of the segment by a fixed permutation (stride 17 of 64): lanes of
    // one instruction then sit far apart along the row, with less similar colours, so their
    // LDS atomics meet the same address less often
    const int x0 = xs + ((lane * 17) & (kWave - 1)) * kPxPerLane;
    const int xlast = min(xs + kSeg, W) - 1;
    const int64_t plane = G.plane;
    const int64_t img = static_cast<int64_t>(b) * 3 * plane + static_cast<int64_t>(y) * W;

    // the pixel loads go first: their latency overlaps the map staging below
    float px[3][4], gy[3][4];
    if (x0 < W) {
        const IO* xin = reinterpret_cast<const IO*>(a.x) + img;
        const IO* gin = reinterpret_cast<const IO*>(a.dy) + img;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            load_px4<IO, VEC>(xin + c * plane, x0, W, px[c]);
            load_px4<IO, VEC>(gin + c * plane, x0, W, gy[c]);
        }
    }

    int iv; uint32_t remv;
    axis_left(G.ay, y, iv, remv);
    const float dv = static_cast<float>(remv) * G.ay.inv;
    const int iv1 = min(iv + 1, h - 1);
    int clo; uint32_t rlo;
    axis_left(G.ax, xs, clo, rlo);
    int chi; uint32_t rhi;
    axis_left(G.ax, xlast, chi, rhi);
    chi = min(chi + 2, w - 1);
    const int ncols = chi - clo + 1;
    const int64_t mplane = G.mplane;

    if (seg != st_seg || iv != st_iv) {
        const MT* m0 = reinterpret_cast<const MT*>(a.map) + static_cast<int64_t>(b) * 9 * mplane +
                       static_cast<int64_t>(iv) * w + clo;
        const int64_t rowd = static_cast<int64_t>(iv1 - iv) * w;
        for (int j = lane; j < ncols; j += kWave) {
            float v0[9], v1[9];
#pragma unroll
            for (int l = 0; l < 9; ++l) {      // all eighteen loads in flight together
                v0[l] = ldf<MT>(m0 + l * mplane + j);
                v1[l] = ldf<MT>(m0 + l * mplane + rowd + j);
            }
            float* dst = raw + j * kBwdRawStride;
#pragma unroll
            for (int l = 0; l < 9; ++l) {
                dst[l] = v0[l];
                dst[12 + l] = v1[l] - v0[l];
            }
        }
        st_seg = seg;
        st_iv = iv;
        wave_sync();
    }
    for (int j = lane; j < ncols; j += kWave) {
        const float* src = raw + j * kBwdRawStride;
#pragma unroll
        for (int l = 0; l < 9; ++l) {
            stage[j * kBwdStride + l] = fmaf(dv, src[12 + l], src[l]);
            dstage[j * kBwdStride + l] = 0;
        }
    }
    wave_sync();

    // a one-column map (a scalar weight per LUT, as in the paper's model): every lane's terms
    // land on column 0, so the wave adds them up first and one lane adds the nine sums
    const bool one_col = FASTMAP && w == 1;
    int msum[9];
#pragma unroll
    for (int l = 0; l < 9; ++l) msum[l] = 0;
    if (x0 < W) {
        float dx[3][4];
        const AxisMap& ax = G.ax;
        int c0; uint32_t rem0;
        axis_left(ax, x0, c0, rem0);
        const float Dm1 = static_cast<float>(D - 1);
        const int Dm2 = D - 2;
        const int rowstep = lut_row_stride(D);
        const int pairstep = lut_pair_stride(D);

        float r0[9], d01[9], d12[9], A0[9], A1[9], A2[9];
        const int j0 = c0 - clo;
        const int j1 = min(c0 + 1, w - 1) - clo;
        const int j2 = min(c0 + 2, w - 1) - clo;
        if (FASTMAP) {
#pragma unroll
            for (int l = 0; l < 9; ++l) {
                const float v0 = stage[j0 * kBwdStride + l];
                const float v1 = stage[j1 * kBwdStride + l];
                const float v2 = stage[j2 * kBwdStride + l];
                r0[l] = v0; d01[l] = v1 - v0; d12[l] = v2 - v1;
                A0[l] = 0.f; A1[l] = 0.f; A2[l] = 0.f;
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
#pragma unroll
            for (int c = 0; c < 3; ++c) dx[c][k] = 0.f;
            if (x0 + k >= W) continue;
            float S[9], ta = 0.f, tb = 0.f, du = 0.f;
            int jk = 0, jk1 = 0;
            if (FASTMAP) {
                const uint32_t n = rem0 + static_cast<uint32_t>(k) * ax.num_step;
                ta = static_cast<float>(min(n, ax.div.d)) * ax.inv;
                tb = static_cast<float>(n > ax.div.d ? n - ax.div.d : 0u) * ax.inv;
#pragma unroll
                for (int l = 0; l < 9; ++l) S[l] = fmaf(tb, d12[l], fmaf(ta, d01[l], r0[l]));
            } else {
                int ck; uint32_t rk;
                axis_left(ax, x0 + k, ck, rk);
                du = static_cast<float>(rk) * ax.inv;
                jk = ck - clo;
                jk1 = min(ck + 1, w - 1) - clo;
#pragma unroll
                for (int l = 0; l < 9; ++l) {
                    const float s0 = stage[jk * kBwdStride + l];
                    S[l] = fmaf(du, stage[jk1 * kBwdStride + l] - s0, s0);
                }
            }
            int ii[3]; float dd[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) decode(px[c][k], Dm1, Dm2, ii[c], dd[c]);
            if (LOSS) {
                // forward output of this pixel (Y_c = sum_p S_{3c+p} phi_{3c+p} + b_c), the loss
                // term against the target held in gy, and dL/dy in its place
                float yv[3] = {bias3[0], bias3[1], bias3[2]};
#pragma unroll
                for (int p = 0; p < 3; ++p) {
                    const int al = (p == 2) ? 1 : 0;
                    const int be = (p == 0) ? 1 : 2;
                    const float da = dd[al], db = dd[be];
                    const float w11 = da * db;
                    const float w10 = da - w11;
                    const float w01 = db - w11;
                    const float w00 = 1.f - da - db + w11;
                    const float* t0 = Tl + p * pairstep + ii[al] * rowstep + kNode * ii[be];
                    const float* t1 = t0 + rowstep;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        float phi = w00 * t0[c];
                        phi = fmaf(w10, t1[c], phi);
                        phi = fmaf(w01, t0[kNode + c], phi);
                        phi = fmaf(w11, t1[kNode + c], phi);
                        yv[c] = fmaf(S[3 * c + p], phi, yv[c]);
                    }
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float d = yv[c] - gy[c][k];
                    if (LOSS == 1) {
                        lacc += fabsf(d);
                        gy[c][k] = d > 0.f ? P.inv_n : (d < 0.f ? -P.inv_n : 0.f);
                    } else {
                        lacc = fmaf(d, d, lacc);
                        gy[c][k] = 2.f * d * P.inv_n;
                    }
                }
            }
            float gx[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int c = 0; c < 3; ++c) dbsum[c] += gy[c][k];
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                const int al = (p == 2) ? 1 : 0;
                const int be = (p == 0) ? 1 : 2;
                const float da = dd[al], db = dd[be];
                const float w11 = da * db;
                const float w10 = da - w11;
                const float w01 = db - w11;
                const float w00 = 1.f - da - db + w11;
                const int slot = p * pairstep + ii[al] * rowstep + kNode * ii[be];
                const float* t0 = Tl + slot;
                const float* t1 = t0 + rowstep;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float T00 = t0[c], T01 = t0[kNode + c], T10 = t1[c], T11 = t1[kNode + c];
                    const float g = gy[c][k] * S[3 * c + p];
                    if (P.want_dT) {
                        int* q0 = dTl + slot;
                        int* q1 = q0 + rowstep;
                        const float gs = g * sT;
                        lds_addi(q0 + c, fixc<EXACT>(gs, w00));
                        lds_addi(q1 + c, fixc<EXACT>(gs, w10));
                        lds_addi(q0 + kNode + c, fixc<EXACT>(gs, w01));
                        lds_addi(q1 + kNode + c, fixc<EXACT>(gs, w11));
                    }
                    gx[al] = fmaf(g, (1.f - db) * (T10 - T00) + db * (T11 - T01), gx[al]);
                    gx[be] = fmaf(g, (1.f - da) * (T01 - T00) + da * (T11 - T10), gx[be]);
                    if (P.want_dmap) {
                        float phi = w00 * T00;
                        phi = fmaf(w10, T10, phi);
                        phi = fmaf(w01, T01, phi);
                        phi = fmaf(w11, T11, phi);
                        const float gp = gy[c][k] * phi;
                        const int l = 3 * c + p;
                        if (FASTMAP) {
                            A0[l] = fmaf(gp, 1.f - ta, A0[l]);
                            A1[l] = fmaf(gp, ta - tb, A1[l]);
                            A2[l] = fmaf(gp, tb, A2[l]);
                        } else {
                            const float gps = gp * sM;
                            lds_addi(dstage + jk * kBwdStride + l, fixc<EXACT>(gps, 1.f - du));
                            lds_addi(dstage + jk1 * kBwdStride + l, fixc<EXACT>(gps, du));
                        }
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float xv = px[c][k];
                dx[c][k] = (xv >= 0.f && xv <= 1.f) ? Dm1 * gx[c] : 0.f;
            }
        }
        if (FASTMAP && P.want_dmap) {
            if (one_col) {
#pragma unroll
                for (int l = 0; l < 9; ++l) msum[l] = fixc<EXACT>(A0[l] + A1[l] + A2[l], sM);
            } else {
#pragma unroll
                for (int l = 0; l < 9; ++l) {
                    lds_addi(dstage + j0 * kBwdStride + l, fixc<EXACT>(A0[l], sM));
                    lds_addi(dstage + j1 * kBwdStride + l, fixc<EXACT>(A1[l], sM));
                    lds_addi(dstage + j2 * kBwdStride + l, fixc<EXACT>(A2[l], sM));
                }
            }
        }
        if (P.want_dx) {
            IO* dxo = reinterpret_cast<IO*>(a.dx) + img;
#pragma unroll
            for (int c = 0; c < 3; ++c) store_px4<IO, VEC>(dxo + c * plane, x0, W, dx[c]);
        }
    }
    if (one_col && P.want_dmap) {   // integer sums: exact in any order
#pragma unroll
        for (int l = 0; l < 9; ++l) {
            int v = msum[l];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) lds_addi(dstage + l, v);
        }
    }
    wave_sync();
    if (P.want_dmap) {
        // distribute the staged column sums to the two map rows around y
        for (int j = lane; j < ncols; j += kWave) {
            const int col = clo + j;
#pragma unroll
            for (int l = 0; l < 9; ++l) {
                const int v = dstage[j * kBwdStride + l];
                if (v == 0) continue;
                if (P.mrows > 0) {
                    // exact split of the fixed-point column sum between the two rows
                    const int v0 = fix(static_cast<float>(v) * (1.f - dv));
                    lds_addi(macc + (l * P.mrows + (iv - row_lo)) * w + col, v0);
                    if (iv1 != iv) lds_addi(macc + (l * P.mrows + (iv1 - row_lo)) * w + col, v - v0);
                } else {
                    const float fv = static_cast<float>(v) * iM;
                    float* dm = a.dmap + static_cast<int64_t>(b) * 9 * mplane + l * mplane;
                    gbl_add(dm + static_cast<int64_t>(iv) * w + col, fv * (1.f - dv));
                    if (iv1 != iv) gbl_add(dm + static_cast<int64_t>(iv1) * w + col, fv * dv);
                }
            }
        }
        wave_sync();
    }
}

// Per-channel sums of |dy| and the largest |dy| over [0, n) of the three channel planes
// starting at p (plane stride `plane`), all three walked together so that a thread's loads
// of the three planes are in flight at once.  Each channel's sum takes its values in the
// same order as abssum_range would.
template <typename IO>
__device__ inline void scan_dy3(const IO* p, int64_t plane, int64_t n, float (&s)[3], float& m, bool& bad) {
    const bool vec = ((plane & 3) == 0) && (reinterpret_cast<uintptr_t>(p) & (4 * sizeof(IO) - 1)) == 0;
    if (!vec) {
        for (int c = 0; c < 3; ++c) abssum_range<IO>(p + c * plane, n, s[c], m, bad);
        return;
    }
    const int64_t n4 = n / 4, step = blockDim.x;
    int64_t v = threadIdx.x;
    for (; v + 3 * step < n4; v += 4 * step) {
        float q[3][4][4];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int u = 0; u < 4; ++u) ld4<IO>(p + c * plane + 4 * (v + u * step), q[c][u]);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int e = 0; e < 4; ++e) abssum_acc(q[c][u][e], s[c], m, bad);
    }
    for (; v < n4; v += step)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float q[4];
            ld4<IO>(p + c * plane + 4 * v, q);
#pragma unroll
            for (int e = 0; e < 4; ++e) abssum_acc(q[e], s[c], m, bad);
        }
    for (int64_t i = n4 * 4 + threadIdx.x; i < n; i += blockDim.x)
#pragma unroll
        for (int c = 0; c < 3; ++c) abssum_acc(ldf<IO>(p + c * plane + i), s[c], m, bad);
}

// Largest |value| over the first n entries of nine map planes (stride mplane) from p: one
// flat walk over the 9n entries with eight loads per thread in flight (the band's map rows
// are short, so a walk per plane would wait for nine rounds of loads).
template <typename MT>
__device__ inline void scan_map9(const MT* p, int64_t mplane, int64_t n, float& m, bool& bad) {
    if (9 * n > INT32_MAX) {
        for (int l = 0; l < 9; ++l) absmax_range<MT>(p + l * mplane, n, m, bad);
        return;
    }
    const uint32_t n32 = static_cast<uint32_t>(n), total = 9u * n32, step = blockDim.x;
    for (uint32_t e0 = threadIdx.x; e0 < total; e0 += 8 * step) {
        float q[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t e = e0 + u * step;
            q[u] = 0.f;
            if (e < total) {
                const uint32_t l = e / n32;
                q[u] = ldf<MT>(p + l * mplane + (e - l * n32));
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) absmax_acc(q[u], m, bad);
    }
}

template <typename IO, typename MT, bool FASTMAP, int LOSS>
__global__ void __launch_bounds__(512) apply_bwd_kernel(BwdDev P) {
    extern __shared__ float smem[];
    const BwdLaunch& a = P.a;
    const int D = a.D;
    const int nlut = lut_floats(D);
    float* Tl = smem;
    int* dTl = reinterpret_cast<int*>(Tl + nlut);
    int* macc = dTl + nlut;
    const int macc_n = P.mrows * 9 * a.w;
    float* aux = reinterpret_cast<float*>(macc + ((macc_n + 3) & ~3));
    const int nw = blockDim.x / kWave;
    const int wave = threadIdx.x / kWave;
    float* raw = aux + wave * P.ncol_max * (kBwdRawStride + 2 * kBwdStride);
    float* stage = raw + P.ncol_max * kBwdRawStride;
    int* dstage = reinterpret_cast<int*>(stage + P.ncol_max * kBwdStride);

    const int lb = logical_block(blockIdx.x, gridDim.x);
    const int b = lb / P.gpi;
    const int j = lb - b * P.gpi;
    const int nseg = (a.W + kSeg - 1) / kSeg;
    const int64_t tpi = static_cast<int64_t>(a.H) * nseg;
    const int64_t t0 = static_cast<int64_t>(j) * P.per;
    const int64_t t1 = min(tpi, t0 + P.per);

    // map rows this band touches
    int row_lo = 0, row_hi = -1;
    if (t0 < t1) {
        const AxisMap ay = make_axis(a.H, a.h);
        uint32_t r;
        axis_left(ay, static_cast<int>(t0 / nseg), row_lo, r);
        axis_left(ay, static_cast<int>((t1 - 1) / nseg), row_hi, r);
        row_hi = min(row_hi + 1, a.h - 1);
    }
    const size_t foff = static_cast<size_t>(b) * 9 * D * a.R;
    stage_luts(Tl, aux, a.U + foff, a.s + static_cast<size_t>(b) * 9 * a.R, a.V + foff, D, a.R,
               min(a.R, 8));
    for (int e = threadIdx.x; e < nlut; e += blockDim.x) dTl[e] = 0;
    for (int e = threadIdx.x; e < macc_n; e += blockDim.x) macc[e] = 0;
    __syncthreads();

    // bounds of the band's contributions -> fixed-point scales
    const int64_t plane = static_cast<int64_t>(a.H) * a.W;
    float sT = 1.f, sM = 1.f;
    bool bad = false;
    float bias3[3] = {0.f, 0.f, 0.f};
    if (LOSS && P.bias) {
#pragma unroll
        for (int c = 0; c < 3; ++c) bias3[c] = P.bias[3 * b + c];
    }
    bool exact = false;
    if ((P.want_dT || P.want_dmap) && t0 < t1) {
        float mdy = 0.f, mmap = 0.f, mT = 0.f;
        float sdy[3] = {0.f, 0.f, 0.f};
        bool nf = false;
        const int64_t e0 = (t0 / nseg) * a.W + (t0 % nseg) * kSeg;
        const int64_t e1 = ((t1 - 1) / nseg) * a.W + min(((t1 - 1) % nseg) * kSeg + kSeg, static_cast<int64_t>(a.W));
        const IO* dyb = reinterpret_cast<const IO*>(a.dy) + static_cast<int64_t>(b) * 3 * plane;
        // dy given: the band's per-channel sums of |dy| (an entry of LUT or map channel l
        // only receives terms of output channel l / 3) and its maximum.  L1: |dy| = 1/n at
        // most.  MSE: |dy| = 2 |y - t| / n with |y_c| <= 3 max|map| max|T| + |b_c| and the
        // band's sums and maximum of |t| (the dy buffer holds the target).
        if (LOSS != 1) scan_dy3<IO>(dyb + e0, plane, e1 - e0, sdy, mdy, nf);
        if (P.want_dT || LOSS == 2) {
            const int64_t mplane = static_cast<int64_t>(a.h) * a.w;
            const MT* mb = reinterpret_cast<const MT*>(a.map) + static_cast<int64_t>(b) * 9 * mplane +
                           static_cast<int64_t>(row_lo) * a.w;
            scan_map9<MT>(mb, mplane, static_cast<int64_t>(row_hi - row_lo + 1) * a.w, mmap, nf);
        }
        if (P.want_dmap || LOSS == 2) {
            // every vertex row of the three pairs: D * kNode contiguous values
            const int RS = lut_row_stride(D), PS = lut_pair_stride(D);
            for (int r = wave; r < 3 * D; r += nw) {
                const int p = r / D;
                const float* row = Tl + p * PS + (r - p * D) * RS;
                for (int k = threadIdx.x & (kWave - 1); k < D * kNode; k += kWave) {
                    const float v = fabsf(row[k]);
                    nf |= !(v <= FLT_MAX);
                    mT = fmaxf(mT, v);
                }
            }
        }
        // one block-wide reduction of the seven values (lanes by butterfly, then waves in order)
        float red[7] = {mdy, sdy[0], sdy[1], sdy[2], mmap, mT, nf ? 1.f : 0.f};
#pragma unroll
        for (int k = 0; k < 7; ++k)
            for (int off = 32; off > 0; off >>= 1) {
                const float o = __shfl_xor(red[k], off, 64);
                red[k] = (k >= 1 && k <= 3) ? red[k] + o : fmaxf(red[k], o);
            }
        if ((threadIdx.x & (kWave - 1)) == 0)
#pragma unroll
            for (int k = 0; k < 7; ++k) aux[wave * 8 + k] = red[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            float m = aux[k];
            for (int i = 1; i < nw; ++i) m = (k >= 1 && k <= 3) ? m + aux[i * 8 + k] : fmaxf(m, aux[i * 8 + k]);
            red[k] = m;
        }
        __syncthreads();   // aux is the waves' staging area from here on
        mdy = red[0];
        float sdm = 0.f;
        if (LOSS != 1) sdm = fmaxf(red[1], fmaxf(red[2], red[3]));
        mmap = red[4];
        mT = red[5];
        bad = red[6] > 0.f;
        const float n = static_cast<float>((t1 - t0) * kSeg);   // band pixels (padding included)
        if (LOSS == 1) {
            mdy = P.inv_n;
            sdm = n * P.inv_n;
        }
        if (LOSS == 2) {
            const float mb = fmaxf(fabsf(bias3[0]), fmaxf(fabsf(bias3[1]), fabsf(bias3[2])));
            const float ymax = 3.f * mmap * mT + mb;
            sdm = 2.f * (n * ymax + sdm) * P.inv_n;
            mdy = 2.f * (ymax + mdy) * P.inv_n;
            bad = bad || !(sdm <= FLT_MAX);
        }
        sT = fix_scale_sum(sdm, mdy, mmap, exact, bad);
        sM = fix_scale_sum(sdm, mdy, mT, exact, bad);
    }
    const float iT = 1.f / sT, iM = 1.f / sM;

    float dbsum[3] = {0.f, 0.f, 0.f};
    float lacc = 0.f;
    const bool base_ok = ((plane | a.W) & 3) == 0 &&
                         ((reinterpret_cast<uintptr_t>(a.x) | reinterpret_cast<uintptr_t>(a.dy) |
                           reinterpret_cast<uintptr_t>(a.dx)) & (4 * sizeof(IO) - 1)) == 0;
    if (t0 < t1) {
        BwdGeo G;
        G.ax = make_axis(a.W, a.w);
        G.ay = make_axis(a.H, a.h);
        G.nseg = nseg;
        G.plane = plane;
        G.mplane = static_cast<int64_t>(a.h) * a.w;
        const float iMx = bad ? __builtin_nanf("") : iM;
        // The band's rows [ya, yb] x segments, walked column-major (same segment, consecutive
        // rows) in one contiguous run per wave, so the staged map rows are reused.
        const int ya = static_cast<int>(t0 / nseg);
        const int nr = static_cast<int>((t1 - 1) / nseg) - ya + 1;
        const int total = nr * nseg;
        const int q = (total + nw - 1) / nw;
        const int k0 = min(total, wave * q);
        const int k1 = min(total, k0 + q);
        int st_seg = -1, st_iv = -1;
        for (int k = k0; k < k1; ++k) {
            const int seg = k / nr;
            const int y = ya + (k - seg * nr);
            const int64_t lt = static_cast<int64_t>(y) * nseg + seg;
            if (lt < t0 || lt >= t1) continue;
            const bool vec = base_ok && seg * kSeg + kSeg <= a.W;
            if (!exact) {
                if (vec)
                    bwd_tile<IO, MT, FASTMAP, true, LOSS, false>(P, G, b, y, seg, Tl, dTl, macc, row_lo, raw, stage,
                                                                 dstage, st_seg, st_iv, sT, sM, iMx, dbsum, bias3, lacc);
                else
                    bwd_tile<IO, MT, FASTMAP, false, LOSS, false>(P, G, b, y, seg, Tl, dTl, macc, row_lo, raw, stage,
                                                                  dstage, st_seg, st_iv, sT, sM, iMx, dbsum, bias3, lacc);
            } else {
                if (vec)
                    bwd_tile<IO, MT, FASTMAP, true, LOSS, true>(P, G, b, y, seg, Tl, dTl, macc, row_lo, raw, stage,
                                                                dstage, st_seg, st_iv, sT, sM, iMx, dbsum, bias3, lacc);
                else
                    bwd_tile<IO, MT, FASTMAP, false, LOSS, true>(P, G, b, y, seg, Tl, dTl, macc, row_lo, raw, stage,
                                                                 dstage, st_seg, st_iv, sT, sM, iMx, dbsum, bias3, lacc);
            }

        }
    }
    __syncthreads();

    if (P.want_dT) {
        float* part = a.dT + (static_cast<size_t>(b) * P.gpi + j) * nlut;
        for (int e = threadIdx.x; e < nlut; e += blockDim.x)
            part[e] = bad ? __builtin_nanf("") : static_cast<float>(dTl[e]) * iT;
    }
    if (P.rowlo && threadIdx.x == 0) P.rowlo[lb] = t0 < t1 ? row_lo : a.h;   // a.h: no rows
    if (P.want_dmap && P.mpart && t0 < t1) {
        float* dst = P.mpart + static_cast<size_t>(lb) * macc_n;
        for (int e = threadIdx.x; e < macc_n; e += blockDim.x)
            dst[e] = bad ? __builtin_nanf("") : static_cast<float>(macc[e]) * iM;
    } else if (P.want_dmap && P.mrows > 0 && t0 < t1) {
        const int64_t mplane = static_cast<int64_t>(a.h) * a.w;
        for (int e = threadIdx.x; e < macc_n; e += blockDim.x) {
            const int l = e / (P.mrows * a.w);
            const int rr = (e / a.w) % P.mrows;
            const int col = e % a.w;
            const int row = row_lo + rr;
            const int v = macc[e];
            if (row < a.h && (v != 0 || bad))
                gbl_add(a.dmap + static_cast<int64_t>(b) * 9 * mplane + l * mplane +
                            static_cast<int64_t>(row) * a.w + col,
                        bad ? __builtin_nanf("") : static_cast<float>(v) * iM);
        }
    }
    if (P.want_db) {
        // the workgroup's dbias: lanes, then waves in order; one value per channel leaves the
        // workgroup (a global atomic per wave would queue on the image's three addresses)
        __shared__ float dbw[3][1024 / kWave];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float v = dbsum[c];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if ((threadIdx.x & 63) == 0) dbw[c][wave] = v;
        }
        __syncthreads();
        if (threadIdx.x < 3) {
            float v = 0.f;
            for (int i = 0; i < nw; ++i) v += dbw[threadIdx.x][i];
            if (P.dbpart) P.dbpart[3 * lb + threadIdx.x] = v;
            else gbl_add(a.dbias + 3 * b + threadIdx.x, v);
        }
    }
    if (LOSS) {
        // this workgroup's loss sum: lanes, then waves in order (aux is free after the barrier)
        for (int off = 32; off > 0; off >>= 1) lacc += __shfl_xor(lacc, off, 64);
        if ((threadIdx.x & 63) == 0) aux[wave] = lacc;
        __syncthreads();
        if (threadIdx.x == 0) {
            float s = 0.f;
            for (int i = 0; i < nw; ++i) s += aux[i];
            P.lpart[lb] = s;
        }
    }
}

// loss = inv_n * sum of the per-workgroup partials, in order (fp64).
// (run by the first wave of a workgroup)
__device__ inline void loss_sum(const float* __restrict__ part, int n, float inv_n, float* __restrict__ out) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 64) acc += part[i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (threadIdx.x == 0) out[0] = static_cast<float>(acc * static_cast<double>(inv_n));
}

// Deterministic mode: dmap and dbias from the per-workgroup partials, added in workgroup
// order.  The workgroups of an image cover consecutive bands, so their first map rows rowlo
// do not decrease with the workgroup index; the ones whose accumulator [rowlo, rowlo + mrows)
// holds row r form a run found by a binary search.  Workgroups without rows carry rowlo = h.
__device__ inline void det_reduce_item(int64_t i, const int* __restrict__ rowlo, const float* __restrict__ mpart,
                                       const float* __restrict__ dbpart, float* __restrict__ dmap,
                                       float* __restrict__ dbias, int B, int gpi, int mrows, int h, int w) {
    const int64_t nmap = dmap ? static_cast<int64_t>(B) * 9 * h * w : 0;
    if (i < nmap) {
        const int col = static_cast<int>(i % w);
        const int r = static_cast<int>((i / w) % h);
        const int l = static_cast<int>((i / (static_cast<int64_t>(w) * h)) % 9);
        const int b = static_cast<int>(i / (static_cast<int64_t>(w) * h * 9));
        const int* rl = rowlo + static_cast<int64_t>(b) * gpi;
        int lo = 0, hi = gpi;           // first j with rl[j] + mrows > r
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (rl[mid] + mrows > r) hi = mid; else lo = mid + 1;
        }
        float acc = 0.f;
        for (int j = lo; j < gpi && rl[j] <= r; ++j)
            acc += mpart[((static_cast<int64_t>(b) * gpi + j) * 9 + l) * mrows * w +
                         static_cast<int64_t>(r - rl[j]) * w + col];
        dmap[i] = acc;
    } else if (dbias && i < nmap + 3 * B) {
        const int k = static_cast<int>(i - nmap), b = k / 3, c = k - 3 * (k / 3);
        float acc = 0.f;
        for (int j = 0; j < gpi; ++j) acc += dbpart[(static_cast<int64_t>(b) * gpi + j) * 3 + c];
        dbias[k] = acc;
    }
}

// Sum the per-workgroup dT partials (fixed order) and apply the chain rule of
// T = U diag(s) V^T: dU = dT V diag(s), dV = dT^T U diag(s), ds_k = sum_i U_ik (dT V)_ik.
__device__ inline void factor_grad_block(int bl, float* sm, const float* __restrict__ part, int gpi,
                                         const float* __restrict__ U, const float* __restrict__ s,
                                         const float* __restrict__ V, float* __restrict__ dU,
                                         float* __restrict__ ds, float* __restrict__ dV, int D, int R) {
    // bl = b*9 + l
    const int b = bl / 9, l = bl - 9 * (bl / 9);
    const int c = l / 3, p = l - 3 * (l / 3);
    const int nlut = lut_floats(D);
    float* dT = sm;                     // [D][D]
    float* Us = dT + D * D;             // [D][R]
    float* Vs = Us + D * R;             // [D][R]
    float* Pm = Vs + D * R;             // [D][R]  dT V
    const float* u = U + static_cast<size_t>(bl) * D * R;
    const float* v = V + static_cast<size_t>(bl) * D * R;
    const float* sv = s + static_cast<size_t>(bl) * R;
    for (int e = threadIdx.x; e < D * D; e += blockDim.x) {
        const int i = e / D, jj = e - (e / D) * D;
        const float* src = part + static_cast<size_t>(b) * gpi * nlut + lut_slot(p, i, jj, c, D);
        // fixed summation order; sixteen independent loads in flight per step
        float acc = 0.f;
        int g = 0;
        for (; g + 16 <= gpi; g += 16) {
            float v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = src[static_cast<size_t>(g + u) * nlut];
#pragma unroll
            for (int u = 0; u < 16; ++u) acc += v[u];
        }
        for (; g < gpi; ++g) acc += src[static_cast<size_t>(g) * nlut];
        dT[e] = acc;
    }
    for (int e = threadIdx.x; e < D * R; e += blockDim.x) { Us[e] = u[e]; Vs[e] = v[e]; }
    __syncthreads();
    for (int e = threadIdx.x; e < D * R; e += blockDim.x) {
        const int i = e / R, k = e - (e / R) * R;
        float accP = 0.f, accQ = 0.f;
        for (int jj = 0; jj < D; ++jj) {
            accP = fmaf(dT[i * D + jj], Vs[jj * R + k], accP);   // (dT V)_ik
            accQ = fmaf(dT[jj * D + i], Us[jj * R + k], accQ);   // (dT^T U)_ik
        }
        Pm[e] = accP;
        dU[static_cast<size_t>(bl) * D * R + e] = accP * sv[k];
        dV[static_cast<size_t>(bl) * D * R + e] = accQ * sv[k];
    }
    __syncthreads();
    for (int k = threadIdx.x; k < R; k += blockDim.x) {
        float acc = 0.f;
        for (int i = 0; i < D; ++i) acc = fmaf(Us[i * R + k], Pm[i * R + k], acc);
        ds[static_cast<size_t>(bl) * R + k] = acc;
    }
}

// Everything that runs after the backward's main kernel, in one launch of 1024-thread
// workgroups: workgroups [0, nfac) sum the dT partials of one LUT channel each and form dU,
// ds, dV; the next nred workgroups (deterministic mode) form dmap and dbias from their
// partials, 1024 entries each; one last workgroup (fused loss) sums the loss partials.
struct PostArgs {
    int nfac, nred, with_loss;
    const float* part; int gpi;
    const float *U, *s, *V;
    float *dU, *ds, *dV;
    int D, R;
    const int* rowlo; const float *mpart, *dbpart;
    float *dmap, *dbias;
    int B, mrows, h, w;
    const float* lpart; int nlp; float inv_n; float* loss;
};

__global__ void __launch_bounds__(1024) bwd_post_kernel(PostArgs A) {
    extern __shared__ float sm[];
    int bid = blockIdx.x;
    if (bid < A.nfac) {
        factor_grad_block(bid, sm, A.part, A.gpi, A.U, A.s, A.V, A.dU, A.ds, A.dV, A.D, A.R);
        return;
    }
    bid -= A.nfac;
    if (bid < A.nred) {
        det_reduce_item(static_cast<int64_t>(bid) * blockDim.x + threadIdx.x, A.rowlo, A.mpart, A.dbpart, A.dmap,
                        A.dbias, A.B, A.gpi, A.mrows, A.h, A.w);
        return;
    }
    if (A.with_loss && threadIdx.x < kWave) loss_sum(A.lpart, A.nlp, A.inv_n, A.loss);
}

// Clears p[0, n) and q[0, m) (either may be empty) in one launch: 16-byte stores over the
// 16-byte-aligned body of each range, element stores for its ends.
__device__ inline void zero_range(float* p, int64_t n, int64_t tid, int64_t nthr) {
    if (n <= 0) return;
    const int64_t head = std::min<int64_t>(n, ((16 - (reinterpret_cast<uintptr_t>(p) & 15)) & 15) / 4);
    const int64_t n4 = (n - head) / 4;
    float4* b = reinterpret_cast<float4*>(p + head);
    for (int64_t i = tid; i < n4; i += nthr) b[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (tid < head) p[tid] = 0.f;
    const int64_t t0 = head + 4 * n4;
    if (tid < n - t0) p[t0 + tid] = 0.f;
}

__global__ void zero_kernel(float* p, int64_t n, float* q, int64_t m) {
    const int64_t tid = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    const int64_t nthr = static_cast<int64_t>(gridDim.x) * blockDim.x;
    zero_range(p, n, tid, nthr);
    zero_range(q, m, tid, nthr);
}

}  // namespace

constexpr int kBwdPartials = 256;   // one workgroup per CU in a single round

int bwd_groups_per_image(int B) { return std::max(1, kBwdPartials / std::max(B, 1)); }

size_t bwd_workspace_bytes(int B, int D) {
    const size_t nlut = static_cast<size_t>(lut_floats(D));
    return sizeof(float) * nlut * static_cast<size_t>(B) * bwd_groups_per_image(B);
}

// Segments per workgroup and the map rows its band can touch (the map-row accumulator's
// height before the LDS check, which may only lower it to 0).
static void bwd_band(int B, int H, int W, int h, int64_t& per, int& mrows) {
    const int gpi = bwd_groups_per_image(B);
    const int nseg = (W + kSeg - 1) / kSeg;
    const int64_t tpi = static_cast<int64_t>(H) * nseg;
    per = (tpi + gpi - 1) / gpi;
    const int64_t band_rows = per / nseg + 2;
    const int64_t mr = (H > 1) ? (band_rows * (h - 1)) / (H - 1) + 3 : 1;
    mrows = static_cast<int>(std::min<int64_t>(h, mr));
}

// Deterministic-mode partials: first map rows (int), dbias partials, map-row accumulators.
struct DetLayout {
    size_t rowlo, dbpart, mpart, total;
};
static DetLayout det_layout(int B, int H, int W, int h, int w) {
    int64_t per;
    int mrows;
    bwd_band(B, H, W, h, per, mrows);
    const size_t nwg = static_cast<size_t>(B) * bwd_groups_per_image(B);
    auto al = [](size_t v) { return (v + 255) & ~static_cast<size_t>(255); };
    DetLayout L;
    L.rowlo = 0;
    L.dbpart = al(nwg * sizeof(int));
    L.mpart = L.dbpart + al(nwg * 3 * sizeof(float));
    L.total = L.mpart + al(nwg * 9 * static_cast<size_t>(mrows) * w * sizeof(float));
    return L;
}

size_t bwd_det_bytes(int B, int H, int W, int h, int w) { return det_layout(B, H, W, h, w).total; }

// LDS of the backward: T (float) and dT (int32), the map-row accumulator (int32), and per
// wave the raw map rows, the blended map row (float) and its gradient (int32); the LUT
// rebuild scratch and the block reductions reuse the staging area.
static size_t bwd_lds(int D, int block, int ncol_max, int mrows, int w, int R) {
    (void)R;
    const size_t nlut = static_cast<size_t>(lut_floats(D));
    const size_t macc = (static_cast<size_t>(mrows) * 9 * w + 3) & ~static_cast<size_t>(3);
    const size_t stage = static_cast<size_t>(block / kWave) * ncol_max * (kBwdRawStride + 2 * kBwdStride);
    const size_t scratch = static_cast<size_t>(2) * 9 * D * 8;
    return sizeof(float) * (2 * nlut + macc + std::max(stage, scratch));
}

// Fused loss of svdlut_apply_loss_bwd: kind (1 = L1, 2 = MSE), forward bias, partial sums
// and the output value.
struct LossArgs {
    int kind;
    const float* bias;
    float* lpart;
    float* loss;
};

static svdlut_status launch_bwd_impl(const BwdLaunch& a, const LossArgs* L, hipStream_t st) {
    const DeviceInfo& di = device_info();
    BwdDev P{};
    P.a = a;
    const int loss = L ? L->kind : 0;
    if (L) {
        P.bias = L->bias;
        P.lpart = L->lpart;
        P.inv_n = static_cast<float>(1.0 / (3.0 * static_cast<double>(a.B) * a.H * a.W));
    }
    P.gpi = bwd_groups_per_image(a.B);
    int mrows = 0;
    bwd_band(a.B, a.H, a.W, a.h, P.per, mrows);
    P.ncol_max = map_cols_bound(a.W, a.w);
    P.fast_map = map_fast_ok(a.W, a.w) ? 1 : 0;
    P.want_dT = a.dU != nullptr;
    P.want_dmap = a.dmap != nullptr;
    P.want_dx = a.dx != nullptr;
    P.want_db = a.dbias != nullptr;
    int block = 0;
    // fine maps need narrow workgroups for their per-wave column staging
    const int blocks[4] = {512, 256, 128, 64};
    for (int pass = 0; pass < 2 && block == 0; ++pass) {
        for (int bk : blocks) {
            if (bwd_lds(a.D, bk, P.ncol_max, mrows, a.w, a.R) <= static_cast<size_t>(di.lds_per_block)) {
                block = bk;
                break;
            }
        }
        if (block == 0) mrows = 0;   // too many map columns: send dmap straight to global atomics
    }
    if (block == 0)
        return fail(SVDLUT_EUNSUPPORTED, "apply_bwd: the map columns one 256-pixel segment touches (" +
                                             std::to_string(P.ncol_max) + ") do not fit the LDS next to T and dT at D = " +
                                             std::to_string(a.D));
    P.mrows = P.want_dmap ? mrows : 0;
    const size_t lds = bwd_lds(a.D, block, P.ncol_max, P.mrows, a.w, a.R);
    const bool det = a.det && (a.dmap || a.dbias);
    if (det) {
        if (a.dmap && P.mrows == 0)
            return fail(SVDLUT_EUNSUPPORTED, "apply_bwd: deterministic mode needs the map-row accumulator, "
                                             "which does not fit the LDS for this map");
        const DetLayout L = det_layout(a.B, a.H, a.W, a.h, a.w);
        char* base = static_cast<char*>(a.det);
        P.rowlo = reinterpret_cast<int*>(base + L.rowlo);
        P.dbpart = a.dbias ? reinterpret_cast<float*>(base + L.dbpart) : nullptr;
        P.mpart = a.dmap ? reinterpret_cast<float*>(base + L.mpart) : nullptr;
    } else {
        const int64_t nm = a.dmap ? static_cast<int64_t>(a.B) * 9 * a.h * a.w : 0;
        const int64_t nb = a.dbias ? static_cast<int64_t>(a.B) * 3 : 0;
        if (nm + nb > 0) {
            const int64_t blocks = std::min<int64_t>(1024, (std::max(nm / 4, nb) + 255) / 256 + 1);
            hipLaunchKernelGGL(zero_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, a.dmap, nm,
                               a.dbias, nb);
        }
    }
    const int grid = a.B * P.gpi;
#define SVDLUT_BWD_L(IO, MT, LS)                                                                \
    do {                                                                                        \
        if (P.fast_map)                                                                         \
            hipLaunchKernelGGL((apply_bwd_kernel<IO, MT, true, LS>), dim3(grid), dim3(block), lds, st, P); \
        else                                                                                    \
            hipLaunchKernelGGL((apply_bwd_kernel<IO, MT, false, LS>), dim3(grid), dim3(block), lds, st, P); \
    } while (0)
#define SVDLUT_BWD(IO, MT)                                                                      \
    do {                                                                                        \
        if (loss == 1) SVDLUT_BWD_L(IO, MT, 1);                                                 \
        else if (loss == 2) SVDLUT_BWD_L(IO, MT, 2);                                            \
        else SVDLUT_BWD_L(IO, MT, 0);                                                           \
    } while (0)
    if (a.io == SVDLUT_F32) {
        if (a.map_dt == SVDLUT_F32) SVDLUT_BWD(float, float); else SVDLUT_BWD(float, __half);
    } else {
        if (a.map_dt == SVDLUT_F32) SVDLUT_BWD(__half, float); else SVDLUT_BWD(__half, __half);
    }
#undef SVDLUT_BWD
#undef SVDLUT_BWD_L
    svdlut_status stt = check_launch("apply_bwd");
    if (stt != SVDLUT_OK) return stt;
    PostArgs Q{};
    Q.nfac = P.want_dT ? a.B * 9 : 0;
    Q.part = a.dT; Q.gpi = P.gpi;
    Q.U = a.U; Q.s = a.s; Q.V = a.V;
    Q.dU = a.dU; Q.ds = a.ds; Q.dV = a.dV;
    Q.D = a.D; Q.R = a.R;
    if (det) {
        const int64_t n = (a.dmap ? static_cast<int64_t>(a.B) * 9 * a.h * a.w : 0) + (a.dbias ? 3 * a.B : 0);
        Q.nred = static_cast<int>((n + 1023) / 1024);
        Q.rowlo = P.rowlo; Q.mpart = P.mpart; Q.dbpart = P.dbpart;
        Q.dmap = a.dmap; Q.dbias = a.dbias;
        Q.B = a.B; Q.mrows = P.mrows; Q.h = a.h; Q.w = a.w;
    }
    if (L) {
        Q.with_loss = 1;
        Q.lpart = L->lpart; Q.nlp = grid; Q.inv_n = P.inv_n; Q.loss = L->loss;
    }
    const int nblk = Q.nfac + Q.nred + Q.with_loss;
    if (nblk > 0) {
        const size_t lds2 = Q.nfac ? sizeof(float) * (static_cast<size_t>(a.D) * a.D +
                                                      3 * static_cast<size_t>(a.D) * a.R) : 0;
        hipLaunchKernelGGL(bwd_post_kernel, dim3(nblk), dim3(1024), lds2, st, Q);
        stt = check_launch("apply_bwd (factor gradients, reductions)");
    }
    return stt;
}

svdlut_status launch_apply_bwd(const BwdLaunch& a, hipStream_t st) { return launch_bwd_impl(a, nullptr, st); }

}  // namespace svdlut

using namespace svdlut;

namespace {

size_t loss_bwd_ws_bytes(int B, int D) {
    return ((bwd_workspace_bytes(B, D) + 255) & ~static_cast<size_t>(255)) +
           sizeof(float) * static_cast<size_t>(B) * bwd_groups_per_image(B);
}

bool dim_ok(int32_t v) { return v >= 1 && v <= kMaxDim; }

}  // namespace

extern "C" {

size_t svdlut_apply_loss_bwd_workspace_size(int32_t B, int32_t D) {
    if (B < 1 || D < 2 || D > kMaxD) return 0;
    return loss_bwd_ws_bytes(B, D);
}

svdlut_status svdlut_apply_loss_bwd(const void* x, const void* target, svdlut_dtype io, const float* U,
                                    const float* s, const float* V, const void* map, svdlut_dtype map_dt,
                                    const float* bias, svdlut_loss_kind kind, float* loss, void* dx, float* dU,
                                    float* ds, float* dV, float* dmap, float* dbias, int32_t B, int32_t H,
                                    int32_t W, int32_t h, int32_t w, int32_t D, int32_t R, void* ws,
                                    size_t ws_bytes, hipStream_t stream) {
    if (!x || !target || !U || !s || !V || !map || !loss || !ws)
        return fail(SVDLUT_EINVAL, "apply_loss_bwd: null pointer");
    if (kind != SVDLUT_LOSS_L1 && kind != SVDLUT_LOSS_MSE) return fail(SVDLUT_EINVAL, "apply_loss_bwd: kind");
    const int nfac = (dU != nullptr) + (ds != nullptr) + (dV != nullptr);
    if (nfac != 0 && nfac != 3) return fail(SVDLUT_EINVAL, "apply_loss_bwd: dU, ds, dV must be all set or all NULL");
    if ((io != SVDLUT_F32 && io != SVDLUT_F16) || (map_dt != SVDLUT_F32 && map_dt != SVDLUT_F16))
        return fail(SVDLUT_EUNSUPPORTED, "apply_loss_bwd: dtype");
    if (B < 1) return fail(SVDLUT_EINVAL, "apply_loss_bwd: B must be >= 1");
    if (!dim_ok(H) || !dim_ok(W) || !dim_ok(h) || !dim_ok(w))
        return fail(SVDLUT_EINVAL, "apply_loss_bwd: H, W, h, w must be in [1, 65535]");
    if (D < 2 || D > kMaxD || R < 1 || R > kMaxR) return fail(SVDLUT_EINVAL, "apply_loss_bwd: D or R out of range");
    if (ws_bytes < loss_bwd_ws_bytes(B, D))
        return fail(SVDLUT_EINVAL, "apply_loss_bwd: workspace smaller than svdlut_apply_loss_bwd_workspace_size()");
    BwdLaunch a{};
    a.x = x; a.dy = target; a.U = U; a.s = s; a.V = V; a.map = map;
    a.dx = dx; a.dU = dU; a.ds = ds; a.dV = dV; a.dmap = dmap; a.dbias = dbias;
    a.dT = static_cast<float*>(ws);
    if ((dmap || dbias) && deterministic_mode()) {
        const size_t base = (loss_bwd_ws_bytes(B, D) + 255) & ~static_cast<size_t>(255);
        const size_t need = base + bwd_det_bytes(B, H, W, h, w);
        if (ws_bytes < need)
            return fail(SVDLUT_EINVAL, "apply_loss_bwd: deterministic mode needs a workspace of " +
                                           std::to_string(need) + " bytes (the usual size plus "
                                           "svdlut_deterministic_workspace_size())");
        a.det = static_cast<char*>(ws) + base;
    }
    a.B = B; a.H = H; a.W = W; a.h = h; a.w = w; a.D = D; a.R = R;
    a.io = io; a.map_dt = map_dt;
    LossArgs L{kind == SVDLUT_LOSS_L1 ? 1 : 2, bias,
               reinterpret_cast<float*>(static_cast<char*>(ws) +
                                        ((bwd_workspace_bytes(B, D) + 255) & ~static_cast<size_t>(255))),
               loss};
    return launch_bwd_impl(a, &L, stream);
}

}  // extern "C"
