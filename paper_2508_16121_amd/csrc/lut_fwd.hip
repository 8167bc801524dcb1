// Forward kernels of the 2D-LUT path: standalone LUT reconstruction and the fused
// reconstruct + spatially weighted 2D-LUT transform (persistent, one launch per batch).
#include "lut_common.h"

#include <algorithm>

namespace svdlut {

// ---------------------------------------------------------------- standalone reconstruction
// One workgroup per LUT: T[i][j] = sum_k U[i][k] s[k] V[j][k].
__global__ void __launch_bounds__(256) reconstruct_kernel(const float* __restrict__ U,
                                                          const float* __restrict__ s,
                                                          const float* __restrict__ V,
                                                          float* __restrict__ T, int D, int R) {
    extern __shared__ float sm[];
    const int n = blockIdx.x;
    float* Us = sm;            // [D][R]
    float* Vs = sm + D * R;    // [D][R]
    const float* u = U + static_cast<size_t>(n) * D * R;
    const float* v = V + static_cast<size_t>(n) * D * R;
    const float* sv = s + static_cast<size_t>(n) * R;
    for (int e = threadIdx.x; e < D * R; e += blockDim.x) {
        Us[e] = u[e] * sv[e % R];
        Vs[e] = v[e];
    }
    __syncthreads();
    float* t = T + static_cast<size_t>(n) * D * D;
    for (int o = threadIdx.x; o < D * D; o += blockDim.x) {
        const int i = o / D, j = o - (o / D) * D;
        float acc = 0.f;
        for (int k = 0; k < R; ++k) acc = fmaf(Us[i * R + k], Vs[j * R + k], acc);
        t[o] = acc;
    }
}

svdlut_status launch_reconstruct(const float* U, const float* s, const float* V, float* T,
                                 int n, int D, int R, hipStream_t st) {
    const size_t lds = 2 * sizeof(float) * D * R;
    hipLaunchKernelGGL(reconstruct_kernel, dim3(n), dim3(256), lds, st, U, s, V, T, D, R);
    return check_launch("reconstruct");
}

// ---------------------------------------------------------------- fused apply
// Work unit ("tile"): one row segment of 64 * PX pixels of one image, processed by one wave
// (PX consecutive pixels per lane; PX = 4, 256-pixel segments, except in an uneven-batch plan
// tuned to PX = 8).  Tiles are numbered image-major, row-major.  Each
// workgroup takes a contiguous chunk of tiles; within each image the chunk is split into
// contiguous per-wave runs.  Before the first tile of an image the workgroup rebuilds that
// image's LUTs into LDS.
//
// Spatial map: per tile the wave stages, for every map column the segment touches, the
// nine map channels blended between the two map rows around the tile's row
// (r_l(col) = (1-dv) m_l[iv][col] + dv m_l[iv+1][col]).  When the map is coarse enough that a
// lane's PX pixels lie within staged columns c0..c0+2 (FASTMAP: (PX-1)(w-1) <= W-1),
// S_l = r0 + a*(r1-r0) + b*(r2-r1) with a = min(t, 1), b = max(t-1, 0), t = u - c0; otherwise
// each pixel blends its own pair of columns.

struct Geo {
    int H, W, h, w;
    int64_t x_off, y_off, map_off;
    int64_t tile0;   // first tile of the image
    int nseg;        // row segments per image row
    bool vec_ok;     // image rows can use aligned 4-element accesses
    AxisMap ax, ay;  // map coordinates along x (W -> w) and y (H -> h)
};

template <int PX>
__device__ __forceinline__ Geo image_geo(const ApplyLaunch& a, int b, int io_bytes) {
    constexpr int SEG = kWave * PX;
    Geo g;
    if (a.descs) {
        const ImgGeom d = a.descs[b];
        g.H = d.H; g.W = d.W; g.h = d.h; g.w = d.w;
        g.x_off = d.x_off; g.y_off = d.y_off; g.map_off = d.map_off;
        g.tile0 = a.tile_start[b];
    } else {
        g.H = a.H; g.W = a.W; g.h = a.h; g.w = a.w;
        const int64_t plane = static_cast<int64_t>(a.H) * a.W;
        g.x_off = static_cast<int64_t>(b) * 3 * plane;
        g.y_off = g.x_off;
        g.map_off = static_cast<int64_t>(b) * 9 * a.h * a.w;
        g.tile0 = static_cast<int64_t>(b) * a.H * ((a.W + SEG - 1) / SEG);
    }
    g.nseg = (g.W + SEG - 1) / SEG;
    const int64_t plane = static_cast<int64_t>(g.H) * g.W;
    // VEC lanes past the row end take the row's last PX pixels, which must lie in the row's
    // last segment: rows of at least PX pixels whose last segment holds at least PX of them
    g.vec_ok = ((g.x_off | g.y_off | plane | g.W) & 3) == 0 && g.W >= PX && (g.W % SEG == 0 || g.W % SEG >= PX) &&
               ((reinterpret_cast<uintptr_t>(a.x) | reinterpret_cast<uintptr_t>(a.y)) &
                (4 * static_cast<uintptr_t>(io_bytes) - 1)) == 0;
    g.ax = make_axis(g.W, g.w);
    g.ay = make_axis(g.H, g.h);
    return g;
}

template <int PX>
__device__ __forceinline__ int image_of_tile(const ApplyLaunch& a, int64_t t) {
    if (!a.descs) {
        const int64_t per = static_cast<int64_t>(a.H) * ((a.W + kWave * PX - 1) / (kWave * PX));
        return static_cast<int>(t / per);
    }
    int lo = 0, hi = a.B - 1;            // largest b with tile_start[b] <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.tile_start[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Pixels of the lane for the tile at row y, segment start xs: 3 channels x PX pixels.  VEC
// (rows 4-element aligned, at least PX long): 4-element vector loads, lanes past the row end
// re-read the row's last PX pixels; otherwise element loads with the index clamped to the row.
template <typename IO, bool VEC, int PX>
__device__ __forceinline__ void load_tile(const ApplyLaunch& a, const Geo& g, int y, int xs, float (&px)[3][PX]) {
    const int lane = threadIdx.x & (kWave - 1);
    const int x0 = min(xs + lane * PX, VEC ? g.W - PX : g.W - 1);
    const int64_t plane = static_cast<int64_t>(g.H) * g.W;
    const IO* xin = reinterpret_cast<const IO*>(a.x) + g.x_off + static_cast<int64_t>(y) * g.W;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int q = 0; q < PX / 4; ++q) {
            float t[4];
            load_px4<IO, VEC>(xin + c * plane, x0 + 4 * q, g.W, t);
#pragma unroll
            for (int e = 0; e < 4; ++e) px[c][4 * q + e] = t[e];
        }
}

// Map columns of the segment starting at xs: first staged column and count.
template <int PX>
__device__ __forceinline__ void seg_columns(const Geo& g, int xs, int& clo, int& ncols) {
    const int xlast = min(xs + kWave * PX, g.W) - 1;
    int chi; uint32_t r;
    axis_left(g.ax, xs, clo, r);
    axis_left(g.ax, xlast, chi, r);
    chi = min(chi + 2, g.w - 1);
    ncols = chi - clo + 1;
}

// Per-wave staging of the forward (floats per map column): the raw rows (top at 0..8, row
// difference at 12..20) and the blended row (nine values).  Usually a wave's lanes read about
// 32 consecutive columns at once, so the strides are odd (13 / 21, scalar accesses) and the
// columns fall on distinct LDS banks; 16-byte-aligned strides of 12 and 24 put 4 and 8 of
// them on each bank and made the 4K apply about 2 % slower (56.4 against 55.0-55.2 us for odd
// pairs from 9 to 13 and 19 to 23).  When a segment spans at most kVecStageCols columns (a
// coarse map, e.g. one weight per image) those aligned strides are conflict-free as well and
// their vector accesses take fewer LDS instructions, so VST selects them.
constexpr int kVecStageCols = 8;
template <bool VST> struct Stg { static constexpr int map = 13, raw = 21; };
template <> struct Stg<true> { static constexpr int map = 12, raw = 24; };
constexpr int kFRawDiff = 12;
inline bool vec_stage(int ncol_max) { return ncol_max <= kVecStageCols; }

// Stage the raw map rows around a tile row for the segment's columns: per column the nine
// channels of row iv ("top") and their difference to row iv+1 ("diff").  Rewritten only when
// the wave moves to another segment or another pair of map rows.
template <typename MT, bool VST>
__device__ __forceinline__ void stage_raw(const ApplyLaunch& a, const Geo& g, int iv, int clo, int ncols,
                                          float* raw) {
    const int lane = threadIdx.x & (kWave - 1);
    const int iv1 = min(iv + 1, g.h - 1);
    const MT* m0 = reinterpret_cast<const MT*>(a.map) + g.map_off + static_cast<int64_t>(iv) * g.w + clo;
    const int64_t rowd = static_cast<int64_t>(iv1 - iv) * g.w;
    const int64_t mplane = static_cast<int64_t>(g.h) * g.w;
    for (int j = lane; j < ncols; j += kWave) {
        const MT* src = m0 + j;
        float v0[9], v1[9];
#pragma unroll
        for (int l = 0; l < 9; ++l) {          // all eighteen loads in flight together
            v0[l] = ldf<MT>(src + l * mplane);
            v1[l] = ldf<MT>(src + l * mplane + rowd);
        }
        float* dst = raw + j * Stg<VST>::raw;
        if (VST) {
            *reinterpret_cast<float4*>(dst) = make_float4(v0[0], v0[1], v0[2], v0[3]);
            *reinterpret_cast<float4*>(dst + 4) = make_float4(v0[4], v0[5], v0[6], v0[7]);
            dst[8] = v0[8];
            *reinterpret_cast<float4*>(dst + 12) =
                make_float4(v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2], v1[3] - v0[3]);
            *reinterpret_cast<float4*>(dst + 16) =
                make_float4(v1[4] - v0[4], v1[5] - v0[5], v1[6] - v0[6], v1[7] - v0[7]);
            dst[20] = v1[8] - v0[8];
        } else {
#pragma unroll
            for (int l = 0; l < 9; ++l) {
                dst[l] = v0[l];
                dst[kFRawDiff + l] = v1[l] - v0[l];
            }
        }
    }
}

// Blend the staged rows for one tile row: stage[col][l] = top + dv * diff.
template <bool VST>
__device__ __forceinline__ void blend_rows(const float* raw, float* stage, int ncols, float dv) {
    const int lane = threadIdx.x & (kWave - 1);
    for (int j = lane; j < ncols; j += kWave) {
        const float* src = raw + j * Stg<VST>::raw;
        float* dst = stage + j * Stg<VST>::map;
        if (VST) {
            const float4 t0 = *reinterpret_cast<const float4*>(src);
            const float4 t1 = *reinterpret_cast<const float4*>(src + 4);
            const float t2 = src[8];
            const float4 d0 = *reinterpret_cast<const float4*>(src + 12);
            const float4 d1 = *reinterpret_cast<const float4*>(src + 16);
            const float d2 = src[20];
            *reinterpret_cast<float4*>(dst) =
                make_float4(fmaf(dv, d0.x, t0.x), fmaf(dv, d0.y, t0.y), fmaf(dv, d0.z, t0.z), fmaf(dv, d0.w, t0.w));
            *reinterpret_cast<float4*>(dst + 4) =
                make_float4(fmaf(dv, d1.x, t1.x), fmaf(dv, d1.y, t1.y), fmaf(dv, d1.z, t1.z), fmaf(dv, d1.w, t1.w));
            dst[8] = fmaf(dv, d2, t2);
        } else {
#pragma unroll
            for (int l = 0; l < 9; ++l) dst[l] = fmaf(dv, src[kFRawDiff + l], src[l]);
        }
    }
}

// Grid slicing state of one tile: the combined planes in LDS, the spatial axis maps and the
// tile row's grid coordinate along y.
struct GridTile {
    const float* Gl;     // [3 channels][3 planes (xy, xc, yc)][Ds][Dsp]
    AxisMap gax;         // W -> Ds
    int iy;
    float dy;
    int Ds, Dsp;
};

template <typename IO, bool FASTMAP, bool VEC, bool GRID, bool VST, int PX>
__device__ __forceinline__ void compute_tile(const ApplyLaunch& a, const Geo& g, const float* Tl,
                                             const float* stage, int clo, int D, int y, int xs,
                                             const float (&px)[3][PX], const float (&bias3)[3],
                                             const GridTile& gt) {
    // Lanes past the row end work on the row's last pixels (the same x0 as load_tile) and
    // store the same values again, so every lane issues the same loads and stores.
    const int lane = threadIdx.x & (kWave - 1);
    const int x0 = min(xs + lane * PX, VEC ? g.W - PX : g.W - 1);
    int c0; uint32_t rem0;
    axis_left(g.ax, x0, c0, rem0);
    const float Dm1 = static_cast<float>(D - 1);
    const int Dm2 = D - 2;
    const int RS = lut_row_stride(D);
    const int PS = lut_pair_stride(D);
    const float RS4 = static_cast<float>(4 * RS), PS4 = static_cast<float>(4 * PS);
    const float Dm2f = static_cast<float>(Dm2);
    (void)PS;
    float out[3][PX];
    float r0[9], d01[9], d12[9];
    if (FASTMAP) {
        const float* s0 = stage + (c0 - clo) * Stg<VST>::map;
        const float* s1 = stage + (min(c0 + 1, g.w - 1) - clo) * Stg<VST>::map;
        const float* s2 = stage + (min(c0 + 2, g.w - 1) - clo) * Stg<VST>::map;
#pragma unroll
        for (int l = 0; l < 9; ++l) {
            const float a0 = s0[l], a1 = s1[l], a2 = s2[l];
            r0[l] = a0; d01[l] = a1 - a0; d12[l] = a2 - a1;
        }
    }
    const uint32_t den = g.ax.div.d;
#pragma unroll
    for (int k = 0; k < PX; ++k) {
        float S[9];
        if (FASTMAP) {
            const uint32_t n = rem0 + static_cast<uint32_t>(k) * g.ax.num_step;
            const float ta = static_cast<float>(min(n, den)) * g.ax.inv;
            const float tb = static_cast<float>(n > den ? n - den : 0u) * g.ax.inv;
#pragma unroll
            for (int l = 0; l < 9; ++l) S[l] = fmaf(tb, d12[l], fmaf(ta, d01[l], r0[l]));
        } else {
            int ck; uint32_t rk;
            axis_left(g.ax, min(x0 + k, g.W - 1), ck, rk);
            const float du = static_cast<float>(rk) * g.ax.inv;
            const float* s0 = stage + (ck - clo) * Stg<VST>::map;
            const float* s1 = stage + (min(ck + 1, g.w - 1) - clo) * Stg<VST>::map;
#pragma unroll
            for (int l = 0; l < 9; ++l) S[l] = fmaf(du, s1[l] - s0[l], s0[l]);
        }
        // decode in float: f = min(floor(q), D-2), d = q - f; LDS byte offsets by float FMA
        // (exact: every value stays below 2^24)
        float fv[3], dd[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float q = fminf(fmaxf(px[c][k], 0.f), 1.f) * Dm1;
            fv[c] = fminf(floorf(q), Dm2f);
            dd[c] = q - fv[c];
        }
        const float dr = dd[0], dg = dd[1], db = dd[2];
        constexpr float NB = 4.f * kNode;   // bytes per vertex
        const float ob[3] = {fv[1] * NB, fmaf(fv[2], NB, PS4), fmaf(fv[2], NB, 2.f * PS4)};
        float acc[3] = {bias3[0], bias3[1], bias3[2]};
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            const float fa = (p == 2) ? fv[1] : fv[0];
            const float da = (p == 2) ? dg : dr;
            const float db2 = (p == 0) ? dg : db;
            const uint32_t boff = static_cast<uint32_t>(fmaf(fa, RS4, ob[p]));
            // bilinear weights: w11 = a b, w10 = a (1-b), w01 = (1-a) b, w00 = (1-a)(1-b)
            const float w11 = da * db2;
            const float w10 = da - w11;
            const float w01 = db2 - w11;
            const float w00 = (1.f - da) - w01;
            const float* t0 = reinterpret_cast<const float*>(reinterpret_cast<const char*>(Tl) + boff);
            const float* t1 = t0 + RS;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float phi = w00 * t0[c];
                phi = fmaf(w10, t1[c], phi);
                phi = fmaf(w01, t0[kNode + c], phi);
                phi = fmaf(w11, t1[kNode + c], phi);
                acc[c] = fmaf(S[3 * c + p], phi, acc[c]);
            }
        }
        if (GRID) {
            // 2D slicing (supp. Eqs. query_grid to bilinear_grid): planes xy (x, y),
            // xc (x, X_c) and yc (y, X_c) of the channel's combined grid
            int ixg; uint32_t rxg;
            axis_left(gt.gax, x0 + k, ixg, rxg);
            const float dxg = static_cast<float>(rxg) * gt.gax.inv;
            const int P = gt.Ds * gt.Dsp;
            const float Dsm1 = static_cast<float>(gt.Ds - 1), Dsm2 = static_cast<float>(gt.Ds - 2);
            const float wy1 = gt.dy, wx1 = dxg;
            const float wxy11 = wx1 * wy1, wxy10 = wx1 - wxy11, wxy01 = wy1 - wxy11;
            const float wxy00 = (1.f - wx1) - wxy01;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float q = fminf(fmaxf(px[c][k], 0.f), 1.f) * Dsm1;
                const float fc = fminf(floorf(q), Dsm2);
                const float dc = q - fc;
                const int ic = static_cast<int>(fc);
                const float* G0 = gt.Gl + 3 * c * P;
                const float* txy = G0 + ixg * gt.Dsp + gt.iy;
                const float* txc = G0 + P + ixg * gt.Dsp + ic;
                const float* tyc = G0 + 2 * P + gt.iy * gt.Dsp + ic;
                float v = wxy00 * txy[0];
                v = fmaf(wxy10, txy[gt.Dsp], v);
                v = fmaf(wxy01, txy[1], v);
                v = fmaf(wxy11, txy[gt.Dsp + 1], v);
                const float wc11x = wx1 * dc, wc10x = wx1 - wc11x, wc01x = dc - wc11x;
                const float wc00x = (1.f - wx1) - wc01x;
                v = fmaf(wc00x, txc[0], v);
                v = fmaf(wc10x, txc[gt.Dsp], v);
                v = fmaf(wc01x, txc[1], v);
                v = fmaf(wc11x, txc[gt.Dsp + 1], v);
                const float wc11y = wy1 * dc, wc10y = wy1 - wc11y, wc01y = dc - wc11y;
                const float wc00y = (1.f - wy1) - wc01y;
                v = fmaf(wc00y, tyc[0], v);
                v = fmaf(wc10y, tyc[gt.Dsp], v);
                v = fmaf(wc01y, tyc[1], v);
                v = fmaf(wc11y, tyc[gt.Dsp + 1], v);
                acc[c] += v;
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c][k] = acc[c];
    }
    const int64_t plane = static_cast<int64_t>(g.H) * g.W;
    IO* yout = reinterpret_cast<IO*>(a.y) + g.y_off + static_cast<int64_t>(y) * g.W;
    if constexpr (PX == 4) {
        store_px4<IO, VEC>(yout, x0, g.W, out[0]);
        store_px4<IO, VEC>(yout + plane, x0, g.W, out[1]);
        store_px4<IO, VEC>(yout + 2 * plane, x0, g.W, out[2]);
    } else {
        // per group of four: without VEC a group that starts past the row end holds only
        // pixels beyond it (the first group's stores cover the row's last pixel) and is skipped
#pragma unroll
        for (int q = 0; q < PX / 4; ++q) {
            if (!VEC && x0 + 4 * q > g.W - 1) continue;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float t[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) t[e] = out[c][4 * q + e];
                store_px4<IO, VEC>(yout + c * plane, x0 + 4 * q, g.W, t);
            }
        }
    }
}

// Largest workgroup an instantiation is compiled for.  Half-precision I/O with grid slicing
// or with per-pixel map columns needs more than the 128 VGPRs per lane that a 1024-thread
// workgroup leaves (it spilled to scratch and ran 4-5x slower), so those variants are built
// for 512 threads (up to 256 VGPRs, 8 waves per CU), as are the 8-pixel-per-lane ones.
template <typename IO, bool FASTMAP, bool GRID, int PX = kPxPerLane>
constexpr int apply_threads() { return (PX > kPxPerLane || (sizeof(IO) == 2 && (GRID || !FASTMAP))) ? 512 : 1024; }

// One image's share [ta, tb) (local row-major tile indices) of a workgroup's chunk.  Inside
// it the tiles are walked column-major (same segment, consecutive rows) in one contiguous
// run per wave, so a wave keeps its staged raw map rows for about h/H of a map cell's
// height in pixel rows and only re-reads the map when the segment or the pair of map rows
// changes.  VEC is uniform per image, so the hot loop has a single load/store form.
template <typename IO, typename MT, bool FASTMAP, bool VEC, bool GRID, bool VST, int PX>
__device__ __forceinline__ void run_image(const ApplyLaunch& a, const Geo& g, int b, int ta, int tb,
                                          int wave, int nw, float* Tl, float* Gl, float* aux, float* stage,
                                          float* raw) {
    const int D = a.D;
    const int ya = ta / g.nseg;
    const int nr = (tb - 1) / g.nseg - ya + 1;
    const int total = nr * g.nseg;
    const int q = (total + nw - 1) / nw;
    const int k0 = min(total, wave * q);
    const int k1 = min(total, k0 + q);
    // first valid tile of the run
    int seg = k0 / nr, yr = k0 - seg * nr, k = k0;
    auto valid = [&](int sg, int r) {
        const int lt = (ya + r) * g.nseg + sg;
        return lt >= ta && lt < tb;
    };
    auto advance = [&](int& sg, int& r, int& kk) {   // to the next valid tile (or kk == k1)
        do {
            ++kk;
            if (++r == nr) { r = 0; ++sg; }
        } while (kk < k1 && !valid(sg, r));
    };
    if (k < k1 && !valid(seg, yr)) advance(seg, yr, k);
    GridTile gt{};
    if (GRID) {
        // Combined planes: slicing is linear in the planes, so the K grids of one output
        // channel (k mod 3 = c) collapse into one grid whose plane is sum_k w^k_plane g^k_plane
        // (the previous image's readers are done: the caller synchronised).
        gt.Ds = a.Ds;
        gt.Dsp = grid_plane_stride(a.Ds);
        const int P = a.Ds * gt.Dsp;
        const float* gsrc = a.grids + static_cast<size_t>(b) * a.K * 3 * a.Ds * a.Ds;
        const float* wsrc = a.gw + static_cast<size_t>(b) * a.K * 3;
        for (int e = threadIdx.x; e < 9 * a.Ds * a.Ds; e += blockDim.x) {
            const int cp = e / (a.Ds * a.Ds);            // 3 * channel + plane
            const int r = e - cp * (a.Ds * a.Ds);
            const int i = r / a.Ds, j = r - i * a.Ds;
            const int c = cp / 3, pl = cp - 3 * c;
            float v = 0.f;
            for (int kk = c; kk < a.K; kk += 3)
                v = fmaf(wsrc[3 * kk + pl], gsrc[(static_cast<size_t>(kk) * 3 + pl) * a.Ds * a.Ds + r], v);
            Gl[cp * P + i * gt.Dsp + j] = v;
        }
        gt.Gl = Gl;
        gt.gax = make_axis(g.W, a.Ds);
    }
    // EARLY (the variants built for 1024 threads): the first tile's pixels are requested
    // before the LUT rebuild, so their memory latency overlaps it, and each later tile's right
    // after the previous tile.  The 512-thread variants measured faster loading each tile's
    // pixels at its start.
    constexpr bool EARLY = apply_threads<IO, FASTMAP, GRID, PX>() == 1024;
    constexpr int SEG = kWave * PX;
    float px[3][PX];
    if (EARLY && k < k1) load_tile<IO, VEC, PX>(a, g, ya + yr, seg * SEG, px);
    const size_t foff = static_cast<size_t>(b) * 9 * D * a.R;
    stage_luts(Tl, aux, a.U + foff, a.s + static_cast<size_t>(b) * 9 * a.R, a.V + foff, D, a.R, min(a.R, 8));
    float bias3[3] = {0.f, 0.f, 0.f};
    if (a.bias) {
        bias3[0] = a.bias[3 * b]; bias3[1] = a.bias[3 * b + 1]; bias3[2] = a.bias[3 * b + 2];
    }
    if (GRID) {
        const float* bsrc = a.gb + static_cast<size_t>(b) * a.K;
        for (int kk = 0; kk < a.K; ++kk) bias3[kk % 3] += bsrc[kk];
    }
    const AxisMap gay = GRID ? make_axis(g.H, a.Ds) : AxisMap{};
    // Each tile stages/blends the map and computes: with 16 waves per CU the other waves
    // cover a wave's load latency (holding a second tile's pixels in registers measured no
    // faster).
    int st_seg = -1, st_iv = -1, clo = 0, ncols = 0;
    while (k < k1) {
        const int y = ya + yr;
        const int xs = seg * SEG;
        if (!EARLY) load_tile<IO, VEC, PX>(a, g, y, xs, px);
        int iv; uint32_t remv;
        axis_left(g.ay, y, iv, remv);
        if (seg != st_seg || iv != st_iv) {
            seg_columns<PX>(g, xs, clo, ncols);
            stage_raw<MT, VST>(a, g, iv, clo, ncols, raw);
            st_seg = seg;
            st_iv = iv;
            wave_sync();
        }
        blend_rows<VST>(raw, stage, ncols, static_cast<float>(remv) * g.ay.inv);
        wave_sync();
        if (GRID) {
            uint32_t ry;
            axis_left(gay, y, gt.iy, ry);
            gt.dy = static_cast<float>(ry) * gay.inv;
        }
        compute_tile<IO, FASTMAP, VEC, GRID, VST, PX>(a, g, Tl, stage, clo, D, y, xs, px, bias3, gt);
        wave_sync();   // the stage region is rewritten for the next tile
        advance(seg, yr, k);
        if (EARLY && k < k1) load_tile<IO, VEC, PX>(a, g, ya + yr, seg * SEG, px);
    }
}

int apply_max_block(svdlut_dtype io, bool fast_map, bool grid, int px) {
    return (px > kPxPerLane || (io == SVDLUT_F16 && (grid || !fast_map))) ? 512 : 1024;
}

// Persistent kernel: workgroup chunk -> per-image sub-ranges -> per-wave runs.
template <typename IO, typename MT, bool FASTMAP, bool GRID, bool VST, int PX = kPxPerLane>
__global__ void __launch_bounds__((apply_threads<IO, FASTMAP, GRID, PX>())) apply_kernel(ApplyLaunch a) {
    extern __shared__ float smem[];
    const int D = a.D;
    float* Tl = smem;
    float* Gl = smem + lut_floats(D);
    float* aux = Gl + (GRID ? ((grid_floats(a.Ds) + 3) & ~3) : 0);
    const int nw = blockDim.x / kWave;
    // wave index as a scalar: everything derived from it (tile runs, rows, segments) stays
    // wave-uniform, so the tile bookkeeping runs on the scalar unit with uniform branches
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    float* stage = aux + wave * a.ncol_max * (Stg<VST>::map + Stg<VST>::raw);
    float* raw = stage + a.ncol_max * Stg<VST>::map;

    const int G = gridDim.x;
    const int lb = logical_block(blockIdx.x, G);
    const int64_t per = (a.total_tiles + G - 1) / G;
    int64_t t0 = static_cast<int64_t>(lb) * per;
    const int64_t t1 = min(a.total_tiles, t0 + per);
    while (t0 < t1) {
        const int b = image_of_tile<PX>(a, t0);
        const Geo g = image_geo<PX>(a, b, sizeof(IO));
        const int64_t img_end = g.tile0 + static_cast<int64_t>(g.H) * g.nseg;
        const int64_t te = min(t1, img_end);
        const int ta = static_cast<int>(t0 - g.tile0);
        const int tb = static_cast<int>(te - g.tile0);
        if (g.vec_ok)
            run_image<IO, MT, FASTMAP, true, GRID, VST, PX>(a, g, b, ta, tb, wave, nw, Tl, Gl, aux, stage, raw);
        else
            run_image<IO, MT, FASTMAP, false, GRID, VST, PX>(a, g, b, ta, tb, wave, nw, Tl, Gl, aux, stage, raw);
        t0 = te;
        __syncthreads();   // every wave is done with Tl and aux before the next image
    }
}

int map_cols_bound(int W, int w, int px) {
    // columns touched by one segment of n = 64 px pixels:
    // c0(last) - c0(first) <= floor((n-1)*(w-1)/(W-1)) + 1, plus 2
    if (w <= 1) return 1;
    const int64_t span = (W > 1) ? (static_cast<int64_t>(kWave * px - 1) * (w - 1)) / (W - 1) : 0;
    return static_cast<int>(std::min<int64_t>(w, span + 4));
}

bool map_fast_ok(int W, int w, int px) {
    // a lane's px pixels must lie within two map cells: (px-1)*(w-1) <= W-1
    return static_cast<int64_t>(px - 1) * (w - 1) <= static_cast<int64_t>(W - 1);
}

size_t apply_lds_bytes(int D, int R, int block, int ncol_max, int Ds) {
    const size_t lut = static_cast<size_t>(lut_floats(D));
    (void)R;
    const size_t grid = Ds > 0 ? static_cast<size_t>((grid_floats(Ds) + 3) & ~3) : 0;
    const size_t scratch = static_cast<size_t>(2) * 9 * D * 8;
    const int per_col = vec_stage(ncol_max) ? Stg<true>::map + Stg<true>::raw : Stg<false>::map + Stg<false>::raw;
    const size_t stage = static_cast<size_t>(block / kWave) * ncol_max * per_col;
    return sizeof(float) * (lut + grid + std::max(scratch, stage));
}

template <typename IO, typename MT, bool FASTMAP, bool GRID, int PX = kPxPerLane>
static void launch_staged(const ApplyLaunch& a, size_t lds, hipStream_t st) {
    if (vec_stage(a.ncol_max))
        hipLaunchKernelGGL((apply_kernel<IO, MT, FASTMAP, GRID, true, PX>), dim3(a.grid), dim3(a.block), lds, st, a);
    else
        hipLaunchKernelGGL((apply_kernel<IO, MT, FASTMAP, GRID, false, PX>), dim3(a.grid), dim3(a.block), lds, st, a);
}

template <typename IO, typename MT>
static void launch_typed(const ApplyLaunch& a, size_t lds, hipStream_t st) {
    if (a.px == kPxWide) {   // validated by launch_apply: piecewise map path, no grids
        launch_staged<IO, MT, true, false, kPxWide>(a, lds, st);
    } else if (a.K > 0) {
        if (a.fast_map) launch_staged<IO, MT, true, true>(a, lds, st);
        else launch_staged<IO, MT, false, true>(a, lds, st);
    } else {
        if (a.fast_map) launch_staged<IO, MT, true, false>(a, lds, st);
        else launch_staged<IO, MT, false, false>(a, lds, st);
    }
}

svdlut_status launch_apply(const ApplyLaunch& a, hipStream_t st) {
    if (a.px != 0 && a.px != kPxPerLane && a.px != kPxWide)
        return fail(SVDLUT_EINVAL, "apply: pixels per lane must be 4 or 8");
    if (a.px == kPxWide && (!a.fast_map || a.K > 0))
        return fail(SVDLUT_EINVAL, "apply: 8 pixels per lane need the piecewise map path and no grids");
    if (a.block > apply_max_block(static_cast<svdlut_dtype>(a.io), a.fast_map != 0, a.K > 0,
                                  a.px == kPxWide ? kPxWide : kPxPerLane))
        return fail(SVDLUT_EINVAL, "apply: workgroup larger than the kernel variant allows");
    const size_t lds = apply_lds_bytes(a.D, a.R, a.block, a.ncol_max, a.K > 0 ? a.Ds : 0);
    if (a.io == SVDLUT_F32) {
        if (a.map_dt == SVDLUT_F32) launch_typed<float, float>(a, lds, st);
        else launch_typed<float, __half>(a, lds, st);
    } else {
        if (a.map_dt == SVDLUT_F32) launch_typed<__half, float>(a, lds, st);
        else launch_typed<__half, __half>(a, lds, st);
    }
    return check_launch("apply");
}

}  // namespace svdlut
