// Backward of the fused bilateral-grid slicing (supplementary Sec. "2D Slicing"): for each
// output channel c the adjoints of the three planes of its combined grid,
//   A_xy[c][ix+a][iy+b] += dy_c wx(a) wy(b),  A_xc[c][ix+a][ic+b] += dy_c wx(a) wc(b),
//   A_yc[c][iy+a][ic+b] += dy_c wy(a) wc(b),
// then per grid k (c = k mod 3): dgrids[k][plane] = w^k_plane A[c][plane],
// dgw[k][plane] = <grids[k][plane], A[c][plane]>, dgb[k] = sum of dy_c; and dx_c gains
// dy_c (Ds-1) (d psi_xc/d p + d psi_yc/d p) of the combined grid inside [0, 1].
//
// Decomposition as in the LUT backward: gpi workgroups per image, each over a contiguous
// band of row segments, adjoints accumulated in LDS as int32 fixed point with a power-of-two
// scale from the band's pixel count and max|dy| (every term is dy_c times weights in [0, 1]),
// written as float partials and summed in a fixed order by a second kernel.  The xy plane's
// contributions of a lane's four pixels are summed in registers first (they share the tile
// row and at most three x vertices), since all lanes of a wave hit the same few vertices.
// The xc and yc planes receive one term per pixel; neighbouring pixels have similar colours,
// so many lanes of a wave add to the same entry (the yc plane's row is the tile's, so up to
// the whole wave).  Those atomics go to ncx / ncy replicas of the planes selected by the lane
// index, which divides the same-address serialisation; the replicas are added in a fixed
// order before the partials are written (integer sums, so the result does not change).
#include "bwd_common.h"

#include <algorithm>

namespace svdlut {

namespace {

struct GridBwdDev {
    const void* x;
    const void* dy;
    void* dx;                 // accumulated: dx += grid part (NULL: skip)
    const float* grids;       // [B][K][3][Ds][Ds]
    const float* gw;          // [B][K][3]
    float* part;              // [B][gpi][9*Ds*Ds + 3]
    int B, H, W, K, Ds, gpi;
    int64_t per;              // row segments per workgroup
    int want_g;
    int ncx, ncy;             // replicas of the xc / yc adjoint planes (powers of two)
};

__device__ __forceinline__ int part_floats(int Ds) { return 9 * Ds * Ds + 3; }

template <typename IO, bool VEC>
__device__ __forceinline__ void grid_bwd_tile(const GridBwdDev& P, int b, int y, int seg, const float* Cl,
                                              int* Al, int* Ayr, int* Axr, int Dsp, const AxisMap& gax, int iy,
                                              float wy, float sc, float (&gsum)[3]) {
    const int lane = threadIdx.x & (kWave - 1);
    const int W = P.W, Ds = P.Ds;
    const int xs = seg * kSeg;
    // lane -> 4-pixel block of the segment by a fixed permutation (stride 17 of 64): lanes of
    // one instruction then sit far apart along the row, with less similar colours, so their
    // LDS atomics meet the same address less often
    const int x0 = xs + ((lane * 17) & (kWave - 1)) * kPxPerLane;
    if (x0 >= W) return;
    const int64_t plane = static_cast<int64_t>(P.H) * W;
    const int64_t img = static_cast<int64_t>(b) * 3 * plane + static_cast<int64_t>(y) * W;
    float px[3][4], gy[3][4];
    const IO* xin = reinterpret_cast<const IO*>(P.x) + img;
    const IO* gin = reinterpret_cast<const IO*>(P.dy) + img;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        load_px4<IO, VEC>(xin + c * plane, x0, W, px[c]);
        load_px4<IO, VEC>(gin + c * plane, x0, W, gy[c]);
    }
    const int PL = Ds * Dsp;
    const float Dsm1 = static_cast<float>(Ds - 1), Dsm2 = static_cast<float>(Ds - 2);
    int ix0; uint32_t r0;
    axis_left(gax, x0, ix0, r0);
    float ax[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};   // xy: [c][x vertex ix0 + n]
    float gx[3][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool on = x0 + k < W;          // clamped duplicates contribute nothing
        int ixk; uint32_t rk;
        axis_left(gax, min(x0 + k, W - 1), ixk, rk);
        const float wx = static_cast<float>(rk) * gax.inv;
        const int n = ixk - ix0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float G = on ? gy[c][k] : 0.f;
            gsum[c] += G;
            const float q = fminf(fmaxf(px[c][k], 0.f), 1.f) * Dsm1;
            const float fc = fminf(floorf(q), Dsm2);
            const float wc = q - fc;
            const int ic = static_cast<int>(fc);
            // xy plane: per-lane sums over the four pixels (at most vertices ix0 .. ix0+2)
            if (n == 0) {
                ax[c][0] = fmaf(G, 1.f - wx, ax[c][0]);
                ax[c][1] = fmaf(G, wx, ax[c][1]);
            } else if (n == 1) {
                ax[c][1] = fmaf(G, 1.f - wx, ax[c][1]);
                ax[c][2] = fmaf(G, wx, ax[c][2]);
            } else if (P.want_g) {            // tiny images: more than one vertex per pixel step
                int* A = Al + (3 * c) * PL;
                const float g0 = G * (1.f - wx) * sc, g1 = G * wx * sc;
                lds_addi(A + ixk * Dsp + iy, fix_mul(g0, 1.f - wy));
                lds_addi(A + ixk * Dsp + iy + 1, fix_mul(g0, wy));
                lds_addi(A + (ixk + 1) * Dsp + iy, fix_mul(g1, 1.f - wy));
                lds_addi(A + (ixk + 1) * Dsp + iy + 1, fix_mul(g1, wy));
            }
            // xc and yc planes
            if (P.want_g) {
                const float gs = G * sc;
                int* Axc = Axr + (c * P.ncx + (lane & (P.ncx - 1))) * PL + ixk * Dsp + ic;
                int* Ayc = Ayr + (c * P.ncy + (lane & (P.ncy - 1))) * PL + iy * Dsp + ic;
                const float wc0 = gs * (1.f - wc), wc1 = gs * wc;
                lds_addi(Axc, fix_mul(wc0, 1.f - wx));
                lds_addi(Axc + 1, fix_mul(wc1, 1.f - wx));
                lds_addi(Axc + Dsp, fix_mul(wc0, wx));
                lds_addi(Axc + Dsp + 1, fix_mul(wc1, wx));
                lds_addi(Ayc, fix_mul(wc0, 1.f - wy));
                lds_addi(Ayc + 1, fix_mul(wc1, 1.f - wy));
                lds_addi(Ayc + Dsp, fix_mul(wc0, wy));
                lds_addi(Ayc + Dsp + 1, fix_mul(wc1, wy));
            }
            // dx through the colour axis of the combined xc and yc planes
            const float* Cxc = Cl + (3 * c + 1) * PL + ixk * Dsp + ic;
            const float* Cyc = Cl + (3 * c + 2) * PL + iy * Dsp + ic;
            const float dxc = (1.f - wx) * (Cxc[1] - Cxc[0]) + wx * (Cxc[Dsp + 1] - Cxc[Dsp]);
            const float dyc = (1.f - wy) * (Cyc[1] - Cyc[0]) + wy * (Cyc[Dsp + 1] - Cyc[Dsp]);
            const float xv = px[c][k];
            gx[c][k] = (xv >= 0.f && xv <= 1.f) ? G * Dsm1 * (dxc + dyc) : 0.f;
        }
    }
    if (P.want_g) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            int* A = Al + (3 * c) * PL;
#pragma unroll
            for (int n = 0; n < 3; ++n) {
                if (ix0 + n > Ds - 1 || ax[c][n] == 0.f) continue;
                const float v = ax[c][n] * sc;
                lds_addi(A + (ix0 + n) * Dsp + iy, fix_mul(v, 1.f - wy));
                lds_addi(A + (ix0 + n) * Dsp + iy + 1, fix_mul(v, wy));
            }
        }
    }
    if (P.dx) {
        IO* dxp = reinterpret_cast<IO*>(P.dx) + img;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float cur[4];
            load_px4<IO, VEC>(dxp + c * plane, x0, W, cur);
            float o[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) o[k] = cur[k] + gx[c][k];
            store_px4<IO, VEC>(dxp + c * plane, x0, W, o);
        }
    }
}

template <typename IO>
__global__ void __launch_bounds__(512) grid_bwd_kernel(GridBwdDev P) {
    extern __shared__ float smem[];
    const int Ds = P.Ds, Dsp = grid_plane_stride(Ds), PL = Ds * Dsp;
    float* Cl = smem;                                   // combined planes [3 c][3 planes][Ds][Dsp]
    int* Al = reinterpret_cast<int*>(Cl + 9 * PL);      // their adjoints, int32 fixed point
    int* Ayr = Al + 9 * PL;                             // yc replicas [3 c][ncy][Ds][Dsp]
    int* Axr = Ayr + 3 * P.ncy * PL;                    // xc replicas [3 c][ncx][Ds][Dsp]
    float* red = reinterpret_cast<float*>(Axr + 3 * P.ncx * PL); // one float per wave
    const int nw = blockDim.x / kWave;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int b = blockIdx.x / P.gpi;
    const int j = blockIdx.x - b * P.gpi;
    const int nseg = (P.W + kSeg - 1) / kSeg;
    const int64_t tpi = static_cast<int64_t>(P.H) * nseg;
    const int64_t t0 = static_cast<int64_t>(j) * P.per;
    const int64_t t1 = min(tpi, t0 + P.per);

    // combined planes (as in the forward) and zeroed adjoints
    const float* gsrc = P.grids + static_cast<size_t>(b) * P.K * 3 * Ds * Ds;
    const float* wsrc = P.gw + static_cast<size_t>(b) * P.K * 3;
    for (int e = threadIdx.x; e < 9 * Ds * Ds; e += blockDim.x) {
        const int cp = e / (Ds * Ds);
        const int r = e - cp * (Ds * Ds);
        const int i = r / Ds, jj = r - i * Ds;
        const int c = cp / 3, pl = cp - 3 * c;
        float v = 0.f;
        for (int kk = c; kk < P.K; kk += 3)
            v = fmaf(wsrc[3 * kk + pl], gsrc[(static_cast<size_t>(kk) * 3 + pl) * Ds * Ds + r], v);
        Cl[cp * PL + i * Dsp + jj] = v;
    }
    for (int e = threadIdx.x; e < (9 + 3 * (P.ncy + P.ncx)) * PL; e += blockDim.x) Al[e] = 0;

    // fixed-point scale from the band's max |dy|
    const int64_t plane = static_cast<int64_t>(P.H) * P.W;
    float mdy = 0.f;
    bool nf = false;
    if (t0 < t1) {
        const int64_t e0 = (t0 / nseg) * P.W + (t0 % nseg) * kSeg;
        const int64_t e1 = ((t1 - 1) / nseg) * P.W + min(((t1 - 1) % nseg) * kSeg + kSeg, static_cast<int64_t>(P.W));
        const IO* dyb = reinterpret_cast<const IO*>(P.dy) + static_cast<int64_t>(b) * 3 * plane;
        for (int c = 0; c < 3; ++c) absmax_range<IO>(dyb + c * plane + e0, e1 - e0, mdy, nf);
    }
    mdy = block_max(mdy, red);
    bool bad = block_max(nf ? 1.f : 0.f, red) > 0.f;
    const float sc = fix_scale(static_cast<float>((t1 - t0) * kSeg), mdy, 1.f, bad);
    __syncthreads();

    const AxisMap gax = make_axis(P.W, Ds);
    const AxisMap gay = make_axis(P.H, Ds);
    const bool base_ok = ((plane | P.W) & 3) == 0 &&
                         ((reinterpret_cast<uintptr_t>(P.x) | reinterpret_cast<uintptr_t>(P.dy) |
                           reinterpret_cast<uintptr_t>(P.dx)) & (4 * sizeof(IO) - 1)) == 0;
    float gsum[3] = {0.f, 0.f, 0.f};
    for (int64_t t = t0 + wave; t < t1; t += nw) {
        const int y = static_cast<int>(t / nseg);
        const int seg = static_cast<int>(t - static_cast<int64_t>(y) * nseg);
        int iy; uint32_t ry;
        axis_left(gay, y, iy, ry);
        const float wy = static_cast<float>(ry) * gay.inv;
        if (base_ok && seg * kSeg + kSeg <= P.W)
            grid_bwd_tile<IO, true>(P, b, y, seg, Cl, Al, Ayr, Axr, Dsp, gax, iy, wy, sc, gsum);
        else
            grid_bwd_tile<IO, false>(P, b, y, seg, Cl, Al, Ayr, Axr, Dsp, gax, iy, wy, sc, gsum);
    }
    __syncthreads();
    if (!P.want_g) return;
    // fold the replicas into the xc and yc planes (fixed order)
    for (int e = threadIdx.x; e < 3 * PL; e += blockDim.x) {
        const int c = e / PL, r = e - c * PL;
        int sy = 0, sx = 0;
        for (int q = 0; q < P.ncy; ++q) sy += Ayr[(c * P.ncy + q) * PL + r];
        for (int q = 0; q < P.ncx; ++q) sx += Axr[(c * P.ncx + q) * PL + r];
        Al[(3 * c + 2) * PL + r] = sy;
        Al[(3 * c + 1) * PL + r] = sx;
    }
    __syncthreads();
    float* out = P.part + (static_cast<size_t>(b) * P.gpi + j) * part_floats(Ds);
    const float isc = bad ? __builtin_nanf("") : 1.f / sc;
    for (int e = threadIdx.x; e < 9 * Ds * Ds; e += blockDim.x) {
        const int cp = e / (Ds * Ds);
        const int r = e - cp * (Ds * Ds);
        const int i = r / Ds, jj = r - i * Ds;
        out[e] = static_cast<float>(Al[cp * PL + i * Dsp + jj]) * isc;
    }
    // sum of dy per channel over the band: waves in a fixed order
    for (int c = 0; c < 3; ++c) {
        float v = gsum[c];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((threadIdx.x & (kWave - 1)) == 0) red[wave] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            float s = 0.f;
            for (int w = 0; w < nw; ++w) s += red[w];
            out[9 * Ds * Ds + c] = s;
        }
        __syncthreads();
    }
}

// One workgroup per (image, grid, plane): fixed-order sum of the partial adjoints, then
// dgrids = w A, dgw = <grids, A>, and (plane 0) dgb = sum of dy of the grid's channel.
__global__ void __launch_bounds__(256) grid_reduce_kernel(const float* __restrict__ part, int gpi, int K, int Ds,
                                                          const float* __restrict__ grids,
                                                          const float* __restrict__ gw,
                                                          float* __restrict__ dgrids, float* __restrict__ dgw,
                                                          float* __restrict__ dgb) {
    __shared__ float red[256];
    const int bkp = blockIdx.x;                 // (b * K + k) * 3 + plane
    const int pl = bkp % 3;
    const int bk = bkp / 3;
    const int k = bk % K, b = bk / K;
    const int c = k % 3;
    const int nf = 9 * Ds * Ds + 3;
    const float* src = part + static_cast<size_t>(b) * gpi * nf + (3 * c + pl) * Ds * Ds;
    const float w = gw[static_cast<size_t>(bk) * 3 + pl];
    const float* g = grids + static_cast<size_t>(bkp) * Ds * Ds;
    float* dg = dgrids + static_cast<size_t>(bkp) * Ds * Ds;
    float dot = 0.f;
    for (int e = threadIdx.x; e < Ds * Ds; e += blockDim.x) {
        float acc = 0.f;
        int q = 0;
        for (; q + 8 <= gpi; q += 8) {     // eight partials in flight, added in workgroup order
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = src[static_cast<size_t>(q + u) * nf + e];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += v[u];
        }
        for (; q < gpi; ++q) acc += src[static_cast<size_t>(q) * nf + e];
        dg[e] = w * acc;
        dot = fmaf(g[e], acc, dot);
    }
    red[threadIdx.x] = dot;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        dgw[static_cast<size_t>(bk) * 3 + pl] = red[0];
        if (pl == 0) {
            const float* gs = part + static_cast<size_t>(b) * gpi * nf + 9 * Ds * Ds + c;
            float acc = 0.f;
            for (int q = 0; q < gpi; ++q) acc += gs[static_cast<size_t>(q) * nf];
            dgb[bk] = acc;
        }
    }
}

}  // namespace

size_t grid_bwd_workspace_bytes(int B, int Ds) {
    return sizeof(float) * static_cast<size_t>(B) * bwd_groups_per_image(B) * (9 * Ds * Ds + 3);
}

svdlut_status launch_grid_bwd(const GridBwdLaunch& a, hipStream_t st) {
    GridBwdDev P{};
    P.x = a.x; P.dy = a.dy; P.dx = a.dx; P.grids = a.grids; P.gw = a.gw; P.part = a.part;
    P.B = a.B; P.H = a.H; P.W = a.W; P.K = a.K; P.Ds = a.Ds;
    P.gpi = bwd_groups_per_image(a.B);
    const int nseg = (a.W + kSeg - 1) / kSeg;
    const int64_t tpi = static_cast<int64_t>(a.H) * nseg;
    P.per = (tpi + P.gpi - 1) / P.gpi;
    P.want_g = a.dgrids != nullptr;
    if (!P.dx && !P.want_g) return SVDLUT_OK;
    const int block = 512;
    // as many replicas as the LDS allows: 16 / 8 at Ds = 17, fewer for larger grids
    const size_t PL = static_cast<size_t>(a.Ds) * grid_plane_stride(a.Ds);
    const size_t lds_cap = static_cast<size_t>(device_info().lds_per_block);
    auto lds_of = [&](int ny, int nx) {
        return sizeof(float) * (2 * static_cast<size_t>(grid_floats(a.Ds)) + 3 * (ny + nx) * PL + block / kWave);
    };
    P.ncy = 16;
    P.ncx = 8;
    while ((P.ncy > 1 || P.ncx > 1) && lds_of(P.ncy, P.ncx) > lds_cap) {
        if (P.ncy >= 2 * P.ncx || P.ncx == 1) P.ncy /= 2;
        else P.ncx /= 2;
    }
    const size_t lds = lds_of(P.ncy, P.ncx);
    const int grid = a.B * P.gpi;
    if (a.io == SVDLUT_F32)
        hipLaunchKernelGGL(grid_bwd_kernel<float>, dim3(grid), dim3(block), lds, st, P);
    else
        hipLaunchKernelGGL(grid_bwd_kernel<__half>, dim3(grid), dim3(block), lds, st, P);
    svdlut_status stt = check_launch("grid_bwd");
    if (stt != SVDLUT_OK || !P.want_g) return stt;
    hipLaunchKernelGGL(grid_reduce_kernel, dim3(a.B * a.K * 3), dim3(256), 0, st, a.part, P.gpi, a.K,
                       a.Ds, a.grids, a.gw, a.dgrids, a.dgw, a.dgb);
    return check_launch("grid_reduce");
}

}  // namespace svdlut
