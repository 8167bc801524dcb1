// Internal declarations shared by the library's translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <string>

#include "../../include/svdlut.h"

namespace svdlut {

constexpr int kMaxD = 40;
constexpr int kMaxR = 64;
constexpr int kMaxDim = 65535;
constexpr int kMaxGenBatch = 4096;   // images per generator call (keeps its int sizes in range)
constexpr int kWave = 64;
constexpr int kPxPerLane = 4;                      // pixels per lane per row segment
constexpr int kSeg = kWave * kPxPerLane;           // pixels per row segment (one wave)
// The uneven-batch plan may also run 8 pixels per lane (512-pixel segments) when every map
// is coarse enough for the piecewise map path at that width and there are no grids.
constexpr int kPxWide = 8;

void set_error(const std::string& msg);
svdlut_status fail(svdlut_status st, const std::string& msg);
svdlut_status check_launch(const char* what);

struct DeviceInfo {
    int device = 0;
    int cus = 256;
    int lds_per_block = 65536;
    int lds_per_cu = 163840;
    std::string arch;
};
const DeviceInfo& device_info();

// ---------------------------------------------------------------- LUT path geometry
// Per-image geometry for the apply kernels.  Offsets are in elements.
struct ImgGeom {
    int32_t H, W, h, w;
    int64_t x_off, y_off, map_off;
};

struct ApplyLaunch {
    const void* x;
    void* y;
    const float* U;
    const float* s;
    const float* V;
    const void* map;
    const float* bias;
    int32_t B, D, R;
    // uniform batch (descs == nullptr): dims below; uneven batch: per-image descs on device
    int32_t H, W, h, w;
    const ImgGeom* descs;          // device, uneven batch only
    const int64_t* tile_start;     // device [B+1] prefix of row segments, uneven batch only
    int64_t total_tiles;
    int32_t ncol_max;              // staged map columns per wave
    int32_t fast_map;              // 1: a lane's pixels lie within two map cells (piecewise path)
    int32_t px;                    // pixels per lane: 4 (0 reads as 4) or kPxWide (plan only)
    int32_t block;                 // threads per workgroup
    int32_t grid;                  // workgroups
    svdlut_dtype io, map_dt;
    // optional 2D bilateral grids (K == 0: none): grids [B][K][3][Ds][Ds], gw [B][K][3], gb [B][K]
    const float* grids;
    const float* gw;
    const float* gb;
    int32_t K, Ds;
};

constexpr int kMaxGrids = 12;
constexpr int kMaxDs = 33;
// LDS floats of the combined grid planes (one xy, xc and yc plane per output channel)
__host__ __device__ inline int grid_plane_stride(int Ds) { return Ds | 1; }
__host__ __device__ inline int grid_floats(int Ds) { return 9 * Ds * grid_plane_stride(Ds); }

size_t apply_lds_bytes(int D, int R, int block, int ncol_max, int Ds = 0);
int apply_max_block(svdlut_dtype io, bool fast_map, bool grid, int px = kPxPerLane);
int map_cols_bound(int W, int w, int px = kPxPerLane);
bool map_fast_ok(int W, int w, int px = kPxPerLane);
svdlut_status launch_apply(const ApplyLaunch& a, hipStream_t st);
svdlut_status launch_reconstruct(const float* U, const float* s, const float* V, float* T,
                                 int n, int D, int R, hipStream_t st);

struct BwdLaunch {
    const void* x;
    const void* dy;
    const float* U;
    const float* s;
    const float* V;
    const void* map;
    void* dx;
    float* dU;
    float* ds;
    float* dV;
    float* dmap;
    float* dbias;
    float* dT;                     // workspace [B][9][D][D]
    // deterministic mode: per-workgroup dmap and dbias partials, bwd_det_bytes(B, H, W, h, w)
    // bytes, summed in a fixed order by a second kernel (nullptr: float atomics)
    void* det;
    int32_t B, H, W, h, w, D, R;
    svdlut_dtype io, map_dt;
};
svdlut_status launch_apply_bwd(const BwdLaunch& a, hipStream_t st);
int bwd_groups_per_image(int B);
size_t bwd_workspace_bytes(int B, int D);
size_t bwd_det_bytes(int B, int H, int W, int h, int w);
bool deterministic_mode();

// Backward of the bilateral-grid slicing; dx (if set) is accumulated into.
struct GridBwdLaunch {
    const void* x;
    const void* dy;
    void* dx;
    const float* grids;
    const float* gw;
    float* part;                   // workspace, grid_bwd_workspace_bytes(B, Ds)
    float* dgrids;                 // [B][K][3][Ds][Ds]; with dgw [B][K][3], dgb [B][K] (all or none)
    float* dgw;
    float* dgb;
    int32_t B, H, W, K, Ds;
    svdlut_dtype io;
};
size_t grid_bwd_workspace_bytes(int B, int Ds);
svdlut_status launch_grid_bwd(const GridBwdLaunch& a, hipStream_t st);

// Unfused original-structure baseline (slicing -> f_s -> 1x1 fusion -> 3D LUT), float32.
struct UnfusedLaunch {
    const float* x;
    float* y;
    const float* grids;            // [B][K][3][Ds][Ds]
    const float* gw;               // [B][K][3]
    const float* gb;               // [B][K]
    const float* Wf;               // [B][3][K+3]
    const float* bf;               // [B][3]
    const float* T3;               // [B][3][D][D][D]
    void* ws;                      // unfused_workspace_bytes(B, H, W, K, D)
    int32_t B, H, W, K, Ds, D;
};
size_t unfused_workspace_bytes(int B, int H, int W, int K, int D);
svdlut_status launch_unfused(const UnfusedLaunch& a, hipStream_t st);

// Standalone 3D-LUT (trilinear) and 1D-LUT (per-channel linear) transforms, fp32 planar.
size_t lut3d_workspace_bytes(int B, int D);
svdlut_status launch_lut3d(const float* x, float* y, const float* T3, int B, int H, int W, int D, void* ws,
                           hipStream_t st);
svdlut_status launch_lut1d(const float* x, float* y, const float* T1, int B, int H, int W, int D, hipStream_t st);

// ---------------------------------------------------------------- generator
svdlut_status launch_loss(const void* y, const void* t, svdlut_dtype io, int64_t n, int kind,
                          float* loss, void* dy, float* partial, int nblocks, hipStream_t st);
int loss_blocks(int64_t n);

}  // namespace svdlut
