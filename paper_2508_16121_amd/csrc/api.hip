// extern "C" entry points of the 2D-LUT path: argument validation (before any HIP call),
// launch configuration, error reporting, and the uneven-batch plan (HIP graph + tuner).
#include "internal.h"
#include "tune_cache.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <vector>

namespace svdlut {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

svdlut_status fail(svdlut_status st, const std::string& msg) {
    set_error(msg);
    return st;
}

svdlut_status check_launch(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(SVDLUT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return SVDLUT_OK;
}

const DeviceInfo& device_info() {
    static std::mutex mu;
    static std::map<int, DeviceInfo> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    DeviceInfo d;
    d.device = dev;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) d.cus = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
        d.lds_per_block = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess && v > 0)
        d.lds_per_cu = v;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) d.arch = prop.gcnArchName;
    (void)hipGetLastError();
    return cache.emplace(dev, d).first->second;
}

size_t bwd_workspace_bytes(int B, int D);

// ---------------------------------------------------------------- deterministic mode
// -1 until first read: then the environment variable SVDLUT_DETERMINISTIC (set, non-empty
// and not "0" turns it on), unless svdlut_set_deterministic chose first.
static std::atomic<int> g_det{-1};

bool deterministic_mode() {
    int v = g_det.load(std::memory_order_relaxed);
    if (v < 0) {
        const char* e = std::getenv("SVDLUT_DETERMINISTIC");
        int want = (e && *e && std::strcmp(e, "0") != 0) ? 1 : 0;
        g_det.compare_exchange_strong(v, want);
        v = g_det.load(std::memory_order_relaxed);
    }
    return v == 1;
}

static size_t align256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

// ---------------------------------------------------------------- validation helpers
static bool dims_ok(int64_t v) { return v >= 1 && v <= kMaxDim; }

static svdlut_status check_lut_dims(int D, int R) {
    if (D < 2 || D > kMaxD) return fail(SVDLUT_EINVAL, "D must be in [2, 40]");
    if (R < 1 || R > kMaxR) return fail(SVDLUT_EINVAL, "R must be in [1, 64]");
    return SVDLUT_OK;
}

static svdlut_status check_dtype(svdlut_dtype t, const char* what) {
    if (t != SVDLUT_F32 && t != SVDLUT_F16)
        return fail(SVDLUT_EUNSUPPORTED, std::string(what) + ": dtype must be SVDLUT_F32 or SVDLUT_F16");
    return SVDLUT_OK;
}

#define SVDLUT_TRY(expr)                          \
    do {                                          \
        const svdlut_status st_ = (expr);         \
        if (st_ != SVDLUT_OK) return st_;         \
    } while (0)

// Default launch shape of the fused apply: one workgroup of the variant's largest size per CU
// (maxb = 1024: 16 waves, the most a 128-VGPR budget allows; 512 for the variants built with
// 256 VGPRs) when its LDS fits, else the largest that fits.
static int default_block(int D, int R, int ncol_max, const DeviceInfo& di, int Ds = 0, int maxb = 1024) {
    for (int b : {1024, 512, 256, 128, 64})
        if (b <= maxb && apply_lds_bytes(D, R, b, ncol_max, Ds) <= static_cast<size_t>(di.lds_per_block)) return b;
    return 0;
}

// Workgroups per CU that can be resident: a variant built for maxb threads per workgroup
// holds 65536 / maxb VGPRs per lane, so a CU fits maxb / 64 of its waves; LDS may allow fewer.
static int blocks_per_cu(int D, int R, int block, int ncol_max, const DeviceInfo& di, int Ds = 0, int maxb = 1024) {
    const size_t lds = apply_lds_bytes(D, R, block, ncol_max, Ds);
    const int by_lds = static_cast<int>(di.lds_per_cu / std::max<size_t>(lds, 1));
    const int by_waves = maxb / std::max(block, kWave);
    return std::max(1, std::min(by_lds, by_waves));
}

// Argument checks of svdlut_apply_bwd and svdlut_apply_bwd_noalloc (no HIP call).
static svdlut_status check_apply_bwd(const void* x, const void* dy, svdlut_dtype io, const float* U, const float* s,
                                     const float* V, const void* map, svdlut_dtype map_dt, const float* dU,
                                     const float* ds, const float* dV, int32_t B, int32_t H, int32_t W, int32_t h,
                                     int32_t w, int32_t D, int32_t R) {
    if (!x || !dy || !U || !s || !V || !map) return fail(SVDLUT_EINVAL, "apply_bwd: null input pointer");
    const int nfac = (dU != nullptr) + (ds != nullptr) + (dV != nullptr);
    if (nfac != 0 && nfac != 3) return fail(SVDLUT_EINVAL, "apply_bwd: dU, ds, dV must be all set or all NULL");
    SVDLUT_TRY(check_dtype(io, "apply_bwd io"));
    SVDLUT_TRY(check_dtype(map_dt, "apply_bwd map"));
    if (B < 1) return fail(SVDLUT_EINVAL, "apply_bwd: B must be >= 1");
    if (!dims_ok(H) || !dims_ok(W) || !dims_ok(h) || !dims_ok(w))
        return fail(SVDLUT_EINVAL, "apply_bwd: H, W, h, w must be in [1, 65535]");
    return check_lut_dims(D, R);
}

// Deterministic mode: whether a backward call needs the partials region (dmap or dbias
// requested), and where it sits: after the first `base` bytes of the workspace, aligned.
static bool det_needed(const float* dmap, const float* dbias) { return (dmap || dbias) && deterministic_mode(); }

static svdlut_status det_region(void* ws, size_t ws_bytes, size_t base, int32_t B, int32_t H, int32_t W, int32_t h,
                                int32_t w, const char* what, void** det) {
    const size_t need = align256(base) + bwd_det_bytes(B, H, W, h, w);
    if (!ws || ws_bytes < need)
        return fail(SVDLUT_EINVAL, std::string(what) + ": deterministic mode needs a workspace of " +
                                       std::to_string(need) + " bytes (the usual size plus "
                                       "svdlut_deterministic_workspace_size())");
    *det = static_cast<char*>(ws) + align256(base);
    return SVDLUT_OK;
}

// The backward launch once the arguments (and the partial buffers) are settled.
static svdlut_status apply_bwd_launch(const void* x, const void* dy, svdlut_dtype io, const float* U, const float* s,
                                      const float* V, const void* map, svdlut_dtype map_dt, void* dx, float* dU,
                                      float* ds, float* dV, float* dmap, float* dbias, int32_t B, int32_t H,
                                      int32_t W, int32_t h, int32_t w, int32_t D, int32_t R, void* ws,
                                      void* det, hipStream_t stream) {
    if (!dx && !dU && !dmap && !dbias) return SVDLUT_OK;
    BwdLaunch a{};
    a.x = x; a.dy = dy; a.U = U; a.s = s; a.V = V; a.map = map;
    a.dx = dx; a.dU = dU; a.ds = ds; a.dV = dV; a.dmap = dmap; a.dbias = dbias;
    a.dT = static_cast<float*>(ws);
    a.det = det;
    a.B = B; a.H = H; a.W = W; a.h = h; a.w = w; a.D = D; a.R = R;
    a.io = io; a.map_dt = map_dt;
    return launch_apply_bwd(a, stream);
}

// ---------------------------------------------------------------- allocation-free backward
// svdlut_apply_bwd_noalloc keeps the backward's dT partials in this library-owned array
// instead of a caller workspace.  Host code never passes the array's name as an address:
// each device's copy is looked up once with hipGetSymbolAddress, with that device current,
// and that pointer is what the kernels receive.
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[SVDLUT_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kScratchDevices] = {};

static svdlut_status scratch_for_current_device(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SVDLUT_EDEVICE, "apply_bwd_noalloc: hipGetDevice failed");
    }
    if (dev < 0 || dev >= kScratchDevices)
        return fail(SVDLUT_EUNSUPPORTED, "apply_bwd_noalloc: device index beyond the library's table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(SVDLUT_EDEVICE, std::string("apply_bwd_noalloc: hipGetSymbolAddress failed: ") +
                                            hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SVDLUT_OK;
}

}  // namespace svdlut

using namespace svdlut;

// ================================================================== C ABI
extern "C" {

const char* svdlut_last_error(void) { return g_last_error.c_str(); }

const char* svdlut_version(void) { return "svdlut-mi355x 0.1 (gfx950)"; }

svdlut_status svdlut_reconstruct(const float* U, const float* s, const float* V, float* T,
                                 int32_t n_luts, int32_t D, int32_t R, hipStream_t stream) {
    if (!U || !s || !V || !T) return fail(SVDLUT_EINVAL, "reconstruct: null pointer");
    if (n_luts < 1) return fail(SVDLUT_EINVAL, "reconstruct: n_luts must be >= 1");
    SVDLUT_TRY(check_lut_dims(D, R));
    return launch_reconstruct(U, s, V, T, n_luts, D, R, stream);
}

// Shared by svdlut_apply and svdlut_apply_grid (K == 0: no grids).
static svdlut_status apply_impl(const void* x, void* y, svdlut_dtype io, const float* U, const float* s,
                                const float* V, const void* map, svdlut_dtype map_dt, const float* bias,
                                const float* grids, const float* gw, const float* gb, int32_t K,
                                int32_t Ds, int32_t B, int32_t H, int32_t W, int32_t h, int32_t w,
                                int32_t D, int32_t R, hipStream_t stream) {
    if (!x || !y || !U || !s || !V || !map) return fail(SVDLUT_EINVAL, "apply: null pointer");
    SVDLUT_TRY(check_dtype(io, "apply io"));
    SVDLUT_TRY(check_dtype(map_dt, "apply map"));
    if (B < 1) return fail(SVDLUT_EINVAL, "apply: B must be >= 1");
    if (!dims_ok(H) || !dims_ok(W) || !dims_ok(h) || !dims_ok(w))
        return fail(SVDLUT_EINVAL, "apply: H, W, h, w must be in [1, 65535]");
    SVDLUT_TRY(check_lut_dims(D, R));
    const DeviceInfo& di = device_info();
    ApplyLaunch a{};
    a.x = x; a.y = y; a.U = U; a.s = s; a.V = V; a.map = map; a.bias = bias;
    a.B = B; a.D = D; a.R = R; a.H = H; a.W = W; a.h = h; a.w = w;
    a.descs = nullptr; a.tile_start = nullptr;
    a.total_tiles = static_cast<int64_t>(B) * H * ((W + kSeg - 1) / kSeg);
    a.ncol_max = map_cols_bound(W, w);
    a.fast_map = map_fast_ok(W, w) ? 1 : 0;
    a.px = kPxPerLane;
    a.grids = grids; a.gw = gw; a.gb = gb; a.K = K; a.Ds = Ds;
    const int lds_ds = K > 0 ? Ds : 0;
    const int maxb = apply_max_block(io, a.fast_map != 0, K > 0);
    a.block = default_block(D, R, a.ncol_max, di, lds_ds, maxb);
    if (a.block == 0) return fail(SVDLUT_EUNSUPPORTED, "apply: map too wide for LDS staging");
    // small frames: narrower workgroups, so that the tiles (one per wave at least) spread over
    // more CUs instead of filling a few 16-wave workgroups; not below 256 threads, since every
    // workgroup rebuilds the LUTs and fewer threads take longer over it (256x256 frame, D = 17:
    // 14.5 us with 64-thread workgroups, 11.3 with 128, 10.0 with 256, 14.6 with 1024)
    while (a.block > 256 && a.total_tiles < static_cast<int64_t>(di.cus) * (a.block / kWave)) a.block /= 2;
    const int64_t max_grid = static_cast<int64_t>(di.cus) * blocks_per_cu(D, R, a.block, a.ncol_max, di, lds_ds, maxb);
    const int64_t tiles_per_block_min = a.block / kWave;   // at least one tile per wave
    a.grid = static_cast<int>(std::max<int64_t>(1, std::min(max_grid, (a.total_tiles + tiles_per_block_min - 1) / tiles_per_block_min)));
    a.io = io; a.map_dt = map_dt;
    return launch_apply(a, stream);
}

svdlut_status svdlut_apply(const void* x, void* y, svdlut_dtype io, const float* U, const float* s,
                           const float* V, const void* map, svdlut_dtype map_dt, const float* bias,
                           int32_t B, int32_t H, int32_t W, int32_t h, int32_t w, int32_t D,
                           int32_t R, hipStream_t stream) {
    return apply_impl(x, y, io, U, s, V, map, map_dt, bias, nullptr, nullptr, nullptr, 0, 0, B, H, W,
                      h, w, D, R, stream);
}

svdlut_status svdlut_apply_grid(const void* x, void* y, svdlut_dtype io, const float* U, const float* s,
                                const float* V, const void* map, svdlut_dtype map_dt, const float* bias,
                                const float* grids, const float* gw, const float* gb, int32_t K,
                                int32_t Ds, int32_t B, int32_t H, int32_t W, int32_t h, int32_t w,
                                int32_t D, int32_t R, hipStream_t stream) {
    if (!grids || !gw || !gb) return fail(SVDLUT_EINVAL, "apply_grid: null grid pointer");
    if (K < 1 || K > kMaxGrids) return fail(SVDLUT_EINVAL, "apply_grid: K must be in [1, 12]");
    if (Ds < 2 || Ds > kMaxDs) return fail(SVDLUT_EINVAL, "apply_grid: Ds must be in [2, 33]");
    return apply_impl(x, y, io, U, s, V, map, map_dt, bias, grids, gw, gb, K, Ds, B, H, W, h, w, D, R,
                      stream);
}

size_t svdlut_unfused_workspace_size(int32_t B, int32_t H, int32_t W, int32_t K, int32_t D) {
    if (B < 1 || !dims_ok(H) || !dims_ok(W) || K < 1 || K > kMaxGrids || D < 2 || D > kMaxD) return 0;
    return unfused_workspace_bytes(B, H, W, K, D);
}

svdlut_status svdlut_unfused_apply(const float* x, float* y, const float* grids, const float* gw,
                                   const float* gb, const float* Wf, const float* bf, const float* T3,
                                   int32_t K, int32_t Ds, int32_t D, int32_t B, int32_t H, int32_t W,
                                   void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!x || !y || !grids || !gw || !gb || !Wf || !bf || !T3 || !ws)
        return fail(SVDLUT_EINVAL, "unfused_apply: null pointer");
    if (B < 1 || !dims_ok(H) || !dims_ok(W)) return fail(SVDLUT_EINVAL, "unfused_apply: bad B, H or W");
    if (K < 1 || K > kMaxGrids) return fail(SVDLUT_EINVAL, "unfused_apply: K must be in [1, 12]");
    if (Ds < 2 || Ds > kMaxDs) return fail(SVDLUT_EINVAL, "unfused_apply: Ds must be in [2, 33]");
    if (D < 2 || D > kMaxD) return fail(SVDLUT_EINVAL, "unfused_apply: D must be in [2, 40]");
    if (sizeof(float) * static_cast<size_t>(K) * 3 * Ds * grid_plane_stride(Ds) > 65536)
        return fail(SVDLUT_EUNSUPPORTED, "unfused_apply: K grids of Ds^2 planes exceed 64 KB of LDS");
    if (ws_bytes < unfused_workspace_bytes(B, H, W, K, D))
        return fail(SVDLUT_EINVAL, "unfused_apply: workspace smaller than svdlut_unfused_workspace_size()");
    UnfusedLaunch a{};
    a.x = x; a.y = y; a.grids = grids; a.gw = gw; a.gb = gb; a.Wf = Wf; a.bf = bf; a.T3 = T3; a.ws = ws;
    a.B = B; a.H = H; a.W = W; a.K = K; a.Ds = Ds; a.D = D;
    return launch_unfused(a, stream);
}

size_t svdlut_lut3d_workspace_size(int32_t B, int32_t D) {
    if (B < 1 || D < 2 || D > kMaxD) return 0;
    return lut3d_workspace_bytes(B, D);
}

svdlut_status svdlut_lut3d_apply(const float* x, float* y, const float* T3, int32_t B, int32_t H, int32_t W,
                                 int32_t D, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!x || !y || !T3 || !ws) return fail(SVDLUT_EINVAL, "lut3d_apply: null pointer");
    if (B < 1 || !dims_ok(H) || !dims_ok(W)) return fail(SVDLUT_EINVAL, "lut3d_apply: bad B, H or W");
    if (D < 2 || D > kMaxD) return fail(SVDLUT_EINVAL, "lut3d_apply: D must be in [2, 40]");
    if (ws_bytes < lut3d_workspace_bytes(B, D))
        return fail(SVDLUT_EINVAL, "lut3d_apply: workspace smaller than svdlut_lut3d_workspace_size()");
    return launch_lut3d(x, y, T3, B, H, W, D, ws, stream);
}

svdlut_status svdlut_lut1d_apply(const float* x, float* y, const float* T1, int32_t B, int32_t H, int32_t W,
                                 int32_t D, hipStream_t stream) {
    if (!x || !y || !T1) return fail(SVDLUT_EINVAL, "lut1d_apply: null pointer");
    if (B < 1 || !dims_ok(H) || !dims_ok(W)) return fail(SVDLUT_EINVAL, "lut1d_apply: bad B, H or W");
    if (D < 2 || D > kMaxD) return fail(SVDLUT_EINVAL, "lut1d_apply: D must be in [2, 40]");
    return launch_lut1d(x, y, T1, B, H, W, D, stream);
}

size_t svdlut_apply_grid_bwd_workspace_size(int32_t B, int32_t D, int32_t Ds) {
    if (B < 1 || D < 2 || D > kMaxD || Ds < 2 || Ds > kMaxDs) return 0;
    return ((bwd_workspace_bytes(B, D) + 255) & ~static_cast<size_t>(255)) + grid_bwd_workspace_bytes(B, Ds);
}

svdlut_status svdlut_apply_grid_bwd(const void* x, const void* dy, svdlut_dtype io, const float* U,
                                    const float* s, const float* V, const void* map, svdlut_dtype map_dt,
                                    const float* grids, const float* gw, int32_t K, int32_t Ds, void* dx,
                                    float* dU, float* ds, float* dV, float* dmap, float* dbias,
                                    float* dgrids, float* dgw, float* dgb, int32_t B, int32_t H, int32_t W,
                                    int32_t h, int32_t w, int32_t D, int32_t R, void* ws, size_t ws_bytes,
                                    hipStream_t stream) {
    if (!grids || !gw) return fail(SVDLUT_EINVAL, "apply_grid_bwd: null grid pointer");
    if (K < 1 || K > kMaxGrids) return fail(SVDLUT_EINVAL, "apply_grid_bwd: K must be in [1, 12]");
    if (Ds < 2 || Ds > kMaxDs) return fail(SVDLUT_EINVAL, "apply_grid_bwd: Ds must be in [2, 33]");
    const int ng = (dgrids != nullptr) + (dgw != nullptr) + (dgb != nullptr);
    if (ng != 0 && ng != 3) return fail(SVDLUT_EINVAL, "apply_grid_bwd: dgrids, dgw, dgb must be all set or all NULL");
    if (B < 1 || !dims_ok(H) || !dims_ok(W)) return fail(SVDLUT_EINVAL, "apply_grid_bwd: bad B, H or W");
    SVDLUT_TRY(check_lut_dims(D, R));
    const size_t lut_ws = (bwd_workspace_bytes(B, D) + 255) & ~static_cast<size_t>(255);
    if ((ng == 3 || dU) && (!ws || ws_bytes < lut_ws + grid_bwd_workspace_bytes(B, Ds)))
        return fail(SVDLUT_EINVAL, "apply_grid_bwd: workspace smaller than svdlut_apply_grid_bwd_workspace_size()");
    SVDLUT_TRY(check_apply_bwd(x, dy, io, U, s, V, map, map_dt, dU, ds, dV, B, H, W, h, w, D, R));
    void* det = nullptr;
    if (det_needed(dmap, dbias))
        SVDLUT_TRY(det_region(ws, ws_bytes, lut_ws + grid_bwd_workspace_bytes(B, Ds), B, H, W, h, w,
                              "apply_grid_bwd", &det));
    // the LUT part writes dx (and the LUT gradients); the grid part then adds into dx
    SVDLUT_TRY(apply_bwd_launch(x, dy, io, U, s, V, map, map_dt, dx, dU, ds, dV, dmap, dbias, B, H, W, h, w, D, R,
                                ws, det, stream));
    GridBwdLaunch g{};
    g.x = x; g.dy = dy; g.dx = dx; g.grids = grids; g.gw = gw;
    g.part = ws ? reinterpret_cast<float*>(static_cast<char*>(ws) + lut_ws) : nullptr;
    g.dgrids = dgrids; g.dgw = dgw; g.dgb = dgb;
    g.B = B; g.H = H; g.W = W; g.K = K; g.Ds = Ds; g.io = io;
    return launch_grid_bwd(g, stream);
}

size_t svdlut_apply_bwd_workspace_size(int32_t B, int32_t D) {
    if (B < 1 || D < 2 || D > kMaxD) return 0;
    return bwd_workspace_bytes(B, D);
}

svdlut_status svdlut_apply_bwd(const void* x, const void* dy, svdlut_dtype io, const float* U,
                               const float* s, const float* V, const void* map, svdlut_dtype map_dt,
                               void* dx, float* dU, float* ds, float* dV, float* dmap, float* dbias,
                               int32_t B, int32_t H, int32_t W, int32_t h, int32_t w, int32_t D,
                               int32_t R, void* ws, size_t ws_bytes, hipStream_t stream) {
    SVDLUT_TRY(check_apply_bwd(x, dy, io, U, s, V, map, map_dt, dU, ds, dV, B, H, W, h, w, D, R));
    const bool factors = dU != nullptr;
    if (factors) {
        if (!ws) return fail(SVDLUT_EINVAL, "apply_bwd: workspace required for dU, ds, dV");
        if (ws_bytes < bwd_workspace_bytes(B, D))
            return fail(SVDLUT_EINVAL, "apply_bwd: workspace smaller than svdlut_apply_bwd_workspace_size()");
    }
    void* det = nullptr;
    if (det_needed(dmap, dbias))
        SVDLUT_TRY(det_region(ws, ws_bytes, bwd_workspace_bytes(B, D), B, H, W, h, w, "apply_bwd", &det));
    return apply_bwd_launch(x, dy, io, U, s, V, map, map_dt, dx, dU, ds, dV, dmap, dbias, B, H, W, h, w, D, R,
                            ws, det, stream);
}

svdlut_status svdlut_apply_bwd_noalloc(const void* x, const void* dy, svdlut_dtype io, const float* U,
                                       const float* s, const float* V, const void* map, svdlut_dtype map_dt,
                                       void* dx, float* dU, float* ds, float* dV, float* dmap, float* dbias,
                                       int32_t B, int32_t H, int32_t W, int32_t h, int32_t w, int32_t D,
                                       int32_t R, hipStream_t stream) {
    SVDLUT_TRY(check_apply_bwd(x, dy, io, U, s, V, map, map_dt, dU, ds, dV, B, H, W, h, w, D, R));
    const bool factors = dU != nullptr;
    const bool det = det_needed(dmap, dbias);
    void* ws = nullptr;
    void* det_ptr = nullptr;
    if (factors || det) {
        // the dT partials first, then (deterministic mode) the dmap and dbias partials
        const size_t need = det ? align256(bwd_workspace_bytes(B, D)) + bwd_det_bytes(B, H, W, h, w)
                                : bwd_workspace_bytes(B, D);
        if (need > static_cast<size_t>(SVDLUT_NOALLOC_SCRATCH_BYTES))
            return fail(SVDLUT_EINVAL, "apply_bwd_noalloc: B = " + std::to_string(B) + ", D = " + std::to_string(D) +
                                           (det ? " (deterministic mode)" : "") + " needs " + std::to_string(need) +
                                           " bytes of scratch, more than the library's " +
                                           std::to_string(static_cast<size_t>(SVDLUT_NOALLOC_SCRATCH_BYTES)));
        SVDLUT_TRY(scratch_for_current_device(&ws));
        if (det) det_ptr = static_cast<char*>(ws) + align256(bwd_workspace_bytes(B, D));
    }
    return apply_bwd_launch(x, dy, io, U, s, V, map, map_dt, dx, dU, ds, dV, dmap, dbias, B, H, W, h, w, D, R,
                            factors ? ws : nullptr, det_ptr, stream);
}

void svdlut_set_deterministic(int32_t on) { g_det.store(on ? 1 : 0); }

int32_t svdlut_get_deterministic(void) { return deterministic_mode() ? 1 : 0; }

size_t svdlut_deterministic_workspace_size(int32_t B, int32_t H, int32_t W, int32_t h, int32_t w) {
    if (B < 1 || !dims_ok(H) || !dims_ok(W) || !dims_ok(h) || !dims_ok(w)) return 0;
    return bwd_det_bytes(B, H, W, h, w);
}

}  // extern "C"

// ================================================================== uneven-batch plan
struct svdlut_plan {
    int B = 0, D = 0, R = 0;
    svdlut_dtype io = SVDLUT_F32, map_dt = SVDLUT_F32;
    std::vector<ImgGeom> descs;
    // per tile width (index 0: 4 pixels per lane, 256-pixel segments; 1: 8, 512-pixel
    // segments): prefix of each image's tiles [B+1], tile count, staged map columns per wave
    std::vector<int64_t> tile_start[2];
    int64_t tiles_w[2] = {0, 0};
    int ncol_w[2] = {1, 1};
    int fast_map = 1;                     // 4 pixels per lane: every map allows the piecewise path
    int wide_ok = 1;                      // 8 pixels per lane allowed (piecewise path at that width)
    int64_t pixels = 0, tiles = 0;        // tiles and ncol_max of the current shape
    int ncol_max = 1;
    int px = svdlut::kPxPerLane;
    int block = 512, grid = 1, bpc = 1;
    int tuned = 0;
    ImgGeom* d_descs = nullptr;
    int64_t* d_tiles[2] = {nullptr, nullptr};
    int device = 0;
    // graph state
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t node = nullptr;
    ApplyLaunch captured{};
    bool have_graph = false;
};

namespace svdlut {

static std::mutex g_tune_mu;
static std::map<std::string, TuneEntry> g_tune;   // problem class -> workgroup shape
static bool g_tune_loaded = false;

static std::string tune_key(const svdlut_plan* p, const DeviceInfo& di) {
    // size class: log2 of the pixel count, and whether every map is coarse enough for FASTMAP
    int lg = 0;
    for (int64_t v = std::max<int64_t>(p->pixels, 1); v > 1; v >>= 1) ++lg;
    std::ostringstream os;
    os << (di.arch.empty() ? "gfx" : di.arch.substr(0, di.arch.find(':'))) << "|io" << p->io << "|map"
       << p->map_dt << "|D" << p->D << "|R" << p->R << "|px2^" << lg << "|fast" << p->fast_map;
    return os.str();
}

// The cache file (JSON, see tune_cache.h) named by SVDLUT_TUNE_CACHE is read once; a
// missing, unreadable or corrupt file leaves the built-in defaults for what it lacks.
static void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("SVDLUT_TUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    if (!f) return;
    std::stringstream ss;
    ss << f.rdbuf();
    parse_tune_cache(ss.str(), g_tune);
}

static void tune_save_locked() {
    const char* path = std::getenv("SVDLUT_TUNE_CACHE");
    if (!path) return;
    std::ofstream f(path);
    if (!f) return;
    f << format_tune_cache(g_tune);
}

static ApplyLaunch plan_args(const svdlut_plan* p, const void* x, void* y, const float* U, const float* s,
                             const float* V, const void* map, const float* bias) {
    ApplyLaunch a{};
    a.x = x; a.y = y; a.U = U; a.s = s; a.V = V; a.map = map; a.bias = bias;
    a.B = p->B; a.D = p->D; a.R = p->R;
    a.H = a.W = a.h = a.w = 0;
    const int wi = p->px == kPxWide ? 1 : 0;
    a.descs = p->d_descs; a.tile_start = p->d_tiles[wi];
    a.total_tiles = p->tiles;
    a.ncol_max = p->ncol_max; a.fast_map = wi ? 1 : p->fast_map;
    a.px = p->px;
    a.block = p->block; a.grid = p->grid;
    a.io = p->io; a.map_dt = p->map_dt;
    return a;
}

static void plan_drop_graph(svdlut_plan* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr; p->graph = nullptr; p->node = nullptr; p->have_graph = false;
}

static svdlut_status plan_capture(svdlut_plan* p, const ApplyLaunch& a) {
    plan_drop_graph(p);
    if (std::getenv("SVDLUT_NO_GRAPH")) return SVDLUT_OK;   // plain launches instead
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
        return fail(SVDLUT_EDEVICE, "plan: stream create failed");
    svdlut_status st = SVDLUT_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        st = fail(SVDLUT_EDEVICE, "plan: begin capture failed");
    } else {
        st = launch_apply(a, cs);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(cs, &g);
        if (st == SVDLUT_OK && e != hipSuccess) st = fail(SVDLUT_EDEVICE, "plan: end capture failed");
        if (st == SVDLUT_OK) {
            p->graph = g;
            size_t n = 0;
            if (hipGraphGetNodes(g, nullptr, &n) != hipSuccess || n != 1) {
                st = fail(SVDLUT_EDEVICE, "plan: captured graph has unexpected shape");
            } else {
                (void)hipGraphGetNodes(g, &p->node, &n);
                if (hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess)
                    st = fail(SVDLUT_EDEVICE, "plan: graph instantiate failed");
            }
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
    }
    (void)hipStreamDestroy(cs);
    (void)hipGetLastError();
    if (st == SVDLUT_OK) {
        p->captured = a;
        p->have_graph = true;
    } else {
        plan_drop_graph(p);
    }
    return st;
}

static bool same_buffers(const ApplyLaunch& a, const ApplyLaunch& b) {
    return a.x == b.x && a.y == b.y && a.U == b.U && a.s == b.s && a.V == b.V && a.map == b.map &&
           a.bias == b.bias && a.block == b.block && a.grid == b.grid && a.px == b.px;
}

// Whether a launch shape is valid for the plan: workgroup size and count within the kernel
// variant's limits and the LDS, 8 pixels per lane only where every map allows it.
static bool plan_shape_ok(const svdlut_plan* p, int block, int bpc, int px, const DeviceInfo& di) {
    if (px != kPxPerLane && px != kPxWide) return false;
    if (px == kPxWide && !p->wide_ok) return false;
    const int wi = px == kPxWide ? 1 : 0;
    const bool fast = wi ? true : p->fast_map != 0;
    const int maxthr = apply_max_block(p->io, fast, false, px);
    if (!tune_entry_ok(TuneEntry{block, bpc, px}) || block > maxthr) return false;
    if (apply_lds_bytes(p->D, p->R, block, p->ncol_w[wi]) > static_cast<size_t>(di.lds_per_block)) return false;
    return bpc <= blocks_per_cu(p->D, p->R, block, p->ncol_w[wi], di, 0, maxthr);
}

static void plan_set_shape(svdlut_plan* p, int block, int bpc, int px, const DeviceInfo& di) {
    const int wi = px == kPxWide ? 1 : 0;
    if (px != p->px || block != p->block || bpc != p->bpc) plan_drop_graph(p);   // another kernel or grid
    p->px = wi ? kPxWide : kPxPerLane;
    p->tiles = p->tiles_w[wi];
    p->ncol_max = p->ncol_w[wi];
    p->block = block;
    p->bpc = bpc;
    const int64_t max_grid = static_cast<int64_t>(di.cus) * bpc;
    const int64_t min_tiles = block / kWave;
    p->grid = static_cast<int>(std::max<int64_t>(1, std::min(max_grid, (p->tiles + min_tiles - 1) / min_tiles)));
}

}  // namespace svdlut

extern "C" {

svdlut_status svdlut_plan_create(const svdlut_image_desc* descs, int32_t B, int32_t D, int32_t R,
                                 svdlut_dtype io, svdlut_dtype map_dt, svdlut_plan** out) {
    if (!descs || !out) return fail(SVDLUT_EINVAL, "plan_create: null pointer");
    *out = nullptr;
    if (B < 1) return fail(SVDLUT_EINVAL, "plan_create: B must be >= 1");
    SVDLUT_TRY(check_lut_dims(D, R));
    SVDLUT_TRY(check_dtype(io, "plan io"));
    SVDLUT_TRY(check_dtype(map_dt, "plan map"));
    auto p = new svdlut_plan();
    p->B = B; p->D = D; p->R = R; p->io = io; p->map_dt = map_dt;
    p->descs.resize(B);
    p->tile_start[0].resize(B + 1);
    p->tile_start[1].resize(B + 1);
    int64_t t = 0, t8 = 0;
    for (int b = 0; b < B; ++b) {
        const svdlut_image_desc& d = descs[b];
        if (!dims_ok(d.H) || !dims_ok(d.W) || !dims_ok(d.h) || !dims_ok(d.w) || d.x_off < 0 || d.y_off < 0 ||
            d.map_off < 0) {
            delete p;
            return fail(SVDLUT_EINVAL, "plan_create: descriptor " + std::to_string(b) + " out of range");
        }
        p->descs[b] = ImgGeom{d.H, d.W, d.h, d.w, d.x_off, d.y_off, d.map_off};
        p->tile_start[0][b] = t;
        p->tile_start[1][b] = t8;
        t += static_cast<int64_t>(d.H) * ((d.W + kSeg - 1) / kSeg);
        t8 += static_cast<int64_t>(d.H) * ((d.W + kWave * kPxWide - 1) / (kWave * kPxWide));
        p->pixels += static_cast<int64_t>(d.H) * d.W;
        p->ncol_w[0] = std::max(p->ncol_w[0], map_cols_bound(d.W, d.w));
        p->ncol_w[1] = std::max(p->ncol_w[1], map_cols_bound(d.W, d.w, kPxWide));
        if (!map_fast_ok(d.W, d.w)) p->fast_map = 0;
        if (!map_fast_ok(d.W, d.w, kPxWide)) p->wide_ok = 0;
    }
    p->tile_start[0][B] = t;
    p->tile_start[1][B] = t8;
    p->tiles_w[0] = t;
    p->tiles_w[1] = t8;
    const DeviceInfo& di = device_info();
    p->device = di.device;
    const std::string key = tune_key(p, di);
    const int maxb = apply_max_block(io, p->fast_map != 0, false);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        auto it = g_tune.find(key);
        if (it != g_tune.end() && plan_shape_ok(p, it->second.block, it->second.bpc, it->second.px, di)) {
            plan_set_shape(p, it->second.block, it->second.bpc, it->second.px, di);
            p->tuned = 1;
        }
    }
    if (!p->tuned) {
        const int blk = default_block(D, R, p->ncol_w[0], di, 0, maxb);
        if (blk == 0) {
            delete p;
            return fail(SVDLUT_EUNSUPPORTED, "plan_create: map too wide for LDS staging");
        }
        plan_set_shape(p, blk, blocks_per_cu(D, R, blk, p->ncol_w[0], di, 0, maxb), kPxPerLane, di);
    }
    if (hipMalloc(reinterpret_cast<void**>(&p->d_descs), sizeof(ImgGeom) * B) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&p->d_tiles[0]), sizeof(int64_t) * (B + 1)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&p->d_tiles[1]), sizeof(int64_t) * (B + 1)) != hipSuccess) {
        (void)hipGetLastError();
        if (p->d_descs) (void)hipFree(p->d_descs);
        if (p->d_tiles[0]) (void)hipFree(p->d_tiles[0]);
        delete p;
        return fail(SVDLUT_ENOMEM, "plan_create: device table allocation failed");
    }
    if (hipMemcpy(p->d_descs, p->descs.data(), sizeof(ImgGeom) * B, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_tiles[0], p->tile_start[0].data(), sizeof(int64_t) * (B + 1), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(p->d_tiles[1], p->tile_start[1].data(), sizeof(int64_t) * (B + 1), hipMemcpyHostToDevice) !=
            hipSuccess) {
        (void)hipFree(p->d_descs);
        (void)hipFree(p->d_tiles[0]);
        (void)hipFree(p->d_tiles[1]);
        delete p;
        return fail(SVDLUT_EDEVICE, "plan_create: descriptor upload failed");
    }
    *out = p;
    return SVDLUT_OK;
}

static svdlut_status check_plan_ptrs(const svdlut_plan* p, const void* x, void* y, const float* U,
                                     const float* s, const float* V, const void* map) {
    if (!p) return fail(SVDLUT_EINVAL, "plan: null plan");
    if (!x || !y || !U || !s || !V || !map) return fail(SVDLUT_EINVAL, "plan: null buffer pointer");
    return SVDLUT_OK;
}

svdlut_status svdlut_plan_launch_direct(svdlut_plan* p, const void* x, void* y, const float* U,
                                        const float* s, const float* V, const void* map, const float* bias,
                                        hipStream_t stream) {
    SVDLUT_TRY(check_plan_ptrs(p, x, y, U, s, V, map));
    return launch_apply(plan_args(p, x, y, U, s, V, map, bias), stream);
}

svdlut_status svdlut_plan_launch(svdlut_plan* p, const void* x, void* y, const float* U, const float* s,
                                 const float* V, const void* map, const float* bias, hipStream_t stream) {
    SVDLUT_TRY(check_plan_ptrs(p, x, y, U, s, V, map));
    const ApplyLaunch a = plan_args(p, x, y, U, s, V, map, bias);
    if (!p->have_graph) {
        const svdlut_status st = plan_capture(p, a);
        if (st != SVDLUT_OK || !p->have_graph) return launch_apply(a, stream);   // plain launch fallback
    } else if (!same_buffers(a, p->captured)) {
        hipKernelNodeParams kp{};
        if (hipGraphKernelNodeGetParams(p->node, &kp) != hipSuccess) {
            (void)hipGetLastError();
            SVDLUT_TRY(plan_capture(p, a));
        } else {
            ApplyLaunch arg = a;
            void* args[1] = {&arg};
            kp.kernelParams = args;
            kp.extra = nullptr;
            if (hipGraphExecKernelNodeSetParams(p->exec, p->node, &kp) != hipSuccess) {
                (void)hipGetLastError();
                SVDLUT_TRY(plan_capture(p, a));
            } else {
                p->captured = a;
            }
        }
    }
    if (!p->have_graph) return launch_apply(a, stream);
    if (hipGraphLaunch(p->exec, stream) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SVDLUT_EDEVICE, "plan_launch: graph launch failed");
    }
    return SVDLUT_OK;
}

svdlut_status svdlut_plan_autotune(svdlut_plan* p, const void* x, void* y, const float* U, const float* s,
                                   const float* V, const void* map, const float* bias, hipStream_t stream) {
    SVDLUT_TRY(check_plan_ptrs(p, x, y, U, s, V, map));
    const DeviceInfo& di = device_info();
    // candidates: tile width (4 pixels per lane, and 8 where every map allows it) x
    // workgroup size x workgroups per CU (powers of two and the most that fit)
    struct Cand { int block, bpc, px; };
    std::vector<Cand> cands;
    for (int px : {kPxPerLane, kPxWide}) {
        if (px == kPxWide && !p->wide_ok) continue;
        const int wi = px == kPxWide ? 1 : 0;
        const int maxthr = apply_max_block(p->io, wi ? true : p->fast_map != 0, false, px);
        for (int blk : {64, 128, 256, 512, 1024}) {
            if (blk > maxthr) continue;
            if (apply_lds_bytes(p->D, p->R, blk, p->ncol_w[wi]) > static_cast<size_t>(di.lds_per_block)) continue;
            const int maxb = blocks_per_cu(p->D, p->R, blk, p->ncol_w[wi], di, 0, maxthr);
            for (int bpc = 1; bpc <= maxb; bpc *= 2) cands.push_back({blk, bpc, px});
            if (maxb & (maxb - 1)) cands.push_back({blk, maxb, px});
        }
    }
    if (cands.empty()) return fail(SVDLUT_EUNSUPPORTED, "plan_autotune: no candidate fits LDS");
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(SVDLUT_EDEVICE, "plan_autotune: event create failed");
    float best = 1e30f;
    Cand bestc = cands[0];
    for (const Cand& c : cands) {
        plan_set_shape(p, c.block, c.bpc, c.px, di);
        const ApplyLaunch a = plan_args(p, x, y, U, s, V, map, bias);
        svdlut_status st = launch_apply(a, stream);   // warm-up
        if (st != SVDLUT_OK) { (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); return st; }
        const int reps = 5;
        (void)hipEventRecord(e0, stream);
        for (int r = 0; r < reps; ++r) launch_apply(a, stream);
        (void)hipEventRecord(e1, stream);
        if (hipEventSynchronize(e1) != hipSuccess) {
            (void)hipEventDestroy(e0); (void)hipEventDestroy(e1);
            return fail(SVDLUT_EDEVICE, "plan_autotune: timing failed");
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) { best = ms; bestc = c; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    plan_set_shape(p, bestc.block, bestc.bpc, bestc.px, di);
    p->tuned = 1;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        g_tune[tune_key(p, di)] = TuneEntry{bestc.block, bestc.bpc, bestc.px};
        tune_save_locked();
    }
    plan_drop_graph(p);
    return SVDLUT_OK;
}

svdlut_status svdlut_plan_set_shape(svdlut_plan* p, int32_t block, int32_t blocks_per_cu, int32_t px_per_lane) {
    if (!p) return fail(SVDLUT_EINVAL, "plan_set_shape: null plan");
    if (px_per_lane != kPxPerLane && px_per_lane != kPxWide)
        return fail(SVDLUT_EINVAL, "plan_set_shape: px_per_lane must be 4 or 8");
    if (!tune_entry_ok(TuneEntry{block, blocks_per_cu, px_per_lane}))
        return fail(SVDLUT_EINVAL, "plan_set_shape: block must be 64, 128, 256, 512 or 1024 and blocks_per_cu in [1, 32]");
    const DeviceInfo& di = device_info();
    if (!plan_shape_ok(p, block, blocks_per_cu, px_per_lane, di))
        return fail(SVDLUT_EUNSUPPORTED, "plan_set_shape: shape not supported for this batch (workgroup size, "
                                         "workgroups per CU or LDS, or 8 pixels per lane with a map too fine)");
    plan_set_shape(p, block, blocks_per_cu, px_per_lane, di);
    return SVDLUT_OK;
}

svdlut_status svdlut_plan_get_info(const svdlut_plan* p, svdlut_plan_info* info) {
    if (!p || !info) return fail(SVDLUT_EINVAL, "plan_get_info: null pointer");
    info->pixels = p->pixels;
    info->tiles = p->tiles;
    info->block = p->block;
    info->grid = p->grid;
    info->tuned = p->tuned;
    info->graph = p->have_graph ? 1 : 0;
    info->tile_px = kWave * p->px;
    info->px_per_lane = p->px;
    info->blocks_per_cu = p->bpc;
    info->reserved = 0;
    return SVDLUT_OK;
}

svdlut_status svdlut_plan_destroy(svdlut_plan* p) {
    if (!p) return SVDLUT_OK;
    plan_drop_graph(p);
    if (p->d_descs) (void)hipFree(p->d_descs);
    if (p->d_tiles[0]) (void)hipFree(p->d_tiles[0]);
    if (p->d_tiles[1]) (void)hipFree(p->d_tiles[1]);
    delete p;
    return SVDLUT_OK;
}

}  // extern "C"
