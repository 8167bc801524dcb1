/*
 * svdlut.h — C ABI of the MI355X (gfx950) hot path of the SVD-decomposed, spatially
 * weighted 2D lookup-table image enhancer (Kim, Lee & Cho, arXiv 2508.16121).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Pointers named x, y, U, s, V, map, T, bias, dx, dy, dU, ds, dV, dmap, dbias, params,
 *    grads, m, v, ws are DEVICE pointers owned by the caller.  The library never frees
 *    or retains them past the call.  Descriptor arrays passed as "host" are read during
 *    the call only.
 *  * Every call is asynchronous on the given hipStream_t (NULL = the legacy default
 *    stream) and returns a status.  Arguments are validated before any HIP call; a
 *    rejected call returns SVDLUT_EINVAL (or SVDLUT_EUNSUPPORTED) and enqueues nothing.
 *    A launch failure returns SVDLUT_EDEVICE.  svdlut_last_error() gives a message for
 *    the calling thread's most recent failure.  Every launch is checked right after it
 *    is enqueued (hipGetLastError), so an error the runtime reports at launch time is
 *    returned by the call that made it, never left for a later one.  An error that
 *    happens while a kernel runs is not seen by the library: the ROCm runtime reports it
 *    at the caller's next synchronisation (hipStreamSynchronize and the like), and a GPU
 *    memory fault terminates the process.  The kernels bound every access by the sizes
 *    validated here, so such faults are not an expected outcome of valid arguments.
 *  * Channels a in {0: r, 1: g, 2: b}.  Colour pairs p in {0: rg, 1: rb, 2: gb} with
 *    (alpha, beta) = (0,1), (0,2), (1,2).  The nine LUTs of an image, and the nine
 *    channels of its spatial map, are indexed l = 3*c + p for output channel c.
 *  * Images are planar: [3][H][W] per image, batches [B][3][H][W], row-major.
 *    Factors: U, V [B][9][D][R] and s [B][9][R], float32.  A LUT is indexed
 *    T_l[i][j] with row i along the pair's first channel (alpha) and column j along its
 *    second (beta): T_l = U_l diag(s_l) V_l^T.  Spatial map [B][9][h][w].
 *  * Gradients are overwritten, never accumulated.
 *  * Limits: 2 <= D <= 40 (the LUTs and their gradients are staged in LDS), 1 <= R <= 64,
 *    1 <= H, W, h, w <= 65535, B >= 1 (B <= 4096 for the generators).
 */
#ifndef SVDLUT_H
#define SVDLUT_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SVDLUT_OK = 0,
    SVDLUT_EINVAL = 1,        /* bad pointer, size or dimension */
    SVDLUT_EUNSUPPORTED = 2,  /* dtype or configuration not supported */
    SVDLUT_ENOMEM = 3,        /* an explicit plan could not allocate its device tables */
    SVDLUT_EDEVICE = 4        /* a HIP call or kernel launch failed */
} svdlut_status;

/* The enumerations take any int32 value across the ABI (the range markers make every value
 * representable, so an unknown one is an EUNSUPPORTED or EINVAL argument, not undefined). */
typedef enum {
    SVDLUT_F32 = 0,
    SVDLUT_F16 = 1,
    SVDLUT_DTYPE_RANGE_MIN_ = -2147483647 - 1,
    SVDLUT_DTYPE_RANGE_MAX_ = 2147483647
} svdlut_dtype;

typedef enum {
    SVDLUT_LOSS_L1 = 0,
    SVDLUT_LOSS_MSE = 1,
    SVDLUT_LOSS_RANGE_MIN_ = -2147483647 - 1,
    SVDLUT_LOSS_RANGE_MAX_ = 2147483647
} svdlut_loss_kind;

/* Message for the calling thread's most recent failed call ("" if none). */
const char* svdlut_last_error(void);
/* Library version string. */
const char* svdlut_version(void);

/*
 * svdlut_reconstruct — 2D LUTs from their rank-R factors (Sec. "Singular Value
 * Decomposition", Eq. gen_LUT_SVD: T = U . S . V^T with S = diag(s)).
 *   U, V: [n_luts][D][R] float32; s: [n_luts][R]; T (out): [n_luts][D][D] float32,
 *   T[n][i][j] = sum_k U[n][i][k] * s[n][k] * V[n][j][k].
 */
svdlut_status svdlut_reconstruct(const float* U, const float* s, const float* V, float* T,
                                 int32_t n_luts, int32_t D, int32_t R, hipStream_t stream);

/*
 * svdlut_apply — spatially weighted 2D-LUT transform of a batch of same-size images, with
 * the LUT reconstruction fused into the launch (each workgroup rebuilds its image's nine
 * LUTs into LDS).  Follows the 2D LUT transform of the supplementary material (Eqs.
 * query_lut, lookup, adjacent, bilinear, weighte_sum) with the scalar LUT weights replaced
 * by a per-pixel weight: Y_c = sum_p S_{3c+p}(y, x) * phi_{3c+p} + bias_c, where
 *   phi_l  = bilinear lookup of T_l at (p_alpha, p_beta), p = min(max(X, 0), 1) (NaN -> 0);
 *            cell i = min(floor(q), D-2) with q = p*(D-1) rounded to float32, delta = q - i;
 *   S_l    = corner-aligned bilinear upsample of map channel l (x' = x/(W-1), y' = y/(H-1);
 *            a size-1 map axis is constant).
 *   x:    [B][3][H][W], dtype io (F32 or F16 storage; arithmetic is float32)
 *   y:    [B][3][H][W] (out), dtype io; F16 output is rounded to nearest even.  No clamp.
 *   map:  [B][9][h][w], dtype map_dt
 *   bias: [B][3] float32 or NULL (= 0)
 */
svdlut_status svdlut_apply(const void* x, void* y, svdlut_dtype io,
                           const float* U, const float* s, const float* V,
                           const void* map, svdlut_dtype map_dt, const float* bias,
                           int32_t B, int32_t H, int32_t W, int32_t h, int32_t w,
                           int32_t D, int32_t R, hipStream_t stream);

/*
 * svdlut_apply_grid — svdlut_apply fused with 2D bilateral-grid slicing (supplementary Sec.
 * "2D Slicing", Eqs. query_grid, lookup_grid, adjacent_grid, bilinear_grid and the weighted
 * sum of the three planes; Sec. "Slicing and LUT Transform", Eq. slicing_transform):
 *   Y_c = (svdlut_apply)_c + sum over grids k with k mod 3 = c of Psi^k,
 *   Psi^k = w^k_xy psi_xy + w^k_xc psi_xc + w^k_yc psi_yc + b^k,
 * where psi_ab is the bilinear lookup of plane ab of grid k at the query
 *   xy: (x', y'),  xc: (x', p_c),  yc: (y', p_c),   c = k mod 3,
 * with x' = x/(W-1), y' = y/(H-1) evaluated exactly as x*(Ds-1)/(W-1) (a size-1 image axis
 * queries 0) and p_c decoded like the LUT colours with Ds vertices.
 *   grids: [B][K][3][Ds][Ds] float32, planes in the order (xy, xc, yc), each indexed
 *          [alpha][beta] = [x][y], [x][c], [y][c]
 *   gw:    [B][K][3] float32 plane weights (w_xy, w_xc, w_yc);  gb: [B][K] float32 biases
 *   K:     1..12 (the paper uses 6: two grids per channel);  Ds: 2..33 (the paper: 17)
 * Other arguments as svdlut_apply.  The library folds the grids of one output channel into
 * one weighted grid per workgroup (slicing is linear in the planes), so the result equals
 * the definition up to float32 rounding.  Errors: as svdlut_apply, plus EINVAL for K or Ds
 * out of range or a null grids/gw/gb.
 */
svdlut_status svdlut_apply_grid(const void* x, void* y, svdlut_dtype io, const float* U, const float* s,
                                const float* V, const void* map, svdlut_dtype map_dt, const float* bias,
                                const float* grids, const float* gw, const float* gb, int32_t K,
                                int32_t Ds, int32_t B, int32_t H, int32_t W, int32_t h, int32_t w,
                                int32_t D, int32_t R, hipStream_t stream);


/*
 * svdlut_unfused_apply — the unfused "original structure" the paper starts from (Sec.
 * "Preliminary"), as a baseline for the fused pass: slicing of K bilateral grids into
 * spatial-feature planes f_s (Eq. slicing; Psi^k as in svdlut_apply_grid, one plane per grid,
 * written to the workspace), the 1x1 convolution X_bar = Wf . concat(X, f_s) + bf written to
 * the workspace (Eq. fusion; input channels ordered r, g, b, f_0 .. f_{K-1}), and the 3D-LUT
 * transform Y_c = trilinear lookup of T3[c] at X_bar (Eq. coloren; LUT indexed [i_r][i_g][i_b],
 * the decode of svdlut_apply with D vertices).  float32 only.
 *   x, y: [B][3][H][W];  grids [B][K][3][Ds][Ds], gw [B][K][3], gb [B][K];  Wf [B][3][K+3],
 *   bf [B][3];  T3 [B][3][D][D][D].
 *   ws: at least svdlut_unfused_workspace_size(B, H, W, K, D) bytes, 256-byte aligned,
 *   caller-owned (holds f_s, X_bar and the packed 3D LUTs).
 * Errors: EINVAL for a null pointer, bad sizes or a short workspace; EUNSUPPORTED when the K
 * grids do not fit 64 KB of LDS.
 */
size_t svdlut_unfused_workspace_size(int32_t B, int32_t H, int32_t W, int32_t K, int32_t D);
svdlut_status svdlut_unfused_apply(const float* x, float* y, const float* grids, const float* gw,
                                   const float* gb, const float* Wf, const float* bf, const float* T3,
                                   int32_t K, int32_t Ds, int32_t D, int32_t B, int32_t H, int32_t W,
                                   void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * svdlut_apply_bwd — gradients of a scalar loss through svdlut_apply, given
 * dy = dL/dY [B][3][H][W] (dtype io).  By the chain rule of the forward:
 *   dT_l[i_a + a][i_b + b] += dy_c * S_l * w_alpha(a) * w_beta(b)   (then dU, ds, dV below)
 *   dmap_l[iv + a][iu + b] += dy_c * phi_l * wv(a) * wu(b)
 *   dx_a = sum over the two pairs containing a of dy_c * S_l * dphi_l/dp_a, times 1 where
 *          0 <= x_a <= 1 and 0 elsewhere (and for NaN)
 *   dbias_c = sum of dy_c over the image
 *   dU = dT V diag(s), dV = dT^T U diag(s), ds_k = sum_ij dT_ij U_ik V_jk.
 * Outputs (each may be NULL to skip it; dU, ds and dV are all NULL or all set):
 *   dx [B][3][H][W] dtype io; dU, dV [B][9][D][R]; ds [B][9][R]; dmap [B][9][h][w]
 *   float32; dbias [B][3] float32.
 * ws: device workspace of at least svdlut_apply_bwd_workspace_size(B, D) bytes, 256-byte
 *   aligned, owned by the caller; contents on entry are ignored.
 * Errors: EINVAL for a null input, a partial (dU, ds, dV) trio, sizes out of range or a short
 *   workspace; EUNSUPPORTED for an unknown dtype, or when the map columns that one 256-pixel
 *   row segment touches cannot be staged in LDS next to T and its fixed-point gradient even
 *   with 64-thread workgroups.  That happens only for D >= 37 with maps finer than about two
 *   thirds of the image width at D = 40 (176 columns per segment fit there); for D <= 36
 *   every map size works (fine maps take narrower workgroups, and their dmap partials go
 *   straight to global memory when the map-row accumulator does not fit).
 * dT is accumulated in fixed point per workgroup and summed in a fixed order, so dU, ds
 * and dV are reproducible, as is dx; dmap and dbias are summed across workgroups with
 * float atomics and depend on their order at the level of float32 rounding, except in
 * deterministic mode (svdlut_set_deterministic), where they are bitwise reproducible too.
 */
size_t svdlut_apply_bwd_workspace_size(int32_t B, int32_t D);

/*
 * Deterministic mode (process-wide; initially on when the environment variable
 * SVDLUT_DETERMINISTIC is set to a non-empty value other than "0").  In this mode the
 * backward entry points (svdlut_apply_bwd, _noalloc, svdlut_apply_grid_bwd,
 * svdlut_apply_loss_bwd) reduce dmap and dbias from per-workgroup partials in a fixed order
 * instead of float atomics, so every output is bitwise reproducible for the same inputs on
 * the same device.  It needs svdlut_deterministic_workspace_size(B, H, W, h, w) more bytes of
 * workspace, placed after the entry point's usual size rounded up to 256 bytes (the whole
 * workspace is then that rounded size plus this), whenever dmap or dbias is requested (a
 * workspace becomes required then even without dU); a shorter one gives EINVAL.  A map whose
 * map-row accumulator does not fit the LDS (very wide maps) gives EUNSUPPORTED in this mode.
 * The generators' backward passes are reproducible in both modes.  The setter may be called
 * at any time between calls; calls already queued keep the mode they were issued with.
 */
void svdlut_set_deterministic(int32_t on);
int32_t svdlut_get_deterministic(void);
size_t svdlut_deterministic_workspace_size(int32_t B, int32_t H, int32_t W, int32_t h, int32_t w);
svdlut_status svdlut_apply_bwd(const void* x, const void* dy, svdlut_dtype io,
                               const float* U, const float* s, const float* V,
                               const void* map, svdlut_dtype map_dt,
                               void* dx, float* dU, float* ds, float* dV,
                               float* dmap, float* dbias,
                               int32_t B, int32_t H, int32_t W, int32_t h, int32_t w,
                               int32_t D, int32_t R, void* ws, size_t ws_bytes,
                               hipStream_t stream);

/*
 * svdlut_apply_bwd_noalloc — svdlut_apply_bwd for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, kernels, outputs and determinism, minus ws and ws_bytes.  The dT partials
 * go to a buffer of SVDLUT_NOALLOC_SCRATCH_BYTES that the library holds in device memory
 * on every GPU it runs on until the process ends; the call itself allocates nothing.  Its
 * contents are ignored on entry (every partial is overwritten), so nothing needs clearing.
 * Every call on one GPU shares that GPU's buffer: calls that overlap in time on one GPU
 * (two streams, two host threads) race and must be serialised by the caller.
 * Errors: those of svdlut_apply_bwd, plus EINVAL when the factor gradients are requested
 * and svdlut_apply_bwd_workspace_size(B, D) exceeds SVDLUT_NOALLOC_SCRATCH_BYTES (e.g. at
 * D = 40 up to B = 369 fits, at D = 33 up to B = 577), or in deterministic mode when that
 * size rounded up to 256 bytes plus svdlut_deterministic_workspace_size(B, H, W, h, w)
 * exceeds it, and EDEVICE if the buffer's address cannot be obtained.
 */
#define SVDLUT_NOALLOC_SCRATCH_BYTES (24u * 1024u * 1024u)
svdlut_status svdlut_apply_bwd_noalloc(const void* x, const void* dy, svdlut_dtype io,
                                       const float* U, const float* s, const float* V,
                                       const void* map, svdlut_dtype map_dt,
                                       void* dx, float* dU, float* ds, float* dV,
                                       float* dmap, float* dbias,
                                       int32_t B, int32_t H, int32_t W, int32_t h, int32_t w,
                                       int32_t D, int32_t R, hipStream_t stream);

/*
 * svdlut_apply_grid_bwd — gradients of a scalar loss through svdlut_apply_grid, given
 * dy = dL/dY.  The LUT and map part is svdlut_apply_bwd (same outputs, same rules); the
 * grid part adds, by the chain rule of the slicing (supp. Sec. "2D Slicing"), per grid k of
 * output channel c = k mod 3:
 *   dgrids[k][plane][a][b] = w^k_plane * sum over pixels of dy_c * w_alpha * w_beta at the
 *                            vertex (a, b) of the plane's query,
 *   dgw[k][plane]          = sum over pixels of dy_c * psi^k_plane,
 *   dgb[k]                 = sum over pixels of dy_c,
 *   dx_c                  += dy_c * (Ds-1) * (d psi_xc/d p + d psi_yc/d p) of the weighted
 *                            grids of channel c, inside [0, 1] (the spatial plane has none).
 *   dgrids [B][K][3][Ds][Ds], dgw [B][K][3], dgb [B][K] float32: all set or all NULL.
 * ws: at least svdlut_apply_grid_bwd_workspace_size(B, D, Ds) bytes (caller-owned, 256-byte
 *   aligned) whenever dU or dgrids is requested.  The grid gradients are accumulated in
 *   fixed point per workgroup and summed in a fixed order, so they are reproducible.
 * Errors: as svdlut_apply_bwd, plus EINVAL for K, Ds out of range, a null grids/gw, a
 * partial (dgrids, dgw, dgb) trio or a short workspace.
 */
size_t svdlut_apply_grid_bwd_workspace_size(int32_t B, int32_t D, int32_t Ds);
svdlut_status svdlut_apply_grid_bwd(const void* x, const void* dy, svdlut_dtype io, const float* U,
                                    const float* s, const float* V, const void* map, svdlut_dtype map_dt,
                                    const float* grids, const float* gw, int32_t K, int32_t Ds, void* dx,
                                    float* dU, float* ds, float* dV, float* dmap, float* dbias,
                                    float* dgrids, float* dgw, float* dgb, int32_t B, int32_t H, int32_t W,
                                    int32_t h, int32_t w, int32_t D, int32_t R, void* ws, size_t ws_bytes,
                                    hipStream_t stream);

/*
 * Batches of images of uneven size.  Image b of a batch lives in packed planar buffers at
 * the element offsets of its descriptor: x + x_off holds its [3][H][W] planes, y + y_off
 * receives them, map + map_off holds its [9][h][w] map.  Factors stay [B][9][D][R].
 */
typedef struct {
    int32_t H, W, h, w;
    int64_t x_off, y_off, map_off;
} svdlut_image_desc;

/*
 * svdlut_plan — one persistent launch over every pixel tile of a batch of uneven images,
 * captured once into a HIP graph and replayed.  Tiles are ordered image-major so that a
 * workgroup rebuilds a given image's LUTs at most once.  Creating a plan uploads the
 * descriptors and the tile prefix tables (one per tile width) to device memory owned by the plan (the only
 * allocation on this path) and picks tile and grid shapes from the autotuner's cache
 * (or the built-in default).  Launching with other buffer addresses than the previous
 * launch updates the graph's kernel arguments in place before the replay.
 *   descs: host array of B descriptors; io / map_dt as for svdlut_apply.
 */
typedef struct svdlut_plan svdlut_plan;

typedef struct {
    int64_t pixels;        /* total pixels of the batch */
    int64_t tiles;         /* work tiles (one row segment each) */
    int32_t block;         /* threads per workgroup */
    int32_t grid;          /* workgroups in the persistent launch */
    int32_t tuned;         /* 1 if the shape came from the autotuner */
    int32_t graph;         /* 1 if launches replay a captured HIP graph */
    int32_t tile_px;       /* pixels of one work tile: a row segment handled by one wave (256 or 512) */
    int32_t px_per_lane;   /* consecutive pixels of a tile per lane (4 or 8) */
    int32_t blocks_per_cu; /* resident workgroups per CU the grid was sized for */
    int32_t reserved;
} svdlut_plan_info;

svdlut_status svdlut_plan_create(const svdlut_image_desc* descs, int32_t B, int32_t D, int32_t R,
                                 svdlut_dtype io, svdlut_dtype map_dt, svdlut_plan** out);
/* Launch shapes.  A tile is one row segment handled by one wave: 4 consecutive pixels per
 * lane (256-pixel segments), or 8 (512-pixel segments; only when every image's map is coarse
 * enough that a lane's 8 pixels lie within two map cells, (8-1)(w-1) <= W-1, built for
 * workgroups of at most 512 threads).  The autotuner times every valid combination of tile
 * width, workgroup size (64 .. 1024 threads) and workgroups per CU (powers of two and the
 * most that fit) on the given buffers (outputs are overwritten), keeps the fastest, records
 * it in the tuning cache (saved as JSON to the file named by the SVDLUT_TUNE_CACHE
 * environment variable when set; entries [block, blocks_per_cu, px_per_lane]) and rebuilds
 * the graph.  The two tile widths compute the map weights of a pixel from different staged
 * columns, so their outputs agree to rounding, not bit for bit; the workgroup shape alone
 * does not change any pixel's arithmetic. */
svdlut_status svdlut_plan_autotune(svdlut_plan* plan, const void* x, void* y,
                                   const float* U, const float* s, const float* V,
                                   const void* map, const float* bias, hipStream_t stream);
svdlut_status svdlut_plan_launch(svdlut_plan* plan, const void* x, void* y,
                                 const float* U, const float* s, const float* V,
                                 const void* map, const float* bias, hipStream_t stream);
/* The same work as a plan launch, without the graph (a plain kernel launch). */
svdlut_status svdlut_plan_launch_direct(svdlut_plan* plan, const void* x, void* y,
                                        const float* U, const float* s, const float* V,
                                        const void* map, const float* bias, hipStream_t stream);
/* Set the launch shape by hand (as the autotuner would): block threads per workgroup (64,
 * 128, 256, 512 or 1024), blocks_per_cu workgroups per CU (1 .. 32), px_per_lane 4 or 8.
 * EINVAL for values outside those sets, EUNSUPPORTED for a shape this batch cannot run (a
 * workgroup larger than the kernel variant allows, more workgroups per CU than fit the LDS,
 * or 8 pixels per lane with a map too fine for it); the plan is unchanged then.  A new shape
 * drops the captured graph; the next launch captures it again. */
svdlut_status svdlut_plan_set_shape(svdlut_plan* plan, int32_t block, int32_t blocks_per_cu,
                                    int32_t px_per_lane);
svdlut_status svdlut_plan_get_info(const svdlut_plan* plan, svdlut_plan_info* info);
svdlut_status svdlut_plan_destroy(svdlut_plan* plan);

/*
 * Loss of an enhanced batch against a target (Sec. "Loss Function": the fidelity term is
 * the mean squared error; the mean absolute error is also provided).
 *   y, target: n elements of dtype io.  loss: one float32 (out) = mean |y - t| or
 *   mean (y - t)^2.  dy (nullable, out, dtype io): dL/dy = sign(y - t)/n (sign(0) = 0) or
 *   2 (y - t)/n.  ws: at least svdlut_loss_workspace_size(n) bytes.
 */
size_t svdlut_loss_workspace_size(int64_t n);
svdlut_status svdlut_loss(const void* y, const void* target, svdlut_dtype io, int64_t n,
                          svdlut_loss_kind kind, float* loss, void* dy,
                          void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * svdlut_apply_loss_bwd — one training pass of the transform fused in a single kernel: the
 * forward output Y of svdlut_apply (bias nullable), the mean L1 or MSE loss of Y against
 * target (loss, one float32, device), dL/dY formed per pixel (L1: sign(Y - t)/n with
 * sign(0) = 0; MSE: 2 (Y - t)/n; n = B*3*H*W), and the gradients of svdlut_apply_bwd for that
 * dL/dY.  The results equal svdlut_apply + svdlut_loss + svdlut_apply_bwd up to float
 * rounding; Y and dL/dY are not written.  Layouts, nullability of dx / dU,ds,dV / dmap /
 * dbias and the determinism notes are those of svdlut_apply_bwd; the loss is summed per
 * workgroup and then in a fixed order, so it is reproducible.
 * ws: svdlut_apply_loss_bwd_workspace_size(B, D) bytes (the dT partials and the loss partials).
 */
size_t svdlut_apply_loss_bwd_workspace_size(int32_t B, int32_t D);
svdlut_status svdlut_apply_loss_bwd(const void* x, const void* target, svdlut_dtype io,
                                    const float* U, const float* s, const float* V,
                                    const void* map, svdlut_dtype map_dt, const float* bias,
                                    svdlut_loss_kind kind, float* loss, void* dx,
                                    float* dU, float* ds, float* dV, float* dmap, float* dbias,
                                    int32_t B, int32_t H, int32_t W, int32_t h, int32_t w,
                                    int32_t D, int32_t R, void* ws, size_t ws_bytes,
                                    hipStream_t stream);

/*
 * Learned generator of the factors and the spatial map from a downsampled image (the
 * paper's backbone + LUT generator, Sec. "Preliminary" Eq. backbone and supplementary
 * Tables backbone / gen_lut, sized as a small CNN):
 *   bilinear downsample to 256x256 (half-pixel centres, no antialias)
 *   5 x [conv3x3 stride 2 pad 1 + ReLU]: 3 -> 16 -> 32 -> 64 -> 128 -> 128
 *   global average pool -> FC 128 -> 9*(D*R + R + D*R): per LUT l the block
 *     [U_l (D x R row-major) | s_l (R) | V_l (D x R)]
 *   map head: conv3x3 stride 1 pad 1, 64 -> 9, on the 32x32 third-layer features
 * Convolutions run on bf16 matrix cores (MFMA) with float32 accumulation; activations are
 * stored as bf16; pooling, FC, bias and optimiser state are float32.
 * params: float32 vector of svdlut_generator_param_count(D, R) values, in order
 *   conv1.w [16][3][3][3], conv1.b [16], conv2.w [32][3][3][16], conv2.b, conv3.w
 *   [64][3][3][32], conv3.b, conv4.w [128][3][3][64], conv4.b, conv5.w [128][3][3][128],
 *   conv5.b, head.w [9][3][3][64], head.b [9], fc.w [9*(2DR+R)][128], fc.b
 *   (convolution weights are [Cout][ky][kx][Cin]).
 * B (images per call) is in [1, 4096] for both generators; the size queries return 0 beyond.
 * ws: workspace of svdlut_generator_workspace_size(B, D, R) bytes holding the
 *   activations of the last forward; svdlut_generator_bwd reads them, so the two calls
 *   must share ws and the parameters must not change between them.
 * Forward outputs: U, V [B][9][D][R], s [B][9][R], map [B][9][32][32], float32.
 * Backward inputs dU, ds, dV, dmap have the same shapes; grads (out) has the layout of
 * params.  Forward and backward are deterministic (fixed-order reductions throughout).
 */
size_t svdlut_generator_param_count(int32_t D, int32_t R);
size_t svdlut_generator_workspace_size(int32_t B, int32_t D, int32_t R);
svdlut_status svdlut_generator_fwd(const float* params, const void* x, svdlut_dtype io,
                                   int32_t B, int32_t H, int32_t W, int32_t D, int32_t R,
                                   float* U, float* s, float* V, float* map,
                                   void* ws, size_t ws_bytes, hipStream_t stream);
svdlut_status svdlut_generator_bwd(const float* params, const float* dU, const float* ds,
                                   const float* dV, const float* dmap, float* grads,
                                   int32_t B, int32_t D, int32_t R,
                                   void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * The paper's own generator (supplementary Sec. "Details of Network Structure", Tables
 * backbone, gen_lut, gen_lut_weight, gen_bilateral, gen_bilateral_weight; with K = 6,
 * Ds = 17, D = 33, R = 8 it has the 160,478 parameters of the component ablation, with K = 0
 * the 109,332 of its LUT-only model):
 *   bilinear downsample to 256x256 (half-pixel centres, no antialias)
 *   5 blocks, m = 8: conv3x3 stride 2 pad 1 (+ bias) -> LeakyReLU(0.2) -> instance norm
 *     (per image and channel, biased variance, eps 1e-5, learned scale and shift; not in
 *     block 5): 3 -> 8 -> 16 -> 32 -> 64 -> 64 channels, 256^2 -> 8^2
 *   dropout 0.5 (keep_mask), 4x4 average pooling to 2x2, flattened to 256 features in
 *     NCHW order (feature 4c + 2py + px)
 *   generators, each FC 256 -> 8 then FC 8 -> n (no activation between):
 *     H_t  n = 9(2DR + R): [U (9 x D x R) | S (9 x R) | V (9 x D x R)], LUT l = 3c + p
 *     H_tw n = 12: per output channel c, (w_rg, w_rb, w_gb, b^c)
 *     H_s  n = 3 K Ds^2 (only when K > 0): grids [K][3][Ds][Ds], planes (xy, xc, yc)
 *     H_sw n = 4K (only when K > 0): per grid k, (w_xy, w_xc, w_yc, b^k)
 * The outputs feed svdlut_apply_grid (or svdlut_apply when K = 0) directly: lut_w is its
 * 9 x 1 x 1 map (h = w = 1), lut_b its bias, grids/gw/gb its grid arguments.
 * Convolutions run on bf16 matrix cores with fp32 accumulation; the normalised activations
 * between blocks are stored as bf16; everything else is fp32.
 * params: float32 vector of svdlut_paper_generator_param_count(D, R, K, Ds) values, in order
 *   conv1.w [8][3][3][3], conv1.b [8], norm1.scale [8], norm1.shift [8], conv2 ... norm4,
 *   conv5.w [64][3][3][64], conv5.b [64], then per generator (t, tw, s, sw)
 *   fc1.w [8][256], fc1.b [8], fc2.w [n][8], fc2.b [n].
 * keep_mask (nullable): uint8 [B][64][8][8] (1 keep, 0 drop); kept values are scaled by 2.
 *   NULL is evaluation mode (no dropout).  The backward must get the forward's mask.
 * ws: svdlut_paper_generator_workspace_size(B, D, R, K, Ds) bytes holding the last
 *   forward's activations; the backward reads them (same ws, same parameters, same B).
 * Forward outputs (float32): U, V [B][9][D][R], s [B][9][R], lut_w [B][9], lut_b [B][3],
 *   grids [B][K][3][Ds][Ds], gw [B][K][3], gb [B][K] (grid outputs ignored and nullable when
 *   K = 0).  Backward inputs have the same shapes; a NULL gradient counts as zero.  grads
 *   (out) has the layout of params and is overwritten.
 * K in [0, 12]; Ds in [2, 33] when K > 0; D in [2, 40]; R in [1, 64].
 * The forward and the backward are deterministic: every reduction (weights, biases, norm
 * scale and shift, FC layers) adds per-workgroup partials in a fixed order, so the same
 * inputs give bitwise the same outputs and gradients on the same device.
 */
size_t svdlut_paper_generator_param_count(int32_t D, int32_t R, int32_t K, int32_t Ds);
size_t svdlut_paper_generator_workspace_size(int32_t B, int32_t D, int32_t R, int32_t K, int32_t Ds);
svdlut_status svdlut_paper_generator_fwd(const float* params, const void* x, svdlut_dtype io,
                                         int32_t B, int32_t H, int32_t W, int32_t D, int32_t R,
                                         int32_t K, int32_t Ds, const uint8_t* keep_mask,
                                         float* U, float* s, float* V, float* lut_w, float* lut_b,
                                         float* grids, float* gw, float* gb,
                                         void* ws, size_t ws_bytes, hipStream_t stream);
svdlut_status svdlut_paper_generator_bwd(const float* params, const uint8_t* keep_mask,
                                         const float* dU, const float* ds, const float* dV,
                                         const float* dlut_w, const float* dlut_b,
                                         const float* dgrids, const float* dgw, const float* dgb,
                                         float* grads, int32_t B, int32_t D, int32_t R, int32_t K,
                                         int32_t Ds, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * The other LUT dimensions the paper weighs the 2D decomposition against (Sec.
 * "Preliminary" and the LUT-dimension analysis: a 3D LUT indexed by all three channels and
 * per-channel 1D LUTs), as standalone float32 transforms of planar x [B][3][H][W] into y
 * (same shape, must not alias x).  Inputs are clamped to [0, 1] and decoded like the 2D
 * LUTs (q = x (D - 1) in float32, cell min(floor(q), D - 2)).
 * svdlut_lut3d_apply: T3 [B][3][D][D][D], output channel c reads t^c[i_r][i_g][i_b] by
 *   trilinear interpolation.  ws: svdlut_lut3d_workspace_size(B, D) bytes (the LUTs
 *   repacked as one float4 per vertex).
 * svdlut_lut1d_apply: T1 [B][3][D], y_c = linear interpolation of t_c at x_c.
 * D in [2, 40].
 */
size_t svdlut_lut3d_workspace_size(int32_t B, int32_t D);
svdlut_status svdlut_lut3d_apply(const float* x, float* y, const float* T3, int32_t B, int32_t H,
                                 int32_t W, int32_t D, void* ws, size_t ws_bytes, hipStream_t stream);
svdlut_status svdlut_lut1d_apply(const float* x, float* y, const float* T1, int32_t B, int32_t H,
                                 int32_t W, int32_t D, hipStream_t stream);

/*
 * svdlut_adam_step — one step of standard Adam (the paper trains with Adam, Sec.
 * "Application Settings"), in place on n float32 values:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr * (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps),   step >= 1.
 */
svdlut_status svdlut_adam_step(float* params, const float* grads, float* m, float* v, int64_t n,
                               float lr, float b1, float b2, float eps, int32_t step,
                               hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* SVDLUT_H */
