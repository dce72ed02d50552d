/* gsr.h - C ABI of the MI355X (gfx950) differentiable tile-based Gaussian rasterizer.
 *
 * The library implements the hot path of LiteGS (arXiv 2503.01199): projection of
 * 3-D Gaussians to screen space with spherical-harmonic colour, Morton ordering
 * with cluster-level culling and compaction (Sec. 3.2), (tile, depth) sorting and
 * binning, front-to-back alpha compositing (Sec. 3, Eq. (1)-(2); App. A.2) and its
 * backward pass (Eq. (3); App. A.1), with the opacity-gradient statistic of Sec. 3.3.
 *
 * Conventions for every call:
 *  - Pointers typed `const float *` / `float *` inside gsr_scene, gsr_grads,
 *    gsr_stats and the image arrays are DEVICE pointers owned by the caller. The
 *    gsr_camera array and every struct passed by pointer are HOST memory, read
 *    during the call only.
 *  - `stream` is a hipStream_t (NULL = the default stream). Every call enqueues
 *    its work on that stream and returns without waiting for the device (counts
 *    that decide launch work are read by the kernels from device memory). Results
 *    are valid once the stream has reached the call's work. Only gsr_frame_inspect,
 *    gsr_frame_release and gsr_stage_times wait.
 *  - The library never allocates device memory. Scratch space comes from a
 *    caller-owned workspace whose size the *_workspace_size calls report.
 *  - Every call returns a gsr_status. Host-side validation happens before any
 *    work is enqueued, so on GSR_ERR_INVALID_ARG or GSR_ERR_WORKSPACE_TOO_SMALL
 *    no output has been touched. gsr_last_error() describes the last failure.
 *  - A context is a host object bound to one device. It is not thread-safe: use
 *    one context per host thread. Separate workspaces on separate streams may
 *    run concurrently.
 */
#ifndef GSR_H
#define GSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GSR_OK = 0,
  GSR_ERR_INVALID_ARG = 1,          /* a null pointer, bad size or option; nothing enqueued */
  GSR_ERR_WORKSPACE_TOO_SMALL = 2,  /* gsr_required_workspace() gives the bytes needed */
  GSR_ERR_DEVICE = 3,               /* a HIP runtime call failed */
  GSR_ERR_UNSUPPORTED = 4
} gsr_status;

typedef enum {
  GSR_FP32 = 0,        /* every raster quantity in FP32 */
  GSR_FP16_BLEND = 1,  /* packed-FP16 blend (Sec. 3.1.2): exponents computed in FP32 and rounded
                          toward zero to FP16; G = 2^e and alpha = min(0.99, o G) in packed FP16
                          (clamp point 0.99 rounded to FP16); T, colour and all gradients FP32.
                          An approximation: its error against FP32 is measured, not bounded. */
  GSR_FP16_BLEND_T = 2 /* as GSR_FP16_BLEND, and the forward's transmittance T is also kept in
                          FP16 (T (1 - alpha) one FP16 fused multiply-add, the 1e-4 stop tested
                          on that FP16 value, the blend weight alpha T formed in FP16): Sec. 3.1.2 keeps
                          G, T and c in half precision; colour accumulates in FP32 here. The
                          backward is that of GSR_FP16_BLEND, starting from the FP16 final T.
                          An approximation whose error is measured, not bounded. */
} gsr_precision;

#define GSR_TILE 16          /* default render tile edge in pixels: one wave64 per 16x16 tile, or
                                per 16x4 band of a tile with a long list (other shapes of 256
                                pixels: gsr_options.tile_width); at most 2^28 tiles per call */
#define GSR_CLUSTER 128      /* primitives per cluster (Sec. 3.2.2) */
#define GSR_MAX_VIEWS 64     /* views per gsr_forward / gsr_backward call, and per gsr_raster_batch */
#define GSR_MAX_BATCH 16     /* prepared frames per gsr_raster_batch call */

typedef struct gsr_context gsr_context;

/* The scene G = {g_i} of Sec. 3: per Gaussian a mean, a covariance given as
 * log-scales and a rotation quaternion, an opacity logit and SH colour
 * coefficients. Structure of arrays, FP32, contiguous, device memory:
 *   means [n,3] world; log_scales [n,3], Sigma = R diag(exp(2 s)) R^T;
 *   quats [n,4] as (w, x, y, z), any non-zero norm (normalised inside);
 *   opacity_logits [n], o = 1/(1 + exp(-l));
 *   sh [n,K,3], K = (sh_degree+1)^2, real orthonormal SH without the
 *   Condon-Shortley phase, colour = max(0, sum_k Y_k(dir) f_k + 1/2). */
typedef struct {
  int64_t n;
  int32_t sh_degree; /* 0..3 */
  const float *means;
  const float *log_scales;
  const float *quats;
  const float *opacity_logits;
  const float *sh;
} gsr_scene;

/* A pinhole view pi_j (HOST memory). x_cam = R x_world + t with x right, y down,
 * z forward; pixel (px, py) has its centre at (px + 1/2, py + 1/2) and a point
 * projects to u = fx x/z + cx, v = fy y/z + cy. Gaussians with z <= near_plane
 * are dropped. bg is composited behind the last blended Gaussian. */
typedef struct {
  int32_t width, height;
  float fx, fy, cx, cy;
  float R[9]; /* row-major */
  float t[3];
  float near_plane;
  float bg[3];
} gsr_camera;

typedef struct {
  int32_t precision;    /* gsr_precision */
  int32_t cluster_cull; /* 1: cull clusters of GSR_CLUSTER consecutive Gaussians against the
                           frusta and compact the visible ones (Sec. 3.2.2); 0: keep all */
  int32_t stats;        /* 1: gsr_backward accumulates the statistic into gsr_stats */
  int32_t deterministic; /* 1: the backward adds the per-tile gradient sums (App. A.1's
                           f_global) as 64-bit fixed-point integers instead of FP32
                           atomics (the integer reduction of Sec. 3.1.2, carried to the
                           device-wide sum, with one exponent shared by all tiles), so
                           gradients and statistic are bitwise reproducible whatever
                           the order in which tiles finish (for one raster schedule,
                           see gsr_set_raster_split). With 2^E the power of two just
                           above max |dL/dI| over the frame (E clamped to [-44, 44]),
                           each per-tile sum is rounded to a multiple of 2^(E-32)
                           (the statistic's square sum: 2^(2E-32)) and saturates at
                           2^31 times that power. The workspace grows by 96 B per
                           record; forward and backward must agree. 0: FP32 atomics. */
  int32_t radius_mode;  /* tile membership of a Gaussian (App. A.1 tile culling leaves out
                           tiles where it has decayed to almost nothing): 0 (default) the
                           tiles of the pixel-centre box of its alpha >= 1/255 ellipse, so
                           tiling is exact; 1 the tiles of the pixel-centre box of the square
                           of half width ceil(3 sqrt(lambda_max)), lambda_max the larger
                           eigenvalue of the screen covariance (the 3-sigma bound, which cuts
                           through the alpha >= 1/255 set of opaque Gaussians: a pixel blends
                           a Gaussian only if its tile is in the rect). */
  int32_t half_reduction; /* 1: the backward packs each pixel strip's colour and opacity
                           gradient sums as FP16 pairs (Sec. 3.1.2: half2 to move more
                           gradient data per reduction step), reduces them over the wave
                           in packed FP16 and adds them across tiles with packed FP16
                           atomics; the geometry gradients and the statistic's square
                           sum stay FP32. An approximation whose error is reported, not
                           bounded; not with deterministic = 1. 0: all FP32. */
  int32_t tile_width;   /* tile shape (Sec. 3.1: tile shape and pixels per thread are
                           parameters of the raster): the width in pixels of a tile of
                           256 pixels, 4, 8, 16, 32 or 64 (height 256 / width: 4x64,
                           8x32, 16x16, 32x8, 64x4); 0 selects 16 (16x16, GSR_TILE). One
                           wave64 walks a tile's list with 4 pixels per lane: lane l owns
                           column l mod width and rows r + S j, j = 0..3, S = min(4,
                           height / 4), r = l / width, or in tiles taller than 16 rows
                           16 (r / 4) + r mod 4. Forward and backward must agree. */
} gsr_options;

/* Parameter gradients, device memory, the shapes of gsr_scene's arrays. Overwritten
 * by gsr_backward (0 for Gaussians that no view sees). */
typedef struct {
  float *means;
  float *log_scales;
  float *quats;
  float *opacity_logits;
  float *sh;
} gsr_grads;

/* Opacity-gradient statistic of Sec. 3.3, device memory, [n] each, ACCUMULATED (+=)
 * by gsr_backward over every (view, pixel) fragment in which the Gaussian is
 * blended: S = sum (dL/do)^2, M = sum dL/do (o the activated opacity), C = count.
 * The caller zeroes them at the start of a densification interval. */
typedef struct {
  float *S;
  float *M;
  uint32_t *C;
} gsr_stats;

/* Counters of the last forward on a workspace (host copy, see gsr_frame_inspect). */
typedef struct {
  int64_t n;               /* Gaussians in the scene */
  int64_t n_visible_slots; /* compact slots = 128 x visible clusters (all when culling is off) */
  int64_t instances;       /* (tile, Gaussian) pairs M */
  int64_t tiles;           /* tiles over all views */
  int64_t pixels;          /* pixels over all views */
  int32_t views;
  int32_t clusters;
  int32_t visible_clusters;
  int32_t split_tiles;     /* tiles the forward rasters as four 16x4 band items (the longest lists) */
  int32_t split_tiles_bwd; /* tiles the backward walks as two items of two bands each */
  int32_t reserved;
} gsr_frame_info;

/* Device pointers into a workspace after gsr_forward, for inspection and tests.
 * Records are indexed r = slot * views + view, slot = compact position.
 *   record      f32[R][12] : u_hi, v_hi, u_lo, v_lo, k1, r, k2, quad4, o, red, green, blue
 *                (screen mean as a float-float pair; exponent in log2 units
 *                 E2 = k1 (dx + r dy)^2 + k2 dy^2, quad4 = a quarter of E2's
 *                 coefficient of j^2)
 *   depth_key   u32[R]     : FP32 bits of the camera-space depth (0xffffffff: invalid)
 *   tiles       u32[R]     : tiles touched
 *   rect        u16[R][4]  : tile rect x0, x1, y0, y1 (inclusive)
 *   compact2full u32[slots]: full Gaussian index of each compact slot (0xffffffff: none)
 *   inst_tile   u32[M], inst_record u32[M]: instances sorted by (tile, depth, record)
 *   ranges      u32[tiles][2]: [start, end) of each tile's instances
 *   pixel_T     f32[pixels] (final transmittance), pixel_last u32[pixels]
 *                 (list position + 1 of the last blended instance)
 *   grad2d      f32[R][12] (after gsr_backward): d/du, d/dv, d/da, d/db, d/dc, d/do,
 *                 d/dred, d/dgreen, d/dblue, S, C, 0 of each record
 *   cluster_bounds f32[clusters][8] : min xyz, max xyz, max log-scale, 0
 *   cluster_visible u32[clusters]
 *   fwd_items   u32[tiles + 3 split_tiles], bwd_items u32[tiles + split_tiles_bwd]:
 *                 the raster schedules, one work item per entry, (global tile << 3) |
 *                 code with code 4 the whole tile, 0..3 a 16x4 band of a tile split
 *                 four ways, 5 and 6 the two halves of a tile split two ways; split
 *                 tiles first, each group in non-increasing list length */
typedef struct {
  const float *record;
  const uint32_t *depth_key;
  const uint32_t *tiles;
  const uint16_t *rect;
  const uint32_t *compact2full;
  const uint32_t *inst_tile;
  const uint32_t *inst_record;
  const uint32_t *ranges;
  const float *pixel_T;
  const uint32_t *pixel_last;
  const float *grad2d;
  const float *cluster_bounds;
  const uint32_t *cluster_visible;
  int64_t pixel_base[GSR_MAX_VIEWS]; /* first pixel of each view in the pixel arrays */
  int64_t tile_base[GSR_MAX_VIEWS];  /* first global tile id of each view */
  const uint32_t *fwd_items;
  const uint32_t *bwd_items;
} gsr_frame_buffers;

/* Context on HIP device `device`. Returns GSR_ERR_DEVICE if the device cannot be used. */
gsr_status gsr_context_create(int device, gsr_context **out);
void gsr_context_destroy(gsr_context *ctx);
/* Message of the last non-OK status on this context (never NULL). */
const char *gsr_last_error(const gsr_context *ctx);
/* Bytes that the last GSR_ERR_WORKSPACE_TOO_SMALL asked for. */
size_t gsr_required_workspace(const gsr_context *ctx);

/* Workspace bytes for one frame of V views whose instance count M is at most
 * max_instances (< 2^30). Needs no device (ctx may be NULL) and validates its
 * arguments exactly as gsr_forward does. M depends on the scene and is known only
 * on the device after projection: a frame whose M exceeds the workspace's capacity
 * drops the excess instances, and gsr_frame_inspect then reports
 * GSR_ERR_WORKSPACE_TOO_SMALL with the bytes that M needs. */
gsr_status gsr_workspace_size(gsr_context *ctx, const gsr_scene *scene, const gsr_camera *cams, int32_t V,
                              const gsr_options *opts, int64_t max_instances, size_t *bytes);

/* Forward render of V views (Sec. 3, Eq. (1)): images[v] is a device pointer to
 * f32 [3, height_v, width_v] (planar RGB), overwritten. The workspace keeps the
 * frame state that gsr_backward needs; do not reuse it for another frame in
 * between. Asynchronous: GSR_ERR_WORKSPACE_TOO_SMALL here means the workspace cannot
 * hold even an empty frame; whether the frame's instances fitted is known from
 * gsr_frame_inspect (if not, the images and a following backward miss the dropped
 * instances: grow the workspace and render again). At most n x V < 2^30 records. */
gsr_status gsr_forward(gsr_context *ctx, const gsr_scene *scene, const gsr_camera *cams, int32_t V,
                       const gsr_options *opts, void *workspace, size_t ws_bytes, float *const *images,
                       void *stream);

/* Every stage of gsr_forward before the raster (cluster cull and compaction of
 * Sec. 3.2, projection, depth sort, binning, tile sort, tile ranges and the raster
 * schedule), enqueued on `stream` with no host wait. Same arguments, validation
 * and errors as gsr_forward, without images. The frame is then rendered by
 * gsr_raster_batch, alone or together with other prepared frames. */
gsr_status gsr_prepare(gsr_context *ctx, const gsr_scene *scene, const gsr_camera *cams, int32_t V,
                       const gsr_options *opts, void *workspace, size_t ws_bytes, void *stream);

/* Bytes of the batch workspace that gsr_raster_batch needs for these prepared
 * frames: the raster work items (4 bytes each; a tile is one item, or four when
 * its list is split into bands, at most one tile in four), rounded up to 256,
 * plus 256 bytes for their count. */
gsr_status gsr_raster_batch_workspace_size(gsr_context *ctx, int32_t n, const void *const *workspaces,
                                           size_t *bytes);

/* One forward-raster launch (Sec. 3, Eq. (1)) over all tiles of n prepared frames
 * (1 <= n <= GSR_MAX_BATCH, distinct workspaces; any scenes and image sizes; at
 * most GSR_MAX_VIEWS views in total, at most 2^28 tiles), scheduled longest tile list first across the
 * frames. images[i][v] is
 * frame i's view v: a device pointer to f32 [3, H, W], overwritten. The frames'
 * gsr_prepare work must be complete or enqueued earlier on `stream` (make `stream`
 * wait for the streams that prepared them). A frame's images are bitwise equal to
 * rendering it alone: tiles are independent and the forward has no atomics.
 * batch_ws: device memory, 256-byte aligned, at least
 * gsr_raster_batch_workspace_size bytes, overwritten (GSR_ERR_WORKSPACE_TOO_SMALL
 * otherwise). Each frame can then be inspected, and differentiated by
 * gsr_backward with the same precision. */
gsr_status gsr_raster_batch(gsr_context *ctx, int32_t n, const void *const *workspaces, float *const *const *images,
                            int32_t precision, void *batch_ws, size_t batch_ws_bytes, void *stream);

/* gsr_raster_batch for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the same
 * launch, with the work-item list in a device-resident scratch array of the library
 * instead of a batch workspace, so the call allocates nothing (the frames' own
 * workspaces, prepared by gsr_prepare, and the images are still the caller's).
 * The scratch holds the items of at most GSR_NOALLOC_MAX_TILES tiles over all n
 * frames (1.8 MB per GPU, held until the process ends); a larger batch returns
 * GSR_ERR_INVALID_ARG before any launch. Every call on one GPU shares that GPU's
 * scratch and leaves its contents there: calls that overlap on one GPU (on
 * different streams, unordered) race and must not be issued. Everything else is
 * as gsr_raster_batch, whose images it reproduces bit for bit. */
#define GSR_NOALLOC_MAX_TILES 262144
gsr_status gsr_raster_batch_noalloc(gsr_context *ctx, int32_t n, const void *const *workspaces,
                                    float *const *const *images, int32_t precision, void *stream);

/* Backward of the last gsr_forward on `workspace` with the same scene, cameras and
 * options (Sec. 3, Eq. (3); App. A.1-A.2). dL_dimages[v] is a device pointer to
 * f32 [3, height_v, width_v]. grads are overwritten; stats (nullable; used when
 * opts->stats = 1) are accumulated. opts->precision must be the forward's. Fully
 * asynchronous. */
gsr_status gsr_backward(gsr_context *ctx, const gsr_scene *scene, const gsr_camera *cams, int32_t V,
                        const gsr_options *opts, void *workspace, size_t ws_bytes,
                        const float *const *dL_dimages, const gsr_grads *grads, const gsr_stats *stats,
                        void *stream);

/* Counters and buffer pointers of the last gsr_forward on `workspace` (info and
 * bufs nullable). Waits until the forward's counters have reached the host.
 * Returns GSR_ERR_WORKSPACE_TOO_SMALL (gsr_required_workspace() = the bytes the
 * frame needs; info still filled, info->instances = the full M) when the frame's
 * instances exceeded the workspace, GSR_ERR_UNSUPPORTED when M reached 2^30, and
 * GSR_ERR_DEVICE if a device-wide wait inside the frame gave up. */
gsr_status gsr_frame_inspect(gsr_context *ctx, const void *workspace, gsr_frame_info *info,
                             gsr_frame_buffers *bufs);

/* Forgets the frame state kept for `workspace` (waits for its forward to finish);
 * call before freeing a workspace whose address may be reused. No-op if none. */
gsr_status gsr_frame_release(gsr_context *ctx, const void *workspace);

/* Densification metric of Sec. 3.3, C * Var = S - M^2 / C (0 where C = 0),
 * evaluated in FP64: out[n] f32, device memory. */
gsr_status gsr_variance(gsr_context *ctx, const gsr_stats *stats, int64_t n, float *out, void *stream);

/* Workspace bytes for gsr_morton_order on n Gaussians (ctx may be NULL). */
gsr_status gsr_morton_workspace_size(gsr_context *ctx, int64_t n, size_t *bytes);

/* Morton order (Sec. 3.2.1): per-axis min/max normalisation of means [n,3] to the
 * unit cube, scaling by 2^21 - 1 with truncation, and interleaving bit k of x, y, z
 * into bits 3k, 3k+1, 3k+2 of a 63-bit code (FP64 arithmetic on the FP32 means:
 * q = trunc(clamp((p - lo)/(hi - lo), 0, 1) * 2097151), 0 on a degenerate axis).
 * perm [n] (i64, device) receives the indices stably sorted by code; codes [n]
 * (u64, device, nullable) the codes in the original order. */
gsr_status gsr_morton_order(gsr_context *ctx, const float *means, int64_t n, void *workspace, size_t ws_bytes,
                            int64_t *perm, uint64_t *codes, void *stream);

/* Workspace bytes for gsr_sort_u32 on n keys of `bits` bits (ctx may be NULL). */
gsr_status gsr_sort_workspace_size(gsr_context *ctx, int64_t n, int32_t bits, size_t *bytes);

/* Stable LSD radix sort of n (< 2^30) 32-bit keys on their low `bits` bits (1..32),
 * 8 bits per one-sweep pass: the sort that orders the records by depth and the
 * instances by tile (App. A.1's binning, in the sorted order Eq. (1) composites).
 * keys [n] (device, each below 2^bits: the passes take whole bytes, so bits above
 * are not ignored) and vals [n] (device; NULL: the values are the positions
 * 0..n-1) are read only; out_keys [n], out_vals [n] (device) receive the keys in
 * ascending order, equal ones in input order, and their values;
 * outputs must not overlap the inputs or each other. Pointers need 4-byte
 * alignment only. workspace: gsr_sort_workspace_size bytes, 256-byte aligned. The
 * call does not wait: the first 32-bit word of the workspace is nonzero once the
 * stream has passed the sort if a device-wide wait gave up (the output is then
 * incomplete); it is zero otherwise. */
gsr_status gsr_sort_u32(gsr_context *ctx, const uint32_t *keys, const uint32_t *vals, int64_t n, int32_t bits,
                        uint32_t *out_keys, uint32_t *out_vals, void *workspace, size_t ws_bytes, void *stream);

/* Gathers rows: dst[a][i, :] = src[a][perm[i], :] for n_arrays arrays of n rows of
 * row_floats[a] floats (device memory; dst and src must not overlap). Applies a
 * Morton order to the parameters and to any optimiser state. */
gsr_status gsr_apply_permutation(gsr_context *ctx, const int64_t *perm, int64_t n, int32_t n_arrays,
                                 const float *const *src, float *const *dst, const int32_t *row_floats,
                                 void *stream);

/* Gradient of the weighted L1 loss L = sum w |I - gt| (the loss of the training
 * step the paper accelerates; the rasterizer itself only sees dL/dI):
 * out[i] = w[i] * sign(image[i] - gt[i]) over `count` floats, device memory. */
gsr_status gsr_l1_grad(gsr_context *ctx, const float *image, const float *w, const float *gt, int64_t count,
                       float *out, void *stream);

/* Rates and constants of one Adam step (Kingma and Ba, Algorithm 1). The paper
 * does not give the rates; 3DGS trains with rates of the order of 1.6e-4 (means),
 * 5e-3 (log-scales), 1e-3 (quaternions), 2.5e-2 (opacity), 2.5e-3 (SH degree 0)
 * and 1.25e-4 (higher SH), betas 0.9 / 0.999 and eps 1e-15. */
typedef struct {
  float lr_means;
  float lr_log_scales;
  float lr_quats;
  float lr_opacity;
  float lr_sh_dc;    /* the first 3 floats of each SH row: the degree-0 coefficient of each colour */
  float lr_sh_rest;  /* the other floats of each SH row */
  float beta1;       /* in [0, 1) */
  float beta2;       /* in [0, 1) */
  float eps;         /* >= 0, added to sqrt(v / (1 - beta2^t)) */
  int32_t reserved;  /* must be 0 */
  int64_t step;      /* t >= 1: this update's number, counted over all updates; both bias
                        corrections use it, for a cluster skipped before as for any other */
} gsr_adam_options;

/* One Adam step at cluster granularity (Sec. 3.2.3): the sparse update of the
 * visible primitives is applied to whole clusters of GSR_CLUSTER consecutive
 * Gaussians, which keeps every read and write of the update on contiguous
 * memory. For every Gaussian i of a cluster c with cluster_visible[c] != 0 and
 * every float x of its parameters, with g its gradient and m, v its moments:
 *   m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
 *   x = x - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps)
 * (FP32; the bias corrections are formed in FP64 once per call). Parameters and
 * both moments of every other cluster are left untouched: they keep their values
 * bit for bit and do not decay.
 *   n, sh_degree: as in gsr_scene; params, exp_avg, exp_avg_sq: the parameters and
 *     the first and second moments, device arrays with gsr_scene's shapes, updated
 *     in place (gsr_grads serves as the holder of five such arrays); grads: the
 *     gradients in the same shapes, read only (gsr_backward's output).
 *   cluster_visible: device u32[ceil(n / GSR_CLUSTER)], nonzero = update the
 *     cluster, e.g. gsr_frame_buffers.cluster_visible of the frame that produced
 *     grads (the clusters its cull kept in any of its views); NULL updates all
 *     (dense Adam).
 * Every array must be 16-byte aligned and no two of the twenty may overlap
 * (GSR_ERR_INVALID_ARG otherwise, as for a null array with n > 0, a degree
 * outside 0..3, step < 1, a beta outside [0, 1) or eps < 0). Asynchronous on
 * `stream`; n = 0 enqueues nothing. */
gsr_status gsr_sparse_adam(gsr_context *ctx, int64_t n, int32_t sh_degree, const uint32_t *cluster_visible,
                           const gsr_grads *params, const gsr_grads *grads, const gsr_grads *exp_avg,
                           const gsr_grads *exp_avg_sq, const gsr_adam_options *opts, void *stream);

/* gsr_backward and gsr_sparse_adam over the frame's kept clusters in one pass (the
 * fused update of Sec. 3.2.3): the projection backward applies the Adam step of
 * gsr_sparse_adam to each Gaussian of a cluster the forward's cull kept, with the
 * gradient it has just computed, and no gradient array is written or read; culled
 * clusters are not touched at all. The scene's arrays are the parameters and are
 * updated IN PLACE (they must be writable device memory; the forward that made the
 * frame read them before the update); exp_avg / exp_avg_sq are the moments, in
 * place. Same arguments and checks as gsr_backward (without grads) and
 * gsr_sparse_adam (with cluster_visible = the frame's flags); stats are accumulated
 * as by gsr_backward. Given the same gradients (a deterministic frame, where the
 * backward's sums do not depend on the order of atomics), the result equals
 * gsr_backward followed by gsr_sparse_adam on the frame's cluster_visible, bit for
 * bit: both apply the same per-float update. */
gsr_status gsr_backward_adam(gsr_context *ctx, const gsr_scene *scene, const gsr_camera *cams, int32_t V,
                             const gsr_options *opts, void *workspace, size_t ws_bytes,
                             const float *const *dL_dimages, const gsr_grads *exp_avg, const gsr_grads *exp_avg_sq,
                             const gsr_adam_options *adam_opts, const gsr_stats *stats, void *stream);

/* Densification of Sec. 3.3: the Gaussians whose opacity-gradient variance metric
 * (gsr_variance's C Var) is largest are split or cloned. The paper fixes the
 * metric only; the thresholds and the split geometry follow the densification of
 * 3DGS that it modifies and are arguments:
 *   candidates: metric >= threshold, the max_candidates largest (ties: lower index
 *     first), compared as the FP32 values given;
 *   a candidate whose largest log-scale exceeds split_log_scale is split into two
 *     children at mean + R(q) (exp(s) * z_c), c = 0, 1, with z_c = noise[i][c][0..2]
 *     (standard normal draws the caller supplies), log-scales s - ln(split_factor)
 *     and the parent's quaternion, opacity and SH; the parent leaves. Any other
 *     candidate is cloned: an exact copy is appended and the original stays;
 *   an original whose opacity logit is below prune_logit leaves (-INFINITY: none).
 * Output rows: the kept originals in index order, then per candidate, largest metric
 * first, its clone or its two children (child 0 first). Means and log-scales of
 * children are computed in FP64 and rounded once. */
typedef struct {
  float threshold;         /* > 0 */
  float split_log_scale;
  float split_factor;      /* > 0 (3DGS divides the scales by 1.6) */
  float prune_logit;
  int64_t max_candidates;  /* >= 0; values above n mean n */
} gsr_densify_options;

/* Workspace bytes for gsr_densify on n Gaussians (ctx may be NULL). */
gsr_status gsr_densify_workspace_size(gsr_context *ctx, int64_t n, int64_t max_candidates, size_t *bytes);

/* One densification (see gsr_densify_options), out of place and asynchronous.
 *   scene: the n input Gaussians (device arrays, read only); metric: f32[n] device;
 *   noise: f32[n][2][3] device (rows of Gaussians that are not split are not read).
 *   out: device arrays of `capacity` rows with gsr_scene's shapes; capacity >= n +
 *     min(max_candidates, n), the largest possible output.
 *   State arrays (e.g. optimiser moments): n_state arrays of row_floats[a] floats per
 *     Gaussian; a kept original's row moves with it, new rows are zero.
 *   workspace: device, 256-byte aligned, gsr_densify_workspace_size bytes.
 *   n_out: device int64 (nullable): receives the output row count, or -1 if a
 *     device-wide wait gave up (the output is then not valid).
 * Inputs and outputs must not overlap (GSR_ERR_INVALID_ARG, as for bad sizes, null
 * arrays, n >= 2^30, more than 16 state arrays or bad options). Re-sorting the
 * output by Morton code afterwards (Sec. 3.2.1 re-sorts after every densification)
 * is gsr_morton_order + gsr_apply_permutation on the n_out rows. */
gsr_status gsr_densify(gsr_context *ctx, const gsr_scene *scene, const float *metric, const float *noise,
                       const gsr_densify_options *opts, const gsr_grads *out, int64_t capacity, int32_t n_state,
                       const float *const *state_in, float *const *state_out, const int32_t *state_row_floats,
                       void *workspace, size_t ws_bytes, int64_t *n_out, void *stream);

/* Opacity decay of Sec. 3.3, the gentler replacement of the opacity reset: each
 * activated opacity o = sigmoid(l) becomes factor * o (the paper halves it), stored
 * back as a logit, in FP64: l = ln(o') - ln(1 - o'). 0 < factor < 1. In place on
 * opacity_logits[n] (device), asynchronous. */
gsr_status gsr_opacity_decay(gsr_context *ctx, float *opacity_logits, int64_t n, float factor, void *stream);

/* Raster schedule of the frames this context prepares from now on (Sec. 3.1 fixes one
 * tile shape; this sets which tiles run in a second one). A work item is normally a
 * whole 16x16 tile, 4 pixels per lane. The forward rasters a tile whose list is
 * longer than split_len entries as four 16x4 band items (1 pixel per lane); the
 * backward walks a tile longer than split_len_bwd as two halves (2 pixels per
 * lane). Longest lists first, at most one tile in four. 0 restores a default (256,
 * 512); UINT32_MAX never splits. Images do not depend on it (a band evaluates its
 * pixels exactly as the whole tile does); gradients only through rounding (a tile
 * walked as two halves adds two per-item sums instead of one). */
gsr_status gsr_set_raster_split(gsr_context *ctx, uint32_t split_len, uint32_t split_len_bwd);

/* Failure injection for tests of the error path (no caller needs it otherwise).
 * The frames this context prepares from now on:
 *   GSR_FAULT_NONE             render normally (the default);
 *   GSR_FAULT_ABORT_BEFORE_SORT raise the abort bit of the frame's error word right
 *                              before the depth sort;
 *   GSR_FAULT_WITHHOLD_STATUS  in the first pass of the tile sort, the block of tile 1
 *                              never publishes its look-back status, so every later
 *                              tile's wait can only end by its time bound (100 ms).
 * Every kernel still exits normally: device-wide waits are bounded by elapsed time,
 * the first one to run out raises the abort bit, every other wait and every later
 * kernel of the frame reads it and leaves, and gsr_frame_inspect then returns
 * GSR_ERR_DEVICE. The next frame prepared on the workspace starts with a clear
 * error word. Returns GSR_ERR_INVALID_ARG for an unknown mode. */
typedef enum {
  GSR_FAULT_NONE = 0,
  GSR_FAULT_ABORT_BEFORE_SORT = 1,
  GSR_FAULT_WITHHOLD_STATUS = 2
} gsr_fault;
gsr_status gsr_set_fault_injection(gsr_context *ctx, int32_t mode);

/* Stages of gsr_forward and gsr_backward, in launch order. */
typedef enum {
  GSR_STAGE_CLUSTER = 0,     /* cluster bounds, frustum cull, compaction list */
  GSR_STAGE_PREPROCESS,      /* projection to screen-space records */
  GSR_STAGE_DEPTH_SORT,      /* stable radix sort of the records by depth */
  GSR_STAGE_OFFSETS,         /* tiles touched in depth order and their prefix sum */
  GSR_STAGE_EMIT,            /* one instance per (record, covered tile) */
  GSR_STAGE_TILE_SORT,       /* stable radix sort of the instances by tile */
  GSR_STAGE_RANGES,          /* per-tile [start, end) */
  GSR_STAGE_RASTER_FWD,      /* alpha compositing */
  GSR_STAGE_ZERO_GRAD,       /* clear the screen-space gradient rows */
  GSR_STAGE_RASTER_BWD,      /* backward compositing with the statistic */
  GSR_STAGE_PREPROCESS_BWD,  /* chain to the parameter gradients */
  GSR_STAGE_COUNT
} gsr_stage;

/* With profiling on, gsr_forward and gsr_backward record a HIP event pair around
 * each stage on the caller's stream (no extra synchronisation). */
gsr_status gsr_set_profiling(gsr_context *ctx, int enable);
/* Milliseconds of each stage of the last profiled gsr_forward / gsr_backward
 * (ms[GSR_STAGE_COUNT]; -1 for a stage that has not run). Waits for the events. */
gsr_status gsr_stage_times(gsr_context *ctx, float *ms);

#ifdef __cplusplus
}
#endif

#endif /* GSR_H */
