// Internal declarations shared by the HIP sources of libgsr (not part of the ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gsr.h"

namespace gsr {

// Launches `kernel` on stream s. A non-null `done` event completes with the kernel
// itself (its completion signal), instead of through a marker enqueued after it:
// a marker makes the next launch in the stream wait for an extra round trip.
// The launchers that take an event return whether a kernel carried it (false
// when there was nothing to launch; the caller then records the event itself).
template <typename K, typename... Args>
inline void launch_tracked(K kernel, unsigned grid, unsigned block, hipStream_t s, hipEvent_t done, Args... args) {
  if (done)
    hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, s, nullptr, done, 0, args...);
  else
    kernel<<<grid, block, 0, s>>>(args...);
}

// Thresholds of the compositing rule (Sec. 3, Eq. (1) with the alpha skip, clamp
// and transmittance stop that the rasterizer applies).
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;
constexpr double kDilation = 0.3;   // screen-space low-pass, px^2
constexpr double kFovClamp = 1.3;   // EWA Jacobian evaluated within 1.3 x the half field of view
constexpr double kLog2e = 1.4426950408889634;
constexpr double kLn2 = 0.6931471805599453;

// Per-view constants, stored in the workspace (device memory).
struct ViewDev {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  float near_plane;
  float bg[3];
  double limx, limy;      // Jacobian clamp limits on x/z and y/z
  double campos[3];       // camera centre -R^T t
  int32_t width, height;
  int32_t tiles_x, tiles_y;
  int32_t tile_base;      // first global tile id of the view
  int32_t tile_wl;        // log2 of the tile width in pixels (tile height 256 >> tile_wl)
  int64_t pixel_base;     // first pixel of the view in the per-pixel arrays
};

// Screen-space record of one (Gaussian, view), 48 bytes = 3 x float4:
//   r0 = {u_hi, v_hi, u_lo, v_lo}    screen mean as a float-float pair
//   r1 = {k1, r, k2, quad}           exponent in log2 units:
//                                      E2(dx, dy) = k1 (dx + r dy)^2 + k2 dy^2,
//                                      quad = coefficient of j^2 along a column
//   r2 = {o, red, green, blue}
struct alignas(16) Record {
  float4 r0, r1, r2;
};

// Per-record screen-space gradient accumulated by the backward raster (12 floats):
// d/du, d/dv, d/da, d/db, d/dc, d/do, d/dred, d/dgreen, d/dblue, S, count, 0, where
// (a, b, c) is the conic of E = -1/2 (a dx^2 + 2 b dx dy + c dy^2) in natural units.
constexpr int kGrad2D = 12;

// Header words of a frame (device memory, cleared at the start of each forward).
enum HeaderWord {
  kHdrVisibleClusters = 0,  // clusters that survived the cull
  kHdrInstances = 1,        // (tile, record) pairs M of the frame
  kHdrInstancesKept = 2,    // min(M, capacity): what the tile sort and raster use
  kHdrRecords = 3,          // active records = 128 * visible clusters * views
  kHdrOverflow = 4,         // 1 when M exceeded the workspace capacity
  kHdrError = 5,            // bit 0: abort (a device-wide wait ran out of time, or the host raised it);
                            // bit 1: a scanned count reached 2^30
  kHdrItems = 6,            // forward raster work items (whole tiles plus the bands of split tiles)
  kHdrItemsBwd = 7,         // backward raster work items
  kHdrGradMax = 8,          // deterministic backward: max |dL/dI| over the frame's views (FP32 bits)
};

// Fixed-point scale of the deterministic backward. A per-tile gradient sum is
// rounded to a multiple of 2^(E - 32), E the binary exponent of max |dL/dI| over
// the frame (max |dL/dI| < 2^E), and the statistic's square sum to a multiple of
// 2^(2E - 32): the sums keep 32 bits below the size of the upstream gradient
// whatever the scale of the loss, and saturate at 2^31 times it. E is clamped to
// [-44, 44] so that both scales stay finite in FP32.
constexpr int kFixedBits = 32;
__device__ __forceinline__ int grad_exponent(const uint32_t* header) {
  const float m = __uint_as_float(header[kHdrGradMax]);
  int e = 0;
  if (m > 0.0f) (void)frexpf(m, &e);
  return e < -44 ? -44 : (e > 44 ? 44 : e);
}

// Error bits of the header's error word. Any set bit makes every later kernel of
// the frame leave at once (frame_aborted): the scans and sorts it would read may
// be incomplete, and indices read from them could point anywhere.
constexpr uint32_t kErrAbort = 1u;
constexpr uint32_t kErrCount = 2u;

// The word is written by earlier kernels of the stream, or by blocks of a running
// look-back kernel (which broadcast their own reading through LDS, since waves may
// read it at different times): read once per wave into a scalar register.
__device__ __forceinline__ bool error_raised(const uint32_t* err) {
  return __builtin_amdgcn_readfirstlane(__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0u;
}
__device__ __forceinline__ bool frame_aborted(const uint32_t* header) { return error_raised(header + kHdrError); }

// Default list lengths above which the raster splits a tile into band items
// (forward: four 16x4 bands; backward: two halves).
constexpr uint32_t kSplitLen = 256;
constexpr uint32_t kSplitLenBwd = 512;

struct Frame {
  // sizes (host)
  int64_t n, ncap, nrec;    // Gaussians, compact slots (128 * clusters), records = ncap * V
  int32_t V, nclusters;
  int64_t tiles, pixels, inst_cap;
  int32_t tile_bits;
  int32_t tile_wl;          // log2 of the tile width (gsr_options.tile_width)
  // device pointers (all inside the workspace)
  uint32_t* header;         // HeaderWord entries
  ViewDev* views;
  float* cluster_bounds;    // [nclusters][8]
  uint32_t* cluster_visible;
  uint32_t* cluster_offset; // exclusive scan of visible
  uint32_t* cluster_list;   // compact cluster -> cluster
  uint32_t* compact2full;   // [ncap]
  Record* rec;              // [nrec]
  uint32_t* dkey;           // [nrec]
  uint32_t* tiles_touched;  // [nrec]
  ushort4* rect;            // [nrec]
  uint32_t *skey[2], *sval[2];   // depth sort buffers [nrec]
  uint32_t* offsets;        // [nrec]
  uint32_t *ikey[2], *ival[2];   // instance buffers [inst_cap]
  uint32_t* inst_tile;      // sorted instances (points into ikey/ival)
  uint32_t* inst_rec;
  uint32_t* inst_mask;      // per instance: byte b nonzero where the forward found a live pixel of band b
                            // with alpha >= 1/255 (the tile sort's spare value buffer)
  uint32_t* ranges;         // [tiles][2]
  uint32_t* tile_order;     // [max_items(tiles)] forward raster work items, longest lists first
  uint32_t* bwd_items;      // [max_items(tiles)] backward raster work items
  float* pix_T;             // [pixels]
  uint32_t* pix_last;       // [pixels]
  float* grad2d;            // [nrec][12]
  float* dmean;              // [ncap][3] mean gradient between the two projection-backward kernels (fused Adam)
  unsigned long long* grad2d_fx;  // [nrec][12] fixed-point sums (deterministic backward), else null
  uint32_t split_len = kSplitLen;         // forward: tiles with longer lists are rastered as four bands
  uint32_t split_len_bwd = kSplitLenBwd;  // backward: tiles with longer lists are walked as two halves
  int32_t radius_mode = 0;                // tile membership: 0 the alpha >= 1/255 box, 1 the 3-sigma square
  uint32_t* ctl;            // look-back / histogram control words, cleared with the header
  size_t ctl_words;
  uint32_t *ctl_cluster_scan, *ctl_depth_sort, *ctl_offsets_scan, *ctl_tile_sort;
  uint32_t* ctl_tile_order = nullptr;  // multi-block raster schedule of large frames (tile_order_ctl_words)
};

// ---------------------------------------------------------------- launchers
// fill.hip
void fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
void fill_f32(float* p, int64_t n, float v, hipStream_t s);

// onesweep.hip: single-pass scan and one-sweep radix sort, counts read from device
// memory (n_dev; n_max bounds the launch). Control words (ctl) must be zero on entry.
// Scan: out[i] = sum_{k<i} src[idx ? idx[k] : k]; total <- sum; list[out[i]] = i where
// the item is non-zero (list nullable).
size_t scan_ctl_words(int64_t n_max);
void scan_u32(const uint32_t* src, const uint32_t* idx, uint32_t* out, int64_t n_max, const uint32_t* n_dev,
              uint32_t* total, uint32_t* list, uint32_t* ctl, uint32_t* err, hipStream_t s);
// Stable LSD radix sort of (key, value) pairs on key bits [0, bits), 8 bits per pass.
// The input is read-only; passes alternate between (kb[0], vb[0]) and (kb[1], vb[1]).
// Returns the index of the pair holding the result, or -1 when no pass was needed
// (then the input is the result). vals_in == nullptr stands for 0..n-1. spatial:
// neighbouring keys tend to share their high bytes (the digit counting then adds
// runs of equal digits at once).
size_t sort_ctl_words(int64_t n_max, int bits);
// withhold >= 0 (tests of the error path only): the first pass's block of that tile
// never publishes its look-back status.
int radix_sort_u32_dev(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* kb[2], uint32_t* vb[2],
                       int64_t n_max, const uint32_t* n_dev, int bits, uint32_t* ctl, uint32_t* err, bool spatial,
                       hipStream_t s, int64_t withhold = -1);
// Raises the abort bit of an error word (tests of the error path).
void raise_abort(uint32_t* err, hipStream_t s);
int radix_sort_u64_dev(const uint64_t* keys_in, const uint32_t* vals_in, uint64_t* kb[2], uint32_t* vb[2],
                       int64_t n_max, const uint32_t* n_dev, int bits, uint32_t* ctl, uint32_t* err, bool spatial,
                       hipStream_t s);

// cluster.hip
constexpr int kViewChunk = 16;
struct ViewChunk {
  ViewDev v[kViewChunk];
};
static_assert(sizeof(ViewChunk) <= 3072, "a view chunk travels in the kernel arguments");
// Copies views [v0, v0 + nv) from the kernel arguments to `views`; the first chunk
// also clears `zero` (zero_words words: the frame header and control words).
void launch_frame_begin(const ViewChunk& chunk, int v0, int nv, ViewDev* views, uint32_t* zero, int64_t zero_words,
                        hipStream_t s);
// Per cluster: bounds (min/max of the means, largest log-scale) and, when cull is
// set, the frustum test against every view (else every cluster is visible).
// The frame start (views and cleared words, as launch_frame_begin) fused into the
// cluster kernel; false (nothing launched) for an empty scene or more than
// kViewChunk views, which take launch_frame_begin + launch_cluster.
bool launch_cluster_begin(const ViewChunk& chunk, int32_t V, ViewDev* views, uint32_t* zero, int64_t zero_words,
                          const float* means, const float* log_scales, int64_t n, int cull, float* bounds,
                          uint32_t* visible, hipStream_t s);
void launch_cluster(const float* means, const float* log_scales, int64_t n, int cull, const ViewDev* views, int32_t V,
                    float* bounds, uint32_t* visible, hipStream_t s);

// preprocess.hip
void launch_preprocess_fwd(const gsr_scene& sc, const Frame& f, hipStream_t s);
struct AdamDev;
// adam null: gradients into g. adam set: no gradient leaves the kernels; the
// Gaussians of kept clusters take the Adam step in place (adam's p, m, v arrays).
// half: the backward raster left the colour and opacity sums as FP16 pairs in slots 6
// and 7 of each gradient row (half_reduction).
void launch_preprocess_bwd(const gsr_scene& sc, const Frame& f, const gsr_grads& g, const gsr_stats* stats,
                           const AdamDev* adam, bool half, hipStream_t s);

// binning.hip (counts read from the frame header)
void launch_emit_instances(const Frame& f, const uint32_t* sorted_rec, hipStream_t s);
void launch_tile_ranges(const Frame& f, const uint32_t* inst_tile, int64_t M_max, hipStream_t s);
bool launch_tile_order(const Frame& f, hipStream_t s, hipEvent_t done);
// Control words the raster schedule of a frame of `tiles` tiles needs (zero when one
// block builds it); they must be zero on entry.
size_t tile_order_ctl_words(int64_t tiles);

// raster_fwd.hip / raster_bwd.hip
struct ImagePtrs {
  float* p[GSR_MAX_VIEWS];
};
struct ConstImagePtrs {
  const float* p[GSR_MAX_VIEWS];
};
bool launch_raster_fwd(const Frame& f, const ImagePtrs& images, int precision, hipStream_t s, hipEvent_t done);

// Batched forward raster over several prepared frames (kernel-argument table).
constexpr int kMaxBatch = GSR_MAX_BATCH;
struct FrameRef {
  const uint32_t* header;   // the frame's header (its error word: an aborted frame's tiles are skipped)
  const ViewDev* views;
  const uint32_t* ranges;
  const uint32_t* inst_rec;
  uint32_t* inst_mask;
  const Record* rec;
  float* pix_T;
  uint32_t* pix_last;
  int32_t V;
  int32_t img_base;  // first image pointer of the frame in the batch's ImagePtrs
};
struct FrameTable {
  FrameRef f[kMaxBatch];
  uint32_t first[kMaxBatch + 1];  // concatenated tile index of each frame's first tile
  int32_t n;
};
static_assert(sizeof(FrameTable) + sizeof(ImagePtrs) <= 3584, "the batch table travels in the kernel arguments");
bool launch_raster_fwd_batch(const FrameTable& tab, const uint32_t* order, const uint32_t* n_items,
                             uint32_t total_tiles, const ImagePtrs& images, int precision, hipStream_t s,
                             hipEvent_t done);
// noalloc.hip: the device-resident scratch of gsr_raster_batch_noalloc (work items
// of at most noalloc_max_tiles() tiles, then their count). noalloc_init(device)
// looks up the device's copy once (hipGetSymbolAddress with the device current);
// noalloc_scratch returns it (null before init) and its size in words.
int64_t noalloc_max_tiles();
hipError_t noalloc_init(int device);
uint32_t* noalloc_scratch(int device, size_t* words);
// Raster work items of the concatenated tiles of a batch of frames (n_items <- count).
void launch_batch_tile_order(const FrameTable& tab, uint32_t total_tiles, uint32_t split_len, uint32_t* order,
                             uint32_t* n_items, hipStream_t s);
// Largest number of raster work items for `tiles` tiles (every split tile adds 3).
int64_t raster_max_items(int64_t tiles);
void launch_raster_bwd(const Frame& f, const ConstImagePtrs& dL, int precision, bool half, hipStream_t s);
// Deterministic backward: header[kHdrGradMax] <- max |dL/dI| over the V images
// (count[v] floats each).
struct ViewCounts {
  int64_t n[GSR_MAX_VIEWS];
};
void launch_grad_absmax(const Frame& f, const ConstImagePtrs& dL, const ViewCounts& counts, hipStream_t s);

// morton.hip
size_t morton_temp_words(int64_t n);
bool morton_order(const float* means, int64_t n, uint32_t* temp, int64_t* perm, uint64_t* codes, hipStream_t s);
void launch_gather_rows(const int64_t* perm, int64_t n, const float* src, float* dst, int32_t row_floats,
                        hipStream_t s);

// variance and loss
void launch_variance(const float* S, const float* M, const uint32_t* C, int64_t n, float* out, hipStream_t s);
void launch_l1_grad(const float* image, const float* w, const float* gt, int64_t n, float* out, hipStream_t s);

// adam.hip: one Adam step over the Gaussians of visible clusters (Sec. 3.2.3).
constexpr int kAdamGroups = 5;  // means, log-scales, quaternions, opacity logits, SH
struct AdamGroupDev {
  float* p;
  const float* g;
  float* m;
  float* v;
  int32_t row;      // floats per Gaussian
  int32_t head;     // leading floats of a row that take step_head (row: all of them)
  float step_head;  // lr / (1 - beta1^t)
  float step_rest;
};
struct AdamDev {
  AdamGroupDev grp[kAdamGroups];
  int64_t n;
  int32_t units;  // float4 units of a full cluster over all groups: GSR_CLUSTER / 4 x sum of rows
  float beta1, beta2, c1, c2, eps;
  float inv_sqrt_bc2;  // 1 / sqrt(1 - beta2^t)
};
// Every pointer 16-byte aligned; visible u32[ceil(n / GSR_CLUSTER)] or null (all).
void launch_sparse_adam(const AdamDev& a, const uint32_t* visible, hipStream_t s);

// One float of an Adam step (Kingma and Ba, Algorithm 1), the bias corrections folded
// into step = lr / (1 - beta1^t) and inv_sqrt_bc2 = 1 / sqrt(1 - beta2^t):
//   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,  p -= step m / (sqrt(v) inv_sqrt_bc2 + eps).
// The separate kernel and the update fused into the projection backward share it, so
// both give the same bits.
__device__ __forceinline__ void adam_float(float& p, float g, float& m, float& v, float step, const AdamDev& a) {
  m = fmaf(a.beta1, m, a.c1 * g);
  v = fmaf(a.beta2, v, a.c2 * (g * g));
  const float den = fmaf(sqrtf(v), a.inv_sqrt_bc2, a.eps);
  p = p - step * (m / den);
}

// densify.hip: densification by the variance metric and opacity decay (Sec. 3.3).
constexpr int kMaxDensCopy = 3 + 16;  // quaternions, opacity logits, SH and up to 16 state arrays
struct DensifyArgs {
  int64_t n, max_candidates;  // max_candidates <= n
  const float *metric, *noise, *means, *log_scales, *quats, *opacity_logits;
  float threshold, split_log_scale, prune_logit;
  double ln_split_factor;
  float *out_means, *out_log_scales;
  int32_t n_copy;  // arrays written through the row map besides the means and log-scales
  const float* copy_in[kMaxDensCopy];
  float* copy_out[kMaxDensCopy];
  int32_t copy_rf[kMaxDensCopy];
  int32_t copy_zero_new[kMaxDensCopy];  // 1: state array (new rows are zero)
  int64_t* n_out;                       // device, nullable: output rows, -1 if a device wait gave up
};
size_t densify_words(int64_t n, int64_t max_candidates);
// n >= 1; ws: densify_words(n, max_candidates) words, 256-byte aligned.
void densify(const DensifyArgs& a, uint32_t* ws, hipStream_t s);
void launch_opacity_decay(float* logits, int64_t n, double factor, hipStream_t s);

}  // namespace gsr
