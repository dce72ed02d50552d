// Host runtime behind the C ABI of include/gsr.h: argument validation, the
// workspace plan, launch sequencing and the per-workspace frame registry.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "gsr_internal.h"

using gsr::Frame;
using gsr::ViewDev;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kHdrBytes = 256;

struct FrameRecord {
  Frame f;
  gsr_scene scene;                     // sizes of the forward's scene (pointers unused)
  gsr_camera cams[GSR_MAX_VIEWS];
  int64_t tile_base[GSR_MAX_VIEWS];
  int64_t pixel_base[GSR_MAX_VIEWS];
  hipEvent_t done = nullptr;           // recorded after the frame's last kernel
  int backwards = 0;                   // backward passes run on this frame
  int precision = -1;                  // precision of the forward raster (-1: prepared, not rastered)
};

}  // namespace

struct gsr_context {
  int device = 0;
  std::string err;
  size_t required = 0;
  std::unordered_map<const void*, FrameRecord> frames;
  bool profiling = false;
  bool events_ready = false;
  hipEvent_t ev[2 * GSR_STAGE_COUNT];
  bool recorded[GSR_STAGE_COUNT] = {};
  uint32_t split_len = gsr::kSplitLen;          // raster schedules of the frames prepared from now on
  uint32_t split_len_bwd = gsr::kSplitLenBwd;
  int32_t fault = GSR_FAULT_NONE;               // failure injection of the frames prepared from now on
};

namespace {

gsr_status fail(gsr_context* ctx, gsr_status st, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
gsr_status fail(gsr_context* ctx, gsr_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  return st;
}

gsr_status check_hip(gsr_context* ctx, hipError_t e, const char* what) {
  if (e == hipSuccess) return GSR_OK;
  return fail(ctx, GSR_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Makes ctx's device current for the duration of a call and restores the caller's.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

struct Planner {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + kAlign - 1) & ~(kAlign - 1);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

int bits_for(int64_t count) {
  int b = 0;
  while (b < 63 && ((int64_t)1 << b) < count) ++b;
  return b;
}

gsr_status validate_scene(gsr_context* ctx, const gsr_scene* sc) {
  if (!sc) return fail(ctx, GSR_ERR_INVALID_ARG, "scene is NULL");
  if (sc->n < 0) return fail(ctx, GSR_ERR_INVALID_ARG, "scene n = %lld < 0", (long long)sc->n);
  if (sc->n > (int64_t)0x7fffffff / 4) return fail(ctx, GSR_ERR_INVALID_ARG, "scene n = %lld too large", (long long)sc->n);
  if (sc->sh_degree < 0 || sc->sh_degree > 3)
    return fail(ctx, GSR_ERR_INVALID_ARG, "sh_degree = %d not in [0, 3]", sc->sh_degree);
  if (sc->n > 0 && (!sc->means || !sc->log_scales || !sc->quats || !sc->opacity_logits || !sc->sh))
    return fail(ctx, GSR_ERR_INVALID_ARG, "a scene array pointer is NULL");
  return GSR_OK;
}

// log2 of the tile width selected by gsr_options.tile_width (validated; 0 means 16)
int tile_wl_of(const gsr_options* o) {
  switch (o->tile_width) {
    case 4: return 2;
    case 8: return 3;
    case 32: return 5;
    case 64: return 6;
    default: return 4;
  }
}

// Tiles of a view under tiles 2^wl wide and 256 >> wl high.
int64_t view_tiles(const gsr_camera& c, int wl) {
  const int tw = 1 << wl, th = 256 >> wl;
  return (int64_t)((c.width + tw - 1) / tw) * ((c.height + th - 1) / th);
}

gsr_status validate_views(gsr_context* ctx, const gsr_camera* cams, int32_t V, int wl) {
  if (!cams) return fail(ctx, GSR_ERR_INVALID_ARG, "cameras are NULL");
  if (V < 1 || V > GSR_MAX_VIEWS) return fail(ctx, GSR_ERR_INVALID_ARG, "V = %d not in [1, %d]", V, GSR_MAX_VIEWS);
  int64_t tiles = 0;
  for (int v = 0; v < V; ++v) {
    const gsr_camera& c = cams[v];
    if (c.width < 1 || c.height < 1 || c.width > 65535 * (1 << wl) || c.height > 65535 * (256 >> wl))
      return fail(ctx, GSR_ERR_INVALID_ARG, "view %d: image %dx%d out of range", v, c.width, c.height);
    if (!(c.fx > 0.0f) || !(c.fy > 0.0f) || !std::isfinite(c.fx) || !std::isfinite(c.fy) ||
        !std::isfinite(c.cx) || !std::isfinite(c.cy))
      return fail(ctx, GSR_ERR_INVALID_ARG, "view %d: bad intrinsics", v);
    if (!(c.near_plane > 0.0f)) return fail(ctx, GSR_ERR_INVALID_ARG, "view %d: near_plane must be > 0", v);
    for (int k = 0; k < 9; ++k)
      if (!std::isfinite(c.R[k])) return fail(ctx, GSR_ERR_INVALID_ARG, "view %d: R not finite", v);
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(c.t[k]) || !std::isfinite(c.bg[k]))
        return fail(ctx, GSR_ERR_INVALID_ARG, "view %d: t or bg not finite", v);
    tiles += view_tiles(c, wl);
  }
  // raster work items carry the tile index in their upper 29 bits
  if (tiles >= ((int64_t)1 << 28)) return fail(ctx, GSR_ERR_INVALID_ARG, "too many tiles (limit 2^28)");
  return GSR_OK;
}

// Records (Gaussian slots x views) are counted and scanned in 30-bit words.
gsr_status validate_records(gsr_context* ctx, const gsr_scene* sc, int32_t V) {
  const int64_t ncap = (sc->n + GSR_CLUSTER - 1) / GSR_CLUSTER * GSR_CLUSTER;
  if (ncap * V >= ((int64_t)1 << 30))
    return fail(ctx, GSR_ERR_INVALID_ARG, "n x views = %lld x %d records: must stay below 2^30", (long long)sc->n, V);
  return GSR_OK;
}

gsr_status validate_opts(gsr_context* ctx, const gsr_options* o) {
  if (!o) return fail(ctx, GSR_ERR_INVALID_ARG, "options are NULL");
  if (o->precision != GSR_FP32 && o->precision != GSR_FP16_BLEND && o->precision != GSR_FP16_BLEND_T)
    return fail(ctx, GSR_ERR_INVALID_ARG, "unknown precision %d", o->precision);
  if (o->cluster_cull != 0 && o->cluster_cull != 1)
    return fail(ctx, GSR_ERR_INVALID_ARG, "cluster_cull must be 0 or 1");
  if (o->stats != 0 && o->stats != 1) return fail(ctx, GSR_ERR_INVALID_ARG, "stats must be 0 or 1");
  if (o->deterministic != 0 && o->deterministic != 1)
    return fail(ctx, GSR_ERR_INVALID_ARG, "deterministic must be 0 or 1");
  if (o->radius_mode != 0 && o->radius_mode != 1) return fail(ctx, GSR_ERR_INVALID_ARG, "radius_mode must be 0 or 1");
  if (o->half_reduction != 0 && o->half_reduction != 1)
    return fail(ctx, GSR_ERR_INVALID_ARG, "half_reduction must be 0 or 1");
  if (o->half_reduction && o->deterministic)
    return fail(ctx, GSR_ERR_INVALID_ARG, "half_reduction and deterministic exclude each other");
  if (o->tile_width != 0 && o->tile_width != 4 && o->tile_width != 8 && o->tile_width != 16 && o->tile_width != 32 &&
      o->tile_width != 64)
    return fail(ctx, GSR_ERR_INVALID_ARG, "tile_width %d not 0, 4, 8, 16, 32 or 64", o->tile_width);
  return GSR_OK;
}

// Lays out one frame in a workspace (or, with ws == nullptr, only sizes it) with
// room for inst_cap instances. Returns the total bytes. Layout: per-scene and
// per-pixel buffers, then the header and control words (cleared together at the
// frame start; their size grows with inst_cap), then the instance buffers.
size_t plan_frame(const gsr_scene* sc, const gsr_camera* cams, int32_t V, int wl, int64_t inst_cap, bool fixed,
                  void* ws, Frame& f) {
  std::memset(&f, 0, sizeof(f));
  f.n = sc->n;
  f.V = V;
  f.nclusters = (int32_t)((sc->n + GSR_CLUSTER - 1) / GSR_CLUSTER);
  f.ncap = (int64_t)f.nclusters * GSR_CLUSTER;
  f.nrec = f.ncap * V;
  f.tiles = 0;
  f.pixels = 0;
  for (int v = 0; v < V; ++v) {
    f.tiles += view_tiles(cams[v], wl);
    f.pixels += (int64_t)cams[v].width * cams[v].height;
  }
  f.tile_bits = bits_for(f.tiles);
  f.tile_wl = wl;
  f.inst_cap = inst_cap;
  Planner P{static_cast<char*>(ws)};
  const size_t nr = (size_t)f.nrec, nc = (size_t)std::max(f.nclusters, 1);
  f.views = P.take<ViewDev>(V);
  f.cluster_bounds = P.take<float>(8 * nc);
  f.cluster_visible = P.take<uint32_t>(nc);
  f.cluster_offset = P.take<uint32_t>(nc);
  f.cluster_list = P.take<uint32_t>(nc);
  f.compact2full = P.take<uint32_t>(std::max<size_t>(f.ncap, 1));
  f.rec = P.take<gsr::Record>(std::max<size_t>(nr, 1));
  f.dkey = P.take<uint32_t>(nr + 1);
  f.tiles_touched = P.take<uint32_t>(nr + 1);
  f.rect = P.take<ushort4>(nr + 1);
  f.skey[0] = P.take<uint32_t>(nr + 1);
  f.skey[1] = P.take<uint32_t>(nr + 1);
  f.sval[0] = P.take<uint32_t>(nr + 1);
  f.sval[1] = P.take<uint32_t>(nr + 1);
  f.offsets = P.take<uint32_t>(nr + 1);
  f.ranges = P.take<uint32_t>(2 * (size_t)f.tiles);
  f.tile_order = P.take<uint32_t>((size_t)gsr::raster_max_items(f.tiles));
  f.bwd_items = P.take<uint32_t>((size_t)gsr::raster_max_items(f.tiles));
  f.pix_T = P.take<float>((size_t)f.pixels);
  f.pix_last = P.take<uint32_t>((size_t)f.pixels);
  f.grad2d = P.take<float>(gsr::kGrad2D * std::max<size_t>(nr, 1));
  f.dmean = P.take<float>(3 * std::max<size_t>(f.ncap, 1));
  f.grad2d_fx = fixed ? P.take<unsigned long long>(gsr::kGrad2D * std::max<size_t>(nr, 1)) : nullptr;
  auto up = [](size_t w) { return (w + 63) & ~(size_t)63; };
  const size_t w_cluster = up(gsr::scan_ctl_words(f.nclusters));
  const size_t w_depth = up(gsr::sort_ctl_words(f.nrec, 32));
  const size_t w_offsets = up(gsr::scan_ctl_words(f.nrec));
  const size_t w_tiles = up(gsr::sort_ctl_words(std::max<int64_t>(inst_cap, 1), f.tile_bits));
  const size_t w_order = up(gsr::tile_order_ctl_words(f.tiles));
  f.ctl_words = w_cluster + w_depth + w_offsets + w_tiles + w_order;
  f.header = P.take<uint32_t>(64 + f.ctl_words);
  if (f.header) {
    f.ctl = f.header + 64;
    f.ctl_cluster_scan = f.ctl;
    f.ctl_depth_sort = f.ctl_cluster_scan + w_cluster;
    f.ctl_offsets_scan = f.ctl_depth_sort + w_depth;
    f.ctl_tile_sort = f.ctl_offsets_scan + w_offsets;
    f.ctl_tile_order = w_order ? f.ctl_tile_sort + w_tiles : nullptr;
  }
  for (int b = 0; b < 2; ++b) {
    f.ikey[b] = P.take<uint32_t>((size_t)std::max<int64_t>(inst_cap, 1));
    f.ival[b] = P.take<uint32_t>((size_t)std::max<int64_t>(inst_cap, 1));
  }
  return (P.off + kAlign - 1) & ~(kAlign - 1);
}

size_t bytes_for_instances(const gsr_scene* sc, const gsr_camera* cams, int32_t V, int wl, int64_t m, bool fixed) {
  Frame f;
  return plan_frame(sc, cams, V, wl, m, fixed, nullptr, f);
}

// Largest instance capacity whose layout fits in ws_bytes (-1 if not even 0 fits).
int64_t instances_for_bytes(const gsr_scene* sc, const gsr_camera* cams, int32_t V, int wl, size_t ws_bytes,
                            bool fixed) {
  if (bytes_for_instances(sc, cams, V, wl, 0, fixed) > ws_bytes) return -1;
  int64_t lo = 0, hi = (int64_t)(ws_bytes / 16) + 1;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (bytes_for_instances(sc, cams, V, wl, mid, fixed) <= ws_bytes) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

struct StageScope {
  gsr_context* ctx;
  int stage;
  hipStream_t s;
  StageScope(gsr_context* c, int st, hipStream_t stream) : ctx(c), stage(st), s(stream) {
    if (ctx->profiling) (void)hipEventRecord(ctx->ev[2 * stage], s);
  }
  ~StageScope() {
    if (ctx->profiling) {
      (void)hipEventRecord(ctx->ev[2 * stage + 1], s);
      ctx->recorded[stage] = true;
    }
  }
};

void release_frame(FrameRecord& fr) {
  if (fr.done) (void)hipEventDestroy(fr.done);
  fr.done = nullptr;
}

void fill_views(const gsr_camera* cams, int32_t V, int wl, ViewDev* out) {
  int64_t tile_base = 0, pixel_base = 0;
  for (int v = 0; v < V; ++v) {
    const gsr_camera& c = cams[v];
    ViewDev& w = out[v];
    std::memset(&w, 0, sizeof(w));
    std::memcpy(w.R, c.R, sizeof(w.R));
    std::memcpy(w.t, c.t, sizeof(w.t));
    w.fx = c.fx;
    w.fy = c.fy;
    w.cx = c.cx;
    w.cy = c.cy;
    w.near_plane = c.near_plane;
    std::memcpy(w.bg, c.bg, sizeof(w.bg));
    w.limx = gsr::kFovClamp * (double)c.width / (2.0 * (double)c.fx);
    w.limy = gsr::kFovClamp * (double)c.height / (2.0 * (double)c.fy);
    const double R[9] = {c.R[0], c.R[1], c.R[2], c.R[3], c.R[4], c.R[5], c.R[6], c.R[7], c.R[8]};
    const double t[3] = {c.t[0], c.t[1], c.t[2]};
    w.campos[0] = -(R[0] * t[0] + R[3] * t[1] + R[6] * t[2]);
    w.campos[1] = -(R[1] * t[0] + R[4] * t[1] + R[7] * t[2]);
    w.campos[2] = -(R[2] * t[0] + R[5] * t[1] + R[8] * t[2]);
    w.width = c.width;
    w.height = c.height;
    w.tiles_x = (c.width + (1 << wl) - 1) >> wl;
    w.tiles_y = (c.height + (256 >> wl) - 1) / (256 >> wl);
    w.tile_wl = wl;
    w.tile_base = (int32_t)tile_base;
    w.pixel_base = pixel_base;
    tile_base += (int64_t)w.tiles_x * w.tiles_y;
    pixel_base += (int64_t)c.width * c.height;
  }
}

}  // namespace

extern "C" {

gsr_status gsr_context_create(int device, gsr_context** out) {
  if (!out) return GSR_ERR_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return GSR_ERR_DEVICE;
  // the device's copy of the no-allocation scratch, looked up once per device
  if (gsr::noalloc_init(device) != hipSuccess) return GSR_ERR_DEVICE;
  gsr_context* ctx = new gsr_context();
  ctx->device = device;
  *out = ctx;
  return GSR_OK;
}

void gsr_context_destroy(gsr_context* ctx) {
  if (!ctx) return;
  {
    DeviceGuard g(ctx->device);
    for (auto& kv : ctx->frames) {
      if (kv.second.done) (void)hipEventSynchronize(kv.second.done);
      release_frame(kv.second);
    }
    ctx->frames.clear();
    if (ctx->events_ready)
      for (int k = 0; k < 2 * GSR_STAGE_COUNT; ++k) (void)hipEventDestroy(ctx->ev[k]);
  }
  delete ctx;
}

const char* gsr_last_error(const gsr_context* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

size_t gsr_required_workspace(const gsr_context* ctx) { return ctx ? ctx->required : 0; }

gsr_status gsr_workspace_size(gsr_context* ctx, const gsr_scene* scene, const gsr_camera* cams, int32_t V,
                              const gsr_options* opts, int64_t max_instances, size_t* bytes) {
  if (!bytes) return fail(ctx, GSR_ERR_INVALID_ARG, "NULL output");
  gsr_status st;
  if ((st = validate_scene(ctx, scene)) || (st = validate_opts(ctx, opts)) ||
      (st = validate_views(ctx, cams, V, tile_wl_of(opts))) ||
      (st = validate_records(ctx, scene, V)))
    return st;
  if (max_instances < 0) return fail(ctx, GSR_ERR_INVALID_ARG, "max_instances < 0");
  if (max_instances >= ((int64_t)1 << 30)) return fail(ctx, GSR_ERR_INVALID_ARG, "max_instances >= 2^30");
  *bytes = bytes_for_instances(scene, cams, V, tile_wl_of(opts), max_instances, opts->deterministic != 0);
  return GSR_OK;
}

namespace {

// Every stage of a frame up to the raster schedule (Cluster-Cull-Compact,
// preprocess, depth sort, offsets, emission, tile sort, ranges, tile order),
// enqueued on `s` without any host wait. With record_done the frame's event
// completes with its last kernel (gsr_forward leaves it to the raster).
gsr_status prepare_frame(gsr_context* ctx, const gsr_scene* scene, const gsr_camera* cams, int32_t V,
                         const gsr_options* opts, void* workspace, size_t ws_bytes, hipStream_t s, bool record_done,
                         FrameRecord** out) {
  gsr_status st;
  bool attached = false;
  if ((st = validate_scene(ctx, scene)) || (st = validate_opts(ctx, opts)) ||
      (st = validate_views(ctx, cams, V, tile_wl_of(opts))) ||
      (st = validate_records(ctx, scene, V)))
    return st;
  if (!workspace) return fail(ctx, GSR_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)workspace & (kAlign - 1)) != 0) return fail(ctx, GSR_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  const bool fixed = opts->deterministic != 0;
  const int wl = tile_wl_of(opts);
  int64_t cap = instances_for_bytes(scene, cams, V, wl, ws_bytes, fixed);
  if (cap < 0) {
    ctx->required = bytes_for_instances(scene, cams, V, wl, 16 * (int64_t)scene->n + 1024, fixed);
    return fail(ctx, GSR_ERR_WORKSPACE_TOO_SMALL, "workspace of %zu bytes < %zu needed before instances", ws_bytes,
                bytes_for_instances(scene, cams, V, wl, 0, fixed));
  }
  cap = std::min<int64_t>(cap, ((int64_t)1 << 30) - 1);
  Frame f;
  const size_t total = plan_frame(scene, cams, V, wl, cap, fixed, workspace, f);
  f.split_len = ctx->split_len;
  f.split_len_bwd = ctx->split_len_bwd;
  f.radius_mode = opts->radius_mode;
  if (total > ws_bytes) return fail(ctx, GSR_ERR_INVALID_ARG, "internal: workspace plan exceeds its size");

  FrameRecord& fr = ctx->frames[workspace];
  if (!fr.done && (st = check_hip(ctx, hipEventCreateWithFlags(&fr.done, hipEventDisableTiming), "frame event")))
    return st;
  fr.scene = *scene;
  std::memcpy(fr.cams, cams, sizeof(gsr_camera) * V);
  fr.backwards = 0;
  fr.precision = -1;

  ViewDev hv[GSR_MAX_VIEWS];
  fill_views(cams, V, wl, hv);
  for (int v = 0; v < V; ++v) {
    fr.tile_base[v] = hv[v].tile_base;
    fr.pixel_base[v] = hv[v].pixel_base;
  }
  for (int k = 0; k < GSR_STAGE_COUNT; ++k) ctx->recorded[k] = false;
  {
    // frame start, then Cluster-Cull-Compact
    StageScope sc_(ctx, GSR_STAGE_CLUSTER, s);
    gsr::ViewChunk first;
    std::memcpy(first.v, hv, sizeof(ViewDev) * std::min(gsr::kViewChunk, (int)V));
    if (!gsr::launch_cluster_begin(first, V, f.views, f.header, (int64_t)(64 + f.ctl_words), scene->means,
                                   scene->log_scales, scene->n, opts->cluster_cull, f.cluster_bounds,
                                   f.cluster_visible, s)) {
      for (int v0 = 0; v0 < V; v0 += gsr::kViewChunk) {
        gsr::ViewChunk chunk;
        const int nv = std::min(gsr::kViewChunk, V - v0);
        std::memcpy(chunk.v, hv + v0, sizeof(ViewDev) * nv);
        gsr::launch_frame_begin(chunk, v0, nv, f.views, f.header, v0 == 0 ? (int64_t)(64 + f.ctl_words) : 0, s);
      }
      gsr::launch_cluster(scene->means, scene->log_scales, scene->n, opts->cluster_cull, f.views, V,
                          f.cluster_bounds, f.cluster_visible, s);
    }
    gsr::scan_u32(f.cluster_visible, nullptr, f.cluster_offset, f.nclusters, nullptr,
                  f.header + gsr::kHdrVisibleClusters, f.cluster_list, f.ctl_cluster_scan, f.header + gsr::kHdrError,
                  s);
  }
  {
    StageScope sc_(ctx, GSR_STAGE_PREPROCESS, s);
    gsr::launch_preprocess_fwd(*scene, f, s);
  }
  const uint32_t* n_rec = f.header + gsr::kHdrRecords;
  uint32_t* err = f.header + gsr::kHdrError;
  const uint32_t* sorted_rec;
  {
    StageScope sc_(ctx, GSR_STAGE_DEPTH_SORT, s);
    uint32_t* kb[2] = {f.skey[0], f.skey[1]};
    uint32_t* vb[2] = {f.sval[0], f.sval[1]};
    if (ctx->fault == GSR_FAULT_ABORT_BEFORE_SORT) gsr::raise_abort(err, s);
    const int r = gsr::radix_sort_u32_dev(f.dkey, nullptr, kb, vb, f.nrec, n_rec, 32, f.ctl_depth_sort, err, true, s);
    sorted_rec = r >= 0 ? vb[r] : vb[0];  // no pass only when there are no records
  }
  {
    // instance offsets: exclusive scan of the tiles touched, in depth order
    StageScope sc_(ctx, GSR_STAGE_OFFSETS, s);
    gsr::scan_u32(f.tiles_touched, sorted_rec, f.offsets, f.nrec, n_rec, f.header + gsr::kHdrInstances, nullptr,
                  f.ctl_offsets_scan, err, s);
  }
  {
    StageScope sc_(ctx, GSR_STAGE_EMIT, s);
    gsr::launch_emit_instances(f, sorted_rec, s);
  }
  {
    StageScope sc_(ctx, GSR_STAGE_TILE_SORT, s);
    uint32_t* ik[2] = {f.ikey[1], f.ikey[0]};
    uint32_t* iv[2] = {f.ival[1], f.ival[0]};
    const int ri = gsr::radix_sort_u32_dev(f.ikey[0], f.ival[0], ik, iv, cap, f.header + gsr::kHdrInstancesKept,
                                           f.tile_bits, f.ctl_tile_sort, err, false, s,
                                           ctx->fault == GSR_FAULT_WITHHOLD_STATUS ? 1 : -1);
    f.inst_tile = ri >= 0 ? ik[ri] : f.ikey[0];
    f.inst_rec = ri >= 0 ? iv[ri] : f.ival[0];
    f.inst_mask = f.inst_rec == f.ival[0] ? f.ival[1] : f.ival[0];  // free once the sort is done
  }
  {
    StageScope sc_(ctx, GSR_STAGE_RANGES, s);
    gsr::launch_tile_ranges(f, f.inst_tile, cap, s);
    attached = gsr::launch_tile_order(f, s, record_done ? fr.done : nullptr);
  }
  if ((st = check_hip(ctx, hipGetLastError(), "frame launches"))) return st;
  if (record_done && !attached && (st = check_hip(ctx, hipEventRecord(fr.done, s), "frame event"))) return st;
  fr.f = f;
  *out = &fr;
  return GSR_OK;
}

}  // namespace

gsr_status gsr_prepare(gsr_context* ctx, const gsr_scene* scene, const gsr_camera* cams, int32_t V,
                       const gsr_options* opts, void* workspace, size_t ws_bytes, void* stream) {
  if (!ctx) return GSR_ERR_INVALID_ARG;
  DeviceGuard guard(ctx->device);
  FrameRecord* fr = nullptr;
  return prepare_frame(ctx, scene, cams, V, opts, workspace, ws_bytes, static_cast<hipStream_t>(stream), true, &fr);
}

gsr_status gsr_forward(gsr_context* ctx, const gsr_scene* scene, const gsr_camera* cams, int32_t V,
                       const gsr_options* opts, void* workspace, size_t ws_bytes, float* const* images,
                       void* stream) {
  if (!ctx) return GSR_ERR_INVALID_ARG;
  if (!images) return fail(ctx, GSR_ERR_INVALID_ARG, "images is NULL");
  for (int v = 0; v < V && v < GSR_MAX_VIEWS; ++v)
    if (!images[v]) return fail(ctx, GSR_ERR_INVALID_ARG, "images[%d] is NULL", v);
  DeviceGuard guard(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  FrameRecord* fr = nullptr;
  gsr_status st = prepare_frame(ctx, scene, cams, V, opts, workspace, ws_bytes, s, false, &fr);
  if (st) return st;
  bool attached = false;
  gsr::ImagePtrs ip;
  std::memset(&ip, 0, sizeof(ip));
  for (int v = 0; v < V; ++v) ip.p[v] = images[v];
  {
    StageScope sc_(ctx, GSR_STAGE_RASTER_FWD, s);
    attached = gsr::launch_raster_fwd(fr->f, ip, opts->precision, s, fr->done);
  }
  if ((st = check_hip(ctx, hipGetLastError(), "forward raster"))) return st;
  if (!attached && (st = check_hip(ctx, hipEventRecord(fr->done, s), "frame event"))) return st;
  fr->precision = opts->precision;
  return GSR_OK;
}

// Batch workspace: the raster work items of the concatenated tiles, then their count.
static size_t batch_items_words(uint64_t tiles) {
  const uint64_t bytes = (uint64_t)gsr::raster_max_items((int64_t)tiles) * 4;
  return (size_t)(((bytes + kAlign - 1) & ~(uint64_t)(kAlign - 1)) / 4);
}
static size_t batch_workspace_bytes(uint64_t tiles) { return batch_items_words(tiles) * 4 + kAlign; }

gsr_status gsr_raster_batch_workspace_size(gsr_context* ctx, int32_t n, const void* const* workspaces,
                                           size_t* bytes) {
  if (!ctx || !bytes || !workspaces || n < 1 || n > gsr::kMaxBatch)
    return fail(ctx, GSR_ERR_INVALID_ARG, "bad arguments to gsr_raster_batch_workspace_size");
  uint64_t tiles = 0;
  for (int i = 0; i < n; ++i) {
    auto it = ctx->frames.find(workspaces[i]);
    if (it == ctx->frames.end()) return fail(ctx, GSR_ERR_INVALID_ARG, "frame %d was not prepared", i);
    tiles += (uint64_t)it->second.f.tiles;
  }
  *bytes = batch_workspace_bytes(tiles);
  return GSR_OK;
}

}  // extern "C"

namespace {

// One batched raster over n prepared frames. With batch_ws set, the work-item list
// lives in the caller's batch workspace; with batch_ws null (the no-allocation
// entry point), in the device-resident scratch of ctx's device.
gsr_status raster_batch_impl(gsr_context* ctx, int32_t n, const void* const* workspaces, float* const* const* images,
                             int32_t precision, void* batch_ws, size_t batch_ws_bytes, bool resident, void* stream) {
  if (!ctx) return GSR_ERR_INVALID_ARG;
  if (n < 1 || n > gsr::kMaxBatch || !workspaces || !images)
    return fail(ctx, GSR_ERR_INVALID_ARG, "n = %d not in [1, %d] or NULL arrays", n, gsr::kMaxBatch);
  if (precision != GSR_FP32 && precision != GSR_FP16_BLEND && precision != GSR_FP16_BLEND_T)
    return fail(ctx, GSR_ERR_INVALID_ARG, "unknown precision %d", precision);
  gsr::FrameTable tab;
  std::memset(&tab, 0, sizeof(tab));
  gsr::ImagePtrs ip;
  std::memset(&ip, 0, sizeof(ip));
  FrameRecord* frs[gsr::kMaxBatch];
  uint64_t tiles = 0;
  int views = 0;
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < i; ++j)
      if (workspaces[j] == workspaces[i]) return fail(ctx, GSR_ERR_INVALID_ARG, "frame %d appears twice", i);
    auto it = ctx->frames.find(workspaces[i]);
    if (it == ctx->frames.end()) return fail(ctx, GSR_ERR_INVALID_ARG, "frame %d was not prepared", i);
    FrameRecord& fr = it->second;
    const Frame& f = fr.f;
    if (views + f.V > GSR_MAX_VIEWS) return fail(ctx, GSR_ERR_INVALID_ARG, "more than %d views in a batch", GSR_MAX_VIEWS);
    if (!images[i]) return fail(ctx, GSR_ERR_INVALID_ARG, "images[%d] is NULL", i);
    for (int v = 0; v < f.V; ++v) {
      if (!images[i][v]) return fail(ctx, GSR_ERR_INVALID_ARG, "images[%d][%d] is NULL", i, v);
      ip.p[views + v] = images[i][v];
    }
    gsr::FrameRef& r = tab.f[i];
    r.header = f.header;
    r.views = f.views;
    r.ranges = f.ranges;
    r.inst_rec = f.inst_rec;
    r.inst_mask = f.inst_mask;
    r.rec = f.rec;
    r.pix_T = f.pix_T;
    r.pix_last = f.pix_last;
    r.V = f.V;
    r.img_base = views;
    tab.first[i] = (uint32_t)tiles;
    tiles += (uint64_t)f.tiles;
    views += f.V;
    frs[i] = &fr;
  }
  if (tiles >= ((uint64_t)1 << 28)) return fail(ctx, GSR_ERR_INVALID_ARG, "too many tiles in a batch (limit 2^28)");
  tab.first[n] = (uint32_t)tiles;
  tab.n = n;
  uint32_t* order = nullptr;
  uint32_t* n_items = nullptr;
  if (resident) {
    if ((int64_t)tiles > gsr::noalloc_max_tiles())
      return fail(ctx, GSR_ERR_INVALID_ARG, "%llu tiles exceed the %lld of the device-resident scratch",
                  (unsigned long long)tiles, (long long)gsr::noalloc_max_tiles());
    size_t words = 0;
    order = gsr::noalloc_scratch(ctx->device, &words);
    if (!order) return fail(ctx, GSR_ERR_DEVICE, "the device-resident scratch was not set up");
    n_items = order + batch_items_words(tiles);
    if (batch_items_words(tiles) + 1 > words) return fail(ctx, GSR_ERR_INVALID_ARG, "internal: scratch too small");
  } else {
    const size_t need = batch_workspace_bytes(tiles);
    if (!batch_ws || batch_ws_bytes < need) {
      ctx->required = need;
      return fail(ctx, GSR_ERR_WORKSPACE_TOO_SMALL, "batch workspace of %zu bytes < %zu", batch_ws_bytes, need);
    }
    if (((uintptr_t)batch_ws & (kAlign - 1)) != 0)
      return fail(ctx, GSR_ERR_INVALID_ARG, "batch workspace not aligned");
    order = static_cast<uint32_t*>(batch_ws);
    n_items = order + batch_items_words(tiles);
  }
  DeviceGuard guard(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  gsr::launch_batch_tile_order(tab, (uint32_t)tiles, ctx->split_len, order, n_items, s);
  const bool attached = gsr::launch_raster_fwd_batch(tab, order, n_items, (uint32_t)tiles, ip, precision, s,
                                                     frs[0]->done);
  gsr_status st = check_hip(ctx, hipGetLastError(), "batched raster");
  if (st) return st;
  for (int i = 0; i < n; ++i) {
    if ((i > 0 || !attached) && (st = check_hip(ctx, hipEventRecord(frs[i]->done, s), "frame event"))) return st;
    frs[i]->precision = precision;
  }
  return GSR_OK;
}

}  // namespace

extern "C" {

gsr_status gsr_raster_batch(gsr_context* ctx, int32_t n, const void* const* workspaces, float* const* const* images,
                            int32_t precision, void* batch_ws, size_t batch_ws_bytes, void* stream) {
  return raster_batch_impl(ctx, n, workspaces, images, precision, batch_ws, batch_ws_bytes, false, stream);
}

gsr_status gsr_raster_batch_noalloc(gsr_context* ctx, int32_t n, const void* const* workspaces,
                                    float* const* const* images, int32_t precision, void* stream) {
  return raster_batch_impl(ctx, n, workspaces, images, precision, nullptr, 0, true, stream);
}

gsr_status gsr_frame_release(gsr_context* ctx, const void* workspace) {
  if (!ctx) return GSR_ERR_INVALID_ARG;
  auto it = ctx->frames.find(workspace);
  if (it == ctx->frames.end()) return GSR_OK;
  DeviceGuard guard(ctx->device);
  gsr_status st = GSR_OK;
  if (it->second.done) st = check_hip(ctx, hipEventSynchronize(it->second.done), "wait for the frame");
  release_frame(it->second);
  ctx->frames.erase(it);
  return st;
}

}  // extern "C"

namespace {

// gsr_backward, and with `adam` set the fused backward + Adam of gsr_backward_adam
// (no gradient arrays then).
gsr_status backward_impl(gsr_context* ctx, const gsr_scene* scene, const gsr_camera* cams, int32_t V,
                         const gsr_options* opts, void* workspace, size_t ws_bytes, const float* const* dL_dimages,
                         const gsr_grads* grads, const gsr_stats* stats, const gsr::AdamDev* adam, void* stream) {
  if (!ctx) return GSR_ERR_INVALID_ARG;
  gsr_status st;
  if ((st = validate_scene(ctx, scene)) || (st = validate_opts(ctx, opts)) ||
      (st = validate_views(ctx, cams, V, tile_wl_of(opts))) ||
      (st = validate_records(ctx, scene, V)))
    return st;
  if (!workspace) return fail(ctx, GSR_ERR_INVALID_ARG, "workspace is NULL");
  auto it = ctx->frames.find(workspace);
  if (it == ctx->frames.end()) return fail(ctx, GSR_ERR_INVALID_ARG, "no forward was run on this workspace");
  FrameRecord& fr = it->second;
  const Frame& f = fr.f;
  if (fr.precision < 0) return fail(ctx, GSR_ERR_INVALID_ARG, "the frame was prepared but never rastered");
  if (fr.precision != opts->precision)
    return fail(ctx, GSR_ERR_INVALID_ARG, "precision %d differs from the forward's %d", opts->precision, fr.precision);
  if ((f.grad2d_fx != nullptr) != (opts->deterministic != 0))
    return fail(ctx, GSR_ERR_INVALID_ARG, "deterministic %d differs from the forward's", opts->deterministic);
  if (f.n != scene->n || f.V != V || fr.scene.sh_degree != scene->sh_degree)
    return fail(ctx, GSR_ERR_INVALID_ARG, "scene or views differ from the forward");
  {
    Frame chk;
    if (f.tile_wl != tile_wl_of(opts))
      return fail(ctx, GSR_ERR_INVALID_ARG, "tile_width %d differs from the forward's", opts->tile_width);
    const size_t total = plan_frame(scene, cams, V, f.tile_wl, f.inst_cap, f.grad2d_fx != nullptr, workspace, chk);
    if (chk.tiles != f.tiles || chk.pixels != f.pixels || chk.grad2d != f.grad2d || total > ws_bytes)
      return fail(ctx, GSR_ERR_INVALID_ARG, "cameras or workspace differ from the forward");
  }
  if (!dL_dimages) return fail(ctx, GSR_ERR_INVALID_ARG, "dL_dimages is NULL");
  for (int v = 0; v < V; ++v)
    if (!dL_dimages[v]) return fail(ctx, GSR_ERR_INVALID_ARG, "dL_dimages[%d] is NULL", v);
  if (!adam && !grads) return fail(ctx, GSR_ERR_INVALID_ARG, "grads is NULL");
  if (!adam && scene->n > 0 &&
      (!grads->means || !grads->log_scales || !grads->quats || !grads->opacity_logits || !grads->sh))
    return fail(ctx, GSR_ERR_INVALID_ARG, "a gradient array pointer is NULL");
  const bool use_stats = opts->stats && stats;
  if (use_stats && scene->n > 0 && (!stats->S || !stats->M || !stats->C))
    return fail(ctx, GSR_ERR_INVALID_ARG, "a statistic array pointer is NULL");
  DeviceGuard guard(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int k = GSR_STAGE_ZERO_GRAD; k < GSR_STAGE_COUNT; ++k) ctx->recorded[k] = false;
  if (fr.backwards > 0) {
    // the forward cleared the rows of its records; a repeated backward clears them again
    StageScope sc_(ctx, GSR_STAGE_ZERO_GRAD, s);
    if (f.grad2d_fx)
      gsr::fill_u32(reinterpret_cast<uint32_t*>(f.grad2d_fx), 2 * gsr::kGrad2D * f.nrec, 0u, s);
    else
      gsr::fill_f32(f.grad2d, gsr::kGrad2D * f.nrec, 0.0f, s);
  }
  gsr::ConstImagePtrs dp;
  std::memset(&dp, 0, sizeof(dp));
  for (int v = 0; v < V; ++v) dp.p[v] = dL_dimages[v];
  {
    StageScope sc_(ctx, GSR_STAGE_RASTER_BWD, s);
    if (f.grad2d_fx) {  // the fixed-point scale follows the upstream gradient's size
      gsr::ViewCounts counts{};
      for (int v = 0; v < V; ++v) counts.n[v] = 3 * (int64_t)cams[v].width * cams[v].height;
      gsr::launch_grad_absmax(f, dp, counts, s);
    }
    gsr::launch_raster_bwd(f, dp, opts->precision, opts->half_reduction != 0, s);
  }
  {
    StageScope sc_(ctx, GSR_STAGE_PREPROCESS_BWD, s);
    const gsr_grads none{};
    gsr::launch_preprocess_bwd(*scene, f, adam ? none : *grads, use_stats ? stats : nullptr, adam,
                               opts->half_reduction != 0, s);
  }
  fr.backwards++;
  return check_hip(ctx, hipGetLastError(), "backward");
}

}  // namespace

extern "C" {

gsr_status gsr_backward(gsr_context* ctx, const gsr_scene* scene, const gsr_camera* cams, int32_t V,
                        const gsr_options* opts, void* workspace, size_t ws_bytes, const float* const* dL_dimages,
                        const gsr_grads* grads, const gsr_stats* stats, void* stream) {
  return backward_impl(ctx, scene, cams, V, opts, workspace, ws_bytes, dL_dimages, grads, stats, nullptr, stream);
}

gsr_status gsr_frame_inspect(gsr_context* ctx, const void* workspace, gsr_frame_info* info, gsr_frame_buffers* bufs) {
  if (!ctx) return GSR_ERR_INVALID_ARG;
  auto it = ctx->frames.find(workspace);
  if (it == ctx->frames.end()) return fail(ctx, GSR_ERR_INVALID_ARG, "no forward was run on this workspace");
  FrameRecord& fr = it->second;
  const Frame& f = fr.f;
  DeviceGuard guard(ctx->device);
  gsr_status st = check_hip(ctx, hipEventSynchronize(fr.done), "wait for the frame");
  if (st) return st;
  // the counters stay in the workspace's header until the next forward on it
  uint32_t h[kHdrBytes / 4];
  if ((st = check_hip(ctx, hipMemcpy(h, f.header, kHdrBytes, hipMemcpyDeviceToHost), "read the frame header")))
    return st;
  const int64_t nvis = h[gsr::kHdrVisibleClusters];
  const int64_t M = h[gsr::kHdrInstances];
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->n = f.n;
    info->n_visible_slots = nvis * GSR_CLUSTER;
    info->instances = M;
    info->tiles = f.tiles;
    info->pixels = f.pixels;
    info->views = f.V;
    info->clusters = f.nclusters;
    info->visible_clusters = (int32_t)nvis;
    info->split_tiles = (int32_t)((h[gsr::kHdrItems] - (uint32_t)f.tiles) / 3);
    info->split_tiles_bwd = (int32_t)(h[gsr::kHdrItemsBwd] - (uint32_t)f.tiles);
  }
  if (bufs) {
    std::memset(bufs, 0, sizeof(*bufs));
    bufs->record = reinterpret_cast<const float*>(f.rec);
    bufs->depth_key = f.dkey;
    bufs->tiles = f.tiles_touched;
    bufs->rect = reinterpret_cast<const uint16_t*>(f.rect);
    bufs->compact2full = f.compact2full;
    bufs->inst_tile = f.inst_tile;
    bufs->inst_record = f.inst_rec;
    bufs->ranges = f.ranges;
    bufs->pixel_T = f.pix_T;
    bufs->pixel_last = f.pix_last;
    bufs->grad2d = f.grad2d;
    bufs->cluster_bounds = f.cluster_bounds;
    bufs->cluster_visible = f.cluster_visible;
    bufs->fwd_items = f.tile_order;
    bufs->bwd_items = f.bwd_items;
    for (int v = 0; v < f.V; ++v) {
      bufs->tile_base[v] = fr.tile_base[v];
      bufs->pixel_base[v] = fr.pixel_base[v];
    }
  }
  if (h[gsr::kHdrError] & 2u) return fail(ctx, GSR_ERR_UNSUPPORTED, "the frame has 2^30 or more instances");
  if (h[gsr::kHdrError]) return fail(ctx, GSR_ERR_DEVICE, "a device-wide scan or sort wait gave up (frame aborted)");
  if (h[gsr::kHdrOverflow]) {
    ctx->required = bytes_for_instances(&fr.scene, fr.cams, f.V, f.tile_wl, M + M / 8 + 1024, f.grad2d_fx != nullptr);
    return fail(ctx, GSR_ERR_WORKSPACE_TOO_SMALL, "frame has %lld instances, workspace holds %lld", (long long)M,
                (long long)f.inst_cap);
  }
  return GSR_OK;
}

gsr_status gsr_variance(gsr_context* ctx, const gsr_stats* stats, int64_t n, float* out, void* stream) {
  if (!ctx) return GSR_ERR_INVALID_ARG;
  if (!stats || n < 0 || (n > 0 && (!stats->S || !stats->M || !stats->C || !out)))
    return fail(ctx, GSR_ERR_INVALID_ARG, "bad arguments to gsr_variance");
  DeviceGuard guard(ctx->device);
  gsr::launch_variance(stats->S, stats->M, stats->C, n, out, static_cast<hipStream_t>(stream));
  return check_hip(ctx, hipGetLastError(), "variance");
}

gsr_status gsr_l1_grad(gsr_context* ctx, const float* image, const float* w, const float* gt, int64_t count,
                       float* out, void* stream) {
  if (!ctx) return GSR_ERR_INVALID_ARG;
  if (count < 0 || (count > 0 && (!image || !w || !gt || !out)))
    return fail(ctx, GSR_ERR_INVALID_ARG, "bad arguments to gsr_l1_grad");
  DeviceGuard guard(ctx->device);
  gsr::launch_l1_grad(image, w, gt, count, out, static_cast<hipStream_t>(stream));
  return check_hip(ctx, hipGetLastError(), "l1 grad");
}

}  // extern "C"

namespace {

// Validates an Adam step over n Gaussians and fills the device constants. grads may
// be null (the fused backward computes them on the fly); every other array must be
// non-null, 16-byte aligned, and no two of the arrays may overlap.
gsr_status build_adam(gsr_context* ctx, int64_t n, int32_t sh_degree, const gsr_grads* params, const gsr_grads* grads,
                      const gsr_grads* exp_avg, const gsr_grads* exp_avg_sq, const gsr_adam_options* opts,
                      gsr::AdamDev& a) {
  if (n < 0 || n > (int64_t(1) << 40) || sh_degree < 0 || sh_degree > 3 || !params || !exp_avg || !exp_avg_sq ||
      !opts)
    return fail(ctx, GSR_ERR_INVALID_ARG, "bad arguments to the Adam step");
  const gsr_adam_options& o = *opts;
  if (o.reserved != 0 || o.step < 1 || !(o.beta1 >= 0.0f && o.beta1 < 1.0f) || !(o.beta2 >= 0.0f && o.beta2 < 1.0f) ||
      !(o.eps >= 0.0f))
    return fail(ctx, GSR_ERR_INVALID_ARG, "Adam step: need step >= 1, betas in [0, 1), eps >= 0");
  const int32_t K = (sh_degree + 1) * (sh_degree + 1);
  const int32_t rows[gsr::kAdamGroups] = {3, 3, 4, 1, 3 * K};
  // the five arrays of each set, in the order of the kernel's groups
  float* arr[4][gsr::kAdamGroups] = {};
  const gsr_grads* sets[4] = {params, grads, exp_avg, exp_avg_sq};
  struct Extent {
    uintptr_t lo, hi;
  };
  std::vector<Extent> ext;
  for (int j = 0; j < 4; ++j) {
    if (!sets[j]) continue;
    const gsr_grads& g = *sets[j];
    float* ptrs[gsr::kAdamGroups] = {g.means, g.log_scales, g.quats, g.opacity_logits, g.sh};
    for (int k = 0; k < gsr::kAdamGroups; ++k) {
      const uintptr_t p = reinterpret_cast<uintptr_t>(ptrs[k]);
      if (n > 0 && (!p || (p & 15u)))
        return fail(ctx, GSR_ERR_INVALID_ARG, "Adam step: every array must be non-null and 16-byte aligned");
      ext.push_back({p, p + uintptr_t(n) * rows[k] * sizeof(float)});
      arr[j][k] = ptrs[k];
    }
  }
  std::sort(ext.begin(), ext.end(), [](const Extent& x, const Extent& y) { return x.lo < y.lo; });
  for (size_t i = 1; i < ext.size() && n > 0; ++i)
    if (ext[i].lo < ext[i - 1].hi) return fail(ctx, GSR_ERR_INVALID_ARG, "Adam step: arrays overlap");

  a = gsr::AdamDev{};
  const double t = double(o.step);
  const double bc1 = 1.0 - std::pow(double(o.beta1), t);
  const double bc2 = 1.0 - std::pow(double(o.beta2), t);
  const float lr[gsr::kAdamGroups] = {o.lr_means, o.lr_log_scales, o.lr_quats, o.lr_opacity, o.lr_sh_dc};
  int32_t row_sum = 0;
  for (int k = 0; k < gsr::kAdamGroups; ++k) {
    gsr::AdamGroupDev& q = a.grp[k];
    q.p = arr[0][k];
    q.g = arr[1][k];
    q.m = arr[2][k];
    q.v = arr[3][k];
    q.row = rows[k];
    q.head = k == 4 ? 3 : rows[k];  // SH: the degree-0 floats take lr_sh_dc, the rest lr_sh_rest
    q.step_head = float(double(lr[k]) / bc1);
    q.step_rest = float(double(k == 4 ? o.lr_sh_rest : lr[k]) / bc1);
    row_sum += rows[k];
  }
  a.n = n;
  a.units = (GSR_CLUSTER / 4) * row_sum;
  a.beta1 = o.beta1;
  a.beta2 = o.beta2;
  a.c1 = float(1.0 - double(o.beta1));
  a.c2 = float(1.0 - double(o.beta2));
  a.eps = o.eps;
  a.inv_sqrt_bc2 = float(1.0 / std::sqrt(bc2));
  return GSR_OK;
}

}  // namespace

extern "C" {

gsr_status gsr_sparse_adam(gsr_context* ctx, int64_t n, int32_t sh_degree, const uint32_t* cluster_visible,
                           const gsr_grads* params, const gsr_grads* grads, const gsr_grads* exp_avg,
                           const gsr_grads* exp_avg_sq, const gsr_adam_options* opts, void* stream) {
  if (!ctx) return GSR_ERR_INVALID_ARG;
  if (!grads) return fail(ctx, GSR_ERR_INVALID_ARG, "bad arguments to gsr_sparse_adam");
  gsr::AdamDev a;
  gsr_status st = build_adam(ctx, n, sh_degree, params, grads, exp_avg, exp_avg_sq, opts, a);
  if (st) return st;
  if (n == 0) return GSR_OK;
  DeviceGuard guard(ctx->device);
  gsr::launch_sparse_adam(a, cluster_visible, static_cast<hipStream_t>(stream));
  return check_hip(ctx, hipGetLastError(), "sparse adam");
}

gsr_status gsr_backward_adam(gsr_context* ctx, const gsr_scene* scene, const gsr_camera* cams, int32_t V,
                             const gsr_options* opts, void* workspace, size_t ws_bytes,
                             const float* const* dL_dimages, const gsr_grads* exp_avg, const gsr_grads* exp_avg_sq,
                             const gsr_adam_options* adam_opts, const gsr_stats* stats, void* stream) {
  if (!ctx) return GSR_ERR_INVALID_ARG;
  if (!scene) return fail(ctx, GSR_ERR_INVALID_ARG, "scene is NULL");
  gsr_grads params;
  params.means = const_cast<float*>(scene->means);
  params.log_scales = const_cast<float*>(scene->log_scales);
  params.quats = const_cast<float*>(scene->quats);
  params.opacity_logits = const_cast<float*>(scene->opacity_logits);
  params.sh = const_cast<float*>(scene->sh);
  gsr::AdamDev a;
  gsr_status st = build_adam(ctx, scene->n, scene->sh_degree, &params, nullptr, exp_avg, exp_avg_sq, adam_opts, a);
  if (st) return st;
  return backward_impl(ctx, scene, cams, V, opts, workspace, ws_bytes, dL_dimages, nullptr, stats, &a, stream);
}

gsr_status gsr_densify_workspace_size(gsr_context* ctx, int64_t n, int64_t max_candidates, size_t* bytes) {
  if (n < 0 || n >= ((int64_t)1 << 30) || max_candidates < 0 || !bytes)
    return fail(ctx, GSR_ERR_INVALID_ARG, "bad arguments to gsr_densify_workspace_size");
  *bytes = n == 0 ? kAlign : gsr::densify_words(n, std::min(max_candidates, n)) * 4 + kAlign;
  return GSR_OK;
}

gsr_status gsr_densify(gsr_context* ctx, const gsr_scene* scene, const float* metric, const float* noise,
                       const gsr_densify_options* opts, const gsr_grads* out, int64_t capacity, int32_t n_state,
                       const float* const* state_in, float* const* state_out, const int32_t* state_row_floats,
                       void* workspace, size_t ws_bytes, int64_t* n_out, void* stream) {
  if (!ctx) return GSR_ERR_INVALID_ARG;
  if (!scene || !opts || !out || n_state < 0 || n_state > gsr::kMaxDensCopy - 3 ||
      (n_state > 0 && (!state_in || !state_out || !state_row_floats)))
    return fail(ctx, GSR_ERR_INVALID_ARG, "bad arguments to gsr_densify");
  const int64_t n = scene->n;
  const gsr_densify_options& o = *opts;
  if (n < 0 || n >= ((int64_t)1 << 30) || scene->sh_degree < 0 || scene->sh_degree > 3)
    return fail(ctx, GSR_ERR_INVALID_ARG, "gsr_densify: bad scene size or degree");
  if (!(o.threshold > 0.0f) || !(o.split_factor > 0.0f) || std::isnan(o.split_log_scale) ||
      std::isnan(o.prune_logit) || o.max_candidates < 0)
    return fail(ctx, GSR_ERR_INVALID_ARG, "gsr_densify: need threshold > 0, split_factor > 0, max_candidates >= 0");
  const int64_t K = std::min(o.max_candidates, n);
  if (capacity < n + K) return fail(ctx, GSR_ERR_INVALID_ARG, "gsr_densify: capacity %lld < n + candidates %lld",
                                    (long long)capacity, (long long)(n + K));
  size_t need = 0;
  gsr_densify_workspace_size(ctx, n, K, &need);
  if (ws_bytes < need) {
    ctx->required = need;
    return fail(ctx, GSR_ERR_WORKSPACE_TOO_SMALL, "densify workspace %zu < %zu", ws_bytes, need);
  }
  if (!workspace || ((uintptr_t)workspace & (kAlign - 1)) != 0)
    return fail(ctx, GSR_ERR_INVALID_ARG, "gsr_densify: workspace must be 256-byte aligned");
  const int32_t K3 = 3 * (scene->sh_degree + 1) * (scene->sh_degree + 1);
  const float* in_p[5] = {scene->means, scene->log_scales, scene->quats, scene->opacity_logits, scene->sh};
  float* out_p[5] = {out->means, out->log_scales, out->quats, out->opacity_logits, out->sh};
  const int32_t rf[5] = {3, 3, 4, 1, K3};
  struct Extent {
    uintptr_t lo, hi;
  };
  std::vector<Extent> ins, outs;
  auto ext = [](const void* p, int64_t rows, int64_t floats) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    return Extent{a, a + uintptr_t(rows) * uintptr_t(floats) * 4};
  };
  for (int k = 0; k < 5; ++k) {
    if (n > 0 && (!in_p[k] || !out_p[k])) return fail(ctx, GSR_ERR_INVALID_ARG, "gsr_densify: null scene array");
    ins.push_back(ext(in_p[k], n, rf[k]));
    outs.push_back(ext(out_p[k], capacity, rf[k]));
  }
  if (n > 0 && (!metric || !noise)) return fail(ctx, GSR_ERR_INVALID_ARG, "gsr_densify: null metric or noise");
  ins.push_back(ext(metric, n, 1));
  ins.push_back(ext(noise, n, 6));
  for (int a = 0; a < n_state; ++a) {
    if (state_row_floats[a] <= 0 || (n > 0 && (!state_in[a] || !state_out[a])))
      return fail(ctx, GSR_ERR_INVALID_ARG, "gsr_densify: state array %d: bad pointer or row size", a);
    ins.push_back(ext(state_in[a], n, state_row_floats[a]));
    outs.push_back(ext(state_out[a], capacity, state_row_floats[a]));
  }
  outs.push_back(Extent{reinterpret_cast<uintptr_t>(workspace), reinterpret_cast<uintptr_t>(workspace) + need});
  if (n_out) outs.push_back(ext(n_out, 1, 2));
  auto meet = [](const Extent& x, const Extent& y) { return x.lo < y.hi && y.lo < x.hi; };
  for (size_t i = 0; i < outs.size(); ++i) {
    for (size_t j = i + 1; j < outs.size(); ++j)
      if (meet(outs[i], outs[j])) return fail(ctx, GSR_ERR_INVALID_ARG, "gsr_densify: outputs overlap");
    for (const Extent& e : ins)
      if (meet(outs[i], e)) return fail(ctx, GSR_ERR_INVALID_ARG, "gsr_densify: an output overlaps an input");
  }
  DeviceGuard guard(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n == 0) {
    if (n_out) gsr::fill_u32(reinterpret_cast<uint32_t*>(n_out), 2, 0u, s);
    return check_hip(ctx, hipGetLastError(), "densify");
  }
  gsr::DensifyArgs a{};
  a.n = n;
  a.max_candidates = K;
  a.metric = metric;
  a.noise = noise;
  a.means = scene->means;
  a.log_scales = scene->log_scales;
  a.quats = scene->quats;
  a.opacity_logits = scene->opacity_logits;
  a.threshold = o.threshold;
  a.split_log_scale = o.split_log_scale;
  a.prune_logit = o.prune_logit;
  a.ln_split_factor = std::log(double(o.split_factor));
  a.out_means = out->means;
  a.out_log_scales = out->log_scales;
  for (int k = 2; k < 5; ++k) {
    a.copy_in[a.n_copy] = in_p[k];
    a.copy_out[a.n_copy] = out_p[k];
    a.copy_rf[a.n_copy] = rf[k];
    a.copy_zero_new[a.n_copy] = 0;
    ++a.n_copy;
  }
  for (int q = 0; q < n_state; ++q) {
    a.copy_in[a.n_copy] = state_in[q];
    a.copy_out[a.n_copy] = state_out[q];
    a.copy_rf[a.n_copy] = state_row_floats[q];
    a.copy_zero_new[a.n_copy] = 1;
    ++a.n_copy;
  }
  a.n_out = n_out;
  gsr::densify(a, static_cast<uint32_t*>(workspace), s);
  return check_hip(ctx, hipGetLastError(), "densify");
}

gsr_status gsr_opacity_decay(gsr_context* ctx, float* opacity_logits, int64_t n, float factor, void* stream) {
  if (!ctx) return GSR_ERR_INVALID_ARG;
  if (n < 0 || (n > 0 && !opacity_logits) || !(factor > 0.0f && factor < 1.0f))
    return fail(ctx, GSR_ERR_INVALID_ARG, "bad arguments to gsr_opacity_decay (need 0 < factor < 1)");
  DeviceGuard guard(ctx->device);
  gsr::launch_opacity_decay(opacity_logits, n, double(factor), static_cast<hipStream_t>(stream));
  return check_hip(ctx, hipGetLastError(), "opacity decay");
}

gsr_status gsr_set_raster_split(gsr_context* ctx, uint32_t split_len, uint32_t split_len_bwd) {
  if (!ctx) return GSR_ERR_INVALID_ARG;
  ctx->split_len = split_len == 0 ? gsr::kSplitLen : split_len;
  ctx->split_len_bwd = split_len_bwd == 0 ? gsr::kSplitLenBwd : split_len_bwd;
  return GSR_OK;
}

gsr_status gsr_set_fault_injection(gsr_context* ctx, int32_t mode) {
  if (!ctx) return GSR_ERR_INVALID_ARG;
  if (mode != GSR_FAULT_NONE && mode != GSR_FAULT_ABORT_BEFORE_SORT && mode != GSR_FAULT_WITHHOLD_STATUS)
    return fail(ctx, GSR_ERR_INVALID_ARG, "unknown fault injection mode %d", mode);
  ctx->fault = mode;
  return GSR_OK;
}

gsr_status gsr_set_profiling(gsr_context* ctx, int enable) {
  if (!ctx) return GSR_ERR_INVALID_ARG;
  DeviceGuard guard(ctx->device);
  if (enable && !ctx->events_ready) {
    for (int k = 0; k < 2 * GSR_STAGE_COUNT; ++k) {
      gsr_status st = check_hip(ctx, hipEventCreate(&ctx->ev[k]), "create profiling events");
      if (st) return st;
    }
    ctx->events_ready = true;
  }
  ctx->profiling = enable != 0;
  return GSR_OK;
}

gsr_status gsr_stage_times(gsr_context* ctx, float* ms) {
  if (!ctx || !ms) return fail(ctx, GSR_ERR_INVALID_ARG, "bad arguments to gsr_stage_times");
  DeviceGuard guard(ctx->device);
  for (int k = 0; k < GSR_STAGE_COUNT; ++k) {
    ms[k] = -1.0f;
    if (!ctx->events_ready || !ctx->recorded[k]) continue;
    gsr_status st = check_hip(ctx, hipEventSynchronize(ctx->ev[2 * k + 1]), "wait for stage events");
    if (st) return st;
    if ((st = check_hip(ctx, hipEventElapsedTime(&ms[k], ctx->ev[2 * k], ctx->ev[2 * k + 1]), "stage time"))) return st;
  }
  return GSR_OK;
}

gsr_status gsr_morton_workspace_size(gsr_context* ctx, int64_t n, size_t* bytes) {
  if (!bytes || n < 0) return fail(ctx, GSR_ERR_INVALID_ARG, "bad arguments to gsr_morton_workspace_size");
  *bytes = gsr::morton_temp_words(n) * 4 + 1024;
  return GSR_OK;
}

gsr_status gsr_morton_order(gsr_context* ctx, const float* means, int64_t n, void* workspace, size_t ws_bytes,
                            int64_t* perm, uint64_t* codes, void* stream) {
  if (!ctx) return GSR_ERR_INVALID_ARG;
  if (n < 0 || n >= ((int64_t)1 << 30) || (n > 0 && (!means || !perm || !workspace)))
    return fail(ctx, GSR_ERR_INVALID_ARG, "bad arguments to gsr_morton_order");
  const size_t need = gsr::morton_temp_words(n) * 4 + 1024;
  if (ws_bytes < need) {
    ctx->required = need;
    return fail(ctx, GSR_ERR_WORKSPACE_TOO_SMALL, "morton workspace %zu < %zu", ws_bytes, need);
  }
  if (((uintptr_t)workspace & (kAlign - 1)) != 0) return fail(ctx, GSR_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  DeviceGuard guard(ctx->device);
  gsr::morton_order(means, n, static_cast<uint32_t*>(workspace), perm, codes, static_cast<hipStream_t>(stream));
  return check_hip(ctx, hipGetLastError(), "morton order");
}

namespace {
// Sort workspace: the error word (padded to 64 words), the control words, then one
// key and one value buffer of n for the passes that do not write the output.
size_t sort_ws_words(int64_t n, int bits) {
  const size_t ctl = (gsr::sort_ctl_words(std::max<int64_t>(n, 1), bits) + 63) & ~(size_t)63;
  return 64 + ctl + 2 * (((size_t)std::max<int64_t>(n, 1) + 63) & ~(size_t)63);
}
}  // namespace

gsr_status gsr_sort_workspace_size(gsr_context* ctx, int64_t n, int32_t bits, size_t* bytes) {
  if (!bytes || n < 0 || n >= ((int64_t)1 << 30) || bits < 1 || bits > 32)
    return fail(ctx, GSR_ERR_INVALID_ARG, "bad arguments to gsr_sort_workspace_size");
  *bytes = sort_ws_words(n, bits) * 4;
  return GSR_OK;
}

gsr_status gsr_sort_u32(gsr_context* ctx, const uint32_t* keys, const uint32_t* vals, int64_t n, int32_t bits,
                        uint32_t* out_keys, uint32_t* out_vals, void* workspace, size_t ws_bytes, void* stream) {
  if (!ctx) return GSR_ERR_INVALID_ARG;
  if (n < 0 || n >= ((int64_t)1 << 30) || bits < 1 || bits > 32 ||
      (n > 0 && (!keys || !out_keys || !out_vals || !workspace)))
    return fail(ctx, GSR_ERR_INVALID_ARG, "bad arguments to gsr_sort_u32");
  const uintptr_t all = (uintptr_t)keys | (uintptr_t)vals | (uintptr_t)out_keys | (uintptr_t)out_vals;
  if ((all & 3u) != 0) return fail(ctx, GSR_ERR_INVALID_ARG, "gsr_sort_u32: arrays need 4-byte alignment");
  auto overlap = [n](const void* a, const void* b) {
    const char *x = static_cast<const char*>(a), *y = static_cast<const char*>(b);
    return a && b && x < y + 4 * n && y < x + 4 * n;
  };
  if (overlap(out_keys, out_vals) || overlap(out_keys, keys) || overlap(out_keys, vals) ||
      overlap(out_vals, keys) || overlap(out_vals, vals))
    return fail(ctx, GSR_ERR_INVALID_ARG, "gsr_sort_u32: outputs overlap the inputs or each other");
  const size_t need = sort_ws_words(n, bits) * 4;
  if (ws_bytes < need) {
    ctx->required = need;
    return fail(ctx, GSR_ERR_WORKSPACE_TOO_SMALL, "sort workspace %zu < %zu", ws_bytes, need);
  }
  if (((uintptr_t)workspace & (kAlign - 1)) != 0) return fail(ctx, GSR_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  if (n == 0) return GSR_OK;
  DeviceGuard guard(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t* err = static_cast<uint32_t*>(workspace);
  const size_t ctl_words = (gsr::sort_ctl_words(n, bits) + 63) & ~(size_t)63;
  uint32_t* ctl = err + 64;
  uint32_t* tk = ctl + ctl_words;
  uint32_t* tv = tk + ((n + 63) & ~(int64_t)63);
  gsr::fill_u32(err, 64 + (int64_t)ctl_words, 0u, s);
  // the last pass writes the outputs: pass p writes buffer p & 1
  const int passes = (bits + 7) / 8;
  const int last = (passes - 1) & 1;
  uint32_t* kb[2] = {last == 0 ? out_keys : tk, last == 1 ? out_keys : tk};
  uint32_t* vb[2] = {last == 0 ? out_vals : tv, last == 1 ? out_vals : tv};
  gsr::radix_sort_u32_dev(keys, vals, kb, vb, n, nullptr, bits, ctl, err, false, s);
  return check_hip(ctx, hipGetLastError(), "sort");
}

gsr_status gsr_apply_permutation(gsr_context* ctx, const int64_t* perm, int64_t n, int32_t n_arrays,
                                 const float* const* src, float* const* dst, const int32_t* row_floats, void* stream) {
  if (!ctx) return GSR_ERR_INVALID_ARG;
  if (n < 0 || n_arrays < 0 || (n > 0 && n_arrays > 0 && (!perm || !src || !dst || !row_floats)))
    return fail(ctx, GSR_ERR_INVALID_ARG, "bad arguments to gsr_apply_permutation");
  for (int a = 0; a < n_arrays; ++a) {
    if (row_floats[a] < 0 || (n > 0 && row_floats[a] > 0 && (!src[a] || !dst[a])))
      return fail(ctx, GSR_ERR_INVALID_ARG, "array %d: bad pointer or row size", a);
    if (src[a] == dst[a] && n > 0 && row_floats[a] > 0)
      return fail(ctx, GSR_ERR_INVALID_ARG, "array %d: src and dst must not overlap", a);
  }
  DeviceGuard guard(ctx->device);
  for (int a = 0; a < n_arrays; ++a)
    gsr::launch_gather_rows(perm, n, src[a], dst[a], row_floats[a], static_cast<hipStream_t>(stream));
  return check_hip(ctx, hipGetLastError(), "apply permutation");
}

}  // extern "C"
