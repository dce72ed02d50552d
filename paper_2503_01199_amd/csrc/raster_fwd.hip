// Forward raster: front-to-back alpha compositing (Sec. 3, Eq. (1)) of each
// tile's depth-ordered list, one wave64 per 16x16 tile.
//
// Each lane walks its 4-pixel strip with the scanline exponent (App. A.2). The
// tile's Gaussian records are staged through LDS in batches of 64 (one gather per
// lane, coalesced on the instance list, loaded straight into LDS and double
// buffered so the next batch arrives during the current one), then read by the
// whole wave as a broadcast. A pixel skips alpha < 1/255, clamps alpha at 0.99 and stops at the
// entry whose blend would take T below 1e-4 (that entry is not blended); the wave
// leaves the list once all its pixels have stopped.
//
// Outputs: the image (planar RGB, background composited behind), and per pixel
// the final colour, T and the list position + 1 of the last blended entry, which
// the backward uses to bound its walk. The colour sum runs in FP64 (gfx950 issues
// an FP64 FMA at the rate of an unpacked FP32 one): the backward takes the colour
// behind an entry as this final colour minus the colour composited up to the
// entry, a difference that in FP32 would lose ~n ulps of the whole colour. P selects the precision of alpha (FP32, or
// the packed-FP16 blend of Sec. 3.1.2).
#include "raster_common.h"

namespace gsr {
namespace {

// One tile gt of a frame (views, ranges, lists and records of that frame); its
// image planes are images.p[img_base + view].
template <int P>
__device__ __forceinline__ void raster_fwd_tile(BatchLDS& bufA, BatchLDS& bufB, const ViewDev* __restrict__ views,
                                                int32_t V, uint32_t gt, const uint32_t* __restrict__ ranges,
                                                const uint32_t* __restrict__ inst_rec, const Record* __restrict__ rec,
                                                const ImagePtrs& images, int img_base, double* __restrict__ pix_rgb,
                                                float* __restrict__ pix_T, uint32_t* __restrict__ pix_last) {
  const int v = view_of_tile(views, V, gt);
  const ViewDev& w = views[v];
  const int W = w.width, H = w.height;
  const int lt = (int)gt - w.tile_base;
  const int tx = lt % w.tiles_x, ty = lt / w.tiles_x;
  const int lane = threadIdx.x;
  const int px = tx * GSR_TILE + (lane & 15);
  const int py0 = ty * GSR_TILE + (lane >> 4);  // rows py0 + 4 j
  const float pxc = (float)px + 0.5f;
  const float pyc = (float)py0 + kStripAnchor + 0.5f;

  // A pixel blends an entry when alpha >= amin; amin is 1/255 while the pixel is
  // live and 2 (unreachable) once it has stopped or lies outside the image.
  float amin[4], T[4];
  double cr[4], cg[4], cb[4];
  uint32_t last[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    amin[j] = ((px < W) && (py0 + kStripStep * j < H)) ? kAlphaMin : 2.0f;
    T[j] = 1.0f;
    cr[j] = cg[j] = cb[j] = 0.0f;
    last[j] = 0;
  }
  const uint32_t s = ranges[2 * gt];
  const uint32_t e = ranges[2 * gt + 1];
  bool live = __any(fminf(fminf(amin[0], amin[1]), fminf(amin[2], amin[3])) < 1.0f);
  // Pipeline: record ids two batches ahead, records one batch ahead (in LDS).
  if (s < e) batch_fetch(bufA, rec, (s + lane < e) ? inst_rec[s + lane] : 0u);
  uint32_t r_next = (s + 64 + lane < e) ? inst_rec[s + 64 + lane] : 0u;
  auto run_batch = [&](const BatchLDS& cur, BatchLDS& nxt, uint32_t b0) __attribute__((always_inline)) {
    __builtin_amdgcn_s_waitcnt(0);  // this batch's records have landed in LDS
    __syncthreads();
    if (b0 + 64 < e) batch_fetch(nxt, rec, r_next);
    r_next = (b0 + 128 + lane < e) ? inst_rec[b0 + 128 + lane] : 0u;
    const int cnt = (int)min(64u, e - b0);
    for (int k = 0; k < cnt; ++k) {
      const Record g = batch_get(cur, k);
      float ev[4], dx, dy;
      strip_exponents(g, pxc, pyc, ev, dx, dy);
      const uint32_t pos1 = b0 - s + (uint32_t)k + 1u;
      float av[4], Gv[4], arv[4];
      strip_alpha<P>(g.r2.x, ev, av, Gv, arv);
      const double cR = g.r2.y, cG = g.r2.z, cB = g.r2.w;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float a = av[j];
        const bool ok = a >= amin[j];
        if (!__any(ok)) continue;  // nobody in this band blends the entry
        const float Tn = T[j] * (1.0f - a);
        const bool stop = ok && (Tn < kTMin);
        const bool blend = ok && !stop;
        const float wt = blend ? a * T[j] : 0.0f;
        cr[j] = __builtin_fma((double)wt, cR, cr[j]);
        cg[j] = __builtin_fma((double)wt, cG, cg[j]);
        cb[j] = __builtin_fma((double)wt, cB, cb[j]);
        T[j] = blend ? Tn : T[j];
        last[j] = blend ? pos1 : last[j];
        amin[j] = stop ? 2.0f : amin[j];
      }
      if (!__any(fminf(fminf(amin[0], amin[1]), fminf(amin[2], amin[3])) < 1.0f)) {
        live = false;
        break;
      }
    }
  };
  for (uint32_t b0 = s; b0 < e && live; b0 += 128) {
    run_batch(bufA, bufB, b0);
    if (b0 + 64 < e && live) run_batch(bufB, bufA, b0 + 64);
  }
  if (px >= W) return;
  float* img = images.p[img_base + v];
  const int64_t plane = (int64_t)W * H;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int py = py0 + kStripStep * j;
    if (py >= H) break;
    const int64_t o = (int64_t)py * W + px;
    const double r = __builtin_fma((double)T[j], (double)w.bg[0], cr[j]);
    const double gg = __builtin_fma((double)T[j], (double)w.bg[1], cg[j]);
    const double b = __builtin_fma((double)T[j], (double)w.bg[2], cb[j]);
    img[o] = (float)r;
    img[plane + o] = (float)gg;
    img[2 * plane + o] = (float)b;
    const int64_t pp = w.pixel_base + o;
    pix_rgb[3 * pp + 0] = r;
    pix_rgb[3 * pp + 1] = gg;
    pix_rgb[3 * pp + 2] = b;
    pix_T[pp] = T[j];
    pix_last[pp] = last[j];
  }
}

template <int P>
__global__ __launch_bounds__(64) void k_raster_fwd(const ViewDev* __restrict__ views, int32_t V,
                                                   const uint32_t* __restrict__ tile_order,
                                                   const uint32_t* __restrict__ ranges,
                                                   const uint32_t* __restrict__ inst_rec,
                                                   const Record* __restrict__ rec, ImagePtrs images,
                                                   double* __restrict__ pix_rgb, float* __restrict__ pix_T,
                                                   uint32_t* __restrict__ pix_last) {
  __shared__ BatchLDS bufA, bufB;  // two objects, so reads of one never wait on loads into the other
  const uint32_t gt = tile_order ? tile_order[blockIdx.x] : blockIdx.x;
  raster_fwd_tile<P>(bufA, bufB, views, V, gt, ranges, inst_rec, rec, images, 0, pix_rgb, pix_T, pix_last);
}

// Several prepared frames in one launch: block b renders work item order[b], an
// index into the frames' concatenated tiles (frame f owns [first[f], first[f+1])).
template <int P>
__global__ __launch_bounds__(64) void k_raster_fwd_batch(FrameTable tab, const uint32_t* __restrict__ order,
                                                         ImagePtrs images) {
  __shared__ BatchLDS bufA, bufB;
  const uint32_t g = order[blockIdx.x];
  int f = 0;
  while (f + 1 < tab.n && tab.first[f + 1] <= g) ++f;
  const FrameRef& fr = tab.f[f];
  raster_fwd_tile<P>(bufA, bufB, fr.views, fr.V, g - tab.first[f], fr.ranges, fr.inst_rec, fr.rec, images,
                     fr.img_base, fr.pix_rgb, fr.pix_T, fr.pix_last);
}

}  // namespace

void launch_raster_fwd_batch(const FrameTable& tab, const uint32_t* order, uint32_t total_tiles,
                             const ImagePtrs& images, int precision, hipStream_t s) {
  if (total_tiles == 0) return;
  if (precision == GSR_FP16_BLEND)
    k_raster_fwd_batch<GSR_FP16_BLEND><<<total_tiles, 64, 0, s>>>(tab, order, images);
  else
    k_raster_fwd_batch<GSR_FP32><<<total_tiles, 64, 0, s>>>(tab, order, images);
}

void launch_raster_fwd(const Frame& f, const ImagePtrs& images, int precision, hipStream_t s) {
  if (f.tiles <= 0) return;
  if (precision == GSR_FP16_BLEND)
    k_raster_fwd<GSR_FP16_BLEND><<<(unsigned)f.tiles, 64, 0, s>>>(f.views, f.V, f.tile_order, f.ranges, f.inst_rec,
                                                                  f.rec, images, f.pix_rgb, f.pix_T, f.pix_last);
  else
    k_raster_fwd<GSR_FP32><<<(unsigned)f.tiles, 64, 0, s>>>(f.views, f.V, f.tile_order, f.ranges, f.inst_rec, f.rec,
                                                            images, f.pix_rgb, f.pix_T, f.pix_last);
}

}  // namespace gsr
