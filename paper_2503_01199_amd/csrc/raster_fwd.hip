// Forward raster: front-to-back alpha compositing (Sec. 3, Eq. (1)) of each
// tile's depth-ordered list, one wave64 per 16x16 tile.
//
// Each lane walks its 4-pixel strip with the scanline exponent (App. A.2). The
// tile's Gaussian records are staged through LDS in batches of 64 (one gather per
// lane, coalesced on the instance list), then read by the whole wave as a
// broadcast. A pixel skips alpha < 1/255, clamps alpha at 0.99 and stops at the
// entry whose blend would take T below 1e-4 (that entry is not blended); the wave
// leaves the list once all its pixels have stopped.
//
// Outputs: the image (planar RGB, background composited behind), and per pixel
// the final colour, T and the list position + 1 of the last blended entry, which
// the backward uses to bound its walk.
#include "raster_common.h"

namespace gsr {
namespace {

__global__ __launch_bounds__(64) void k_raster_fwd(const ViewDev* __restrict__ views, int32_t V,
                                                   const uint32_t* __restrict__ tile_order,
                                                   const uint32_t* __restrict__ ranges,
                                                   const uint32_t* __restrict__ inst_rec,
                                                   const Record* __restrict__ rec, ImagePtrs images,
                                                   float* __restrict__ pix_rgb, float* __restrict__ pix_T,
                                                   uint32_t* __restrict__ pix_last) {
  __shared__ Record batch[64];
  const uint32_t gt = tile_order ? tile_order[blockIdx.x] : blockIdx.x;
  const int v = view_of_tile(views, V, gt);
  const ViewDev& w = views[v];
  const int W = w.width, H = w.height;
  const int lt = (int)gt - w.tile_base;
  const int tx = lt % w.tiles_x, ty = lt / w.tiles_x;
  const int lane = threadIdx.x;
  const int px = tx * GSR_TILE + (lane & 15);
  const int py0 = ty * GSR_TILE + (lane >> 4) * 4;
  const float pxc = (float)px + 0.5f;
  const float pyc = (float)py0 + 0.5f;

  // A pixel blends an entry when alpha >= amin; amin is 1/255 while the pixel is
  // live and 2 (unreachable) once it has stopped or lies outside the image.
  float amin[4], T[4], cr[4], cg[4], cb[4];
  uint32_t last[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    amin[j] = ((px < W) && (py0 + j < H)) ? kAlphaMin : 2.0f;
    T[j] = 1.0f;
    cr[j] = cg[j] = cb[j] = 0.0f;
    last[j] = 0;
  }
  const uint32_t s = ranges[2 * gt];
  const uint32_t e = ranges[2 * gt + 1];
  bool live = __any(fminf(fminf(amin[0], amin[1]), fminf(amin[2], amin[3])) < 1.0f);
  // Record gathers are pipelined: ids two batches ahead, records one batch ahead.
  uint32_t r_next = (s + 64 + lane < e) ? inst_rec[s + 64 + lane] : 0u;
  Record g_cur = {};
  if (s + lane < e) g_cur = rec[inst_rec[s + lane]];
  for (uint32_t b0 = s; b0 < e && live; b0 += 64) {
    __syncthreads();
    batch[lane] = g_cur;
    __syncthreads();
    if (b0 + 64 + lane < e) g_cur = rec[r_next];
    r_next = (b0 + 128 + lane < e) ? inst_rec[b0 + 128 + lane] : 0u;
    const int cnt = (int)min(64u, e - b0);
    for (int k = 0; k < cnt; ++k) {
      const Record g = batch[k];
      float ev[4], dx, dy;
      strip_exponents(g, pxc, pyc, ev, dx, dy);
      const uint32_t pos1 = b0 - s + (uint32_t)k + 1u;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float G, araw;
        const float a = alpha_of(g.r2.x, ev[j], G, araw);
        const bool ok = a >= amin[j];
        const float Tn = T[j] * (1.0f - a);
        const bool stop = ok && (Tn < kTMin);
        const bool blend = ok && !stop;
        const float wt = blend ? a * T[j] : 0.0f;
        cr[j] = __builtin_fmaf(wt, g.r2.y, cr[j]);
        cg[j] = __builtin_fmaf(wt, g.r2.z, cg[j]);
        cb[j] = __builtin_fmaf(wt, g.r2.w, cb[j]);
        T[j] = blend ? Tn : T[j];
        last[j] = blend ? pos1 : last[j];
        amin[j] = stop ? 2.0f : amin[j];
      }
      if (!__any(fminf(fminf(amin[0], amin[1]), fminf(amin[2], amin[3])) < 1.0f)) {
        live = false;
        break;
      }
    }
  }
  if (px >= W) return;
  float* img = images.p[v];
  const int64_t plane = (int64_t)W * H;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int py = py0 + j;
    if (py >= H) break;
    const int64_t o = (int64_t)py * W + px;
    const float r = __builtin_fmaf(T[j], w.bg[0], cr[j]);
    const float gg = __builtin_fmaf(T[j], w.bg[1], cg[j]);
    const float b = __builtin_fmaf(T[j], w.bg[2], cb[j]);
    img[o] = r;
    img[plane + o] = gg;
    img[2 * plane + o] = b;
    const int64_t pp = w.pixel_base + o;
    pix_rgb[3 * pp + 0] = r;
    pix_rgb[3 * pp + 1] = gg;
    pix_rgb[3 * pp + 2] = b;
    pix_T[pp] = T[j];
    pix_last[pp] = last[j];
  }
}

}  // namespace

void launch_raster_fwd(const Frame& f, const ImagePtrs& images, int precision, hipStream_t s) {
  (void)precision;
  if (f.tiles <= 0) return;
  k_raster_fwd<<<(unsigned)f.tiles, 64, 0, s>>>(f.views, f.V, f.tile_order, f.ranges, f.inst_rec, f.rec, images,
                                                f.pix_rgb, f.pix_T, f.pix_last);
}

}  // namespace gsr
