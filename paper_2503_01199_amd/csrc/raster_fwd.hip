// Forward raster: front-to-back alpha compositing (Sec. 3, Eq. (1)) of each
// tile's depth-ordered list, one wave64 per work item: a 16x16 tile, or one 16x4
// band of a tile whose list is long (the longest lists would otherwise set the
// launch's duration; a band item walks the same list for a quarter of the pixels).
//
// Each lane walks its 4-pixel strip with the scanline exponent (App. A.2). The
// tile's Gaussian records are staged through LDS in batches of 32 (one gather per
// lane, coalesced on the instance list, loaded straight into LDS and double
// buffered so the next batch arrives during the current one), then read by the
// whole wave as a broadcast. A pixel skips alpha < 1/255, clamps alpha at 0.99 and stops at the
// entry whose blend would take T below 1e-4 (that entry is not blended); the wave
// leaves the list once all its pixels have stopped.
//
// Outputs: the image (planar RGB, background composited behind), per pixel the
// final T and the list position + 1 of the last blended entry, from which the
// backward starts its back-to-front walk, and per instance a band mask (byte b
// nonzero where a live pixel of band b had alpha >= 1/255) that lets the backward
// skip bands and entries that blend nowhere. P selects the precision of alpha (FP32, or
// the packed-FP16 blend of Sec. 3.1.2).
#include "raster_common.h"

namespace gsr {
namespace {

// 32 records per batch: 3 KB of LDS per wave for the two buffers, so LDS no longer
// caps the waves a CU holds below what the registers allow.
constexpr int kBatch = 32;
using FwdBatch = BatchLDS<kBatch>;

// Exponent bound below which no pixel can reach alpha >= 1/255: o 2^e >= 1/255 needs
// e >= log2(1/255) - log2(o). The FP32 walk tests a band's exponents against this
// bound, less a margin of 2^-10 (a relative 6.8e-4 in o 2^e, far above the few ulp by
// which v_log_f32, v_exp_f32 and the product round), before it evaluates alpha: a
// band that fails for every lane cannot blend (its exact test would fail too), so it
// skips the quarter-rate exponential and the alpha arithmetic. The bound is computed
// once per batch, lane k for entry k, and read per entry from that lane.
constexpr float kLog2AlphaMinLessMargin = -7.99435343685885793f - 0.0009765625f;

// One work item of a frame (views, ranges, lists and records of that frame): tile
// gt whole (NB = 4 pixels per lane) or its band `band` (NB = 1); its image planes
// are images.p[img_base + view].
template <int P, int NB>
__device__ __forceinline__ void raster_fwd_item(FwdBatch& bufA, FwdBatch& bufB, const ViewDev* __restrict__ views,
                                                int32_t V, uint32_t gt, int band, const uint32_t* __restrict__ ranges,
                                                const uint32_t* __restrict__ inst_rec,
                                                uint32_t* __restrict__ inst_mask, const Record* __restrict__ rec,
                                                const ImagePtrs& images, int img_base, float* __restrict__ pix_T,
                                                uint32_t* __restrict__ pix_last) {
  const int v = view_of_tile(views, V, gt);
  const ViewDev& w = views[v];
  const int W = w.width, H = w.height;
  const int lt = (int)gt - w.tile_base;
  const int tx = lt % w.tiles_x, ty = lt / w.tiles_x;
  const int lane = threadIdx.x;
  float soff[NB], sg[NB];
  const LaneStrip q = lane_strip<NB>(w, tx, ty, band, lane, soff);
  const int px = q.px, py0 = q.py0, step = q.step;  // rows py0 + step j
  const float pxc = q.pxc, pyc = q.pyc;
  strip_sigmas<NB>(soff, sg);

  // A pixel blends an entry when alpha >= amin; amin is 1/255 while the pixel is
  // live and 2 (unreachable) once it has stopped or lies outside the image.
  float amin[NB], T[NB], cr[NB], cg[NB], cb[NB];
  uint32_t last[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    amin[j] = ((px < W) && (py0 + step * j < H)) ? kAlphaMin : 2.0f;
    T[j] = 1.0f;
    cr[j] = cg[j] = cb[j] = 0.0f;
    last[j] = 0;
  }
  // lm[j]: the lanes whose pixel j is live, as a wave mask (scalar registers),
  // refreshed by the bands that blend, so that the test for a wave with no live
  // pixel left takes no vector instruction
  uint64_t lm[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) lm[j] = __ballot(amin[j] < 1.0f);
  auto any_live = [&]() __attribute__((always_inline)) {
    uint64_t m = lm[0];
#pragma unroll
    for (int j = 1; j < NB; ++j) m |= lm[j];
    return m != 0;
  };
  const uint32_t s = ranges[2 * gt];
  const uint32_t e = ranges[2 * gt + 1];
  bool live = any_live();
  // Pipeline: record ids two batches ahead, records one batch ahead (in LDS).
  if (s < e) batch_fetch(bufA, rec, (lane < kBatch && s + lane < e) ? inst_rec[s + lane] : 0u);
  uint32_t r_next = (lane < kBatch && s + kBatch + lane < e) ? inst_rec[s + kBatch + lane] : 0u;
  constexpr bool kPrefilter = P == GSR_FP32;
  auto run_batch = [&](const FwdBatch& cur, FwdBatch& nxt, uint32_t b0) __attribute__((always_inline)) {
    __builtin_amdgcn_s_waitcnt(0);  // this batch's records have landed in LDS
    __syncthreads();
    // lane k: the exponent bound of entry k (lanes past the batch repeat an entry)
    const float eth_lane =
        kPrefilter ? kLog2AlphaMinLessMargin - __builtin_amdgcn_logf(cur.part[2][lane & (kBatch - 1)].x) : 0.0f;
    if (b0 + kBatch < e) batch_fetch(nxt, rec, r_next);
    r_next = (lane < kBatch && b0 + 2 * kBatch + lane < e) ? inst_rec[b0 + 2 * kBatch + lane] : 0u;
    const int cnt = (int)min((uint32_t)kBatch, e - b0);
    uint64_t bm[NB];  // bit k of bm[j]: band j has a live pixel with alpha >= 1/255 at entry b0 + k
#pragma unroll
    for (int j = 0; j < NB; ++j) bm[j] = 0;
    for (int k = 0; k < cnt; ++k) {
      const Record g = batch_get(cur, k);
      float ev[NB], dx, dy;
      strip_exponents<NB>(g, pxc, pyc, sg, ev, dx, dy);
      uint32_t pos1 = b0 - s + (uint32_t)k + 1u;
      asm volatile("" : "+v"(pos1));  // one register copy per entry, not one per band select
      float av[NB], Gv[NB], arv[NB];
      float eth = 0.0f;
      if constexpr (kPrefilter)
        eth = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, eth_lane), k));
      else
        strip_alpha<P, NB>(g.r2.x, ev, av, Gv, arv);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if constexpr (kPrefilter) {
          if (!__any(ev[j] >= eth)) continue;  // no pixel of the band can reach 1/255
          av[j] = alpha_of(g.r2.x, ev[j], Gv[j], arv[j]);
        }
        const float a = av[j];
        const bool ok = a >= amin[j];
        if (!__any(ok)) continue;  // nobody in this band blends the entry
        bm[j] |= 1ull << k;
        float Tn, wt0;
        if constexpr (P == GSR_FP16_BLEND_T) {
          // T kept in FP16 (T[j] holds an FP16 value; a is one too): T (1 - a) and a T
          // each one FP16 operation
          const _Float16 Th = (_Float16)T[j], ah = (_Float16)a;
          Tn = (float)__builtin_fmaf16(-Th, ah, Th);
          wt0 = (float)(ah * Th);
        } else {
          Tn = __builtin_fmaf(-T[j], a, T[j]);  // T (1 - a), one rounding
          wt0 = a * T[j];
        }
        const bool below = Tn < kTMin;  // one compare serves both outcomes
        const bool stop = ok && below;
        const bool blend = ok && !below;
        const float wt = blend ? wt0 : 0.0f;
        cr[j] = __builtin_fmaf(wt, g.r2.y, cr[j]);
        cg[j] = __builtin_fmaf(wt, g.r2.z, cg[j]);
        cb[j] = __builtin_fmaf(wt, g.r2.w, cb[j]);
        T[j] = blend ? Tn : T[j];
        last[j] = blend ? pos1 : last[j];
        amin[j] = stop ? 2.0f : amin[j];
        lm[j] = __ballot(amin[j] < 1.0f);
      }
      if (!any_live()) {
        live = false;
        break;
      }
    }
    // lane k stores entry k's mask, byte j for band j (entries past a break stay 0:
    // every pixel of the item has stopped before them)
    if (lane < cnt) {
      uint32_t mk = 0;
#pragma unroll
      for (int j = 0; j < NB; ++j) mk |= (uint32_t)((bm[j] >> lane) & 1ull) << (8 * j);
      if constexpr (NB == 4)
        inst_mask[b0 + lane] = mk;
      else
        reinterpret_cast<uint8_t*>(inst_mask)[4 * (size_t)(b0 + lane) + band] = (uint8_t)mk;
    }
  };
  for (uint32_t b0 = s; b0 < e && live; b0 += 2 * kBatch) {
    run_batch(bufA, bufB, b0);
    if (b0 + kBatch < e && live) run_batch(bufB, bufA, b0 + kBatch);
  }
  if (px >= W) return;
  float* img = images.p[img_base + v];
  const int64_t plane = (int64_t)W * H;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int py = py0 + step * j;
    if (py >= H) break;
    const int64_t o = (int64_t)py * W + px;
    img[o] = __builtin_fmaf(T[j], w.bg[0], cr[j]);
    img[plane + o] = __builtin_fmaf(T[j], w.bg[1], cg[j]);
    img[2 * plane + o] = __builtin_fmaf(T[j], w.bg[2], cb[j]);
    const int64_t pp = w.pixel_base + o;
    pix_T[pp] = T[j];
    pix_last[pp] = last[j];
  }
}

// Work item `item` of a frame: a whole tile or one band of a split tile.
template <int P>
__device__ __forceinline__ void raster_fwd_work(FwdBatch& bufA, FwdBatch& bufB, const ViewDev* views, int32_t V,
                                                uint32_t item, uint32_t tile_offset, const uint32_t* ranges,
                                                const uint32_t* inst_rec, uint32_t* inst_mask, const Record* rec,
                                                const ImagePtrs& images, int img_base, float* pix_T,
                                                uint32_t* pix_last) {
  const uint32_t gt = (item >> 3) - tile_offset;
  const uint32_t code = item & 7u;
  if (code == kItemWhole)
    raster_fwd_item<P, 4>(bufA, bufB, views, V, gt, 0, ranges, inst_rec, inst_mask, rec, images, img_base, pix_T,
                          pix_last);
  else
    raster_fwd_item<P, 1>(bufA, bufB, views, V, gt, (int)code, ranges, inst_rec, inst_mask, rec, images, img_base,
                          pix_T, pix_last);
}

// One frame: block b renders work item items[b] (blocks past the count leave).
template <int P>
__global__ __launch_bounds__(64) void k_raster_fwd(const ViewDev* __restrict__ views, int32_t V,
                                                   const uint32_t* __restrict__ items,
                                                   const uint32_t* __restrict__ header,
                                                   const uint32_t* __restrict__ ranges,
                                                   const uint32_t* __restrict__ inst_rec,
                                                   uint32_t* __restrict__ inst_mask,
                                                   const Record* __restrict__ rec, ImagePtrs images,
                                                   float* __restrict__ pix_T, uint32_t* __restrict__ pix_last) {
  __shared__ FwdBatch bufA, bufB;  // two objects, so reads of one never wait on loads into the other
  if (blockIdx.x >= header[kHdrItems] || frame_aborted(header)) return;
  raster_fwd_work<P>(bufA, bufB, views, V, items[blockIdx.x], 0, ranges, inst_rec, inst_mask, rec, images, 0,
                     pix_T, pix_last);
}

// Several prepared frames in one launch: block b renders work item order[b], whose
// tile indexes the frames' concatenated tiles (frame f owns [first[f], first[f+1])).
template <int P>
__global__ __launch_bounds__(64) void k_raster_fwd_batch(FrameTable tab, const uint32_t* __restrict__ order,
                                                         const uint32_t* __restrict__ n_items, ImagePtrs images) {
  __shared__ FwdBatch bufA, bufB;
  if (blockIdx.x >= *n_items) return;
  const uint32_t item = order[blockIdx.x];
  const uint32_t g = item >> 3;
  int f = 0;
  while (f + 1 < tab.n && tab.first[f + 1] <= g) ++f;
  const FrameRef& fr = tab.f[f];
  if (frame_aborted(fr.header)) return;  // that frame gave up: its lists may be garbage
  raster_fwd_work<P>(bufA, bufB, fr.views, fr.V, item, tab.first[f], fr.ranges, fr.inst_rec, fr.inst_mask, fr.rec,
                     images, fr.img_base, fr.pix_T, fr.pix_last);
}

}  // namespace

bool launch_raster_fwd_batch(const FrameTable& tab, const uint32_t* order, const uint32_t* n_items,
                             uint32_t total_tiles, const ImagePtrs& images, int precision, hipStream_t s,
                             hipEvent_t done) {
  if (total_tiles == 0) return false;
  const unsigned grid = (unsigned)max_items(total_tiles);
  if (precision == GSR_FP16_BLEND)
    launch_tracked(k_raster_fwd_batch<GSR_FP16_BLEND>, grid, 64, s, done, tab, order, n_items, images);
  else if (precision == GSR_FP16_BLEND_T)
    launch_tracked(k_raster_fwd_batch<GSR_FP16_BLEND_T>, grid, 64, s, done, tab, order, n_items, images);
  else
    launch_tracked(k_raster_fwd_batch<GSR_FP32>, grid, 64, s, done, tab, order, n_items, images);
  return true;
}

bool launch_raster_fwd(const Frame& f, const ImagePtrs& images, int precision, hipStream_t s, hipEvent_t done) {
  if (f.tiles <= 0) return false;
  const unsigned grid = (unsigned)max_items(f.tiles);
  const uint32_t* header = f.header;
  if (precision == GSR_FP16_BLEND)
    launch_tracked(k_raster_fwd<GSR_FP16_BLEND>, grid, 64, s, done, (const ViewDev*)f.views, f.V,
                   (const uint32_t*)f.tile_order, header, (const uint32_t*)f.ranges, (const uint32_t*)f.inst_rec,
                   f.inst_mask, (const Record*)f.rec, images, f.pix_T, f.pix_last);
  else if (precision == GSR_FP16_BLEND_T)
    launch_tracked(k_raster_fwd<GSR_FP16_BLEND_T>, grid, 64, s, done, (const ViewDev*)f.views, f.V,
                   (const uint32_t*)f.tile_order, header, (const uint32_t*)f.ranges, (const uint32_t*)f.inst_rec,
                   f.inst_mask, (const Record*)f.rec, images, f.pix_T, f.pix_last);
  else
    launch_tracked(k_raster_fwd<GSR_FP32>, grid, 64, s, done, (const ViewDev*)f.views, f.V,
                   (const uint32_t*)f.tile_order, header, (const uint32_t*)f.ranges, (const uint32_t*)f.inst_rec,
                   f.inst_mask, (const Record*)f.rec, images, f.pix_T, f.pix_last);
  return true;
}

}  // namespace gsr
