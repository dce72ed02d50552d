// Backward raster: per-Gaussian screen-space gradients (Sec. 3, Eq. (3);
// App. A.1) and the opacity-gradient statistic (Sec. 3.3), one wave64 per work item
// (a tile, or two 16x4 bands of a tile with a long list).
//
// The wave walks its tile's list back to front, from the furthest pixel's last
// blended entry, recomputing alpha as the forward did; an entry is blended at a
// pixel when it lies before the pixel's last blended position and alpha >= 1/255
// (the forward's decisions). Each pixel starts from the forward's final T and the
// colour behind its last entry, T_final bg. For each blended (pixel, Gaussian) pair
// the T before the entry is T after it divided by (1 - alpha), and with the colour
// behind it R (a running sum of the later entries' contributions, so its rounding
// stays relative to R itself) and the upstream gradient g = dL/dI:
//   dL/dc     += T alpha g                                  (Eq. (3))
//   dL/dalpha  = T (g . c) - (g . R) / (1 - alpha)
//   g_o        = dL/dalpha * G  (zero where alpha is clamped)  -> statistic S, M, C
//   dL/dE      = g_o * o
// Per lane, the exponent gradients of its strip are summed against s^0, s^1, s^2,
// s the row offset from the strip's anchor (App. A.2, Eq. (10)-(11)) and turned into gradients of the screen mean and
// conic at the strip's anchor. The f_pixel and f_tile stages of App. A.1
// thus end in ONE wave reduction (DPP row shifts and row broadcasts) per
// (tile, Gaussian), and f_global is ONE atomic add per gradient per tile, issued
// as a single 11-lane atomic instruction on the record's contiguous 48-byte row.
#include "raster_common.h"

namespace gsr {
namespace {

template <int CTRL>
__device__ __forceinline__ float dpp_row_shr(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, true));
}

// v_permlane32_swap / v_permlane16_swap (gfx950): exchange the upper 32 lanes of the
// first operand with the lower 32 lanes of the second, resp. the odd 16-lane rows
// of the first with the even rows of the second.
__device__ __forceinline__ void swap32(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}
__device__ __forceinline__ void swap16(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}

// Transposed wave reduction of 12 per-lane values v[0..11]. Two swap-and-add
// stages halve the registers while halving the lanes each value spans (so each
// add reduces two values at once), then a 4-step DPP row reduction finishes the
// 16-lane rows. On return w[i] holds, in lanes 15, 31, 47 and 63, the wave totals
// of values 4i, 4i+2, 4i+1 and 4i+3.
__device__ __forceinline__ void wave_reduce12(float v[12], float w[3]) {
  float u[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    float a = v[2 * i], b = v[2 * i + 1];
    swap32(a, b);
    u[i] = a + b;  // lanes 0-31: value 2i, lanes 32-63: value 2i+1
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    float a = u[2 * i], b = u[2 * i + 1];
    swap16(a, b);
    w[i] = a + b;  // rows 0, 1, 2, 3: values 4i, 4i+2, 4i+1, 4i+3
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) w[i] += dpp_row_shr<0x111>(w[i]);
#pragma unroll
  for (int i = 0; i < 3; ++i) w[i] += dpp_row_shr<0x112>(w[i]);
#pragma unroll
  for (int i = 0; i < 3; ++i) w[i] += dpp_row_shr<0x114>(w[i]);
#pragma unroll
  for (int i = 0; i < 3; ++i) w[i] += dpp_row_shr<0x118>(w[i]);
}

// One work item: tile gt whole (NB = 4 pixels per lane), or its two bands from
// `band` on (NB = 2, at their row offsets from the whole strip's anchor).
template <int P, int NB>
__device__ __forceinline__ void raster_bwd_item(BatchLDS& bufA, BatchLDS& bufB, uint32_t* recA, uint32_t* recB,
                                                const ViewDev* __restrict__ views, int32_t V, uint32_t gt, int band,
                                                const uint32_t* __restrict__ ranges,
                                                const uint32_t* __restrict__ inst_rec,
                                                const Record* __restrict__ rec, const ConstImagePtrs& dL,
                                                const float* __restrict__ pix_T,
                                                const uint32_t* __restrict__ pix_last, float* __restrict__ grad2d) {
  const int v = view_of_tile(views, V, gt);
  const ViewDev& w = views[v];
  const int W = w.width, H = w.height;
  const int lt = (int)gt - w.tile_base;
  const int tx = lt % w.tiles_x, ty = lt / w.tiles_x;
  const int lane = threadIdx.x;
  const int px = tx * GSR_TILE + (lane & 15);
  const int ys = ty * GSR_TILE + (lane >> 4);  // first row of the lane's whole-tile strip
  const int py0 = ys + kStripStep * band;      // rows py0 + 4 j
  const float pxc = (float)px + 0.5f;
  const float pyc = (float)ys + kStripAnchor + 0.5f;
  float soff[NB];
  strip_offsets<NB>(band, soff);
  const int64_t plane = (int64_t)W * H;
  const float* g_img = dL.p[v];

  // Per pixel: upstream gradient g, T after the entries walked so far (from the
  // back), g . (colour behind the next entry), and the list position after its
  // last blend.
  float gI[NB][3], T[NB], gR[NB];
  uint32_t last[NB];
  uint32_t mymax = 0;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    T[j] = 1.0f;
    gR[j] = 0.0f;
    last[j] = 0;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) gI[j][ch] = 0.0f;
    if (px < W && py0 + kStripStep * j < H) {
      const int64_t o = (int64_t)(py0 + kStripStep * j) * W + px;
      const int64_t pp = w.pixel_base + o;
      last[j] = pix_last[pp];
      T[j] = pix_T[pp];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) gI[j][ch] = g_img[ch * plane + o];
      gR[j] = T[j] * __builtin_fmaf(gI[j][2], w.bg[2], __builtin_fmaf(gI[j][1], w.bg[1], gI[j][0] * w.bg[0]));
      mymax = max(mymax, last[j]);
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) mymax = max(mymax, (uint32_t)__shfl_xor((int)mymax, d, 64));
  const uint32_t s = ranges[2 * gt];
  const uint32_t e = min(ranges[2 * gt + 1], s + mymax);
  if (e <= s) return;

  // Batches from the back: the first one processed starts at the last multiple of 64
  // below e. Pipeline as in the forward, in reverse: record ids two batches ahead,
  // records one batch ahead (in LDS).
  const uint32_t first = s + ((e - s - 1) / 64) * 64;
  {
    const uint32_t r0 = (first + lane < e) ? inst_rec[first + lane] : 0u;
    batch_fetch(bufA, rec, r0);
    recA[lane] = r0;
  }
  uint32_t r_next = (first >= s + 64) ? inst_rec[first - 64 + lane] : 0u;
  // per-entry accumulators; zero at the start and again after each reduction that
  // consumes them (an entry that blends nowhere leaves them at zero)
  float S0 = 0.f, S1 = 0.f, S2 = 0.f, dcr = 0.f, dcg = 0.f, dcb = 0.f, dop = 0.f, ss = 0.f, nfrag = 0.f;
  auto run_batch = [&](const BatchLDS& cur, const uint32_t* cur_rec, BatchLDS& nxt, uint32_t* nxt_rec,
                       uint32_t b0) __attribute__((always_inline)) {
    __builtin_amdgcn_s_waitcnt(0);  // this batch's records have landed in LDS
    __syncthreads();
    if (b0 >= s + 64) {
      batch_fetch(nxt, rec, r_next);
      nxt_rec[lane] = r_next;
    }
    r_next = (b0 >= s + 128) ? inst_rec[b0 - 128 + lane] : 0u;
    const int cnt = (int)min(64u, e - b0);
    for (int k = cnt - 1; k >= 0; --k) {
      const Record g = batch_get(cur, k);
      float ev[NB], dx, dy;
      strip_exponents<NB>(g, pxc, pyc, soff, ev, dx, dy);
      const uint32_t pos = b0 - s + (uint32_t)k;
      const float o = g.r2.x;
      float av[NB], Gv[NB], arv[NB];
      strip_alpha<P, NB>(o, ev, av, Gv, arv);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const float a = av[j], G = Gv[j], araw = arv[j];
        const bool blend = (pos < last[j]) && (a >= kAlphaMin);
        if (blend) {
          nfrag += 1.0f;
          const float inv = __builtin_amdgcn_rcpf(1.0f - a);
          const float Tb = T[j] * inv;  // T before this entry
          const float wt = a * Tb;
          const float gc = __builtin_fmaf(gI[j][2], g.r2.w, __builtin_fmaf(gI[j][1], g.r2.z, gI[j][0] * g.r2.y));
          dcr = __builtin_fmaf(wt, gI[j][0], dcr);
          dcg = __builtin_fmaf(wt, gI[j][1], dcg);
          dcb = __builtin_fmaf(wt, gI[j][2], dcb);
          // dL/dalpha = T (g . c) - (g . colour behind) / (1 - alpha)
          const float dA = __builtin_fmaf(Tb, gc, -gR[j] * inv);
          const float go = (araw <= alpha_clamp<P>()) ? dA * G : 0.0f;
          const float dE = go * o;
          S0 += dE;
          S1 = __builtin_fmaf(soff[j], dE, S1);
          S2 = __builtin_fmaf(soff[j] * soff[j], dE, S2);
          dop += go;
          ss = __builtin_fmaf(go, go, ss);
          gR[j] = __builtin_fmaf(wt, gc, gR[j]);  // now the colour behind the previous entry
          T[j] = Tb;
        }
      }
      if (!__any(nfrag > 0.0f)) continue;  // nobody blended this entry
      // exponent -> conic (a, b, c) and mean (u, v) gradients at the strip anchor
      // (pixel j is s_j rows below it):
      //   E_j = -1/2 (a dx^2 + 2 b dx (dy - s_j) + c (dy - s_j)^2), d = mean - anchor
      const float ca = -2.0f * (float)kLn2 * g.r1.x;
      const float cb = ca * g.r1.y;
      const float cc = -2.0f * (float)kLn2 * g.r1.w;
      const float gu = __builtin_fmaf(cb, S1, -__builtin_fmaf(ca, dx, cb * dy) * S0);
      const float gv = __builtin_fmaf(cc, S1, -__builtin_fmaf(cb, dx, cc * dy) * S0);
      const float ga = -0.5f * dx * dx * S0;
      const float gb = __builtin_fmaf(dx, S1, -dx * dy * S0);
      const float gcn = __builtin_fmaf(dy, S1, __builtin_fmaf(-0.5f * dy * dy, S0, -0.5f * S2));
      float vals[12] = {gu, gv, ga, gb, gcn, dop, dcr, dcg, dcb, ss, nfrag, 0.0f};
      float tot[3];
      wave_reduce12(vals, tot);
      S0 = S1 = S2 = dcr = dcg = dcb = dop = ss = nfrag = 0.f;
      // lanes 15, 31, 47, 63 of tot[i] hold slots 4i, 4i+2, 4i+1, 4i+3 (slot 11 is padding)
      if ((lane & 15) == 15) {
        const int row = lane >> 4;
        const int sub = (row == 0) ? 0 : (row == 1) ? 2 : (row == 2) ? 1 : 3;
        float* dst = grad2d + (int64_t)cur_rec[k] * kGrad2D + sub;
        unsafeAtomicAdd(dst, tot[0]);
        unsafeAtomicAdd(dst + 4, tot[1]);
        if (sub != 3) unsafeAtomicAdd(dst + 8, tot[2]);
      }
    }
  };
  for (int64_t b0 = first; b0 >= (int64_t)s; b0 -= 128) {
    run_batch(bufA, recA, bufB, recB, (uint32_t)b0);
    if (b0 >= (int64_t)s + 64) run_batch(bufB, recB, bufA, recA, (uint32_t)(b0 - 64));
  }
}

template <int P>
__global__ __launch_bounds__(64) void k_raster_bwd(const ViewDev* __restrict__ views, int32_t V,
                                                   const uint32_t* __restrict__ items,
                                                   const uint32_t* __restrict__ n_items,
                                                   const uint32_t* __restrict__ ranges,
                                                   const uint32_t* __restrict__ inst_rec,
                                                   const Record* __restrict__ rec, ConstImagePtrs dL,
                                                   const float* __restrict__ pix_T,
                                                   const uint32_t* __restrict__ pix_last,
                                                   float* __restrict__ grad2d) {
  __shared__ BatchLDS bufA, bufB;  // two objects, so reads of one never wait on loads into the other
  __shared__ uint32_t recA[64], recB[64];
  if (blockIdx.x >= *n_items) return;
  const uint32_t item = items[blockIdx.x];
  const uint32_t gt = item >> 3;
  const uint32_t code = item & 7u;
  if (code == kItemWhole)
    raster_bwd_item<P, 4>(bufA, bufB, recA, recB, views, V, gt, 0, ranges, inst_rec, rec, dL, pix_T, pix_last,
                          grad2d);
  else  // half of a split tile
    raster_bwd_item<P, 2>(bufA, bufB, recA, recB, views, V, gt, 2 * (int)(code - kItemHalf), ranges, inst_rec, rec,
                          dL, pix_T, pix_last, grad2d);
}

}  // namespace

void launch_raster_bwd(const Frame& f, const ConstImagePtrs& dL, int precision, hipStream_t s) {
  if (f.tiles <= 0) return;
  const unsigned grid = (unsigned)max_items(f.tiles);
  const uint32_t* n_items = f.header + kHdrItemsBwd;
  if (precision == GSR_FP16_BLEND)
    k_raster_bwd<GSR_FP16_BLEND><<<grid, 64, 0, s>>>(f.views, f.V, f.bwd_items, n_items, f.ranges, f.inst_rec,
                                                     f.rec, dL, f.pix_T, f.pix_last, f.grad2d);
  else
    k_raster_bwd<GSR_FP32><<<grid, 64, 0, s>>>(f.views, f.V, f.bwd_items, n_items, f.ranges, f.inst_rec, f.rec, dL,
                                               f.pix_T, f.pix_last, f.grad2d);
}

}  // namespace gsr
