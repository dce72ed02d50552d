// Backward raster: per-Gaussian screen-space gradients (Sec. 3, Eq. (3);
// App. A.1) and the opacity-gradient statistic (Sec. 3.3), one wave64 per tile.
//
// The wave re-walks its tile's list front to back up to the furthest pixel's last
// blended entry, recomputing alpha and T exactly as the forward did. For each
// blended (pixel, Gaussian) pair with T before the entry, the colour behind it R
// (final colour minus everything composited up to and including the entry) and
// the upstream gradient g = dL/dI:
//   dL/dc     += T alpha g                                  (Eq. (3))
//   dL/dalpha  = T (g . c) - (g . R) / (1 - alpha)
//   g_o        = dL/dalpha * G  (zero where alpha is clamped)  -> statistic S, M, C
//   dL/dE      = g_o * o
// Per lane, the exponent gradients of its strip are summed against s^0, s^1, s^2,
// s the row offset from the strip's anchor (App. A.2, Eq. (10)-(11)) and turned into gradients of the screen mean and
// conic at the strip's first pixel. The f_pixel and f_tile stages of App. A.1
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

template <int P>
__global__ __launch_bounds__(64) void k_raster_bwd(const ViewDev* __restrict__ views, int32_t V,
                                                   const uint32_t* __restrict__ tile_order,
                                                   const uint32_t* __restrict__ ranges,
                                                   const uint32_t* __restrict__ inst_rec,
                                                   const Record* __restrict__ rec, ConstImagePtrs dL,
                                                   const double* __restrict__ pix_rgb,
                                                   const uint32_t* __restrict__ pix_last,
                                                   float* __restrict__ grad2d) {
  __shared__ BatchLDS bufA, bufB;  // two objects, so reads of one never wait on loads into the other
  __shared__ uint32_t recA[64], recB[64];
  const uint32_t gt = tile_order ? tile_order[blockIdx.x] : blockIdx.x;
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
  const int64_t plane = (int64_t)W * H;
  const float* g_img = dL.p[v];

  // Per pixel: upstream gradient g, g . I_final, g . (colour composited so far), T
  // and the list position after its last blend. The colour behind entry k is
  // I_final - C_{<=k}, so g . (colour behind) = gIf - gC; both run in FP64, as the
  // forward's colour sum does, so the difference keeps its relative precision
  // behind entries near the front of deep lists.
  float gI[4][3], T[4];
  double gIf[4], gC[4];
  uint32_t last[4];
  uint32_t mymax = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    T[j] = 1.0f;
    gC[j] = 0.0;
    gIf[j] = 0.0;
    last[j] = 0;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) gI[j][ch] = 0.0f;
    if (px < W && py0 + kStripStep * j < H) {
      const int64_t o = (int64_t)(py0 + kStripStep * j) * W + px;
      const int64_t pp = w.pixel_base + o;
      last[j] = pix_last[pp];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        gI[j][ch] = g_img[ch * plane + o];
        gIf[j] = __builtin_fma((double)gI[j][ch], pix_rgb[3 * pp + ch], gIf[j]);
      }
      mymax = max(mymax, last[j]);
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) mymax = max(mymax, (uint32_t)__shfl_xor((int)mymax, d, 64));
  const uint32_t s = ranges[2 * gt];
  const uint32_t e = min(ranges[2 * gt + 1], s + mymax);

  // Pipeline: record ids two batches ahead, records one batch ahead (in LDS).
  if (s < e) {
    const uint32_t r0 = (s + lane < e) ? inst_rec[s + lane] : 0u;
    batch_fetch(bufA, rec, r0);
    recA[lane] = r0;
  }
  uint32_t r_next = (s + 64 + lane < e) ? inst_rec[s + 64 + lane] : 0u;
  auto run_batch = [&](const BatchLDS& cur, const uint32_t* cur_rec, BatchLDS& nxt, uint32_t* nxt_rec,
                       uint32_t b0) __attribute__((always_inline)) {
    __builtin_amdgcn_s_waitcnt(0);  // this batch's records have landed in LDS
    __syncthreads();
    if (b0 + 64 < e) {
      batch_fetch(nxt, rec, r_next);
      nxt_rec[lane] = r_next;
    }
    r_next = (b0 + 128 + lane < e) ? inst_rec[b0 + 128 + lane] : 0u;
    const int cnt = (int)min(64u, e - b0);
    for (int k = 0; k < cnt; ++k) {
      const Record g = batch_get(cur, k);
      float ev[4], dx, dy;
      strip_exponents(g, pxc, pyc, ev, dx, dy);
      const uint32_t pos = b0 - s + (uint32_t)k;
      const float o = g.r2.x;
      float S0 = 0.f, S1 = 0.f, S2 = 0.f, dcr = 0.f, dcg = 0.f, dcb = 0.f, dop = 0.f, ss = 0.f, nfrag = 0.f;
      float av[4], Gv[4], arv[4];
      strip_alpha<P>(o, ev, av, Gv, arv);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float a = av[j], G = Gv[j], araw = arv[j];
        const bool blend = (pos < last[j]) && (a >= kAlphaMin);
        if (blend) {
          nfrag += 1.0f;
          const float wt = a * T[j];
          const float gc = __builtin_fmaf(gI[j][2], g.r2.w, __builtin_fmaf(gI[j][1], g.r2.z, gI[j][0] * g.r2.y));
          dcr = __builtin_fmaf(wt, gI[j][0], dcr);
          dcg = __builtin_fmaf(wt, gI[j][1], dcg);
          dcb = __builtin_fmaf(wt, gI[j][2], dcb);
          gC[j] = __builtin_fma((double)wt, (double)gc, gC[j]);
          const float one_m_a = 1.0f - a;
          const float behind = (float)(gIf[j] - gC[j]);  // g . (colour behind this entry)
          // dL/dalpha = T (g . c) - (g . colour behind) / (1 - alpha)
          const float dA = __builtin_fmaf(T[j], gc, -behind * __builtin_amdgcn_rcpf(one_m_a));
          const float go = (araw <= alpha_clamp<P>()) ? dA * G : 0.0f;
          const float dE = go * o;
          S0 += dE;
          S1 = __builtin_fmaf(kStripOffset[j], dE, S1);
          S2 = __builtin_fmaf(kStripOffset[j] * kStripOffset[j], dE, S2);
          dop += go;
          ss = __builtin_fmaf(go, go, ss);
          T[j] *= one_m_a;
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
  for (uint32_t b0 = s; b0 < e; b0 += 128) {
    run_batch(bufA, recA, bufB, recB, b0);
    if (b0 + 64 < e) run_batch(bufB, recB, bufA, recA, b0 + 64);
  }
}

}  // namespace

void launch_raster_bwd(const Frame& f, const ConstImagePtrs& dL, int precision, hipStream_t s) {
  if (f.tiles <= 0) return;
  if (precision == GSR_FP16_BLEND)
    k_raster_bwd<GSR_FP16_BLEND><<<(unsigned)f.tiles, 64, 0, s>>>(f.views, f.V, f.tile_order, f.ranges, f.inst_rec,
                                                                  f.rec, dL, f.pix_rgb, f.pix_last, f.grad2d);
  else
    k_raster_bwd<GSR_FP32><<<(unsigned)f.tiles, 64, 0, s>>>(f.views, f.V, f.tile_order, f.ranges, f.inst_rec, f.rec,
                                                            dL, f.pix_rgb, f.pix_last, f.grad2d);
}

}  // namespace gsr
