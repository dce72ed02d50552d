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
// Per lane, the exponent gradients of its strip are summed against j^0, j^1, j^2
// (App. A.2, Eq. (10)-(11)) and turned into gradients of the screen mean and
// conic at the strip's first pixel. The f_pixel and f_tile stages of App. A.1
// thus end in ONE wave reduction (DPP row shifts and row broadcasts) per
// (tile, Gaussian), and f_global is ONE atomic add per gradient per tile, issued
// as a single 11-lane atomic instruction on the record's contiguous 48-byte row.
#include "raster_common.h"

namespace gsr {
namespace {

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_move(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, true));
}

// Sum over the wave; the total lands in lane 63.
__device__ __forceinline__ float wave_sum_to_last(float x) {
  x += dpp_move<0x111, 0xf>(x);  // row_shr:1
  x += dpp_move<0x112, 0xf>(x);  // row_shr:2
  x += dpp_move<0x114, 0xf>(x);  // row_shr:4
  x += dpp_move<0x118, 0xf>(x);  // row_shr:8  -> lane 15 of each row holds the row sum
  x += dpp_move<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x += dpp_move<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3 -> lane 63 holds the total
  return x;
}

__device__ __forceinline__ float lane63(float x) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63)); }

__global__ __launch_bounds__(64) void k_raster_bwd(const ViewDev* __restrict__ views, int32_t V,
                                                   const uint32_t* __restrict__ ranges,
                                                   const uint32_t* __restrict__ inst_rec,
                                                   const Record* __restrict__ rec, ConstImagePtrs dL,
                                                   const float* __restrict__ pix_rgb,
                                                   const uint32_t* __restrict__ pix_last,
                                                   float* __restrict__ grad2d) {
  __shared__ Record batch[64];
  __shared__ uint32_t brec[64];
  const uint32_t gt = blockIdx.x;
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
  const int64_t plane = (int64_t)W * H;
  const float* g_img = dL.p[v];

  float gI[4][3], Rb[4][3], T[4];
  uint32_t last[4];
  uint32_t mymax = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    T[j] = 1.0f;
    last[j] = 0;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) gI[j][ch] = Rb[j][ch] = 0.0f;
    if (px < W && py0 + j < H) {
      const int64_t o = (int64_t)(py0 + j) * W + px;
      const int64_t pp = w.pixel_base + o;
      last[j] = pix_last[pp];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        gI[j][ch] = g_img[ch * plane + o];
        Rb[j][ch] = pix_rgb[3 * pp + ch];
      }
      mymax = max(mymax, last[j]);
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) mymax = max(mymax, (uint32_t)__shfl_xor((int)mymax, d, 64));
  const uint32_t s = ranges[2 * gt];
  const uint32_t e = min(ranges[2 * gt + 1], s + mymax);
  for (uint32_t b0 = s; b0 < e; b0 += 64) {
    const uint32_t idx = b0 + lane;
    __syncthreads();
    if (idx < e) {
      const uint32_t r = inst_rec[idx];
      brec[lane] = r;
      batch[lane] = rec[r];
    }
    __syncthreads();
    const int cnt = (int)min(64u, e - b0);
    for (int k = 0; k < cnt; ++k) {
      const Record g = batch[k];
      float ev[4], dx, dy;
      strip_exponents(g, pxc, pyc, ev, dx, dy);
      const uint32_t pos = b0 - s + (uint32_t)k;
      const float o = g.r2.x;
      float S0 = 0.f, S1 = 0.f, S2 = 0.f, dcr = 0.f, dcg = 0.f, dcb = 0.f, dop = 0.f, ss = 0.f, nfrag = 0.f;
      bool any = false;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float G, araw;
        const float a = alpha_of(o, ev[j], G, araw);
        const bool blend = (pos < last[j]) && (a >= kAlphaMin);
        if (blend) {
          const float wt = a * T[j];
          dcr = __builtin_fmaf(wt, gI[j][0], dcr);
          dcg = __builtin_fmaf(wt, gI[j][1], dcg);
          dcb = __builtin_fmaf(wt, gI[j][2], dcb);
          Rb[j][0] = __builtin_fmaf(-wt, g.r2.y, Rb[j][0]);
          Rb[j][1] = __builtin_fmaf(-wt, g.r2.z, Rb[j][1]);
          Rb[j][2] = __builtin_fmaf(-wt, g.r2.w, Rb[j][2]);
          const float gc = __builtin_fmaf(gI[j][2], g.r2.w, __builtin_fmaf(gI[j][1], g.r2.z, gI[j][0] * g.r2.y));
          const float gR = __builtin_fmaf(gI[j][2], Rb[j][2], __builtin_fmaf(gI[j][1], Rb[j][1], gI[j][0] * Rb[j][0]));
          const float one_m_a = 1.0f - a;
          const float dA = __builtin_fmaf(T[j], gc, -gR * __builtin_amdgcn_rcpf(one_m_a));
          const float dAr = (araw <= kAlphaMax) ? dA : 0.0f;
          const float go = dAr * G;
          const float dE = go * o;
          S0 += dE;
          S1 = __builtin_fmaf((float)j, dE, S1);
          S2 = __builtin_fmaf((float)(j * j), dE, S2);
          dop += go;
          ss = __builtin_fmaf(go, go, ss);
          nfrag += 1.0f;
          T[j] *= one_m_a;
          any = true;
        }
      }
      if (!__any(any)) continue;
      // exponent -> conic (a, b, c) and mean (u, v) gradients at the strip start:
      //   E_j = -1/2 (a dx^2 + 2 b dx (dy - j) + c (dy - j)^2), d = mean - pixel
      const float ca = -2.0f * (float)kLn2 * g.r1.x;
      const float cb = ca * g.r1.y;
      const float cc = -2.0f * (float)kLn2 * g.r1.w;
      const float gu = __builtin_fmaf(cb, S1, -__builtin_fmaf(ca, dx, cb * dy) * S0);
      const float gv = __builtin_fmaf(cc, S1, -__builtin_fmaf(cb, dx, cc * dy) * S0);
      const float ga = -0.5f * dx * dx * S0;
      const float gb = __builtin_fmaf(dx, S1, -dx * dy * S0);
      const float gcn = __builtin_fmaf(dy, S1, __builtin_fmaf(-0.5f * dy * dy, S0, -0.5f * S2));
      float vals[11] = {gu, gv, ga, gb, gcn, dop, dcr, dcg, dcb, ss, nfrag};
      float mine = 0.0f;
#pragma unroll
      for (int q = 0; q < 11; ++q) {
        const float tot = lane63(wave_sum_to_last(vals[q]));
        mine = (lane == q) ? tot : mine;
      }
      if (lane < 11) unsafeAtomicAdd(grad2d + (int64_t)brec[k] * kGrad2D + lane, mine);
    }
  }
}

}  // namespace

void launch_raster_bwd(const Frame& f, const ConstImagePtrs& dL, int precision, hipStream_t s) {
  (void)precision;
  if (f.tiles <= 0) return;
  k_raster_bwd<<<(unsigned)f.tiles, 64, 0, s>>>(f.views, f.V, f.ranges, f.inst_rec, f.rec, dL, f.pix_rgb,
                                                f.pix_last, f.grad2d);
}

}  // namespace gsr
