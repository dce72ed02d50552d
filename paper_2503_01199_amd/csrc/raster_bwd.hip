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
// Per lane, the opacity gradients of its strip are summed against s^0, s^1, s^2,
// s the row offset from the strip's anchor (App. A.2, Eq. (10)-(11)); times o they
// are the exponent-gradient sums, turned into gradients of the screen mean and
// conic at the anchor. The f_pixel and f_tile stages of App. A.1 thus end in ONE
// transposed wave reduction (permlane swaps, then DPP row shifts) per (tile,
// Gaussian); the fragment count is a popcount of the blend masks on the scalar
// unit. f_global is ONE atomic add per gradient per tile, issued as three 4-lane
// atomic instructions on the record's contiguous 48-byte row (FP32), or, for a
// bitwise reproducible backward, on its 96-byte row of 64-bit fixed-point sums.
#include <algorithm>

#include "raster_common.h"

namespace gsr {
namespace {

constexpr int kBatch = 64;  // records per LDS batch
// Entries whose wave totals are staged in LDS before one pass turns them into
// gradients and issues their atomics (a divisor of kBatch).
constexpr int kGroup = 16;
static_assert(kBatch % kGroup == 0 && kGroup <= 16, "a group's atomics take one pass of four lanes per entry");

// Deterministic backward: per-tile sums become two's-complement fixed point (round
// to nearest, saturating) at the frame's scale (grad_exponent), so that the
// device-wide integer sum does not depend on the order in which tiles add.
__device__ __forceinline__ unsigned long long to_fixed(float v, float scale) {
  const float x = fminf(fmaxf(v * scale, -0x1p63f), 0x1.fffffep62f);
  return (unsigned long long)(long long)__builtin_rintf(x);
}
using BwdBatch = BatchLDS<kBatch>;

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

// Transposed wave reduction of 10 per-lane values v[0..9] (slots 10 and 11 are
// zero). Two swap-and-add stages halve the registers while halving the lanes each
// value spans (so each add reduces two values at once), then a 4-step DPP row
// reduction finishes the 16-lane rows. On return w[i] holds, in lanes 15, 31, 47
// and 63, the wave totals of slots 4i, 4i+2, 4i+1 and 4i+3.
__device__ __forceinline__ void wave_reduce10(const float v[10], float w[3]) {
  float u[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    float a = v[2 * i], b = v[2 * i + 1];
    swap32(a, b);
    u[i] = a + b;  // lanes 0-31: value 2i, lanes 32-63: value 2i+1
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    float a = u[2 * i], b = (i < 2) ? u[2 * i + 1] : 0.0f;
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

__device__ __forceinline__ void swap32u(uint32_t& a, uint32_t& b) {
  const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
  a = r[0];
  b = r[1];
}
__device__ __forceinline__ void swap16u(uint32_t& a, uint32_t& b) {
  const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
  a = r[0];
  b = r[1];
}
__device__ __forceinline__ half2_t as_h2(uint32_t x) { return __builtin_bit_cast(half2_t, x); }
__device__ __forceinline__ uint32_t as_u32(half2_t x) { return __builtin_bit_cast(uint32_t, x); }

// The same transposed reduction for the half_reduction layout: 6 FP32 values v (the
// screen-mean and conic gradients and the square sum) and 2 packed FP16 pairs h0
// (red, green), h1 (blue, opacity). On return, in lanes 15, 31, 47 and 63: w0 holds
// v0, v2, v1, v3; w1 holds v4, 0, v5, 0; w2 holds h0, 0, h1, 0 (packed FP16 sums).
__device__ __forceinline__ void wave_reduce_half(const float v[6], half2_t h0, half2_t h1, float& w0, float& w1,
                                                 half2_t& w2) {
  float u[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    float a = v[2 * i], b = v[2 * i + 1];
    swap32(a, b);
    u[i] = a + b;
  }
  uint32_t pa = as_u32(h0), pb = as_u32(h1);
  swap32u(pa, pb);
  const half2_t u3 = as_h2(pa) + as_h2(pb);
  {
    float a = u[0], b = u[1];
    swap16(a, b);
    w0 = a + b;
  }
  {
    float a = u[2], b = 0.0f;
    swap16(a, b);
    w1 = a + b;
  }
  {
    uint32_t a = as_u32(u3), b = 0u;
    swap16u(a, b);
    w2 = as_h2(a) + as_h2(b);
  }
  w0 += dpp_row_shr<0x111>(w0);
  w1 += dpp_row_shr<0x111>(w1);
  w2 = w2 + as_h2((uint32_t)__builtin_amdgcn_update_dpp(0, (int)as_u32(w2), 0x111, 0xf, 0xf, true));
  w0 += dpp_row_shr<0x112>(w0);
  w1 += dpp_row_shr<0x112>(w1);
  w2 = w2 + as_h2((uint32_t)__builtin_amdgcn_update_dpp(0, (int)as_u32(w2), 0x112, 0xf, 0xf, true));
  w0 += dpp_row_shr<0x114>(w0);
  w1 += dpp_row_shr<0x114>(w1);
  w2 = w2 + as_h2((uint32_t)__builtin_amdgcn_update_dpp(0, (int)as_u32(w2), 0x114, 0xf, 0xf, true));
  w0 += dpp_row_shr<0x118>(w0);
  w1 += dpp_row_shr<0x118>(w1);
  w2 = w2 + as_h2((uint32_t)__builtin_amdgcn_update_dpp(0, (int)as_u32(w2), 0x118, 0xf, 0xf, true));
}

// One work item: tile gt whole (NB = 4 pixels per lane), or its two bands from
// `band` on (NB = 2, at their row offsets from the whole strip's anchor).
template <int P, int NB, bool kFixed, bool kHalf>
__device__ __forceinline__ void raster_bwd_item(BwdBatch& bufA, BwdBatch& bufB, uint32_t* recA, uint32_t* recB,
                                                float4* __restrict__ stage,
                                                const ViewDev* __restrict__ views, int32_t V, uint32_t gt, int band,
                                                const uint32_t* __restrict__ ranges,
                                                const uint32_t* __restrict__ inst_rec,
                                                const uint32_t* __restrict__ inst_mask,
                                                const Record* __restrict__ rec, const ConstImagePtrs& dL,
                                                const float* __restrict__ pix_T,
                                                const uint32_t* __restrict__ pix_last, float* __restrict__ grad2d,
                                                unsigned long long* __restrict__ grad_fx, float fx_lin, float fx_sq) {
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
    if (px < W && py0 + step * j < H) {
      const int64_t o = (int64_t)(py0 + step * j) * W + px;
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
  mymax = (uint32_t)__builtin_amdgcn_readfirstlane((int)mymax);  // equal in every lane: keep the loop bounds scalar
  const uint32_t s = ranges[2 * gt];
  const uint32_t e = min(ranges[2 * gt + 1], s + mymax);
  if (e <= s) return;

  // Batches from the back: the first one processed starts at the last multiple of
  // kBatch below e. Pipeline as in the forward, in reverse: record ids two batches
  // ahead, records (in LDS) and the forward's band masks (lane k: entry k) one
  // batch ahead.
  const bool batch_lane = lane < kBatch;
  const uint32_t first = s + ((e - s - 1) / kBatch) * kBatch;
  uint32_t maskA, maskB = 0;
  {
    const uint32_t r0 = (batch_lane && first + lane < e) ? inst_rec[first + lane] : 0u;
    batch_fetch(bufA, rec, r0);
    if (batch_lane) recA[lane] = r0;
    maskA = (batch_lane && first + lane < e) ? inst_mask[first + lane] : 0u;
  }
  // the item's bands in the mask bytes: all four, or two from `band` on
  const uint32_t mask_shift = 8u * (uint32_t)band;
  const uint32_t mask_keep = NB == 4 ? 0xFFFFFFFFu : 0xFFFFu;
  uint32_t r_next = (batch_lane && first >= s + kBatch) ? inst_rec[first - kBatch + lane] : 0u;
  // per-entry accumulators; zero at the start and again after each reduction that
  // consumes them (an entry that blends nowhere leaves them at zero). The opacity
  // gradients g_o are summed against s^0 (dop), s^1 and s^2; times o they are the
  // exponent-gradient sums S0, S1, S2.
  float P1 = 0.f, P2 = 0.f, dcr = 0.f, dcg = 0.f, dcb = 0.f, dop = 0.f, ss = 0.f;

  // Gradients of a group of staged entries (FP32 path). Each lane reduces, against
  // its pixels' offsets X = dx, Y_j = dy - s_j from the Gaussian's mean, the sums
  // (dop, sum g_o X, sum g_o Y, sum g_o X^2, sum g_o X Y, sum g_o Y^2, dcr, dcg, dcb,
  // ss); row r of an entry's stage holds their wave totals in slots (sub, sub + 4,
  // sub + 8), sub = 0, 2, 1, 3 for r = 0..3, slot 10 being the fragment count.
  // Lane i converts entry k0 + i: with the exponent E = -1/2 (a X^2 + 2 b X Y +
  // c Y^2) and w = o g_o,
  //   dL/du = -(a sum wX + b sum wY), dL/dv = -(b sum wX + c sum wY),
  //   dL/da = -1/2 sum wX^2, dL/db = -sum wXY, dL/dc = -1/2 sum wY^2:
  // the per-pixel chain rule with its linear pieces taken after the wave sum (o and
  // the conic are the entry's). The entry's 12 output slots go back to its stage;
  // then four lanes per entry add one 16-byte quarter of its gradient row each (one
  // atomic per gradient per tile).
  auto flush = [&](const BwdBatch& cur, const uint32_t* cur_rec, int k0, uint32_t stg) __attribute__((always_inline)) {
    wave_lds_sync();
    if (lane < kGroup && ((stg >> lane) & 1u)) {
      const Record g = batch_get(cur, k0 + lane);
      float4* st = stage + 4 * lane;
      const float4 q0 = st[0], q1 = st[1], q2 = st[2], q3 = st[3];
      const float o = g.r2.x;
      const float wX = o * q2.x, wY = o * q1.x, wXX = o * q3.x, wXY = o * q0.y, wYY = o * q2.y;
      const float ca = -2.0f * (float)kLn2 * g.r1.x;
      const float cb = ca * g.r1.y;
      const float cc = -8.0f * (float)kLn2 * g.r1.w;  // the record holds c / (-8 ln 2)
      const float gu = -__builtin_fmaf(ca, wX, cb * wY);
      const float gv = -__builtin_fmaf(cb, wX, cc * wY);
      st[0] = make_float4(gu, gv, -0.5f * wXX, -wXY);
      st[1] = make_float4(-0.5f * wYY, q0.x, q1.y, q3.y);  // conic c, opacity, red, green
      st[2] = make_float4(q0.z, q2.z, q1.z, 0.0f);         // blue, square sum, count
    }
    wave_lds_sync();
    const int e = lane >> 2, sub = lane & 3;
    if ((stg >> e) & 1u) {
      const float* sv = reinterpret_cast<const float*>(stage + 4 * e) + sub;
      const int64_t row = (int64_t)cur_rec[k0 + e] * kGrad2D + sub;
      if constexpr (kFixed) {
        unsigned long long* dst = grad_fx + row;
        atomicAdd(dst, to_fixed(sv[0], fx_lin));
        atomicAdd(dst + 4, to_fixed(sv[4], fx_lin));
        // slot 9 is the square sum of the statistic, slot 10 the fragment count
        if (sub != 3)
          atomicAdd(dst + 8, sub == 2 ? (unsigned long long)(uint32_t)sv[8] << kFixedBits
                                      : to_fixed(sv[8], sub == 1 ? fx_sq : fx_lin));
      } else {
        float* dst = grad2d + row;
        unsafeAtomicAdd(dst, sv[0]);
        unsafeAtomicAdd(dst + 4, sv[4]);
        if (sub != 3) unsafeAtomicAdd(dst + 8, sv[8]);
      }
    }
    wave_lds_sync();  // the group's stage is read before the next group writes it
  };

  auto run_batch = [&](const BwdBatch& cur, const uint32_t* cur_rec, uint32_t cur_mask, BwdBatch& nxt,
                       uint32_t* nxt_rec, uint32_t& nxt_mask, uint32_t b0) __attribute__((always_inline)) {
    __builtin_amdgcn_s_waitcnt(0);  // this batch's records have landed in LDS
    __syncthreads();
    if (b0 >= s + kBatch) {
      batch_fetch(nxt, rec, r_next);
      if (batch_lane) nxt_rec[lane] = r_next;
      nxt_mask = batch_lane ? inst_mask[b0 - kBatch + lane] : 0u;
    }
    r_next = (batch_lane && b0 >= s + 2 * kBatch) ? inst_rec[b0 - 2 * kBatch + lane] : 0u;
    const int cnt = (int)min((uint32_t)kBatch, e - b0);
    uint32_t stg = 0;  // entries of the current group staged (scalar)
    for (int k = cnt - 1; k >= 0; --k) {
      const uint32_t m = ((uint32_t)__builtin_amdgcn_readlane((int)cur_mask, k) >> mask_shift) & mask_keep;
      if (m != 0) {  // else no pixel of the item blends this entry
        const Record g = batch_get(cur, k);
        float dx, dy;
        const StripTerms et = strip_terms(g, pxc, pyc, dx, dy);
        const uint32_t pos = b0 - s + (uint32_t)k;
        const float o = g.r2.x;
        uint32_t nfrag = 0;  // blended pixels of this entry over the wave (scalar)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          if (((m >> (8 * j)) & 0xFFu) == 0) continue;  // no pixel of band j blends it
          float G, araw;
          const float a = pixel_alpha<P>(o, et.at(sg[j]), G, araw);
          const bool before = pos < last[j], visible = a >= kAlphaMin;
          const bool blend = before && visible;
          nfrag += (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(before) &
                                                  __builtin_amdgcn_ballot_w64(visible));
          if (blend) {
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
            dop += go;
            P1 = __builtin_fmaf(soff[j], go, P1);
            P2 = __builtin_fmaf(soff[j] * soff[j], go, P2);
            ss = __builtin_fmaf(go, go, ss);
            gR[j] = __builtin_fmaf(wt, gc, gR[j]);  // now the colour behind the previous entry
            T[j] = Tb;
          }
        }
        if constexpr (kHalf) {
          if (nfrag != 0) {
            const float S0 = o * dop, S1 = o * P1, S2 = o * P2;  // dL/dE sums
            // exponent -> conic (a, b, c) and mean (u, v) gradients at the strip
            // anchor (pixel j is s_j rows below it):
            //   E_j = -1/2 (a dx^2 + 2 b dx (dy - s_j) + c (dy - s_j)^2), d = mean - anchor
            const float ca = -2.0f * (float)kLn2 * g.r1.x;
            const float cb = ca * g.r1.y;
            const float cc = -8.0f * (float)kLn2 * g.r1.w;  // the record holds c / (-8 ln 2)
            const float gu = __builtin_fmaf(cb, S1, -__builtin_fmaf(ca, dx, cb * dy) * S0);
            const float gv = __builtin_fmaf(cc, S1, -__builtin_fmaf(cb, dx, cc * dy) * S0);
            const float ga = -0.5f * dx * dx * S0;
            const float gb = __builtin_fmaf(dx, S1, -dx * dy * S0);
            const float gcn = __builtin_fmaf(dy, S1, __builtin_fmaf(-0.5f * dy * dy, S0, -0.5f * S2));
            // colour and opacity sums as FP16 pairs (round to nearest), reduced packed
            const float v6[6] = {gu, gv, ga, gb, gcn, ss};
            const half2_t h0 = {(_Float16)dcr, (_Float16)dcg};
            const half2_t h1 = {(_Float16)dcb, (_Float16)dop};
            float t0, t1;
            half2_t t2;
            wave_reduce_half(v6, h0, h1, t0, t1, t2);
            P1 = P2 = dcr = dcg = dcb = dop = ss = 0.f;
            if ((lane & 15) == 15) {
              const int row = lane >> 4;
              const int sub = (row == 0) ? 0 : (row == 1) ? 2 : (row == 2) ? 1 : 3;
              float* dst = grad2d + (int64_t)cur_rec[k] * kGrad2D;
              unsafeAtomicAdd(dst + sub, t0);
              // t1 rows: conic c (slot 4), padding (the fragment count goes there: slot
              // 10), square sum (slot 9); t2 rows: (red, green) into slot 6, (blue,
              // opacity) into 7
              if (row != 3) unsafeAtomicAdd(dst + (row == 0 ? 4 : row == 1 ? 10 : 9), row == 1 ? (float)nfrag : t1);
              if (row == 0 || row == 2)
                __builtin_amdgcn_global_atomic_fadd_v2f16(
                    (__attribute__((address_space(1))) half2_t*)(reinterpret_cast<half2_t*>(dst + (row == 0 ? 6 : 7))),
                    t2);
            }
          }
        } else if (nfrag != 0) {
          // sums against the offsets X = dx, Y_j = dy - s_j of the lane's pixels
          const float wX = dx * dop;
          const float wY = __builtin_fmaf(dy, dop, -P1);
          const float wYY = __builtin_fmaf(dy, wY, __builtin_fmaf(-dy, P1, P2));
          const float vals[10] = {dop, wX, wY, dx * wX, dx * wY, wYY, dcr, dcg, dcb, ss};
          float tot[3];
          wave_reduce10(vals, tot);
          P1 = P2 = dcr = dcg = dcb = dop = ss = 0.f;
          if ((lane & 15) == 15) {
            const int row = lane >> 4;
            stage[4 * (k & (kGroup - 1)) + row] = make_float4(tot[0], tot[1], row == 1 ? (float)nfrag : tot[2], 0.0f);
          }
          stg |= 1u << (k & (kGroup - 1));
        }
      }
      if constexpr (!kHalf) {
        if ((k & (kGroup - 1)) == 0 && stg != 0) {
          flush(cur, cur_rec, k, stg);
          stg = 0;
        }
      }
    }
  };
  for (int64_t b0 = first; b0 >= (int64_t)s; b0 -= 2 * kBatch) {
    run_batch(bufA, recA, maskA, bufB, recB, maskB, (uint32_t)b0);
    if (b0 >= (int64_t)s + kBatch) run_batch(bufB, recB, maskB, bufA, recA, maskA, (uint32_t)(b0 - kBatch));
  }
}

template <int P, bool kFixed, bool kHalf>
__global__ __launch_bounds__(64) void k_raster_bwd(const ViewDev* __restrict__ views, int32_t V,
                                                   const uint32_t* __restrict__ items,
                                                   const uint32_t* __restrict__ header,
                                                   const uint32_t* __restrict__ ranges,
                                                   const uint32_t* __restrict__ inst_rec,
                                                   const uint32_t* __restrict__ inst_mask,
                                                   const Record* __restrict__ rec, ConstImagePtrs dL,
                                                   const float* __restrict__ pix_T,
                                                   const uint32_t* __restrict__ pix_last,
                                                   float* __restrict__ grad2d,
                                                   unsigned long long* __restrict__ grad_fx) {
  __shared__ BwdBatch bufA, bufB;  // two objects, so reads of one never wait on loads into the other
  __shared__ uint32_t recA[kBatch], recB[kBatch];
  __shared__ float4 stage[kHalf ? 1 : 4 * kGroup];
  if (blockIdx.x >= header[kHdrItemsBwd] || frame_aborted(header)) return;
  const uint32_t item = items[blockIdx.x];
  const uint32_t gt = item >> 3;
  const uint32_t code = item & 7u;
  float fx_lin = 0.0f, fx_sq = 0.0f;
  if constexpr (kFixed) {
    const int E = grad_exponent(header);
    fx_lin = __builtin_ldexpf(1.0f, kFixedBits - E);
    fx_sq = __builtin_ldexpf(1.0f, kFixedBits - 2 * E);
  }
  if (code == kItemWhole)
    raster_bwd_item<P, 4, kFixed, kHalf>(bufA, bufB, recA, recB, stage, views, V, gt, 0, ranges, inst_rec, inst_mask, rec, dL,
                                  pix_T, pix_last, grad2d, grad_fx, fx_lin, fx_sq);
  else  // half of a split tile
    raster_bwd_item<P, 2, kFixed, kHalf>(bufA, bufB, recA, recB, stage, views, V, gt, 2 * (int)(code - kItemHalf), ranges,
                                  inst_rec, inst_mask, rec, dL, pix_T, pix_last, grad2d, grad_fx, fx_lin, fx_sq);
}

// max |dL/dI| over the views' images into header[kHdrGradMax] (zeroed before): the
// bits of a non-negative float order as unsigned integers, so an atomic max on them
// is the maximum whatever the order of the blocks. A few blocks (one per CU) each
// reduce a strided share with 16-byte loads and add one atomic: same-address
// atomics serialise, so one per wave cost tens of microseconds.
constexpr int kAbsMaxBlocks = 256;
__global__ __launch_bounds__(256) void k_grad_absmax(ConstImagePtrs dL, ViewCounts counts, int32_t V,
                                                     uint32_t* __restrict__ header) {
  __shared__ float wmax[4];
  if (frame_aborted(header)) return;
  float m = 0.0f;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int v = 0; v < V; ++v) {
    const float* g = dL.p[v];
    const int64_t n = counts.n[v];
    const bool aligned = (reinterpret_cast<uintptr_t>(g) & 15u) == 0;
    const int64_t n4 = aligned ? n / 4 : 0;
    const float4* g4 = reinterpret_cast<const float4*>(g);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride) {
      const float4 x = g4[i];
      m = fmaxf(m, fmaxf(fmaxf(fabsf(x.x), fabsf(x.y)), fmaxf(fabsf(x.z), fabsf(x.w))));
    }
    for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) m = fmaxf(m, fabsf(g[i]));
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
    if (m > 0.0f) atomicMax(header + kHdrGradMax, __float_as_uint(m));
  }
}

template <int P, bool kFixed, bool kHalf = false>
void launch_bwd(const Frame& f, const ConstImagePtrs& dL, hipStream_t s) {
  const unsigned grid = (unsigned)max_items(f.tiles);
  k_raster_bwd<P, kFixed, kHalf><<<grid, 64, 0, s>>>(f.views, f.V, f.bwd_items, f.header, f.ranges,
                                              f.inst_rec, f.inst_mask, f.rec, dL, f.pix_T, f.pix_last, f.grad2d,
                                              f.grad2d_fx);
}

}  // namespace

void launch_grad_absmax(const Frame& f, const ConstImagePtrs& dL, const ViewCounts& counts, hipStream_t s) {
  fill_u32(f.header + kHdrGradMax, 1, 0u, s);
  int64_t total = 0;
  for (int v = 0; v < f.V; ++v) total += counts.n[v];
  const int64_t g = std::min<int64_t>(std::max<int64_t>((total + 1023) / 1024, 1), kAbsMaxBlocks);
  k_grad_absmax<<<(unsigned)g, 256, 0, s>>>(dL, counts, f.V, f.header);
}

void launch_raster_bwd(const Frame& f, const ConstImagePtrs& dL, int precision, bool half, hipStream_t s) {
  if (f.tiles <= 0) return;
  if (precision == GSR_FP16_BLEND_T) precision = GSR_FP16_BLEND;  // the same alphas; T restarts from the final T
  const bool fixed = f.grad2d_fx != nullptr;
  if (half && !fixed) {
    if (precision == GSR_FP16_BLEND)
      launch_bwd<GSR_FP16_BLEND, false, true>(f, dL, s);
    else
      launch_bwd<GSR_FP32, false, true>(f, dL, s);
    return;
  }
  if (precision == GSR_FP16_BLEND)
    fixed ? launch_bwd<GSR_FP16_BLEND, true>(f, dL, s) : launch_bwd<GSR_FP16_BLEND, false>(f, dL, s);
  else
    fixed ? launch_bwd<GSR_FP32, true>(f, dL, s) : launch_bwd<GSR_FP32, false>(f, dL, s);
}

}  // namespace gsr
