// Per-wave arithmetic shared by the forward and backward raster kernels.
//
// Tile/thread mapping: one wave64 per tile of 256 pixels, TW = 2^tile_wl wide and
// TH = 256 / TW high (16x16 by default); lane l owns pixel column l % TW and the
// 4-pixel vertical strip of rows l / TW + S j, j = 0..3, with the row step
// S = TH / 4 (the scanline of App. A.2 runs along y). Step j of every lane thus
// covers the compact TW x S band of rows S j .. S j + S - 1 (16x4 in a 16x16 tile),
// so an entry that blends no pixel of a band skips that band wave-wide. Tiles taller
// than 16 rows (8x32, 4x64) are stacks of 16-row blocks walked the same way (S = 4;
// band j is then row slab j of every block: lane_strip). A tile
// whose list is long is instead split into its 4 bands, one wave each with one
// pixel per lane (NB = 1), so that the longest lists do not set the kernel's
// duration. A band item evaluates its pixel with the same strip anchor and row
// offset as the whole-tile walk, so every pixel's arithmetic is the same whichever
// way its tile is scheduled (a batch of frames may split other tiles than each
// frame alone, and the backward may walk another schedule than the forward). Both
// kernels evaluate the exponent and alpha through the functions below with an
// explicit operation sequence (the library is built without FP contraction), so
// the backward re-derives exactly the forward's blend decisions and transmittances.
#pragma once

#include "gsr_internal.h"

namespace gsr {

// Raster work items: (tile << 3) | code. kItemWhole (4) is the whole tile, 4
// pixels per lane; codes 0..3 are band `code` of a tile split four ways, 1 pixel per
// lane; kItemHalf + h (5, 6) are bands 2h and 2h + 1 of a tile split two ways, 2
// pixels per lane. By default the forward splits tiles with more than kSplitLen
// (gsr_internal.h) entries four ways; the backward, whose per-entry wave reduction and atomics are
// repeated by every item of a tile, splits those with more than kSplitLenBwd
// entries two ways (both thresholds can be set per context). Either takes the
// longest first, at most one tile in kSplitShare.
constexpr uint32_t kItemWhole = 4;
constexpr uint32_t kItemHalf = 5;
constexpr int64_t kSplitShare = 4;
__host__ __device__ constexpr int64_t max_items(int64_t tiles) { return tiles + 3 * ((tiles + kSplitShare - 1) / kSplitShare); }
// A lane's pixels in a work item of a view's tile (tx, ty): column px, the rows
// py0 + step j of its NB pixels (band `band` onwards), and the strip anchor, the
// centre row of the lane's whole-tile strip (1.5 steps below its first row;
// anchoring at the centre halves the largest offset, and so the extrapolation of
// the scanline form, against anchoring at the first pixel). s[j] = step (band + j
// - 3/2) is pixel j's row offset from the anchor (exact in FP32); the exponent is
// evaluated at the scaled offsets sigma_j = -2 s_j (strip_sigmas).
struct LaneStrip {
  int px, py0, step;
  float pxc, pyc;  // anchor pixel centre
};

template <int NB>
__device__ __forceinline__ LaneStrip lane_strip(const ViewDev& w, int tx, int ty, int band, int lane, float s[NB]) {
  const int wl = w.tile_wl, hl = 8 - wl;
  LaneStrip q;
  // row step TH / 4, at most 4: a tile taller than 16 rows is a stack of 16-row
  // blocks, lane row lr owning rows 16 (lr / 4) + lr % 4 + 4 j of it, so that no
  // strip spans more than 13 rows (the scanline form extrapolates over +-6 rows at
  // most, as in a 16x16 tile)
  const int lr = lane >> wl;
  q.step = hl > 4 ? 4 : 1 << (hl - 2);
  q.px = (tx << wl) + (lane & ((1 << wl) - 1));
  const int ys = (ty << hl) + (hl > 4 ? ((lr >> 2) << 4) + (lr & 3) : lr);  // first row of the lane's strip
  q.py0 = ys + q.step * band;
  q.pxc = (float)q.px + 0.5f;
  q.pyc = (float)ys + 1.5f * (float)q.step + 0.5f;
#pragma unroll
  for (int j = 0; j < NB; ++j) s[j] = (float)q.step * ((float)(band + j) - 1.5f);
  return q;
}

template <int NB>
__device__ __forceinline__ void strip_sigmas(const float s[NB], float sg[NB]) {
#pragma unroll
  for (int j = 0; j < NB; ++j) sg[j] = -2.0f * s[j];
}

// Exponent of the 2-D Gaussian (Eq. (2)) in log2 units at row offsets s[j] from a
// strip anchor whose pixel centre is (pxc, pyc). Following the scanline split of
// App. A.2 (Eq. (8)-(9)), it is Basic + Linear s + Quad s^2, with Basic and Linear
// computed once per strip from the factored form
//   E2 = k1 (dx + r dy)^2 + k2 dy^2,   d = screen mean - anchor centre,
// whose two terms never cancel; the per-pixel cost is two FMAs. In the scaled offset
// sigma = -2 s the form is Basic + sigma (L + sigma Q/4) with L = -Linear/2: the record
// holds Q/4 and L needs no product by -2, and since the scalings are by powers of two
// the value is the same, bit for bit, as Basic + s (Linear + s Q).
struct StripTerms {
  float basic, lin, quad4;
  // exponent at scaled row offset sg = -2 s from the anchor
  __device__ __forceinline__ float at(float sg) const {
    return __builtin_fmaf(sg, __builtin_fmaf(sg, quad4, lin), basic);
  }
};

__device__ __forceinline__ StripTerms strip_terms(const Record& g, float pxc, float pyc, float& dx, float& dy) {
  dx = (g.r0.x - pxc) + g.r0.z;
  dy = (g.r0.y - pyc) + g.r0.w;
  const float D = __builtin_fmaf(g.r1.y, dy, dx);
  const float t1 = g.r1.x * D;
  const float t2 = g.r1.z * dy;
  StripTerms t;
  t.basic = __builtin_fmaf(t1, D, t2 * dy);
  t.lin = __builtin_fmaf(t1, g.r1.y, t2);
  t.quad4 = g.r1.w;
  return t;
}

template <int NB>
__device__ __forceinline__ void strip_exponents(const Record& g, float pxc, float pyc, const float sg[NB],
                                                float e[NB], float& dx, float& dy) {
  const StripTerms t = strip_terms(g, pxc, pyc, dx, dy);
#pragma unroll
  for (int j = 0; j < NB; ++j) e[j] = t.at(sg[j]);
}

// G = 2^e (v_exp_f32) and alpha = min(0.99, o G); araw = o G before the clamp.
__device__ __forceinline__ float alpha_of(float o, float e, float& G, float& araw) {
  G = __builtin_amdgcn_exp2f(e);
  araw = o * G;
  return fminf(kAlphaMax, araw);
}

// FP16 blend (Sec. 3.1.2): the strip's exponents, computed in FP32, are rounded to
// FP16 (toward zero, two per instruction); G = 2^e (v_exp_f16) and alpha =
// min(0.99, o G) are evaluated on pixel pairs in packed FP16. Transmittance,
// colour and all gradients stay FP32, taking these alphas as exact.
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
extern "C" __device__ _Float16 __ocml_exp2_f16(_Float16);
constexpr float kAlphaMaxH = 0.990234375f;  // 0.99 rounded to FP16: the clamp point of the FP16 blend

template <int NB>
__device__ __forceinline__ void strip_alpha_h(float o, const float e[NB], float a[NB], float G[NB], float araw[NB]) {
  const _Float16 oh = (_Float16)o;
  const half2_t o2 = {oh, oh};
  const half2_t cap = {(_Float16)kAlphaMax, (_Float16)kAlphaMax};
#pragma unroll
  for (int p = 0; p < (NB + 1) / 2; ++p) {
    const float e1 = (2 * p + 1 < NB) ? e[2 * p + 1] : e[2 * p];
    const half2_t eh = __builtin_bit_cast(half2_t, __builtin_amdgcn_cvt_pkrtz(e[2 * p], e1));
    const half2_t g = {__ocml_exp2_f16(eh.x), __ocml_exp2_f16(eh.y)};
    const half2_t r = o2 * g;
    const half2_t al = __builtin_elementwise_min(cap, r);
    a[2 * p] = (float)al.x;
    G[2 * p] = (float)g.x;
    araw[2 * p] = (float)r.x;
    if (2 * p + 1 < NB) {
      a[2 * p + 1] = (float)al.y;
      G[2 * p + 1] = (float)g.y;
      araw[2 * p + 1] = (float)r.y;
    }
  }
}

// Alpha of the NB strip pixels at precision P (GSR_FP32, or the FP16 blend of
// GSR_FP16_BLEND and GSR_FP16_BLEND_T).
template <int P, int NB>
__device__ __forceinline__ void strip_alpha(float o, const float e[NB], float a[NB], float G[NB], float araw[NB]) {
  if constexpr (P == GSR_FP16_BLEND || P == GSR_FP16_BLEND_T) {
    strip_alpha_h<NB>(o, e, a, G, araw);
  } else {
#pragma unroll
    for (int j = 0; j < NB; ++j) a[j] = alpha_of(o, e[j], G[j], araw[j]);
  }
}

// Alpha of one pixel at precision P: the same value, operation for operation, as
// strip_alpha gives that pixel (the FP16 pair operations act elementwise).
template <int P>
__device__ __forceinline__ float pixel_alpha(float o, float e, float& G, float& araw) {
  if constexpr (P == GSR_FP16_BLEND || P == GSR_FP16_BLEND_T) {
    const half2_t eh = __builtin_bit_cast(half2_t, __builtin_amdgcn_cvt_pkrtz(e, e));
    const _Float16 g = __ocml_exp2_f16(eh.x);
    const _Float16 r = (_Float16)o * g;
    const _Float16 al = __builtin_elementwise_min((_Float16)kAlphaMax, r);
    G = (float)g;
    araw = (float)r;
    return (float)al;
  } else {
    return alpha_of(o, e, G, araw);
  }
}

// The value of o G above which alpha is clamped (and its derivative is 0).
template <int P>
constexpr float alpha_clamp() {
  return P == GSR_FP32 ? kAlphaMax : kAlphaMaxH;
}

// A batch of B records (B a power of two, at most 64) in LDS, stored as three
// planes of float4 (r0, r1, r2) and filled by direct global-to-LDS loads
// (global_load_lds_dwordx4): lane l < B has its record part land at plane + 16 l
// without passing through registers, so the next batch is in flight while the
// wave works on the current one. Lanes past the end of the list load record 0
// (always valid; those slots are never read). The batch size trades the batch
// overhead (a barrier and a fetch per batch) against LDS per wave, which bounds
// how many waves a CU holds.
template <int B>
struct BatchLDS {
  float4 part[3][B];
};

template <int B>
__device__ __forceinline__ void batch_fetch(BatchLDS<B>& dst, const Record* __restrict__ rec, uint32_t r) {
  if (B < 64 && (int)threadIdx.x >= B) return;
  const float4* src = reinterpret_cast<const float4*>(rec + r);
#pragma unroll
  for (int p = 0; p < 3; ++p)
    __builtin_amdgcn_global_load_lds((const void*)(src + p),
                                     (__attribute__((address_space(3))) void*)(&dst.part[p][0]), 16, 0, 0);
}

template <int B>
__device__ __forceinline__ Record batch_get(const BatchLDS<B>& b, int k) {
  Record g;
  g.r0 = b.part[0][k];
  g.r1 = b.part[1][k];
  g.r2 = b.part[2][k];
  return g;
}

// A wave's LDS instructions execute in issue order, so its lanes exchange data
// through LDS behind a compiler-level barrier alone.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Locate the view of global tile gt (views are few; the loop is wave-uniform).
__device__ __forceinline__ int view_of_tile(const ViewDev* views, int32_t V, uint32_t gt) {
  int v = 0;
  while (v + 1 < V && (uint32_t)views[v + 1].tile_base <= gt) ++v;
  return v;
}

}  // namespace gsr
