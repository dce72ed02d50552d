// Per-wave arithmetic shared by the forward and backward raster kernels.
//
// Tile/thread mapping: one wave64 per 16x16 tile; lane l owns pixel column l % 16
// and the 4-pixel vertical strip of rows 4*(l/16) .. 4*(l/16)+3 (the scanline of
// App. A.2 runs along y). Both kernels evaluate the exponent and alpha through
// the functions below with an explicit operation sequence (the library is built
// without FP contraction), so the backward re-derives exactly the forward's
// blend decisions and transmittances.
#pragma once

#include "gsr_internal.h"

namespace gsr {

// Exponent of the 2-D Gaussian (Eq. (2)) in log2 units at the 4 pixels of a strip
// whose first pixel centre is (pxc, pyc). Following the scanline split of
// App. A.2 (Eq. (8)-(9)), it is Basic + Linear j + Quad j^2 with Basic and Linear
// computed once per strip from the factored form
//   E2 = k1 (dx + r dy)^2 + k2 dy^2,   d = screen mean - pixel centre,
// whose two terms never cancel; the per-pixel cost is two FMAs.
__device__ __forceinline__ void strip_exponents(const Record& g, float pxc, float pyc, float e[4], float& dx,
                                                float& dy) {
  dx = (g.r0.x - pxc) + g.r0.z;
  dy = (g.r0.y - pyc) + g.r0.w;
  const float D = __builtin_fmaf(g.r1.y, dy, dx);
  const float t1 = g.r1.x * D;
  const float t2 = g.r1.z * dy;
  const float basic = __builtin_fmaf(t1, D, t2 * dy);
  const float lin = -2.0f * __builtin_fmaf(t1, g.r1.y, t2);
  const float quad = g.r1.w;
  e[0] = basic;
  e[1] = __builtin_fmaf(1.0f, __builtin_fmaf(1.0f, quad, lin), basic);
  e[2] = __builtin_fmaf(2.0f, __builtin_fmaf(2.0f, quad, lin), basic);
  e[3] = __builtin_fmaf(3.0f, __builtin_fmaf(3.0f, quad, lin), basic);
}

// G = 2^e (v_exp_f32) and alpha = min(0.99, o G); araw = o G before the clamp.
__device__ __forceinline__ float alpha_of(float o, float e, float& G, float& araw) {
  G = __builtin_amdgcn_exp2f(e);
  araw = o * G;
  return fminf(kAlphaMax, araw);
}

// Locate the view of global tile gt (views are few; the loop is wave-uniform).
__device__ __forceinline__ int view_of_tile(const ViewDev* views, int32_t V, uint32_t gt) {
  int v = 0;
  while (v + 1 < V && (uint32_t)views[v + 1].tile_base <= gt) ++v;
  return v;
}

}  // namespace gsr
