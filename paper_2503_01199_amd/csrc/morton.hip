// Morton codes and spatial reorder (Sec. 3.2.1).
//
// Positions are normalised per axis to the unit cube by the scene's min/max,
// scaled by 2^21 - 1 and truncated to 21-bit integers, whose bits are interleaved
// into a 63-bit Z-order code (bit k of x, y, z -> bits 3k, 3k+1, 3k+2). The
// normalisation runs in FP64 on the FP32 means, q = trunc(clamp((p - lo)/(hi - lo),
// 0, 1) * 2097151), so the codes are a reproducible function of the inputs. The
// permutation is the stable radix sort of the codes.
#include <math.h>

#include "gsr_internal.h"

namespace gsr {
namespace {

constexpr int kBoundsBlocks = 1024;

__global__ __launch_bounds__(256) void k_bounds_partial(const float* __restrict__ means, int64_t n,
                                                        float* __restrict__ part) {
  float lo[3] = {INFINITY, INFINITY, INFINITY};
  float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float m = means[3 * i + a];
      lo[a] = fminf(lo[a], m);
      hi[a] = fmaxf(hi[a], m);
    }
  }
  __shared__ float red[6][4];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], __shfl_xor(lo[a], d, 64));
      hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], d, 64));
    }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int a = 0; a < 3; ++a) {
      red[a][w] = lo[a];
      red[3 + a][w] = hi[a];
    }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int a = threadIdx.x;
    float x = red[a][0];
    for (int q = 1; q < 4; ++q) x = a < 3 ? fminf(x, red[a][q]) : fmaxf(x, red[a][q]);
    part[blockIdx.x * 6 + a] = x;
  }
}

// One wave per axis bound (6 waves): lanes stride over the block partials.
__global__ void k_bounds_final(const float* __restrict__ part, int G, float* __restrict__ bounds) {
  const int a = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  if (a >= 6) return;
  float x = a < 3 ? INFINITY : -INFINITY;
  for (int b = lane; b < G; b += 64) x = a < 3 ? fminf(x, part[6 * b + a]) : fmaxf(x, part[6 * b + a]);
  for (int d = 32; d >= 1; d >>= 1) {
    const float y = __shfl_xor(x, d, 64);
    x = a < 3 ? fminf(x, y) : fmaxf(x, y);
  }
  if (lane == 0) bounds[a] = x;
}

// 21 bits of v spread to every third bit of a 64-bit word.
__device__ __forceinline__ uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | (x << 32)) & 0x001f00000000ffffull;
  x = (x | (x << 16)) & 0x001f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

__global__ void k_morton_encode(const float* __restrict__ means, int64_t n, const float* __restrict__ bounds,
                                uint64_t* __restrict__ codes_sort, uint64_t* __restrict__ codes_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t code = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double lo = bounds[a], hi = bounds[3 + a];
    double u = 0.0;
    if (hi > lo) u = ((double)means[3 * i + a] - lo) / (hi - lo);
    u = fmin(fmax(u, 0.0), 1.0);
    const uint32_t q = (uint32_t)(u * 2097151.0);
    code |= spread3(q) << a;
  }
  codes_sort[i] = code;
  if (codes_out) codes_out[i] = code;
}

__global__ void k_perm_out(const uint32_t* __restrict__ vals, int64_t n, int64_t* __restrict__ perm,
                           const uint32_t* __restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // a sort that gave up leaves the order as it is (the identity is a valid
  // permutation, so a caller's gather stays in bounds)
  const bool ok = !error_raised(err);
  if (i < n) perm[i] = ok ? (int64_t)vals[i] : i;
}

__global__ void k_gather_rows(const int64_t* __restrict__ perm, int64_t n, const float* __restrict__ src,
                              float* __restrict__ dst, int32_t rf) {
  const int64_t total = n * rf;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t / rf;
    const int64_t c = t - i * rf;
    dst[t] = src[perm[i] * rf + c];
  }
}

size_t align_words(size_t w) { return (w + 63) & ~(size_t)63; }

}  // namespace

size_t morton_temp_words(int64_t n) {
  return align_words(6 * kBoundsBlocks) + 64 + 3 * align_words((size_t)n * 2) + 2 * align_words((size_t)n) +
         align_words(sort_ctl_words(n, 63)) + 64;
}

bool morton_order(const float* means, int64_t n, uint32_t* temp, int64_t* perm, uint64_t* codes, hipStream_t s) {
  if (n <= 0) return true;
  float* part = (float*)temp;
  float* bounds = (float*)(temp + align_words(6 * kBoundsBlocks));
  uint32_t* p = temp + align_words(6 * kBoundsBlocks) + 64;
  uint64_t* ck[2];
  ck[0] = (uint64_t*)p;
  p += align_words((size_t)n * 2);
  ck[1] = (uint64_t*)p;
  p += align_words((size_t)n * 2);
  uint64_t* cin = (uint64_t*)p;
  p += align_words((size_t)n * 2);
  uint32_t* vb[2];
  vb[0] = p;
  p += align_words((size_t)n);
  vb[1] = p;
  p += align_words((size_t)n);
  uint32_t* err = p;
  p += 64;
  uint32_t* ctl = p;
  fill_u32(err, 64 + (int64_t)sort_ctl_words(n, 63), 0u, s);
  int G = (int)((n + 255) / 256);
  if (G > kBoundsBlocks) G = kBoundsBlocks;
  k_bounds_partial<<<G, 256, 0, s>>>(means, n, part);
  k_bounds_final<<<1, 384, 0, s>>>(part, G, bounds);
  k_morton_encode<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(means, n, bounds, cin, codes);
  const int r = radix_sort_u64_dev(cin, nullptr, ck, vb, n, nullptr, 63, ctl, err, false, s);
  k_perm_out<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(vb[r], n, perm, err);
  return true;
}

void launch_gather_rows(const int64_t* perm, int64_t n, const float* src, float* dst, int32_t row_floats,
                        hipStream_t s) {
  if (n <= 0 || row_floats <= 0) return;
  int64_t g = (n * row_floats + 255) / 256;
  if (g > 65536) g = 65536;
  k_gather_rows<<<(unsigned)g, 256, 0, s>>>(perm, n, src, dst, row_floats);
}

}  // namespace gsr
