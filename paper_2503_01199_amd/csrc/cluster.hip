// Cluster-Cull-Compact (Sec. 3.2.2): clusters of GSR_CLUSTER consecutive
// (Morton-ordered) Gaussians, one bounding record per cluster, a frustum test per
// cluster and view, and the list of visible clusters whose Gaussians the
// preprocess then reads as one contiguous, coalesced stream.
#include <math.h>

#include "gsr_internal.h"

namespace gsr {
namespace {

// Frame start: views from the kernel arguments into the workspace, and the frame's
// header and control words cleared (fill kernels, not memset nodes, so the frame
// stays capturable in a graph).
__global__ void k_frame_begin(ViewChunk chunk, int v0, int nv, ViewDev* __restrict__ views, uint32_t* __restrict__ zero,
                              int64_t zero_words) {
  constexpr int kWords = sizeof(ViewDev) / 4;
  static_assert(sizeof(ViewDev) % 4 == 0, "ViewDev is copied by words");
  if (blockIdx.x == 0) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(chunk.v);
    uint32_t* dst = reinterpret_cast<uint32_t*>(views + v0);
    for (int k = threadIdx.x; k < nv * kWords; k += blockDim.x) dst[k] = src[k];
  }
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < zero_words; k += (int64_t)gridDim.x * blockDim.x)
    zero[k] = 0u;
}

// max / min over the box [lo, hi] of the affine function c . p + c0
__device__ inline float box_max(const float* c, float c0, const float* lo, const float* hi) {
  float s = c0;
#pragma unroll
  for (int a = 0; a < 3; ++a) s += c[a] > 0.0f ? c[a] * hi[a] : c[a] * lo[a];
  return s;
}

__device__ inline float box_min(const float* c, float c0, const float* lo, const float* hi) {
  float s = c0;
#pragma unroll
  for (int a = 0; a < 3; ++a) s += c[a] > 0.0f ? c[a] * lo[a] : c[a] * hi[a];
  return s;
}

// A cluster is culled in a view when no Gaussian in it can have a non-empty
// screen footprint there. For a Gaussian with camera-space mean (tx, ty, tz),
// tz > near, largest scale s and opacity o < 1, the footprint half-width is
//   rx = sqrt(2 ln(255 o) cov_xx) <= sqrt(2 ln 255) ((fx/tz) sqrt(1 + limx^2) s + sqrt(0.3)),
// so the footprint lies left of the image if
//   tx + ((cx + g)/fx) tz < -sqrt(2 ln 255) sqrt(1 + limx^2) s,
// with g = sqrt(0.3 * 2 ln 255) + guard. The left side is affine in the world
// position, so its maximum over the cluster's box of means decides for the whole
// cluster. The other three sides are symmetric; all means behind the near plane
// also cull. A guard of 2 px and 1% on the radius cover FP32 rounding. The
// camera rotation is assumed orthonormal.
__device__ bool cluster_visible_in(const ViewDev& w, const float* lo, const float* hi, float smax) {
  const float sqK = 3.33170f * 1.01f;  // sqrt(2 ln 255) with margin
  const float guard = 1.8241f + 2.0f;  // sqrt(0.3 * 2 ln 255) + 2 px
  const float* rx = w.R;
  const float* ry = w.R + 3;
  const float* rz = w.R + 6;
  if (box_max(rz, w.t[2], lo, hi) <= w.near_plane) return false;
  const float rhox = sqK * sqrtf(1.0f + (float)(w.limx * w.limx)) * smax;
  const float rhoy = sqK * sqrtf(1.0f + (float)(w.limy * w.limy)) * smax;
  float cf[3];
  float k = (w.cx + guard) / w.fx;  // left
  for (int a = 0; a < 3; ++a) cf[a] = rx[a] + k * rz[a];
  if (box_max(cf, w.t[0] + k * w.t[2], lo, hi) < -rhox) return false;
  k = (w.cx - (float)w.width - guard) / w.fx;  // right
  for (int a = 0; a < 3; ++a) cf[a] = rx[a] + k * rz[a];
  if (box_min(cf, w.t[0] + k * w.t[2], lo, hi) > rhox) return false;
  k = (w.cy + guard) / w.fy;  // top
  for (int a = 0; a < 3; ++a) cf[a] = ry[a] + k * rz[a];
  if (box_max(cf, w.t[1] + k * w.t[2], lo, hi) < -rhoy) return false;
  k = (w.cy - (float)w.height - guard) / w.fy;  // bottom
  for (int a = 0; a < 3; ++a) cf[a] = ry[a] + k * rz[a];
  if (box_min(cf, w.t[1] + k * w.t[2], lo, hi) > rhoy) return false;
  return true;
}

// One wave per cluster of 128 Gaussians (two per lane): min/max of the means and the
// largest log-scale (output [8]: min xyz, max xyz, max log-scale, 0), then the
// frustum test against every view. kBegin (frames of at most kViewChunk views): the
// kernel also starts the frame, as k_frame_begin would: the views come from the
// kernel arguments (block 0 copies them to `views` for the later kernels) and the
// blocks clear the header and control words, which no block of this kernel reads.
template <bool kBegin>
__global__ __launch_bounds__(64) void k_cluster(const float* __restrict__ means, const float* __restrict__ log_scales,
                                                int64_t n, int cull, const ViewDev* __restrict__ views, int32_t V,
                                                float* __restrict__ bounds, uint32_t* __restrict__ visible,
                                                ViewChunk chunk, ViewDev* __restrict__ views_out,
                                                uint32_t* __restrict__ zero, int64_t zero_words) {
  const int64_t c = blockIdx.x;
  const int lane = threadIdx.x;
  if constexpr (kBegin) {
    constexpr int kWords = sizeof(ViewDev) / 4;
    if (c == 0) {
      const uint32_t* src = reinterpret_cast<const uint32_t*>(chunk.v);
      uint32_t* dst = reinterpret_cast<uint32_t*>(views_out);
      for (int k = lane; k < V * kWords; k += 64) dst[k] = src[k];
    }
    for (int64_t k = c * 64 + lane; k < zero_words; k += (int64_t)gridDim.x * 64) zero[k] = 0u;
  }
  float lo[3] = {INFINITY, INFINITY, INFINITY};
  float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  float mls = -INFINITY;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int64_t i = c * GSR_CLUSTER + k * 64 + lane;
    if (i < n) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const float m = means[3 * i + a];
        lo[a] = fminf(lo[a], m);
        hi[a] = fmaxf(hi[a], m);
        mls = fmaxf(mls, log_scales[3 * i + a]);
      }
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], __shfl_xor(lo[a], d, 64));
      hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], d, 64));
    }
    mls = fmaxf(mls, __shfl_xor(mls, d, 64));
  }
  if (lane < 8) {
    const float vals[8] = {lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], mls, 0.0f};
    float v = vals[0];
#pragma unroll
    for (int k = 1; k < 8; ++k) v = (lane == k) ? vals[k] : v;
    bounds[c * 8 + lane] = v;
  }
  if (lane == 0) {
    uint32_t vis = 1;
    if (cull) {
      vis = 0;
      const float smax = expf(mls);
      for (int v = 0; v < V && !vis; ++v)
        vis = cluster_visible_in(kBegin ? chunk.v[v] : views[v], lo, hi, smax) ? 1u : 0u;
    }
    visible[c] = vis;
  }
}

}  // namespace

void launch_frame_begin(const ViewChunk& chunk, int v0, int nv, ViewDev* views, uint32_t* zero, int64_t zero_words,
                        hipStream_t s) {
  int64_t g = (zero_words + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  k_frame_begin<<<(unsigned)g, 256, 0, s>>>(chunk, v0, nv, views, zero, zero_words);
}

void launch_cluster(const float* means, const float* log_scales, int64_t n, int cull, const ViewDev* views, int32_t V,
                    float* bounds, uint32_t* visible, hipStream_t s) {
  const int64_t nc = (n + GSR_CLUSTER - 1) / GSR_CLUSTER;
  if (nc > 0)
    k_cluster<false><<<(unsigned)nc, 64, 0, s>>>(means, log_scales, n, cull, views, V, bounds, visible, ViewChunk{},
                                                 nullptr, nullptr, 0);
}

bool launch_cluster_begin(const ViewChunk& chunk, int32_t V, ViewDev* views, uint32_t* zero, int64_t zero_words,
                          const float* means, const float* log_scales, int64_t n, int cull, float* bounds,
                          uint32_t* visible, hipStream_t s) {
  const int64_t nc = (n + GSR_CLUSTER - 1) / GSR_CLUSTER;
  if (nc <= 0 || V > kViewChunk) return false;
  k_cluster<true><<<(unsigned)nc, 64, 0, s>>>(means, log_scales, n, cull, views, V, bounds, visible, chunk, views,
                                              zero, zero_words);
  return true;
}

}  // namespace gsr
