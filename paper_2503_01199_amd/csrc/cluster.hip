// Cluster-Cull-Compact (Sec. 3.2.2): clusters of GSR_CLUSTER consecutive
// (Morton-ordered) Gaussians, one bounding record per cluster, a frustum test per
// cluster and view, and the list of visible clusters whose Gaussians the
// preprocess then reads as one contiguous, coalesced stream.
#include <math.h>

#include "gsr_internal.h"

namespace gsr {
namespace {

// One wave per cluster of 128 Gaussians (two per lane): min/max of the means and
// the largest log-scale. Output [8]: min xyz, max xyz, max log-scale, 0.
__global__ __launch_bounds__(64) void k_cluster_bounds(const float* __restrict__ means,
                                                       const float* __restrict__ log_scales, int64_t n,
                                                       float* __restrict__ bounds) {
  const int64_t c = blockIdx.x;
  const int lane = threadIdx.x;
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
}

// max over the box [lo, hi] of the affine function c . p + c0
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
// also cull. A guard of 2 px and 1% on the radius cover FP32 rounding.
__global__ void k_cluster_cull(const float* __restrict__ bounds, int32_t nclusters, const ViewDev* __restrict__ views,
                               int32_t V, uint32_t* __restrict__ visible) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nclusters) return;
  const float* b = bounds + 8 * (int64_t)c;
  const float lo[3] = {b[0], b[1], b[2]};
  const float hi[3] = {b[3], b[4], b[5]};
  const float smax = expf(b[6]);
  const float sqK = 3.33170f * 1.01f;  // sqrt(2 ln 255) with margin
  const float guard = 1.8241f + 2.0f;  // sqrt(0.3 * 2 ln 255) + 2 px
  uint32_t vis = 0;
  for (int v = 0; v < V && !vis; ++v) {
    const ViewDev& w = views[v];
    const float* rx = w.R;
    const float* ry = w.R + 3;
    const float* rz = w.R + 6;
    if (box_max(rz, w.t[2], lo, hi) <= w.near_plane) continue;
    const float rhox = sqK * sqrtf(1.0f + (float)(w.limx * w.limx)) * smax;
    const float rhoy = sqK * sqrtf(1.0f + (float)(w.limy * w.limy)) * smax;
    float cf[3];
    // left
    float k = (w.cx + guard) / w.fx;
    for (int a = 0; a < 3; ++a) cf[a] = rx[a] + k * rz[a];
    if (box_max(cf, w.t[0] + k * w.t[2], lo, hi) < -rhox) continue;
    // right
    k = (w.cx - (float)w.width - guard) / w.fx;
    for (int a = 0; a < 3; ++a) cf[a] = rx[a] + k * rz[a];
    if (box_min(cf, w.t[0] + k * w.t[2], lo, hi) > rhox) continue;
    // top
    k = (w.cy + guard) / w.fy;
    for (int a = 0; a < 3; ++a) cf[a] = ry[a] + k * rz[a];
    if (box_max(cf, w.t[1] + k * w.t[2], lo, hi) < -rhoy) continue;
    // bottom
    k = (w.cy - (float)w.height - guard) / w.fy;
    for (int a = 0; a < 3; ++a) cf[a] = ry[a] + k * rz[a];
    if (box_min(cf, w.t[1] + k * w.t[2], lo, hi) > rhoy) continue;
    vis = 1;
  }
  visible[c] = vis;
}

__global__ void k_cluster_list(const uint32_t* __restrict__ visible, const uint32_t* __restrict__ offset,
                               int32_t nclusters, uint32_t* __restrict__ list) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < nclusters && visible[c]) list[offset[c]] = (uint32_t)c;
}

}  // namespace

void launch_cluster_bounds(const float* means, const float* log_scales, int64_t n, float* bounds, hipStream_t s) {
  const int64_t nc = (n + GSR_CLUSTER - 1) / GSR_CLUSTER;
  if (nc > 0) k_cluster_bounds<<<(unsigned)nc, 64, 0, s>>>(means, log_scales, n, bounds);
}

void launch_cluster_cull(const float* bounds, int32_t nclusters, const ViewDev* views, int32_t V,
                         uint32_t* visible, hipStream_t s) {
  if (nclusters > 0) k_cluster_cull<<<(nclusters + 255) / 256, 256, 0, s>>>(bounds, nclusters, views, V, visible);
}

void launch_cluster_list(const uint32_t* visible, const uint32_t* offset, int32_t nclusters, uint32_t* list,
                         hipStream_t s) {
  if (nclusters > 0) k_cluster_list<<<(nclusters + 255) / 256, 256, 0, s>>>(visible, offset, nclusters, list);
}

}  // namespace gsr
