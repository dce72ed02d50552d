// Adam at cluster granularity (Sec. 3.2.3).
//
// The sparse update of the per-view visible primitives is applied to whole
// clusters of GSR_CLUSTER consecutive Gaussians: a cluster that the frame's cull
// kept is updated in full, every other cluster is left alone (parameters and both
// moments). Because a cluster is a run of consecutive rows, each of its parameter
// groups is one contiguous slice of that group's array, 128 x row floats long, so
// the update streams full 16-byte lines and never scatters.
//
// A block takes two consecutive clusters and skips a culled one after reading its
// flag (one cluster per block, or four, measured slower: more short-lived blocks,
// or a worse balance). It walks a cluster's five slices as one list of float4
// units (means, log-scales, quaternions, opacity logits, SH), four units per
// thread at a time with every load of the four issued before the first store;
// loads and stores are non-temporal, since no float is touched twice. The
// partial last cluster takes a scalar walk.
//
// Per float (Kingma and Ba, Algorithm 1, with the bias corrections folded into
// constants the host computes in FP64):
//   m' = b1 m + (1 - b1) g,   v' = b2 v + (1 - b2) g^2,
//   p' = p - (lr / (1 - b1^t)) m' / (sqrt(v') / sqrt(1 - b2^t) + eps).
#include "gsr_internal.h"

namespace gsr {
namespace {

constexpr int kAdamThreads = 256;
constexpr int kAdamBatch = 4;                      // float4 units in flight per thread
constexpr int kAdamPer = 2;                        // consecutive clusters per block
constexpr int kUnitsPerRowFloat = GSR_CLUSTER / 4;  // float4 units of a full cluster per float of a row

// Every float is read once and written once: loads and stores are non-temporal.
typedef float adam_v4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 load_stream(const float* p) {
  const adam_v4 x = __builtin_nontemporal_load(reinterpret_cast<const adam_v4*>(p));
  return make_float4(x.x, x.y, x.z, x.w);
}
__device__ __forceinline__ void store_stream(float* p, const float (&x)[4]) {
  const adam_v4 y = {x[0], x[1], x[2], x[3]};
  __builtin_nontemporal_store(y, reinterpret_cast<adam_v4*>(p));
}

// Rate of float `r` of a row (r < row): the group's head floats take step_head.
__device__ __forceinline__ float adam_rate(const AdamGroupDev& q, uint32_t r) {
  return r < (uint32_t)q.head ? q.step_head : q.step_rest;
}

// Unit u of a full cluster -> group index and the unit's position in its slice.
__device__ __forceinline__ int unit_group(const AdamDev& a, int32_t& u) {
  int k = 0;
#pragma unroll
  for (int q = 0; q < kAdamGroups - 1; ++q) {
    const int32_t nq = kUnitsPerRowFloat * a.grp[q].row;
    if (k == q && u >= nq) {
      u -= nq;
      k = q + 1;
    }
  }
  return k;
}

// The full cluster that starts at Gaussian `first`.
__device__ __forceinline__ void adam_cluster_vec(const AdamDev& a, int64_t first) {
  const int32_t units = a.units;
  for (int32_t base = threadIdx.x; base < units; base += kAdamThreads * kAdamBatch) {
    float4 P[kAdamBatch], G[kAdamBatch], M[kAdamBatch], V[kAdamBatch];
    int64_t at[kAdamBatch];
    int grp[kAdamBatch];
    uint32_t r0[kAdamBatch];
#pragma unroll
    for (int j = 0; j < kAdamBatch; ++j) {
      int32_t u = base + j * kAdamThreads;
      const bool ok = u < units;
      if (!ok) u = 0;  // clamped: loaded but never stored
      const int k = unit_group(a, u);
      grp[j] = ok ? k : -1;
      int32_t row = a.grp[0].row;
      const float* gp = a.grp[0].g;
      const float* pp = a.grp[0].p;
      const float* mp = a.grp[0].m;
      const float* vp = a.grp[0].v;
#pragma unroll
      for (int q = 1; q < kAdamGroups; ++q) {
        if (k == q) {
          row = a.grp[q].row;
          gp = a.grp[q].g;
          pp = a.grp[q].p;
          mp = a.grp[q].m;
          vp = a.grp[q].v;
        }
      }
      const int64_t e = first * row + 4 * (int64_t)u;  // float index of the unit in its group array
      at[j] = e;
      r0[j] = (uint32_t)(4 * u) % (uint32_t)row;  // the slice starts on a row boundary
      P[j] = load_stream(pp + e);
      G[j] = load_stream(gp + e);
      M[j] = load_stream(mp + e);
      V[j] = load_stream(vp + e);
    }
#pragma unroll
    for (int j = 0; j < kAdamBatch; ++j) {
      if (grp[j] < 0) continue;
      const int k = grp[j];
      AdamGroupDev q = a.grp[0];
#pragma unroll
      for (int s = 1; s < kAdamGroups; ++s)
        if (k == s) q = a.grp[s];
      float p[4] = {P[j].x, P[j].y, P[j].z, P[j].w};
      const float g[4] = {G[j].x, G[j].y, G[j].z, G[j].w};
      float m[4] = {M[j].x, M[j].y, M[j].z, M[j].w};
      float v[4] = {V[j].x, V[j].y, V[j].z, V[j].w};
      uint32_t r = r0[j];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        adam_float(p[t], g[t], m[t], v[t], adam_rate(q, r), a);
        r = (r + 1 == (uint32_t)q.row) ? 0u : r + 1;
      }
      store_stream(q.p + at[j], p);
      store_stream(q.m + at[j], m);
      store_stream(q.v + at[j], v);
    }
  }
}

__device__ __forceinline__ void adam_cluster_scalar(const AdamDev& a, int64_t first, int32_t count) {
#pragma unroll
  for (int k = 0; k < kAdamGroups; ++k) {
    const AdamGroupDev q = a.grp[k];
    const int32_t len = count * q.row;
    const int64_t start = first * q.row;
    for (int32_t e = threadIdx.x; e < len; e += kAdamThreads) {
      float p = q.p[start + e], m = q.m[start + e], v = q.v[start + e];
      adam_float(p, q.g[start + e], m, v, adam_rate(q, (uint32_t)e % (uint32_t)q.row), a);
      q.p[start + e] = p;
      q.m[start + e] = m;
      q.v[start + e] = v;
    }
  }
}

__global__ __launch_bounds__(kAdamThreads) void k_sparse_adam(AdamDev a, const uint32_t* __restrict__ visible) {
  const int64_t nc = (a.n + GSR_CLUSTER - 1) / GSR_CLUSTER;
  for (int i = 0; i < kAdamPer; ++i) {
    const int64_t c = (int64_t)blockIdx.x * kAdamPer + i;
    if (c >= nc) break;
    if (visible != nullptr && visible[c] == 0u) continue;
    const int64_t first = c * GSR_CLUSTER;
    const int64_t left = a.n - first;
    if (left >= GSR_CLUSTER)
      adam_cluster_vec(a, first);
    else
      adam_cluster_scalar(a, first, (int32_t)left);
  }
}

}  // namespace

void launch_sparse_adam(const AdamDev& a, const uint32_t* visible, hipStream_t s) {
  const int64_t nc = (a.n + GSR_CLUSTER - 1) / GSR_CLUSTER;
  if (nc > 0) k_sparse_adam<<<(unsigned)((nc + kAdamPer - 1) / kAdamPer), kAdamThreads, 0, s>>>(a, visible);
}

}  // namespace gsr
