// Densification driven by the opacity-gradient variance metric, and opacity decay
// (Sec. 3.3).
//
// Candidates are the Gaussians with the largest C Var metric at or above a
// threshold, at most max_candidates of them, ties to the lower index. Selection
// is a stable radix sort of one 32-bit key per Gaussian: the complemented FP32
// bits of a qualifying metric (all of them positive, so the bits order like the
// values and the complement sorts largest first) and 0xffffffff for the rest.
// Qualifying keys then form a prefix of the sorted list, whose end one thread
// finds. A candidate whose largest log-scale exceeds a bound is split into two
// children placed by caller-supplied normal draws; the others are cloned. The
// split parents and the originals below an opacity bound leave.
//
// The output is described by a row map: kept originals in index order (an
// exclusive scan of the keep flags gives their rows), then each candidate's clone
// or two children in rank order (an exclusive scan of the children counts per
// rank). Every array is then written through the map in one gather; the means and
// log-scales of children are computed in FP64 on the way. Counts stay on the
// device; the new row count is written for the caller.
#include <algorithm>

#include "gsr_internal.h"

namespace gsr {
namespace {

constexpr int kThreads = 256;
enum : uint32_t { kOpNone = 0, kOpClone = 1, kOpSplit = 2 };
enum : uint32_t { kKindKept = 0, kKindClone = 1, kKindChild0 = 2, kKindChild1 = 3 };
enum : int {
  kDhCandidates = 0,  // k = min(qualifying, max_candidates)
  kDhKept = 1,        // originals kept
  kDhChildren = 2,    // rows appended (1 per clone, 2 per split)
  kDhRows = 3,        // output rows
  kDhQualifying = 4,  // Gaussians with metric >= threshold
};

unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

__global__ void k_dens_keys(const float* __restrict__ metric, int64_t n, float thr, uint32_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const float m = metric[i];
  keys[i] = (m >= thr) ? ~__float_as_uint(m) : 0xffffffffu;  // thr > 0: a qualifying m is positive
}

// The end of the qualifying prefix of the sorted keys (the header starts at zero, so
// an empty prefix needs no writer).
__global__ void k_dens_count(const uint32_t* __restrict__ skeys, int64_t n, int64_t kmax,
                             uint32_t* __restrict__ hdr) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  if (skeys[i] != 0xffffffffu && (i + 1 == n || skeys[i + 1] == 0xffffffffu)) {
    hdr[kDhQualifying] = (uint32_t)(i + 1);
    hdr[kDhCandidates] = (uint32_t)min<int64_t>(i + 1, kmax);
  }
}

// Rank r < k: candidate svals[r] (svals null: the identity) is split or cloned.
// Every kernel that indexes with sorted values or scanned positions leaves when a
// device-wide wait of the round gave up (the error word): those may be garbage.
__global__ void k_dens_mark(const uint32_t* __restrict__ svals, int64_t kmax, const uint32_t* __restrict__ hdr,
                            const float* __restrict__ log_scales, float split_ls, uint32_t* __restrict__ op,
                            uint32_t* __restrict__ cc, const uint32_t* __restrict__ err) {
  if (error_raised(err)) return;
  const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (r >= kmax) return;
  if (r >= (int64_t)hdr[kDhCandidates]) {
    cc[r] = 0u;
    return;
  }
  const uint32_t i = svals ? svals[r] : (uint32_t)r;
  const float* s = log_scales + 3 * (int64_t)i;
  const bool split = fmaxf(fmaxf(s[0], s[1]), s[2]) > split_ls;
  op[i] = split ? kOpSplit : kOpClone;
  cc[r] = split ? 2u : 1u;
}

__global__ void k_dens_keep(const uint32_t* __restrict__ op, const float* __restrict__ logits, float prune,
                            int64_t n, uint32_t* __restrict__ keep) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  keep[i] = (op[i] != kOpSplit && !(logits[i] < prune)) ? 1u : 0u;
}

__global__ void k_dens_map_kept(const uint32_t* __restrict__ keep, const uint32_t* __restrict__ pos, int64_t n,
                                uint32_t* __restrict__ src, uint32_t* __restrict__ kind,
                                const uint32_t* __restrict__ err) {
  if (error_raised(err)) return;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n || keep[i] == 0u) return;
  src[pos[i]] = (uint32_t)i;
  kind[pos[i]] = kKindKept;
}

__global__ void k_dens_map_new(const uint32_t* __restrict__ svals, const uint32_t* __restrict__ cc,
                               const uint32_t* __restrict__ coff, int64_t kmax, uint32_t* __restrict__ hdr,
                               const uint32_t* __restrict__ err, uint32_t* __restrict__ src,
                               uint32_t* __restrict__ kind, int64_t* __restrict__ n_out) {
  const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool bad = error_raised(err);
  if (r == 0) {  // no output rows after a wait gave up: the later gathers do nothing
    const uint32_t rows = bad ? 0u : hdr[kDhKept] + hdr[kDhChildren];
    hdr[kDhRows] = rows;
    if (n_out) *n_out = bad ? -1 : (int64_t)rows;
  }
  if (bad || r >= kmax || cc[r] == 0u) return;
  const uint32_t i = svals ? svals[r] : (uint32_t)r;
  const uint32_t base = hdr[kDhKept] + coff[r];
  if (cc[r] == 1u) {
    src[base] = i;
    kind[base] = kKindClone;
  } else {
    src[base] = i;
    kind[base] = kKindChild0;
    src[base + 1] = i;
    kind[base + 1] = kKindChild1;
  }
}

// out[j, :] = in[src[j], :] for the j < rows of the output; state arrays (zero_new)
// take zeros in rows that are not kept originals.
__global__ void k_dens_gather(const uint32_t* __restrict__ src, const uint32_t* __restrict__ kind,
                              const uint32_t* __restrict__ hdr, int64_t rows_max, const float* __restrict__ in,
                              float* __restrict__ out, int32_t rf, int zero_new) {
  const int64_t rows = min<int64_t>(rows_max, hdr[kDhRows]);
  const int64_t total = rows * rf;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
    const int64_t j = t / rf;
    const int64_t c = t - j * rf;
    out[t] = (zero_new && kind[j] != kKindKept) ? 0.0f : in[(int64_t)src[j] * rf + c];
  }
}

// Means and log-scales of the output rows: children at mean + R(q) (exp(s) * z_c)
// with log-scales s - ln(factor), in FP64; every other row copied.
__global__ void k_dens_geometry(const uint32_t* __restrict__ src, const uint32_t* __restrict__ kind,
                                const uint32_t* __restrict__ hdr, int64_t rows_max, const float* __restrict__ means,
                                const float* __restrict__ log_scales, const float* __restrict__ quats,
                                const float* __restrict__ noise, double ln_factor, float* __restrict__ out_means,
                                float* __restrict__ out_log_scales) {
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t rows = min<int64_t>(rows_max, hdr[kDhRows]);
  if (j >= rows) return;
  const int64_t i = src[j];
  const uint32_t kd = kind[j];
  if (kd < kKindChild0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      out_means[3 * j + a] = means[3 * i + a];
      out_log_scales[3 * j + a] = log_scales[3 * i + a];
    }
    return;
  }
  double w = quats[4 * i], x = quats[4 * i + 1], y = quats[4 * i + 2], z = quats[4 * i + 3];
  const double inv = 1.0 / sqrt(w * w + x * x + y * y + z * z);
  w *= inv;
  x *= inv;
  y *= inv;
  z *= inv;
  const double R[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                          {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                          {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
  const float* zc = noise + 6 * i + 3 * (kd - kKindChild0);
  double d[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) d[a] = exp((double)log_scales[3 * i + a]) * (double)zc[a];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    out_means[3 * j + a] = (float)((double)means[3 * i + a] + (R[a][0] * d[0] + R[a][1] * d[1] + R[a][2] * d[2]));
    out_log_scales[3 * j + a] = (float)((double)log_scales[3 * i + a] - ln_factor);
  }
}

__global__ void k_opacity_decay(float* __restrict__ logits, int64_t n, double factor) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const double o = factor / (1.0 + exp(-(double)logits[i]));
  logits[i] = (float)(log(o) - log1p(-o));
}

size_t align64(size_t w) { return (w + 63) & ~(size_t)63; }

struct DensLayout {
  size_t keys, kb0, kb1, vb0, vb1, op, keep, pos, cc, coff, src, kind, hdr, err, ctl_sort, ctl_scan1, ctl_scan2,
      total;
};

DensLayout dens_layout(int64_t n, int64_t kmax) {
  DensLayout L{};
  size_t w = 0;
  auto take = [&](size_t words) {
    const size_t at = w;
    w += align64(words);
    return at;
  };
  const size_t N = (size_t)n, K = (size_t)std::max<int64_t>(kmax, 1);
  L.keys = take(N);
  L.kb0 = take(N);
  L.kb1 = take(N);
  L.vb0 = take(N);
  L.vb1 = take(N);
  L.op = take(N);
  L.keep = take(N);
  L.pos = take(N);
  L.cc = take(K);
  L.coff = take(K);
  L.src = take(N + K);
  L.kind = take(N + K);
  L.hdr = take(64);  // header, error word and control words: cleared together
  L.err = take(64);
  L.ctl_sort = take(sort_ctl_words(n, 32));
  L.ctl_scan1 = take(scan_ctl_words(n));
  L.ctl_scan2 = take(scan_ctl_words(K));
  L.total = w;
  return L;
}

}  // namespace

size_t densify_words(int64_t n, int64_t max_candidates) { return dens_layout(n, max_candidates).total; }

void densify(const DensifyArgs& a, uint32_t* ws, hipStream_t s) {
  const int64_t n = a.n, K = a.max_candidates;
  const DensLayout L = dens_layout(n, K);
  uint32_t* hdr = ws + L.hdr;
  uint32_t* err = ws + L.err;
  fill_u32(hdr, (int64_t)(L.total - L.hdr), 0u, s);
  fill_u32(ws + L.op, n, 0u, s);
  k_dens_keys<<<blocks_for(n), kThreads, 0, s>>>(a.metric, n, a.threshold, ws + L.keys);
  uint32_t* kb[2] = {ws + L.kb0, ws + L.kb1};
  uint32_t* vb[2] = {ws + L.vb0, ws + L.vb1};
  const int r = radix_sort_u32_dev(ws + L.keys, nullptr, kb, vb, n, nullptr, 32, ws + L.ctl_sort, err, false, s);
  const uint32_t* skeys = r < 0 ? ws + L.keys : kb[r];
  const uint32_t* svals = r < 0 ? nullptr : vb[r];
  k_dens_count<<<blocks_for(n), kThreads, 0, s>>>(skeys, n, K, hdr);
  if (K > 0)
    k_dens_mark<<<blocks_for(K), kThreads, 0, s>>>(svals, K, hdr, a.log_scales, a.split_log_scale, ws + L.op,
                                                  ws + L.cc, err);
  k_dens_keep<<<blocks_for(n), kThreads, 0, s>>>(ws + L.op, a.opacity_logits, a.prune_logit, n, ws + L.keep);
  scan_u32(ws + L.keep, nullptr, ws + L.pos, n, nullptr, hdr + kDhKept, nullptr, ws + L.ctl_scan1, err, s);
  if (K > 0)
    scan_u32(ws + L.cc, nullptr, ws + L.coff, K, nullptr, hdr + kDhChildren, nullptr, ws + L.ctl_scan2, err, s);
  k_dens_map_kept<<<blocks_for(n), kThreads, 0, s>>>(ws + L.keep, ws + L.pos, n, ws + L.src, ws + L.kind, err);
  k_dens_map_new<<<blocks_for(std::max<int64_t>(K, 1)), kThreads, 0, s>>>(svals, ws + L.cc, ws + L.coff, K, hdr, err,
                                                                     ws + L.src, ws + L.kind, a.n_out);
  const int64_t rows_max = n + K;
  k_dens_geometry<<<blocks_for(rows_max), kThreads, 0, s>>>(ws + L.src, ws + L.kind, hdr, rows_max, a.means,
                                                            a.log_scales, a.quats, a.noise, a.ln_split_factor,
                                                            a.out_means, a.out_log_scales);
  for (int q = 0; q < a.n_copy; ++q) {
    const int64_t floats = rows_max * a.copy_rf[q];
    const unsigned g = (unsigned)std::min<int64_t>(std::max<int64_t>(1, (floats + kThreads - 1) / kThreads), 65536);
    k_dens_gather<<<g, kThreads, 0, s>>>(ws + L.src, ws + L.kind, hdr, rows_max, a.copy_in[q], a.copy_out[q],
                                         a.copy_rf[q], a.copy_zero_new[q]);
  }
}

void launch_opacity_decay(float* logits, int64_t n, double factor, hipStream_t s) {
  if (n > 0) k_opacity_decay<<<blocks_for(n), kThreads, 0, s>>>(logits, n, factor);
}

}  // namespace gsr
