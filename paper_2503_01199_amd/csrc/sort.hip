// Stable LSD radix sort of (key, value) pairs, 8 bits per pass.
//
// Each pass: a per-block digit histogram (blocks own contiguous chunks, so block
// order is input order), an exclusive scan of the digit-major histogram (giving
// every (digit, block) its output offset), and a scatter in which each block walks
// its chunk in tiles of 256 items. Within a tile, items with equal digits are
// ranked by wave64 ballots over the 8 digit bits (lanes with the same digit form a
// "peer" mask; the rank is the population count of the lower peers), and by the
// per-wave counts of earlier waves, which keeps the sort stable.
#include "gsr_internal.h"

namespace gsr {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxBlocks = 2048;

template <typename K>
__global__ __launch_bounds__(kThreads) void k_radix_hist(const K* __restrict__ keys, int64_t n, int shift,
                                                         int64_t chunk, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  const int lane = threadIdx.x & 63;
  for (int64_t i0 = beg; i0 < end; i0 += kThreads) {
    const int64_t i = i0 + threadIdx.x;
    const bool valid = i < end;
    const uint32_t d = valid ? (uint32_t)(keys[i] >> shift) & 255u : 0u;
    // aggregate equal digits within the wave before touching LDS
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bal = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? bal : ~bal;
    }
    const uint64_t lower = peers & ((1ull << lane) - 1ull);
    if (valid && lower == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

template <typename K>
__global__ __launch_bounds__(kThreads) void k_radix_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                            K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                            int64_t n, int shift, int64_t chunk,
                                                            const uint32_t* __restrict__ offs) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wc[kWaves][256];
  const int t = threadIdx.x;
  const int w = t >> 6;
  const int lane = t & 63;
  base[t] = offs[(size_t)t * gridDim.x + blockIdx.x];
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  for (int64_t i0 = beg; i0 < end; i0 += kThreads) {
    const int64_t i = i0 + t;
    const bool valid = i < end;
    const K key = valid ? kin[i] : (K)0;
    const uint32_t val = valid ? (vin ? vin[i] : (uint32_t)i) : 0u;
    const uint32_t d = (uint32_t)(key >> shift) & 255u;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) wc[q][t] = 0;
    __syncthreads();
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bal = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? bal : ~bal;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & ((1ull << lane) - 1ull));
    if (valid && rank == 0) wc[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = base[d] + rank;
      for (int q = 0; q < w; ++q) pos += wc[q][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) add += wc[q][t];
    base[t] += add;
    __syncthreads();
  }
}

template <typename K>
__global__ void k_copy_pairs(const K* __restrict__ kin, const uint32_t* __restrict__ vin, K* __restrict__ kout,
                             uint32_t* __restrict__ vout, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    kout[i] = kin[i];
    vout[i] = vin ? vin[i] : (uint32_t)i;
  }
}

template <typename K>
int radix_sort(const K* keys_in, const uint32_t* vals_in, K* kb[2], uint32_t* vb[2], int64_t n, int bits,
               uint32_t* temp, hipStream_t s) {
  if (n <= 0) return 0;
  if (bits <= 0) {
    int g = (int)((n + 255) / 256);
    if (g > 65536) g = 65536;
    k_copy_pairs<K><<<g, 256, 0, s>>>(keys_in, vals_in, kb[0], vb[0], n);
    return 0;
  }
  int64_t G = (n + 2047) / 2048;
  if (G > kMaxBlocks) G = kMaxBlocks;
  if (G < 1) G = 1;
  const int64_t chunk = (n + G - 1) / G;
  uint32_t* hist = temp;
  uint32_t* offs = temp + 256 * kMaxBlocks;
  uint32_t* stemp = temp + 2 * 256 * kMaxBlocks;
  const K* kcur = keys_in;
  const uint32_t* vcur = vals_in;
  int out = 0;
  for (int shift = 0; shift < bits; shift += 8) {
    k_radix_hist<K><<<(unsigned)G, kThreads, 0, s>>>(kcur, n, shift, chunk, hist);
    scan_exclusive_u32(hist, offs, 256 * G, nullptr, stemp, s);
    k_radix_scatter<K><<<(unsigned)G, kThreads, 0, s>>>(kcur, vcur, kb[out], vb[out], n, shift, chunk, offs);
    kcur = kb[out];
    vcur = vb[out];
    out ^= 1;
  }
  return out ^ 1;
}

}  // namespace

size_t radix_temp_words() { return 2 * 256 * (size_t)kMaxBlocks + scan_temp_words(256 * (int64_t)kMaxBlocks); }

int radix_sort_u32(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* kb[2], uint32_t* vb[2], int64_t n,
                   int bits, uint32_t* temp, hipStream_t s) {
  return radix_sort<uint32_t>(keys_in, vals_in, kb, vb, n, bits, temp, s);
}

int radix_sort_u64(const uint64_t* keys_in, const uint32_t* vals_in, uint64_t* kb[2], uint32_t* vb[2], int64_t n,
                   int bits, uint32_t* temp, hipStream_t s) {
  return radix_sort<uint64_t>(keys_in, vals_in, kb, vb, n, bits, temp, s);
}

}  // namespace gsr
