// Device-wide exclusive prefix sum of u32 arrays (reduce, recursive scan of the
// block sums, downsweep) and small fill kernels.
#include "gsr_internal.h"

namespace gsr {
namespace {

constexpr int kThreads = 256;
constexpr int kRounds = 16;
constexpr int kBlockItems = kThreads * kRounds;  // 4096 items per block

__device__ inline uint32_t wave_inclusive_scan(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// Exclusive scan of one value per thread over a 256-thread block; also returns
// the block total. Contains two barriers.
__device__ inline uint32_t block_exclusive_scan(uint32_t x, uint32_t& total) {
  __shared__ uint32_t wsum[kThreads / 64];
  const uint32_t incl = wave_inclusive_scan(x);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kThreads / 64; ++i) {
    const uint32_t s = wsum[i];
    off += (i < w) ? s : 0u;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return off + incl - x;
}

__global__ __launch_bounds__(kThreads) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                          uint32_t* __restrict__ partials) {
  const int64_t base = (int64_t)blockIdx.x * kBlockItems;
  uint32_t s = 0;
#pragma unroll 4
  for (int r = 0; r < kRounds; ++r) {
    const int64_t i = base + r * kThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  uint32_t tot;
  block_exclusive_scan(s, tot);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// Exclusive scan of the block's 4096 items in 16 coalesced rounds, offset by the
// scanned block sum. in may alias out. The last block stores the grand total.
__global__ __launch_bounds__(kThreads) void k_scan_down(const uint32_t* in, uint32_t* out, int64_t n,
                                                        const uint32_t* __restrict__ partials,
                                                        uint32_t* __restrict__ total) {
  const int64_t base = (int64_t)blockIdx.x * kBlockItems;
  uint32_t carry = partials ? partials[blockIdx.x] : 0u;
  for (int r = 0; r < kRounds; ++r) {
    const int64_t i = base + r * kThreads + threadIdx.x;
    const uint32_t x = i < n ? in[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(x, tot);
    if (i < n) out[i] = carry + ex;
    carry += tot;
  }
  if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = carry;
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_f32(float* p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

int grid_for(int64_t n, int threads) {
  int64_t g = (n + threads - 1) / threads;
  if (g > 65536) g = 65536;
  return g < 1 ? 1 : (int)g;
}

}  // namespace

size_t scan_temp_words(int64_t n) {
  size_t words = 0;
  int64_t m = n;
  while (m > kBlockItems) {
    m = (m + kBlockItems - 1) / kBlockItems;
    words += (size_t)m + 64;
  }
  return words + 64;
}

void scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, uint32_t* temp,
                        hipStream_t s) {
  if (n <= 0) {
    if (total) fill_u32(total, 1, 0u, s);
    return;
  }
  const int64_t nb = (n + kBlockItems - 1) / kBlockItems;
  if (nb == 1) {
    k_scan_down<<<1, kThreads, 0, s>>>(in, out, n, nullptr, total);
    return;
  }
  uint32_t* partials = temp;
  k_scan_reduce<<<(unsigned)nb, kThreads, 0, s>>>(in, n, partials);
  scan_exclusive_u32(partials, partials, nb, nullptr, temp + nb + 64, s);
  k_scan_down<<<(unsigned)nb, kThreads, 0, s>>>(in, out, n, partials, total);
}

void fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return;
  k_fill_u32<<<grid_for(n, 256), 256, 0, s>>>(p, n, v);
}

void fill_f32(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return;
  k_fill_f32<<<grid_for(n, 256), 256, 0, s>>>(p, n, v);
}

}  // namespace gsr
