// Single-pass device-wide scan and one-sweep LSD radix sort with decoupled
// look-back, both driven by counts that live in device memory (so a frame is
// enqueued without waiting on the host).
//
// Look-back protocol: block b owns tile b and waits only on lower tiles, whose blocks
// the dispatcher has placed before it (workgroups are dispatched in id order; an
// atomic ticket per block would cost a serialised device-scope atomic per block on
// one address, ~20 us per pass here). A block publishes its tile aggregate, adds
// the aggregates of the earlier tiles of its group of 32, and walks back over the
// groups' status words until it meets an inclusive prefix; a group's last tile
// publishes the group's aggregate and then its inclusive prefix (look_back_grouped).
// Grids hold one block per tile of the largest possible count; blocks past the
// count on the device leave at once. A status word
// is (flag << 30 | value): flag 0 = not ready, 1 = aggregate, 2 = inclusive
// prefix. Values must stay below 2^30: a larger prefix sets the count bit of the
// error word (the result is then wrong but every access stays in bounds).
//
// Waits: every wait is bounded by elapsed time (kWaitTicks) and reads the error
// word on each round. A wait that runs out raises the word's abort bit; any raised
// bit ends every other wait at its next round and makes every block skip its
// writes, and every later kernel of the frame checks the word at entry and leaves.
// A protocol or scheduling failure therefore surfaces within one bound as an
// error status of the frame, instead of as minutes of per-block spinning.
#include <algorithm>

#include "gsr_internal.h"

namespace gsr {
namespace {

constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagPrefix = 2u << 30;
constexpr uint32_t kValueMask = (1u << 30) - 1u;
// s_memrealtime counts at a constant 100 MHz on gfx9 parts: 100 ms. A legitimate
// wait lasts as long as earlier tiles take to publish (microseconds; at most the
// pass itself, ~2 ms on the largest sorts here).
constexpr uint64_t kWaitTicks = 100ull * 100000ull;

__device__ __forceinline__ uint32_t ld_status(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_status(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Deadline of one wait. over(): the error word is raised (by another block, or by
// the host), or the deadline has passed, in which case this wait raises the abort
// bit itself.
struct WaitBound {
  uint64_t t0;
  __device__ WaitBound() : t0(__builtin_amdgcn_s_memrealtime()) {}
  __device__ bool over(uint32_t* err) const {
    if (ld_status(err) != 0u) return true;
    if (__builtin_amdgcn_s_memrealtime() - t0 > kWaitTicks) {
      atomicOr(err, kErrAbort);
      return true;
    }
    return false;
  }
};

// Block entry: the error word and the item count (n_dev, or n_host when null), read
// once for the whole block by one thread, both loads in one round trip (waves could
// otherwise read the word at different times while other blocks raise it). A raised
// word means an earlier stage gave up and the count may be garbage: the caller
// leaves without using it. Every thread must call it; it also clears the block's
// incomplete-wait flag (block_incomplete).
struct BlockStart {
  bool error;
  int64_t n;
};
__device__ __forceinline__ BlockStart block_start(uint32_t* err, const uint32_t* n_dev, int64_t n_host,
                                                  uint32_t& s_incomplete) {
  __shared__ uint32_t s_err;
  __shared__ int64_t s_n;
  if (threadIdx.x == 0) {
    const uint32_t e = ld_status(err);
    const int64_t n = n_dev ? (int64_t)ld_status(n_dev) : n_host;
    s_err = e;
    s_n = n;
    s_incomplete = 0u;
  }
  __syncthreads();
  return {s_err != 0u, s_n};
}

// After the look-back: whether any thread's waits ended before its prefix was
// complete (they end early only when the error word is raised). Every thread must
// call it with its own look-back's completion; it synchronises the block.
__device__ __forceinline__ bool block_incomplete(bool complete, uint32_t& s_incomplete) {
  if (!complete) s_incomplete = 1u;
  __syncthreads();
  return s_incomplete != 0u;
}

// Sum, in status column `col` (stride `stride` words between entries), of the
// values from entry b down to the nearest inclusive prefix, that prefix included
// (entries below 0 count as an empty prefix). The walk reads kWindow entries per
// round trip (kFirstWindow in the first: the nearest prefix is usually the entry
// just below, and every status read goes past the XCD's L2) and consumes them in
// order, waiting on entries not yet published.
constexpr int kWindow = 16;
constexpr int kFirstWindow = 4;

__device__ uint32_t walk_back(const uint32_t* status, int64_t b, int64_t stride, int col, uint32_t* err,
                              bool& complete) {
  uint32_t excl = 0;
  const WaitBound bound;
  bool found = false;
  int win = kFirstWindow;
  while (!found) {
    uint32_t st[kWindow];
#pragma unroll
    for (int q = 0; q < kWindow; ++q)
      st[q] = q >= win ? 0u : b - q >= 0 ? ld_status(status + (b - q) * stride + col) : kFlagPrefix;
    const int read = win;
    win = kWindow;
    int used = 0;
#pragma unroll
    for (int q = 0; q < kWindow; ++q) {
      if (found || used < q) continue;  // stop at a prefix or at the first status not yet published
      const uint32_t flag = st[q] & ~kValueMask;
      if (flag == 0) continue;
      excl += st[q] & kValueMask;
      used = q + 1;
      if (flag == kFlagPrefix) found = true;
    }
    if (found) break;
    b -= used;
    if (used < read) {  // stopped at a status not yet published: wait a little
      if (bound.over(err)) break;
      __builtin_amdgcn_s_sleep(1);
    }
  }
  complete = found;
  return excl;
}

// Two-level look-back for many tiles. Tiles form groups of kGroup; a tile adds
// the aggregates of the earlier tiles of its group (published right after they
// rank, so one round trip) and walks back over whole groups, whose last tile
// publishes the group's aggregate and then its inclusive prefix. An inclusive
// prefix thus reaches kWindow * kGroup tiles further per round trip, instead of
// kWindow. Every wait is on a lower tile, so in-order dispatch guarantees
// progress. tstat: [tiles][stride] per-tile aggregates; gstat: [groups][stride].
constexpr int kGroup = 32;

// The look-back in two steps, so that a caller can do other work between them
// while its aggregate reaches the later tiles: look_back_publish publishes the
// tile's aggregate (returned, clipped to the value range); look_back_gather then
// waits for the exclusive prefix. publish = false (tests of the error path only):
// the tile never publishes. complete: the prefix found is whole (false only when a
// wait gave up).
__device__ __forceinline__ uint32_t look_back_publish(uint32_t* tstat, int64_t tile, int64_t stride, int col,
                                                      uint32_t agg, uint32_t* err, bool publish = true) {
  if (agg > kValueMask) {
    atomicOr(err, kErrCount);
    agg &= kValueMask;
  }
  if (publish) st_status(tstat + tile * stride + col, kFlagAgg | agg);
  return agg;
}

__device__ uint32_t look_back_gather(uint32_t* tstat, uint32_t* gstat, int64_t tile, int64_t stride, int col,
                                     uint32_t agg, uint32_t* err, bool& complete, bool publish = true) {
  const int64_t g = tile / kGroup, g0 = g * kGroup;
  const bool last = publish && tile % kGroup == kGroup - 1;
  // exclusive sum over the group's earlier tiles g0 .. tile - 1
  uint32_t E = 0;
  const WaitBound bound;
  for (;;) {
    uint32_t v[kGroup - 1];
#pragma unroll
    for (int q = 0; q < kGroup - 1; ++q) {  // all loads in flight at once (the condition is uniform)
      const int64_t j = tile - 1 - q;
      v[q] = j >= g0 ? ld_status(tstat + j * stride + col) : kFlagAgg;
    }
    bool ready = true;
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < kGroup - 1; ++q) {
      ready = ready && (v[q] & ~kValueMask) != 0;
      sum += v[q] & kValueMask;
    }
    if (ready) {
      E = sum;
      break;
    }
    if (bound.over(err)) {
      E = sum;
      complete = false;
      return E;  // the prefix is partial: publish nothing further
    }
    __builtin_amdgcn_s_sleep(1);
  }
  if (last) st_status(gstat + g * stride + col, kFlagAgg | ((E + agg) & kValueMask));
  bool walked = true;
  const uint32_t X = g > 0 ? walk_back(gstat, g - 1, stride, col, err, walked) : 0u;
  complete = walked;
  if ((uint64_t)X + E + agg > kValueMask) atomicOr(err, kErrCount);
  if (last && walked) st_status(gstat + g * stride + col, kFlagPrefix | ((X + E + agg) & kValueMask));
  return X + E;
}

__device__ __forceinline__ uint32_t look_back_grouped(uint32_t* tstat, uint32_t* gstat, int64_t tile, int64_t stride,
                                                      int col, uint32_t agg, uint32_t* err, bool& complete,
                                                      bool publish = true) {
  agg = look_back_publish(tstat, tile, stride, col, agg, err, publish);
  return look_back_gather(tstat, gstat, tile, stride, col, agg, err, complete, publish);
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// ------------------------------------------------------------------ scan
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;  // 2048

// out[k] = sum_{i<k} in(i) for k < n, n = *n_dev (or n_host when n_dev is null).
// in(i) = src[idx ? idx[i] : i]. total (nullable) receives the sum of all n items;
// when list != nullptr, every i with in(i) != 0 also writes list[out[i]] = i.
__global__ __launch_bounds__(kScanThreads) void k_scan(const uint32_t* __restrict__ src,
                                                       const uint32_t* __restrict__ idx, uint32_t* __restrict__ out,
                                                       int64_t n_host, const uint32_t* __restrict__ n_dev,
                                                       uint32_t* __restrict__ total, uint32_t* __restrict__ list,
                                                       uint32_t* __restrict__ ctl, uint32_t* __restrict__ err) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  __shared__ uint32_t s_excl, s_incomplete;
  const BlockStart bs = block_start(err, n_dev, n_host, s_incomplete);
  if (bs.error) return;  // an earlier stage gave up: its counts and indices may be garbage
  const int64_t n = bs.n;
  const int t = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int64_t base = tile * kScanTile;
  if (base >= n && !(tile == 0 && n == 0)) return;
  uint32_t v[kScanItems];
  uint32_t sum = 0;
  const int64_t first = base + (int64_t)t * kScanItems;
  if (n > 0) {
    // all loads first (indices clamped into range, so none sits behind a branch),
    // then the gathers, then the masking: the memory round trips overlap
    uint32_t j[kScanItems];
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
      const int64_t i = first + q < n ? first + q : n - 1;
      j[q] = idx ? idx[i] : (uint32_t)i;
    }
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) v[q] = src[j[q]];
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
      v[q] = first + q < n ? v[q] : 0u;
      sum += v[q];
    }
  } else {
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) v[q] = 0u;
  }
  const uint32_t incl = wave_incl_scan(sum);
  if ((t & 63) == 63) wsum[t >> 6] = incl;
  __syncthreads();
  uint32_t agg = 0, off = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; ++w) {
    off += (w < (t >> 6)) ? wsum[w] : 0u;
    agg += wsum[w];
  }
  bool complete = true;
  if (t == 0) {
    const int64_t tiles = max<int64_t>(1, (n_host + kScanTile - 1) / kScanTile);
    s_excl = look_back_grouped(ctl + 1, ctl + 1 + tiles, tile, 1, 0, agg, err, complete);
  }
  if (block_incomplete(complete, s_incomplete)) return;  // a wait gave up: the prefix may be partial
  uint32_t run = s_excl + off + incl - sum;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    const int64_t i = first + q;
    if (i < n) {
      out[i] = run;
      if (list && v[q]) list[run] = (uint32_t)i;
    }
    run += v[q];
  }
  if (total && (base + kScanTile >= n) && t == kScanThreads - 1) *total = run;
}

// ------------------------------------------------------------------ radix sort
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;
constexpr int kSortTile = kSortThreads * kSortRounds;  // 2048 items per tile
constexpr int kHistBlocks = 512;
constexpr int64_t kHistChunk = 4096;  // keys per histogram block at least
constexpr int kMaxPasses = 8;
constexpr int64_t kWideSortItems = int64_t(1) << 24;  // from this capacity: 4096-item tiles, 16-byte histogram loads

// Items per one-sweep tile for a sort of capacity n_max: 4096 from kWideSortItems on
// (digits leave in longer runs, the look-back has fewer tiles), else 2048. 1024-item
// tiles, which give small sorts more blocks than CUs (the room's depth sort of 409k
// records has 200 tiles of 2048 for 256 CUs), measured slower: 12.7 against 11.5 us
// per depth-sort pass (the look-back chain doubles).
inline int64_t sort_tile_items(int64_t n_max) { return n_max >= kWideSortItems ? 2 * kSortTile : kSortTile; }

// Lanes of the wave holding the same 8-bit digit d (restricted to `valid` lanes).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint64_t bal = __ballot((d >> b) & 1u);
    peers &= ((d >> b) & 1u) ? bal : ~bal;
  }
  return peers;
}

// Digit histograms of every pass in one read of the keys, merged into hist[p][d]
// (which starts at zero); each scatter block scans its pass's 256 counts into digit
// offsets itself. Counting needs no ranks. With kRuns (keys in spatial order, whose high bytes repeat), each thread
// takes 8 consecutive keys and adds each run of equal digits to its LDS counter
// with one atomic, since per-key atomics on one address would serialise within an
// instruction; otherwise each key adds 1 directly.
// Blocks take at least kHistChunk keys each (their number is chosen from the count
// on the device, so the same-address atomics of the final merge stay few). Blocks
// beyond the needed number leave at once.
template <typename K, bool kRuns>
__global__ __launch_bounds__(kSortThreads) void k_os_hist(const K* __restrict__ keys, int64_t n_host,
                                                          const uint32_t* __restrict__ n_dev, int passes,
                                                          uint32_t* __restrict__ hist, const uint32_t* __restrict__ err) {
  __shared__ uint32_t h[kMaxPasses][256];
  // the error word (set by an earlier kernel only: the same for every wave) and the
  // count, loaded together; a raised word means the count may be garbage
  const uint32_t e = ld_status(err);
  const int64_t n = n_dev ? (int64_t)ld_status(n_dev) : n_host;
  if (e != 0u) return;
  int64_t nb = (n + kHistChunk - 1) / kHistChunk;
  if (nb < 1) nb = 1;
  if (nb > gridDim.x) nb = gridDim.x;
  if (blockIdx.x >= nb) return;
  const int t = threadIdx.x;
  const int lane = t & 63;
  for (int p = 0; p < passes; ++p) h[p][t] = 0;
  __syncthreads();
  if constexpr (!kRuns && sizeof(K) == 4) {
    // Large sorts of 32-bit keys: four per 16-byte load, so a thread has 32 keys in
    // flight (two blocks per CU with one key per load leave too few bytes in flight
    // for HBM). Small sorts keep one key per load, which spreads them over more
    // iterations.
    if (n_host >= kWideSortItems && (reinterpret_cast<uintptr_t>(keys) & 15u) == 0) {
      constexpr int64_t kStep = (int64_t)kSortTile * 4;
      for (int64_t base = (int64_t)blockIdx.x * kStep; base < n; base += nb * kStep) {
        uint4 q[kSortRounds];
#pragma unroll
        for (int r = 0; r < kSortRounds; ++r) {
          const int64_t i = base + 4 * ((int64_t)r * kSortThreads + t);
          if (i + 3 < n) {
            q[r] = *reinterpret_cast<const uint4*>(keys + i);
          } else {
            q[r].x = (uint32_t)keys[i < n ? i : n - 1];
            q[r].y = (uint32_t)keys[i + 1 < n ? i + 1 : n - 1];
            q[r].z = (uint32_t)keys[i + 2 < n ? i + 2 : n - 1];
            q[r].w = (uint32_t)keys[i + 3 < n ? i + 3 : n - 1];
          }
        }
#pragma unroll
        for (int r = 0; r < kSortRounds; ++r) {
          const int64_t i = base + 4 * ((int64_t)r * kSortThreads + t);
          const uint32_t e[4] = {q[r].x, q[r].y, q[r].z, q[r].w};
#pragma unroll
          for (int c = 0; c < 4; ++c)
            if (i + c < n)
              for (int p = 0; p < passes; ++p) atomicAdd(&h[p][(e[c] >> (8 * p)) & 255u], 1u);
        }
      }
      goto merge;
    }
  }
  for (int64_t base = (int64_t)blockIdx.x * kSortTile; base < n; base += nb * kSortTile) {
    if constexpr (!kRuns) {
      K key[kSortRounds];
#pragma unroll
      for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = base + r * kSortThreads + t;
        key[r] = keys[i < n ? i : n - 1];
      }
#pragma unroll
      for (int r = 0; r < kSortRounds; ++r) {
        if (base + r * kSortThreads + t < n)
          for (int p = 0; p < passes; ++p) atomicAdd(&h[p][(uint32_t)(key[r] >> (8 * p)) & 255u], 1u);
      }
      continue;
    }
    const int64_t first = base + (int64_t)t * kSortRounds;  // this thread's consecutive keys
    K key[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) key[r] = keys[first + r < n ? first + r : n - 1];
    const int nv = (int)max<int64_t>(0, min<int64_t>(kSortRounds, n - first));  // valid keys of the thread
    for (int p = 0; p < passes; ++p) {
      uint32_t prev = (uint32_t)(key[0] >> (8 * p)) & 255u, run = nv > 0 ? 1u : 0u;
#pragma unroll
      for (int r = 1; r < kSortRounds; ++r) {
        if (r >= nv) break;
        const uint32_t d = (uint32_t)(key[r] >> (8 * p)) & 255u;
        if (d == prev) {
          ++run;
        } else {
          atomicAdd(&h[p][prev], run);
          prev = d;
          run = 1;
        }
      }
      if (run) atomicAdd(&h[p][prev], run);
    }
  }
merge:
  __syncthreads();
  for (int p = 0; p < passes; ++p)
    if (h[p][t]) atomicAdd(&hist[p * 256 + t], h[p][t]);
}

// One pass: block b takes tile b of kTile items. Wave w owns the contiguous quarter
// [w kTile/4, (w+1) kTile/4) of the tile and ranks it round by round (64 consecutive
// items per round, coalesced): the lanes holding the same 8-bit digit find each
// other by ballots, and a per-wave running count per digit in LDS gives each item
// its rank among the wave's earlier items of that digit. Ordering by (wave, round,
// lane) is the input order, so the ranks are stable. The block then learns the
// per-digit counts of all earlier tiles by look-back and scatters; the tile is first
// reordered by digit in LDS, so that consecutive threads store consecutive positions
// of each digit's run (a direct per-item scatter writes 256 short runs from
// scattered lanes). The per-wave counters take 4 KB of LDS whatever the tile size,
// so more blocks fit on a CU than with per-round counters; the tile is staged
// before the look-back, so that keys and values leave the registers first. A
// 4096-item tile of 32-bit keys is held to 128 registers: four blocks per CU.
template <typename K, int R>
__global__ __launch_bounds__(kSortThreads) __attribute__((amdgpu_waves_per_eu(R > 8 && sizeof(K) == 4 ? 4 : 1))) void k_os_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                             K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                             int64_t n_host, const uint32_t* __restrict__ n_dev,
                                                             int shift, const uint32_t* __restrict__ hist,
                                                             uint32_t* __restrict__ ctl, uint32_t* __restrict__ err,
                                                             int64_t withhold) {
  constexpr int kTile = kSortThreads * R;  // items per tile: R rounds of one item per thread
  constexpr int kWaves = kSortThreads / 64;
  constexpr int kQuarter = kTile / kWaves;  // items per wave
  __shared__ uint32_t wcnt[kWaves][256];    // running count, then exclusive offset, per (wave, digit)
  __shared__ __align__(16) K s_key[kTile];
  __shared__ uint32_t s_val[kTile];
  __shared__ uint32_t gofs[256], ldig[256], wtot[kWaves], htot[kWaves];
  __shared__ uint32_t s_incomplete;
  const BlockStart bs = block_start(err, n_dev, n_host, s_incomplete);
  if (bs.error) return;  // an earlier stage gave up: its counts may be garbage
  const int64_t n = bs.n;
  const int t = threadIdx.x;
  const int w = t >> 6;
  const int lane = t & 63;
  {
    const int64_t tile = blockIdx.x;
    const int64_t base = tile * kTile;
    if (base >= n) return;  // uniform over the block
#pragma unroll
    for (int q = 0; q < 4; ++q) wcnt[w][lane + 64 * q] = 0;
    const int64_t wbase = base + (int64_t)w * kQuarter + lane;  // round r: item wbase + 64 r
    K key[R];
    uint32_t rd[R];  // rank among the wave's items of the same digit, | digit << 16 (256: past the end)
    uint32_t val[R];
    // every round's loads first (indices clamped into range, so none sits behind a
    // branch and their round trips overlap), then the ranking; tiles of up to 2048
    // items load their values with the keys too, larger ones after the ranking (so
    // that the ranking's registers are not held by them)
    constexpr bool kEarlyVals = R <= 8;
    // the pass's count of digit t over all keys (loaded with the values); its
    // exclusive scan over the digits is the digit's first output position
    uint32_t hcount = kEarlyVals ? hist[t] : 0u;
    auto load_vals = [&]() __attribute__((always_inline)) {
      if (vin) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int64_t i = wbase + 64 * r;
          val[r] = vin[i < n ? i : n - 1];
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) val[r] = (uint32_t)(wbase + 64 * r);
      }
    };
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = wbase + 64 * r;
      key[r] = kin[i < n ? i : n - 1];
    }
    if constexpr (kEarlyVals) load_vals();
    // the wave's counters are zero before its first read (LDS runs a wave's
    // instructions in order)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool valid = wbase + 64 * r < n;
      const uint32_t d = valid ? (uint32_t)(key[r] >> shift) & 255u : 256u;
      const uint64_t peers = match_digit(d & 255u, valid);
      const uint32_t before = valid ? wcnt[w][d] : 0u;
      const uint32_t below = (uint32_t)__popcll(peers & ((1ull << lane) - 1ull));
      rd[r] = (before + below) | (d << 16);
      if (valid && below == 0) wcnt[w][d] = before + (uint32_t)__popcll(peers);
      // the next round reads what this one wrote (in order within the wave)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if constexpr (!kEarlyVals) {
      load_vals();
      hcount = hist[t];
    }
    __syncthreads();
    // thread d: exclusive offsets of digit d over the waves, then the tile total,
    // published at once (the staging below overlaps its way to the later tiles)
    uint32_t run = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
      const uint32_t c = wcnt[q][t];
      wcnt[q][t] = run;
      run += c;
    }
    const int64_t tiles = (n_host + kTile - 1) / kTile;
    const uint32_t agg = look_back_publish(ctl + 64, tile, 256, t, run, err, tile != withhold);
    // exclusive scans over the digits: the tile's totals (tile-local digit offsets)
    // and the pass's counts (the digits' output offsets)
    const uint32_t incl = wave_incl_scan(run);
    const uint32_t hincl = wave_incl_scan(hcount);
    if (lane == 63) {
      wtot[w] = incl;
      htot[w] = hincl;
    }
    __syncthreads();
    uint32_t woff = 0, hoff = 0;
    for (int q = 0; q < w; ++q) {
      woff += wtot[q];
      hoff += htot[q];
    }
    ldig[t] = woff + incl - run;
    const uint32_t digit_off = hoff + hincl - hcount;
    __syncthreads();
    // the tile sorted by digit (stable) in LDS; its place in the output needs only
    // the earlier tiles' counts, learnt next
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t d = rd[r] >> 16;
      if (d < 256u) {
        const uint32_t lpos = ldig[d] + wcnt[w][d] + (rd[r] & 0xFFFFu);
        s_key[lpos] = key[r];
        s_val[lpos] = val[r];
      }
    }
    bool complete = true;
    const uint32_t prior = look_back_gather(ctl + 64, ctl + 64 + tiles * 256, tile, 256, t, agg, err, complete,
                                            tile != withhold);
    gofs[t] = digit_off + prior;
    // a wait gave up: the prefixes may be partial (the barrier also orders the LDS writes)
    if (block_incomplete(complete, s_incomplete)) return;
    const int nv = (int)min<int64_t>(kTile, n - base);
    for (int q = t; q < nv; q += kSortThreads) {
      const K k = s_key[q];
      const uint32_t d = (uint32_t)(k >> shift) & 255u;
      const uint32_t pos = gofs[d] + ((uint32_t)q - ldig[d]);
      kout[pos] = k;
      vout[pos] = s_val[q];
    }
  }
}

template <typename K>
int radix_sort_os(const K* keys_in, const uint32_t* vals_in, K* kb[2], uint32_t* vb[2], int64_t n_max,
                  const uint32_t* n_dev, int bits, uint32_t* ctl, uint32_t* err, bool runs, hipStream_t s,
                  int64_t withhold = -1) {
  const int passes = (bits + 7) / 8;
  if (n_max <= 0 || passes == 0) return -1;
  uint32_t* hist = ctl;                        // [passes][256]
  uint32_t* pass_ctl = ctl + kMaxPasses * 256;  // per pass: 64 reserved words, tile then group status [.][256]
  // Large sorts take 4096-item tiles: each 8-bit digit of a tile then leaves in runs
  // of ~16 items instead of ~8, and the look-back has half the tiles. Smaller sorts
  // keep 2048, which gives more blocks (sort_ctl_words sizes the control words for
  // the same choice).
  const int64_t tile_items = sort_tile_items(n_max);
  const int64_t tiles = (n_max + tile_items - 1) / tile_items;
  const int64_t pass_words = 64 + (tiles + (tiles + kGroup - 1) / kGroup) * 256;
  int64_t hb = (n_max + kHistChunk - 1) / kHistChunk;
  if (hb > kHistBlocks) hb = kHistBlocks;
  if (hb < 1) hb = 1;
  if (runs)
    k_os_hist<K, true><<<(unsigned)hb, kSortThreads, 0, s>>>(keys_in, n_max, n_dev, passes, hist, err);
  else
    k_os_hist<K, false><<<(unsigned)hb, kSortThreads, 0, s>>>(keys_in, n_max, n_dev, passes, hist, err);
  const K* kcur = keys_in;
  const uint32_t* vcur = vals_in;
  int out = 0;
  for (int p = 0; p < passes; ++p) {
    const int64_t wh = p == 0 ? withhold : -1;
    if (tile_items == 2 * kSortTile)
      k_os_scatter<K, 2 * kSortRounds><<<(unsigned)tiles, kSortThreads, 0, s>>>(
          kcur, vcur, kb[out], vb[out], n_max, n_dev, 8 * p, hist + p * 256, pass_ctl + p * pass_words, err, wh);
    else
      k_os_scatter<K, kSortRounds><<<(unsigned)tiles, kSortThreads, 0, s>>>(
          kcur, vcur, kb[out], vb[out], n_max, n_dev, 8 * p, hist + p * 256, pass_ctl + p * pass_words, err, wh);
    kcur = kb[out];
    vcur = vb[out];
    out ^= 1;
  }
  return out ^ 1;
}

}  // namespace

size_t scan_ctl_words(int64_t n_max) {
  const int64_t tiles = std::max<int64_t>(1, (n_max + kScanTile - 1) / kScanTile);
  return 64 + (size_t)(tiles + (tiles + kGroup - 1) / kGroup) + 64;
}

size_t sort_ctl_words(int64_t n_max, int bits) {
  const int passes = (bits + 7) / 8;
  const int64_t tile_items = sort_tile_items(n_max);
  const int64_t tiles = (n_max + tile_items - 1) / tile_items;
  return kMaxPasses * 256 + (size_t)passes * (64 + (tiles + (tiles + kGroup - 1) / kGroup) * 256);
}

void scan_u32(const uint32_t* src, const uint32_t* idx, uint32_t* out, int64_t n_max, const uint32_t* n_dev,
              uint32_t* total, uint32_t* list, uint32_t* ctl, uint32_t* err, hipStream_t s) {
  const int64_t tiles = n_max > 0 ? (n_max + kScanTile - 1) / kScanTile : 1;
  k_scan<<<(unsigned)tiles, kScanThreads, 0, s>>>(src, idx, out, n_max, n_dev, total, list, ctl, err);
}

int radix_sort_u32_dev(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* kb[2], uint32_t* vb[2],
                       int64_t n_max, const uint32_t* n_dev, int bits, uint32_t* ctl, uint32_t* err, bool spatial,
                       hipStream_t s, int64_t withhold) {
  return radix_sort_os<uint32_t>(keys_in, vals_in, kb, vb, n_max, n_dev, bits, ctl, err, spatial, s, withhold);
}

namespace {
__global__ void k_raise_abort(uint32_t* err) { atomicOr(err, kErrAbort); }
}  // namespace

void raise_abort(uint32_t* err, hipStream_t s) { k_raise_abort<<<1, 1, 0, s>>>(err); }

int radix_sort_u64_dev(const uint64_t* keys_in, const uint32_t* vals_in, uint64_t* kb[2], uint32_t* vb[2],
                       int64_t n_max, const uint32_t* n_dev, int bits, uint32_t* ctl, uint32_t* err, bool spatial,
                       hipStream_t s) {
  return radix_sort_os<uint64_t>(keys_in, vals_in, kb, vb, n_max, n_dev, bits, ctl, err, spatial, s);
}

}  // namespace gsr
