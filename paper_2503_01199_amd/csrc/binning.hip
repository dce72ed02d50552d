// Binning: expand each depth-sorted record into one instance per covered tile and
// delimit each tile's instances after the tile sort.
//
// The records are first stably sorted by depth key (ties keep record order); the
// instances are then emitted in that order and stably sorted by global tile id.
// The result is each tile's list in (depth, record) order, the same order as a
// stable sort of 64-bit (tile << 32 | depth) keys emitted in record order, but it
// moves 4-byte keys and sorts the instances on the tile bits only.
#include <algorithm>

#include "raster_common.h"

namespace gsr {
namespace {

// One thread per sorted record k < (active records); its instances go to its
// scanned offset, tiles in row-major order of its rect. A record with more than
// kEmitAlone tiles is written by its whole wave instead, lanes on consecutive
// positions, one such record after another (found by a ballot, broadcast by lane
// reads): left to one lane, the largest rects hold their wave long after the others
// are done (on 8 orbit views of a 3M-Gaussian scene the slowest lane's count
// averages 4x a wave's mean). When the frame has more instances than the workspace
// holds, the list is cut at the capacity (the record that straddles it writes its
// first tiles only), so [0, kept) is always complete, and the overflow flag is
// raised. The first threads also clear the per-tile ranges.
constexpr int kEmitThreads = 128;
constexpr uint32_t kEmitAlone = 4;

__global__ __launch_bounds__(kEmitThreads) void k_emit(const uint32_t* __restrict__ sorted_rec,
                                                       const uint32_t* __restrict__ offsets,
                                                       const uint32_t* __restrict__ tiles,
                                                       const ushort4* __restrict__ rect,
                                                       const ViewDev* __restrict__ views, int32_t V,
                                                       uint32_t* __restrict__ header, int64_t cap,
                                                       uint32_t* __restrict__ inst_tile,
                                                       uint32_t* __restrict__ inst_rec, uint32_t* __restrict__ ranges,
                                                       int64_t ntiles) {
  if (frame_aborted(header)) return;  // the depth sort or offsets scan gave up
  const int64_t k = (int64_t)blockIdx.x * kEmitThreads + threadIdx.x;
  for (int64_t q = k; q < 2 * ntiles; q += (int64_t)gridDim.x * kEmitThreads) ranges[q] = 0u;
  if (k == 0) {
    const uint32_t M = header[kHdrInstances];
    header[kHdrInstancesKept] = (uint32_t)min((int64_t)M, cap);
    if ((int64_t)M > cap) header[kHdrOverflow] = 1u;
  }
  const int64_t nrec = header[kHdrRecords];
  if (k - (threadIdx.x & 63) >= nrec) return;  // the whole wave
  uint32_t r = 0, cnt = 0;
  int64_t o = 0;
  if (k < nrec) {
    r = sorted_rec[k];
    cnt = tiles[r];
    o = offsets[k];
  }
  const bool live = cnt > 0 && o < cap;
  const bool alone = live && cnt > kEmitAlone;
  ushort4 b = make_ushort4(0, 0, 0, 0);
  int32_t base = 0, tx = 0;
  if (live) {  // every lane loads its own rect and view first, large records too
    b = rect[r];
    const int v = (int)(r % (uint32_t)V);
    base = views[v].tile_base;
    tx = views[v].tiles_x;
  }
  if (live && !alone) {
    const int64_t end = min(o + (int64_t)cnt, cap);
    for (int y = b.z; y <= b.w && o < end; ++y)
      for (int x = b.x; x <= b.y && o < end; ++x) {
        inst_tile[o] = (uint32_t)(base + y * tx + x);
        inst_rec[o] = r;
        ++o;
      }
  }
  uint64_t big = __builtin_amdgcn_ballot_w64(alone);
  const int lane = (int)(threadIdx.x & 63);
  while (big) {  // wave-uniform; every value comes from the owning lane's registers
    const int src = __builtin_ctzll(big);
    big &= big - 1;
    const uint32_t rr = (uint32_t)__shfl((int)r, src, 64);
    const int64_t o0 = (int64_t)(uint32_t)__shfl((int)(uint32_t)o, src, 64);
    const int64_t n_here = min((int64_t)(uint32_t)__shfl((int)cnt, src, 64), cap - o0);
    const int32_t x0 = __shfl((int)b.x, src, 64);
    const int32_t y0 = __shfl((int)b.z, src, 64);
    const uint32_t width = (uint32_t)(__shfl((int)b.y, src, 64) - x0 + 1);
    const int32_t tbase = __shfl(base, src, 64);
    const int32_t ttx = __shfl(tx, src, 64);
    for (int64_t idx = lane; idx < n_here; idx += 64) {
      const uint32_t row = (uint32_t)idx / width;
      const uint32_t col = (uint32_t)idx - row * width;
      inst_tile[o0 + idx] = (uint32_t)(tbase + (y0 + (int32_t)row) * ttx + x0 + (int32_t)col);
      inst_rec[o0 + idx] = rr;
    }
  }
}

// Each thread takes four consecutive instances (one 16-byte load) and compares each
// with its neighbours; the first and last instance of a tile write its range.
__global__ void k_ranges(const uint32_t* __restrict__ inst_tile, const uint32_t* __restrict__ header,
                         uint32_t* __restrict__ ranges) {
  constexpr uint32_t kNone = 0xffffffffu;  // no tile id (ids stay below 2^28)
  if (frame_aborted(header)) return;  // the tile sort gave up: tile ids may be out of range
  const int64_t M = header[kHdrInstancesKept];
  const int64_t G = (M + 3) / 4;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < G; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k0 = 4 * q;
    uint32_t t[6];  // instances k0 - 1 .. k0 + 4, kNone outside [0, M)
    if (k0 + 4 <= M) {
      const uint4 v = *reinterpret_cast<const uint4*>(inst_tile + k0);
      t[1] = v.x, t[2] = v.y, t[3] = v.z, t[4] = v.w;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) t[1 + j] = k0 + j < M ? inst_tile[k0 + j] : kNone;
    }
    t[0] = k0 > 0 ? inst_tile[k0 - 1] : kNone;
    t[5] = k0 + 4 < M ? inst_tile[k0 + 4] : kNone;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (t[1 + j] == kNone) break;
      if (t[j] != t[1 + j]) ranges[2 * (int64_t)t[1 + j]] = (uint32_t)(k0 + j);
      if (t[2 + j] != t[1 + j]) ranges[2 * (int64_t)t[1 + j] + 1] = (uint32_t)(k0 + j + 1);
    }
  }
}

// Raster schedules (tiles are independent and a pixel's arithmetic does not
// depend on how its tile is split, so the schedule changes no image): one block
// buckets the list lengths (clamped to 4095) in LDS in descending order and scans
// the buckets, giving each tile its rank. For each list, the ns longest tiles with
// more than its split length (ns at most a quarter of the tiles) become 4 (forward)
// or 2 (backward) band items each, placed first; every other tile is one whole
// item, after them; both groups in descending length. The item counts go to
// *n_items (and *n_bwd). Within a bucket ranks come from LDS atomics, in no fixed
// order, except in a bucket that holds both a list's last split tile and its first
// whole one (the cap cuts through tiles of equal length): there ranks follow the
// tile index, so which tiles are split never depends on the order of atomics (a
// split changes how the backward rounds its per-item sums).
constexpr int kOrderThreads = 1024;
constexpr int kOrderBuckets = 4096;
constexpr int kOrderUnroll = 8;  // list lengths loaded per thread before they are counted

// Bucket of a list length: descending length, lengths clamped to kOrderBuckets - 1.
__device__ __forceinline__ uint32_t order_bucket(uint32_t len) {
  return kOrderBuckets - 1 - min(len, (uint32_t)(kOrderBuckets - 1));
}

// List length of concatenated tile i: one frame, or a batch of frames (a short
// uniform search over the frames' first tiles).
struct OneFrame {
  const uint32_t* ranges;
  const uint32_t* header;
  __device__ bool aborted() const { return frame_aborted(header); }
  __device__ uint32_t len(int64_t i) const { return ranges[2 * i + 1] - ranges[2 * i]; }
};
// A frame that gave up counts as empty here (its ranges may be garbage); the raster
// skips its items.
struct ManyFrames {
  FrameTable tab;
  __device__ bool aborted() const { return false; }
  __device__ uint32_t len(int64_t i) const {
    int f = 0;
    while (f + 1 < tab.n && tab.first[f + 1] <= (uint32_t)i) ++f;
    if (frame_aborted(tab.f[f].header)) return 0u;
    const int64_t t = i - tab.first[f];
    return tab.f[f].ranges[2 * t + 1] - tab.f[f].ranges[2 * t];
  }
};

// Item codes of band group b of a tile split `ways` ways.
__device__ __forceinline__ uint32_t split_code(uint32_t ways, uint32_t b) { return ways == 4 ? b : kItemHalf + b; }

// Places tile i, of rank pos, in an item list that splits its ns first tiles.
template <typename W>
__device__ __forceinline__ void place_items(W* items, uint32_t i, uint32_t pos, uint32_t ns, uint32_t ways) {
  if (pos < ns) {
    for (uint32_t b = 0; b < ways; ++b) items[ways * pos + b] = (W)((i << 3) | split_code(ways, b));
  } else {
    items[(ways - 1) * ns + pos] = (W)((i << 3) | kItemWhole);
  }
}

// Up to kStageTiles tiles an item fits in 16 bits and both lists are built in LDS,
// then stored with coalesced writes (one CU issuing ~3 scattered 4-byte stores per
// tile is otherwise the kernel's bottleneck); larger frames store items directly.
constexpr int64_t kStageTiles = 8192;
static_assert(kStageTiles <= (int64_t)kOrderThreads * kOrderUnroll, "a staged frame is counted in one round");
constexpr int kStageItems = (int)(kStageTiles + 3 * ((kStageTiles + kSplitShare - 1) / kSplitShare));

template <class Len>
__global__ __launch_bounds__(kOrderThreads) void k_tile_order(Len L, int64_t T, uint32_t split_len,
                                                              uint32_t split_len_bwd, uint32_t* __restrict__ items,
                                                              uint32_t* __restrict__ n_items,
                                                              uint32_t* __restrict__ bwd,
                                                              uint32_t* __restrict__ n_bwd) {
  __shared__ uint16_t s_items[2][kStageItems];
  const bool staged = T <= kStageTiles;
  __shared__ uint32_t h[kOrderBuckets];
  __shared__ uint32_t wsum[kOrderThreads / 64];
  __shared__ uint32_t nlong[2];
  __shared__ uint32_t edge[2];  // bucket holding the forward's / backward's last split rank (none: kOrderBuckets)
  __shared__ uint32_t wcnt[2][kOrderThreads / 64];
  if (L.aborted()) return;  // the item counts stay 0: no raster work
  const int t = threadIdx.x;
  for (int b = t; b < kOrderBuckets; b += kOrderThreads) h[b] = 0;
  if (t < 2) {
    nlong[t] = 0;
    edge[t] = kOrderBuckets;
  }
  __syncthreads();
  uint32_t my_long = 0, my_long_b = 0;
  // a staged frame (T <= kOrderThreads * kOrderUnroll) takes one round, whose lengths
  // the placement below reuses instead of loading them again
  uint32_t kept[kOrderUnroll];
  for (int64_t i0 = t; i0 < T; i0 += (int64_t)kOrderThreads * kOrderUnroll) {
    uint32_t len[kOrderUnroll];
#pragma unroll
    for (int q = 0; q < kOrderUnroll; ++q) {  // unconditional loads (index clamped), so all are in flight at once
      const int64_t i = i0 + (int64_t)q * kOrderThreads;
      const uint32_t l = L.len(i < T ? i : T - 1);
      len[q] = i < T ? l : 0u;
      kept[q] = len[q];
    }
#pragma unroll
    for (int q = 0; q < kOrderUnroll; ++q) {
      if (i0 + (int64_t)q * kOrderThreads >= T) continue;
      atomicAdd(&h[order_bucket(len[q])], 1u);
      my_long += len[q] > split_len ? 1u : 0u;
      my_long_b += len[q] > split_len_bwd ? 1u : 0u;
    }
  }
  // wave sums first: a same-address atomic from every lane is serialised lane by
  // lane on the CU's one scalar unit (~6 us for 16 waves and two counters)
  for (int d = 32; d > 0; d >>= 1) {
    my_long += __shfl_xor(my_long, d, 64);
    my_long_b += __shfl_xor(my_long_b, d, 64);
  }
  if ((t & 63) == 0) {
    atomicAdd(&nlong[0], my_long);
    if (bwd) atomicAdd(&nlong[1], my_long_b);
  }
  __syncthreads();
  const uint32_t cap = (uint32_t)((T + kSplitShare - 1) / kSplitShare);
  const uint32_t ns = min(nlong[0], cap);
  const uint32_t ns_b = min(nlong[1], cap);
  // exclusive scan of the buckets, 4 per thread
  uint32_t v[4], sum = 0;
  for (int q = 0; q < 4; ++q) {
    v[q] = h[4 * t + q];
    sum += v[q];
  }
  uint32_t incl = sum;
  const int lane = t & 63;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) wsum[t >> 6] = incl;
  __syncthreads();
  uint32_t off = incl - sum;
  for (int w = 0; w < (t >> 6); ++w) off += wsum[w];
  __syncthreads();
  for (int q = 0; q < 4; ++q) {
    // a list's split edge: the bucket that holds both its last split rank, ns - 1,
    // and the first whole one, ns (the quarter cap cuts through equal lengths)
    if (ns > 0 && off < ns && ns < off + v[q]) edge[0] = 4 * t + q;
    if (bwd && ns_b > 0 && off < ns_b && ns_b < off + v[q]) edge[1] = 4 * t + q;
    h[4 * t + q] = off;
    off += v[q];
  }
  __syncthreads();
  // Edge buckets: ranks in tile-index order. Each thread takes a contiguous run of
  // tiles, counts its edge tiles, and a block scan of the counts gives its first rank.
  const uint32_t e0 = edge[0], e1 = edge[1];
  if (e0 < kOrderBuckets || e1 < kOrderBuckets) {
    const int64_t per = (T + kOrderThreads - 1) / kOrderThreads;
    const int64_t lo = min<int64_t>(T, (int64_t)t * per), hi = min<int64_t>(T, lo + per);
    uint32_t c0 = 0, c1 = 0;
    for (int64_t i = lo; i < hi; ++i) {
      const uint32_t b = order_bucket(L.len(i));
      c0 += b == e0 ? 1u : 0u;
      c1 += (b == e1 && e1 != e0) ? 1u : 0u;
    }
    uint32_t x0 = c0, x1 = c1;
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y0 = __shfl_up(x0, d, 64), y1 = __shfl_up(x1, d, 64);
      if (lane >= d) {
        x0 += y0;
        x1 += y1;
      }
    }
    if (lane == 63) {
      wcnt[0][t >> 6] = x0;
      wcnt[1][t >> 6] = x1;
    }
    __syncthreads();
    uint32_t r0 = x0 - c0, r1 = x1 - c1;
    for (int w = 0; w < (t >> 6); ++w) {
      r0 += wcnt[0][w];
      r1 += wcnt[1][w];
    }
    const uint32_t s0 = e0 < kOrderBuckets ? h[e0] : 0u, s1 = e1 < kOrderBuckets ? h[e1] : 0u;
    for (int64_t i = lo; i < hi; ++i) {
      const uint32_t b = order_bucket(L.len(i));
      if (b != e0 && b != e1) continue;
      const uint32_t pos = (b == e0) ? s0 + r0++ : s1 + r1++;
      if (staged) {
        place_items(s_items[0], (uint32_t)i, pos, ns, 4);
        if (bwd) place_items(s_items[1], (uint32_t)i, pos, ns_b, 2);
      } else {
        place_items(items, (uint32_t)i, pos, ns, 4);
        if (bwd) place_items(bwd, (uint32_t)i, pos, ns_b, 2);
      }
    }
  }
  for (int64_t i0 = t; i0 < T; i0 += (int64_t)kOrderThreads * kOrderUnroll) {
    uint32_t len[kOrderUnroll];
#pragma unroll
    for (int q = 0; q < kOrderUnroll; ++q) {  // larger frames: unconditional loads again (index clamped)
      const int64_t i = i0 + (int64_t)q * kOrderThreads;
      const uint32_t l = staged ? kept[q] : L.len(i < T ? i : T - 1);
      len[q] = i < T ? l : 0u;
    }
#pragma unroll
    for (int q = 0; q < kOrderUnroll; ++q) {
      const int64_t i = i0 + (int64_t)q * kOrderThreads;
      if (i >= T) continue;
      const uint32_t b = order_bucket(len[q]);
      if (b == e0 || b == e1) continue;  // placed above
      const uint32_t pos = atomicAdd(&h[b], 1u);
      if (staged) {
        place_items(s_items[0], (uint32_t)i, pos, ns, 4);
        if (bwd) place_items(s_items[1], (uint32_t)i, pos, ns_b, 2);
      } else {
        place_items(items, (uint32_t)i, pos, ns, 4);
        if (bwd) place_items(bwd, (uint32_t)i, pos, ns_b, 2);
      }
    }
  }
  const uint32_t ni = (uint32_t)T + 3 * ns, nb = (uint32_t)T + ns_b;
  if (staged) {
    __syncthreads();
    for (uint32_t k = t; k < ni; k += kOrderThreads) items[k] = s_items[0][k];
    if (bwd)
      for (uint32_t k = t; k < nb; k += kOrderThreads) bwd[k] = s_items[1][k];
  }
  if (t == 0) {
    *n_items = ni;
    if (bwd) *n_bwd = nb;
  }
}

// Frames of more than kStageTiles tiles: the same schedule from three launches over
// many blocks (one block storing the items of the 65k tiles of 8 full-HD views took
// 155 us). Block g takes the chunk of kOrderChunk tiles from g kOrderChunk. Control
// words: bucket starts [4096], meta [64] (ns, ns_b, the edge buckets), then per
// block its bucket counts [4096] and long-list counts [2].
constexpr int64_t kOrderChunk = 4096;  // tiles per block: 4 per thread
constexpr int kOrderMeta = kOrderBuckets;
constexpr int kOrderBlk = kOrderBuckets + 64;
constexpr int kOrderBlkWords = kOrderBuckets + 2;

// The chunk's count per length bucket and of long lists (written whole: no atomics
// across blocks).
template <class Len>
__global__ __launch_bounds__(kOrderThreads) void k_order_count(Len L, int64_t T, uint32_t split_len,
                                                               uint32_t split_len_bwd, uint32_t* __restrict__ ctl) {
  __shared__ uint32_t h[kOrderBuckets];
  __shared__ uint32_t nl[2];
  if (L.aborted()) return;
  const int t = threadIdx.x;
  for (int b = t; b < kOrderBuckets; b += kOrderThreads) h[b] = 0;
  if (t < 2) nl[t] = 0;
  __syncthreads();
  const int64_t c0 = (int64_t)blockIdx.x * kOrderChunk;
  uint32_t my_long = 0, my_long_b = 0;
  uint32_t len[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t i = c0 + q * kOrderThreads + t;
    len[q] = L.len(i < T ? i : T - 1);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (c0 + q * kOrderThreads + t >= T) continue;
    atomicAdd(&h[order_bucket(len[q])], 1u);
    my_long += len[q] > split_len ? 1u : 0u;
    my_long_b += len[q] > split_len_bwd ? 1u : 0u;
  }
  for (int d = 32; d > 0; d >>= 1) {
    my_long += __shfl_xor(my_long, d, 64);
    my_long_b += __shfl_xor(my_long_b, d, 64);
  }
  if ((t & 63) == 0) {
    atomicAdd(&nl[0], my_long);
    atomicAdd(&nl[1], my_long_b);
  }
  __syncthreads();
  uint32_t* blk = ctl + kOrderBlk + (int64_t)blockIdx.x * kOrderBlkWords;
  for (int b = t; b < kOrderBuckets; b += kOrderThreads) blk[b] = h[b];
  if (t < 2) blk[kOrderBuckets + t] = nl[t];
}

// Bucket starts (exclusive scan of the totals), the split counts, the edge buckets
// and the item counts (one block).
template <class Len>
__global__ __launch_bounds__(kOrderThreads) void k_order_scan(Len L, int64_t T, uint32_t* __restrict__ ctl,
                                                              uint32_t* __restrict__ n_items,
                                                              uint32_t* __restrict__ n_bwd) {
  __shared__ uint32_t wsum[kOrderThreads / 64];
  __shared__ uint32_t edge[2];
  __shared__ uint32_t nl[2];
  if (L.aborted()) return;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int64_t G = (T + kOrderChunk - 1) / kOrderChunk;
  if (t < 2) {
    edge[t] = kOrderBuckets;
    uint32_t c = 0;
    for (int64_t g = 0; g < G; ++g) c += ctl[kOrderBlk + g * kOrderBlkWords + kOrderBuckets + t];
    nl[t] = c;
  }
  uint32_t v[4] = {0, 0, 0, 0}, sum = 0;
  for (int64_t g = 0; g < G; ++g) {
    const uint32_t* blk = ctl + kOrderBlk + g * kOrderBlkWords;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] += blk[4 * t + q];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) sum += v[q];
  uint32_t incl = sum;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) wsum[t >> 6] = incl;
  __syncthreads();
  const uint32_t cap = (uint32_t)((T + kSplitShare - 1) / kSplitShare);
  const uint32_t ns = min(nl[0], cap);
  const uint32_t ns_b = min(nl[1], cap);
  uint32_t off = incl - sum;
  for (int w = 0; w < (t >> 6); ++w) off += wsum[w];
  for (int q = 0; q < 4; ++q) {
    if (ns > 0 && off < ns && ns < off + v[q]) edge[0] = 4 * t + q;
    if (n_bwd && ns_b > 0 && off < ns_b && ns_b < off + v[q]) edge[1] = 4 * t + q;
    ctl[4 * t + q] = off;
    off += v[q];
  }
  __syncthreads();
  if (t == 0) {
    ctl[kOrderMeta + 0] = ns;
    ctl[kOrderMeta + 1] = ns_b;
    ctl[kOrderMeta + 2] = edge[0];
    ctl[kOrderMeta + 3] = edge[1];
    *n_items = (uint32_t)T + 3 * ns;
    if (n_bwd) *n_bwd = (uint32_t)T + ns_b;
  }
}

// Places the block's chunk: thread t takes its tiles 4t .. 4t + 3. A tile's rank is
// its bucket's start, plus the bucket's tiles in the chunks before (their counts),
// plus its rank within the chunk: in index order in an edge bucket (a block scan),
// in no particular order in any other (LDS atomics).
template <class Len>
__global__ __launch_bounds__(kOrderThreads) void k_order_place(Len L, int64_t T, const uint32_t* __restrict__ ctl,
                                                               uint32_t* __restrict__ items,
                                                               uint32_t* __restrict__ bwd) {
  __shared__ uint32_t base[kOrderBuckets];  // the block's first rank per bucket
  __shared__ uint32_t h[kOrderBuckets];     // chunk ranks handed out per bucket
  __shared__ uint32_t wsum[2][kOrderThreads / 64];
  if (L.aborted()) return;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const uint32_t ns = ctl[kOrderMeta + 0], ns_b = ctl[kOrderMeta + 1];
  const uint32_t e0 = ctl[kOrderMeta + 2], e1 = ctl[kOrderMeta + 3];
  const int64_t g = blockIdx.x;
  for (int b = t; b < kOrderBuckets; b += kOrderThreads) {
    uint32_t x = ctl[b];
    for (int64_t q = 0; q < g; ++q) x += ctl[kOrderBlk + q * kOrderBlkWords + b];
    base[b] = x;
    h[b] = 0;
  }
  __syncthreads();
  const int64_t i0 = g * kOrderChunk + 4 * (int64_t)t;
  uint32_t bk[4], rk[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) bk[q] = order_bucket(L.len(i0 + q < T ? i0 + q : T - 1));
  uint32_t c_e0 = 0, c_e1 = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    rk[q] = 0;
    if (i0 + q >= T) continue;
    if (bk[q] == e0) rk[q] = c_e0++;
    else if (bk[q] == e1) rk[q] = c_e1++;
    else rk[q] = atomicAdd(&h[bk[q]], 1u);
  }
  // ranks of the edge tiles of lower threads (index order)
  uint32_t x0 = c_e0, x1 = c_e1;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y0 = __shfl_up(x0, d, 64), y1 = __shfl_up(x1, d, 64);
    if (lane >= d) {
      x0 += y0;
      x1 += y1;
    }
  }
  if (lane == 63) {
    wsum[0][t >> 6] = x0;
    wsum[1][t >> 6] = x1;
  }
  __syncthreads();
  uint32_t r0 = x0 - c_e0, r1 = x1 - c_e1;
  for (int w = 0; w < (t >> 6); ++w) {
    r0 += wsum[0][w];
    r1 += wsum[1][w];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t i = i0 + q;
    if (i >= T) continue;
    const uint32_t pos = base[bk[q]] + rk[q] + (bk[q] == e0 ? r0 : bk[q] == e1 ? r1 : 0u);
    place_items(items, (uint32_t)i, pos, ns, 4);
    if (bwd) place_items(bwd, (uint32_t)i, pos, ns_b, 2);
  }
}

}  // namespace

size_t tile_order_ctl_words(int64_t tiles) {
  return tiles > kStageTiles ? kOrderBlk + (size_t)((tiles + kOrderChunk - 1) / kOrderChunk) * kOrderBlkWords : 0;
}

bool launch_tile_order(const Frame& f, hipStream_t s, hipEvent_t done) {
  if (f.tiles <= 0) return false;
  if (f.tiles > kStageTiles && f.ctl_tile_order) {
    const OneFrame L{f.ranges, f.header};
    const unsigned g = (unsigned)((f.tiles + kOrderChunk - 1) / kOrderChunk);
    k_order_count<<<g, kOrderThreads, 0, s>>>(L, (int64_t)f.tiles, f.split_len, f.split_len_bwd, f.ctl_tile_order);
    k_order_scan<<<1, kOrderThreads, 0, s>>>(L, (int64_t)f.tiles, f.ctl_tile_order, f.header + kHdrItems,
                                             f.header + kHdrItemsBwd);
    launch_tracked(k_order_place<OneFrame>, g, kOrderThreads, s, done, L, (int64_t)f.tiles, f.ctl_tile_order,
                   f.tile_order, f.bwd_items);
    return true;
  }
  launch_tracked(k_tile_order<OneFrame>, 1, kOrderThreads, s, done, OneFrame{f.ranges, f.header}, (int64_t)f.tiles,
                 f.split_len, f.split_len_bwd, f.tile_order, f.header + kHdrItems, f.bwd_items,
                 f.header + kHdrItemsBwd);
  return true;
}

void launch_batch_tile_order(const FrameTable& tab, uint32_t total_tiles, uint32_t split_len, uint32_t* order,
                             uint32_t* n_items, hipStream_t s) {
  if (total_tiles == 0) return;
  k_tile_order<ManyFrames><<<1, kOrderThreads, 0, s>>>(ManyFrames{tab}, total_tiles, split_len, 0u, order, n_items,
                                                       nullptr, nullptr);
}

int64_t raster_max_items(int64_t tiles) { return max_items(tiles); }

void launch_emit_instances(const Frame& f, const uint32_t* sorted_rec, hipStream_t s) {
  int64_t n = std::max<int64_t>(f.nrec, 2 * f.tiles);
  int64_t g = (n + kEmitThreads - 1) / kEmitThreads;
  if (g < 1) g = 1;
  k_emit<<<(unsigned)g, kEmitThreads, 0, s>>>(sorted_rec, f.offsets, f.tiles_touched, f.rect, f.views, f.V,
                                              f.header, f.inst_cap, f.ikey[0], f.ival[0], f.ranges, f.tiles);
}

void launch_tile_ranges(const Frame& f, const uint32_t* inst_tile, int64_t M_max, hipStream_t s) {
  if (M_max <= 0) return;
  // grid-stride over the count on the device; the grid covers typical frames in one sweep
  const int64_t g = std::min<int64_t>((M_max + 4 * 256 - 1) / (4 * 256), 4096);
  k_ranges<<<(unsigned)g, 256, 0, s>>>(inst_tile, f.header, f.ranges);
}

}  // namespace gsr
