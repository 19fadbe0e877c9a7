// Partitioned insert and lookup: filters larger than one workgroup's LDS
// processed slice by slice, with streaming memory traffic only.
//
// The filter is cut into slices of S = 2^slice_shift consecutive blocks (a
// slice fits one workgroup's LDS). Block selection is monotone in the high
// half of the hash, so every key belongs to exactly one slice. The batch is
// cut into G contiguous chunks, one per partitioning workgroup. Kernels:
//
//   count     workgroup g counts the keys of chunk g per slice -> hist[g][s]
//   colsum    column sums of hist over blocks of 256 rows
//   colscan   start[g][s] = sum of hist[< g][s]; tot[s] = sum over g
//   offsets   offsets[s] = sum of round4(tot[< s]): slice s's keys begin at a
//             multiple of four keys (32 bytes)
//   scatter   workgroup g walks chunk g in tiles, sorts each tile by slice in
//             LDS and writes each slice's run with consecutive lanes at the
//             slice cursor offsets[s] + start[g][s] + (keys already written);
//             for lookups it also records pos[i], where key i's result sits
//             among the chunk's results
//   slice     one workgroup per slice loads the slice into LDS; insert ORs the
//             slice's keys into it and stores it back with plain stores,
//             lookup tests the slice's keys against it and writes one result
//             byte per key in partitioned order
//   unpermute lookups only: workgroup g writes out[i] = result[pos[i]] for
//             chunk g; each slice's results for chunk g are one contiguous
//             run, read front to back
//
// No global atomics touch the filter or the partition. The partition order
// is deterministic up to the order of equal-slice keys inside one tile, and a
// filter is the OR of all masks, so inserts never depend on it; lookups are
// pure and return to input order through pos. Lookup chunks hold at most
// 65,536 keys, so positions are 16-bit.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"
#include "sbbf_device.h"

namespace sbbf {
namespace {

constexpr uint32_t kPartThreads = 1024;    // count, scan, slice and unpermute kernels
constexpr uint32_t kMaxSlices = 4096;       // slices per partitioned filter
constexpr uint32_t kScatterThreads = 1024;
constexpr uint32_t kScatterPer = 7;        // keys per thread per scatter tile
constexpr uint32_t kScatterGroup = 8;      // keys per aligned group written by the scatter (64 bytes)
constexpr uint32_t kTile = kScatterThreads * kScatterPer;
constexpr uint32_t kScanRows = 256;    // rows per colsum/colscan workgroup (16 segments of 16)
constexpr uint32_t kScanCols = 64;     // columns per colsum/colscan workgroup
constexpr uint32_t kSliceSteps = 2;    // 256-key steps per wave per slice-loop iteration
// Lookup chunks are at most this many keys so that one chunk's result bytes
// fit one workgroup's LDS in the unpermute kernel and positions fit 16 bits.
constexpr uint32_t kLookupChunk = 65536u;

__device__ __forceinline__ uint32_t slice_of(uint64_t h, uint32_t num_blocks, uint32_t slice_shift) {
  return block_of((uint32_t)(h >> 32), num_blocks) >> slice_shift;
}

// Slice of a hash relative to the first slice of the partition (slice_base:
// 0 for one level; a group's first slice in the second level of a two-level
// partition, whose keys all lie in that group), clamped into [0, num_slices)
// so that no key can index past the per-slice arrays.
__device__ __forceinline__ uint32_t local_slice(uint64_t h, uint32_t num_blocks, uint32_t slice_shift,
                                                uint32_t slice_base, uint32_t num_slices) {
  return min(slice_of(h, num_blocks, slice_shift) - slice_base, num_slices - 1u);
}

__device__ __forceinline__ void chunk_range(uint32_t g, uint32_t chunk, uint32_t n, uint32_t *b, uint32_t *e) {
  const uint64_t lo = (uint64_t)g * chunk;
  *b = (uint32_t)min<uint64_t>(lo, n);
  *e = (uint32_t)min<uint64_t>(lo + chunk, n);
}

__global__ void __launch_bounds__(kPartThreads)
part_count_kernel(const uint64_t *__restrict__ hashes, uint32_t n, uint32_t chunk, uint32_t num_blocks,
                  uint32_t slice_shift, uint32_t slice_base, uint32_t num_slices, uint32_t keys,
                  uint32_t *__restrict__ hist_out) {
  extern __shared__ uint32_t hist[];
  for (uint32_t i = threadIdx.x; i < num_slices; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  uint32_t b, e;
  chunk_range(blockIdx.x, chunk, n, &b, &e);
  for (uint32_t i = b + threadIdx.x; i < e; i += blockDim.x) {
    const uint32_t s =
        local_slice(as_hash(load_hash<0>(hashes + i), keys), num_blocks, slice_shift, slice_base, num_slices);
    __hip_atomic_fetch_add(hist + s, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __syncthreads();
  uint32_t *row = hist_out + (uint64_t)blockIdx.x * num_slices;
  for (uint32_t i = threadIdx.x; i < num_slices; i += blockDim.x) row[i] = hist[i];
}

// Column prefix sums of hist[groups][num_slices], two kernels over a grid of
// (column blocks of 64) x (row blocks of 256). In both, thread (seg, c) of a
// workgroup handles column c over the 16 rows of segment seg.
__device__ __forceinline__ uint32_t segment_sum(const uint32_t *__restrict__ hist, uint32_t groups,
                                                uint32_t num_slices, uint32_t r0, uint32_t col) {
  uint32_t v[16];
#pragma unroll
  for (uint32_t k = 0; k < 16u; ++k) {
    const uint32_t r = r0 + k;
    v[k] = (r < groups && col < num_slices) ? hist[(uint64_t)r * num_slices + col] : 0u;
  }
  uint32_t s = 0;
#pragma unroll
  for (uint32_t k = 0; k < 16u; ++k) s += v[k];
  return s;
}

// blocksum[rb][col] = sum of hist over the 256 rows of row block rb.
__global__ void __launch_bounds__(kPartThreads)
part_colsum_kernel(const uint32_t *__restrict__ hist, uint32_t groups, uint32_t num_slices,
                   uint32_t *__restrict__ blocksum) {
  __shared__ uint32_t seg_sum[16][kScanCols];
  const uint32_t c = threadIdx.x % kScanCols, seg = threadIdx.x / kScanCols;
  const uint32_t col = blockIdx.x * kScanCols + c;
  seg_sum[seg][c] = segment_sum(hist, groups, num_slices, blockIdx.y * kScanRows + seg * 16u, col);
  __syncthreads();
  if (seg == 0 && col < num_slices) {
    uint32_t s = 0;
#pragma unroll
    for (uint32_t k = 0; k < 16u; ++k) s += seg_sum[k][c];
    blocksum[(uint64_t)blockIdx.y * num_slices + col] = s;
  }
}

// start[r][col] = sum of hist[< r][col]; the last row block also writes tot.
__global__ void __launch_bounds__(kPartThreads)
part_colscan_kernel(const uint32_t *__restrict__ hist, uint32_t groups, uint32_t num_slices,
                    const uint32_t *__restrict__ blocksum, uint32_t *__restrict__ start,
                    uint32_t *__restrict__ tot) {
  __shared__ uint32_t seg_sum[16][kScanCols];
  __shared__ uint32_t carry[kScanCols];
  const uint32_t c = threadIdx.x % kScanCols, seg = threadIdx.x / kScanCols;
  const uint32_t col = blockIdx.x * kScanCols + c;
  const uint32_t r0 = blockIdx.y * kScanRows + seg * 16u;
  seg_sum[seg][c] = segment_sum(hist, groups, num_slices, r0, col);
  if (seg == 0) {
    uint32_t s = 0;
    if (col < num_slices)
      for (uint32_t rb = 0; rb < blockIdx.y; ++rb) s += blocksum[(uint64_t)rb * num_slices + col];
    carry[c] = s;
  }
  __syncthreads();
  uint32_t run = carry[c];
  for (uint32_t k = 0; k < seg; ++k) run += seg_sum[k][c];
  if (col >= num_slices) return;
#pragma unroll
  for (uint32_t k = 0; k < 16u; ++k) {
    const uint32_t r = r0 + k;
    if (r < groups) {
      start[(uint64_t)r * num_slices + col] = run;
      run += hist[(uint64_t)r * num_slices + col];
    }
  }
  if (blockIdx.y == gridDim.y - 1u && seg == 15u) tot[col] = run;
}

// One workgroup: offsets[s] = sum of round4(tot[< s]); offsets[num_slices] is
// the padded total. Thread t owns slices 4t .. 4t+3 (num_slices <= 4096).
__global__ void __launch_bounds__(kPartThreads)
part_offsets_kernel(const uint32_t *__restrict__ tot, uint32_t num_slices, uint32_t *__restrict__ offsets) {
  __shared__ uint32_t wsum[16];
  uint32_t c[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const uint32_t s = threadIdx.x * 4u + r;
    c[r] = s < num_slices ? (tot[s] + 3u) & ~3u : 0u;
  }
  uint32_t run = block_scan_owned<4>(c, wsum);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const uint32_t s = threadIdx.x * 4u + r;
    if (s < num_slices) offsets[s] = run;
    run += c[r];
    if (s + 1u == num_slices) offsets[num_slices] = run;
  }
}

// Scatter LDS for groups of L keys (L = 1: no carry). The stage holds one
// tile's keys sorted by slice, each slice's run preceded by the keys carried
// over from the previous tile, so its size is kTile + (L - 1) * (slices),
// slices = R * kScatterThreads.
constexpr uint32_t stage_keys(uint32_t L, uint32_t R) { return kTile + (L - 1u) * R * kScatterThreads; }

constexpr size_t scatter_lds_bytes(uint32_t num_slices, bool with_pos, uint32_t L, uint32_t R) {
  return (size_t)stage_keys(L, R) * 8u + (size_t)num_slices * (with_pos ? 20u : 16u) + 64u;
}

struct ScatterLds {
  uint64_t *stage;  // [stage_keys(L)] keys sorted by slice
  uint2 *info;      // [P] staged position k < info.y of slice s goes to k + info.x
  uint32_t *hist;   // [P] keys per slice in the tile (ranks come from it)
  uint32_t *sbase;  // [P] staged position of the tile's first key of slice s
  uint32_t *pdelta; // [P] (lookups) chunk result position of staged position k is k + pdelta[s]
  uint32_t *wsum;   // [16]
};

// Hashes of tile t0 for this thread: index t0 + t * kScatterThreads + thread,
// clamped to the chunk's last key so loads never branch. Lookups load them
// through the caches and inserts with the non-temporal hint: measured on
// MI355X at 1e8 inserts and 2e8 lookups into 128 MiB, that order is 6 %
// faster for the lookup scatter (and its slice kernel) and 5 % faster for
// the insert scatter than the other.
template <bool kCached>
__device__ __forceinline__ void load_tile(const uint64_t *__restrict__ hashes, uint32_t t0, uint32_t e,
                                          uint64_t (&h)[kScatterPer]) {
  constexpr uint32_t kLoad = kCached ? (uint32_t)SBBF_HASH_LOAD_CACHED : 0u;
#pragma unroll
  for (uint32_t t = 0; t < kScatterPer; ++t) {
    const uint32_t i = t0 + t * kScatterThreads + threadIdx.x;
    h[t] = load_hash<kLoad>(hashes + (i < e ? i : e - 1u));
  }
}

// Per-slice state of one scatter workgroup, kept by the thread that owns the
// slice: where the chunk's next key of the slice goes, how many of its keys
// came before (lookups), and the keys carried over from the previous tile
// (fewer than L, the tail of a group of L keys that is not yet complete).
template <int R>
struct SliceCursor {
  uint32_t cursor[R], pbase[R], carry[R], carry_at[R];
};

// Fixed-capacity buckets of the count-free insert partition. Scatter
// workgroup g (of G = gridDim.x) writes its keys of slice s to bucket
// s * G + g (a slice's buckets are adjacent), which holds up to cap keys (a
// multiple of 8) from position (s * G + g) * cap; count[s * G + g] is the
// bucket's key count rounded up to a multiple of four (padded with copies of
// its last key: a key inserted twice sets the same bits). Keys that find their
// bucket full go to ovf (ovf_n of them, at most ovf_cap), which a
// global-atomic pass inserts afterwards.
struct Buckets {
  uint32_t cap;
  uint32_t *count;
  uint64_t *ovf;
  uint32_t *ovf_n;
  uint32_t ovf_cap;
};

// End (exclusive) of scatter workgroup g's bucket of slice s.
__device__ __forceinline__ uint32_t bucket_end(uint32_t g, uint32_t s, uint32_t cap) {
  return (s * gridDim.x + g + 1u) * cap;
}

// One tile of the scatter: rank every key within its slice (LDS atomics),
// scan the slice counts (plus carried keys), stage the keys sorted by slice
// behind each slice's carried keys, and write every complete, aligned group
// of L keys with consecutive lanes; the incomplete tail of each slice's run
// stays in the stage as the next tile's carry. kFull: the whole tile is
// inside the chunk (no per-key guards).
template <bool kWithPos, int R, uint32_t L, bool kBucket, bool kFull>
__device__ __forceinline__ void scatter_tile(uint64_t (&h)[kScatterPer], uint32_t t0, uint32_t e,
                                             const uint32_t *__restrict__ new_chunk_hist, uint32_t num_blocks,
                                             uint32_t slice_shift, uint32_t slice_base, uint32_t num_slices,
                                             uint32_t keys,
                                             const ScatterLds &S, SliceCursor<R> &C, uint64_t *__restrict__ out_keys,
                                             uint16_t *__restrict__ out_pos, const Buckets &Bk) {
  // Keys are hashed here, where the prefetched tile is first used.
  if (keys) {
#pragma unroll
    for (uint32_t t = 0; t < kScatterPer; ++t) h[t] = key_hash(h[t]);
  }
  static_assert(L == 1u || R <= 2, "carried groups need at most two slices per thread");
  static_assert(!kBucket || (L >= 4u && !kWithPos), "buckets are for inserts with carried groups");
  constexpr uint32_t kCarryMax = L > 1u ? L - 1u : 1u;
  const uint32_t own = threadIdx.x * R;
  if constexpr (kWithPos) {
    // First tile of a new chunk: positions restart at that chunk's slice
    // prefix (new_chunk_hist is its count row; it is uniform).
    if (new_chunk_hist != nullptr) {
      uint32_t c0[R];
#pragma unroll
      for (int r = 0; r < R; ++r) c0[r] = own + r < num_slices ? new_chunk_hist[own + r] : 0u;
      uint32_t run0 = block_scan_owned<R, kScatterThreads>(c0, S.wsum);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        C.pbase[r] = run0;
        run0 += c0[r];
      }
    }
  }
  uint32_t s[kScatterPer], rank[kScatterPer];
#pragma unroll
  for (uint32_t t = 0; t < kScatterPer; ++t) {
    const uint32_t i = t0 + t * kScatterThreads + threadIdx.x;
    s[t] = local_slice(h[t], num_blocks, slice_shift, slice_base, num_slices);
    rank[t] = __hip_atomic_fetch_add(S.hist + s[t], (kFull || i < e) ? 1u : 0u, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  lds_barrier();
  uint32_t c[R], m[R];
  uint64_t carried[R][kCarryMax];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t sl = own + r;
    c[r] = sl < num_slices ? S.hist[sl] : 0u;
    if (sl < num_slices) S.hist[sl] = 0u;  // ready for the next tile (ranked after two more barriers)
    if constexpr (L > 1u) {
#pragma unroll
      for (uint32_t j = 0; j < kCarryMax; ++j) carried[r][j] = j < C.carry[r] ? S.stage[C.carry_at[r] + j] : 0ull;
    }
    m[r] = C.carry[r] + c[r];
  }
  uint32_t total;
  // Every thread has read its carried keys before the barrier inside the scan,
  // so the stage can be rewritten after it.
  uint32_t run = block_scan_owned<R, kScatterThreads>(m, S.wsum, &total);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t sl = own + r;
    if constexpr (L > 1u) {
#pragma unroll
      for (uint32_t j = 0; j < kCarryMax; ++j)
        if (j < C.carry[r]) S.stage[run + j] = carried[r][j];
    }
    const uint32_t first = C.cursor[r] - C.carry[r];  // global position of staged position `run`
    const uint32_t end = C.cursor[r] + c[r];
    uint32_t aligned = end & ~(L - 1u);
    // Buckets: once the run passes the bucket's end, the bucket is written up
    // to its end and the rest of the run goes to the overflow list, uncarried.
    bool spill = false;
    if constexpr (kBucket) {
      const uint32_t cap_end = bucket_end(blockIdx.x, sl, Bk.cap);
      spill = end > cap_end;
      if (spill) aligned = cap_end;
    }
    const uint32_t wlen = aligned > first ? aligned - first : 0u;  // keys written by this tile
    if (sl < num_slices) {
      S.info[sl] = make_uint2(first - run, run + wlen);
      S.sbase[sl] = run + C.carry[r];
      if constexpr (kWithPos) S.pdelta[sl] = C.pbase[r] - (run + C.carry[r]);
    }
    C.carry[r] = spill ? 0u : m[r] - wlen;
    C.carry_at[r] = run + wlen;
    C.cursor[r] = end;
    C.pbase[r] += c[r];
    run += m[r];
  }
  lds_barrier();
#pragma unroll
  for (uint32_t t = 0; t < kScatterPer; ++t) {
    const uint32_t i = t0 + t * kScatterThreads + threadIdx.x;
    if (kFull || i < e) {
      const uint32_t k = S.sbase[s[t]] + rank[t];
      S.stage[k] = h[t];
      // Positions are read back only by the unpermute kernel, after the
      // slice phase: stored non-temporally (3 % faster lookups on MI355X).
      if constexpr (kWithPos) __builtin_nontemporal_store((uint16_t)(k + S.pdelta[s[t]]), out_pos + i);
    }
  }
  lds_barrier();
#pragma unroll
  for (uint32_t t = 0; t < kScatterPer + (L - 1u) * R; ++t) {
    const uint32_t k = t * kScatterThreads + threadIdx.x;
    if ((L == 1u && kFull) || k < total) {
      const uint64_t key = S.stage[k];
      const uint32_t sl = local_slice(key, num_blocks, slice_shift, slice_base, num_slices);
      const uint2 in = S.info[sl];
      if (L == 1u || k < in.y) {
        out_keys[k + in.x] = key;
      } else if constexpr (kBucket) {
        // past the bucket's end: to the overflow list (carried keys are not)
        if (k + in.x >= bucket_end(blockIdx.x, sl, Bk.cap)) {
          const uint32_t o = __hip_atomic_fetch_add(Bk.ovf_n, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (o < Bk.ovf_cap) Bk.ovf[o] = key;
        }
      }
    }
  }
  // The next tile's first barrier orders these reads of stage and info
  // before they are rewritten.
}

// Workgroup g partitions chunk g. For lookups it also writes, for every key i
// of the chunk, the 16-bit position of its result inside the chunk's own
// results (the chunk's runs of all slices laid end to end in slice order),
// which is what the unpermute kernel reads back from LDS.
template <bool kWithPos, int R, uint32_t L, bool kBucket>
__global__ void __launch_bounds__(kScatterThreads)
part_scatter_kernel(const uint64_t *__restrict__ hashes, uint32_t n, uint32_t chunk, uint32_t chunks_per_group,
                    uint32_t num_blocks, uint32_t slice_shift, uint32_t slice_base, uint32_t num_slices,
                    const uint32_t *__restrict__ offsets, const uint32_t *__restrict__ start,
                    const uint32_t *__restrict__ hist_rows, uint32_t keys, uint64_t *__restrict__ out_keys,
                    uint16_t *__restrict__ out_pos, Buckets Bk) {
  extern __shared__ unsigned long long smem[];
  ScatterLds S;
  S.stage = reinterpret_cast<uint64_t *>(smem);
  S.info = reinterpret_cast<uint2 *>(S.stage + stage_keys(L, R));
  S.hist = reinterpret_cast<uint32_t *>(S.info + num_slices);
  S.sbase = S.hist + num_slices;
  S.pdelta = S.sbase + num_slices;
  S.wsum = kWithPos ? S.pdelta + num_slices : S.pdelta;

  // This workgroup takes chunks u0 .. u0 + chunks_per_group - 1.
  const uint32_t u0 = blockIdx.x * chunks_per_group;
  uint32_t b, e;
  chunk_range(blockIdx.x, chunk * chunks_per_group, n, &b, &e);
  const uint32_t own = threadIdx.x * R;
  if (b >= e) {  // whole workgroup
    if constexpr (kBucket) {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (own + r < num_slices) Bk.count[(own + r) * gridDim.x + blockIdx.x] = 0u;
    }
    return;
  }

  const uint32_t *my_start = kBucket ? nullptr : start + (uint64_t)u0 * num_slices;
  const uint32_t *my_hist = kWithPos ? hist_rows + (uint64_t)u0 * num_slices : nullptr;
  SliceCursor<R> C;
  uint32_t c[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t sl = own + r;
    if constexpr (kBucket)
      C.cursor[r] = bucket_end(blockIdx.x, sl, Bk.cap) - Bk.cap;
    else
      C.cursor[r] = sl < num_slices ? offsets[sl] + my_start[sl] : 0u;
    C.carry[r] = 0u;
    C.carry_at[r] = 0u;
    C.pbase[r] = 0u;
    c[r] = kWithPos && sl < num_slices ? my_hist[sl] : 0u;
    if (sl < num_slices) S.hist[sl] = 0u;
  }
  if constexpr (kWithPos) {
    uint32_t run = block_scan_owned<R, kScatterThreads>(c, S.wsum);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      C.pbase[r] = run;
      run += c[r];
    }
  }
  lds_barrier();

  // Tiles alternate between two register sets so the next tile's loads are
  // issued before this tile's stores and need no register copies.
  const uint32_t nfull = (e - b) / kTile;
  uint64_t ha[kScatterPer], hb[kScatterPer];
  load_tile<kWithPos>(hashes, b, e, ha);
  uint32_t t0 = b, k = 0;
#define SBBF_SCATTER_TILE(FULL, H)                                                                            \
  scatter_tile<kWithPos, R, L, kBucket, FULL>(                                                                \
      H, t0, e, kWithPos && t0 != b && t0 % chunk == 0u ? hist_rows + (uint64_t)(t0 / chunk) * num_slices : nullptr, \
      num_blocks, slice_shift, slice_base, num_slices, keys, S, C, out_keys, out_pos, Bk)
  for (; k + 2u <= nfull; k += 2u) {
    load_tile<kWithPos>(hashes, t0 + kTile, e, hb);
    SBBF_SCATTER_TILE(true, ha);
    t0 += kTile;
    load_tile<kWithPos>(hashes, t0 + kTile, e, ha);
    SBBF_SCATTER_TILE(true, hb);
    t0 += kTile;
  }
  if (k < nfull) {
    load_tile<kWithPos>(hashes, t0 + kTile, e, hb);
    SBBF_SCATTER_TILE(true, ha);
    t0 += kTile;
    if (t0 < e) SBBF_SCATTER_TILE(false, hb);
  } else if (t0 < e) {
    SBBF_SCATTER_TILE(false, ha);
  }
#undef SBBF_SCATTER_TILE
  // The last incomplete group of every slice: its keys are still in the
  // stage (nothing rewrites it after the last tile's staging barrier).
  if constexpr (L > 1u) {
#pragma unroll
    for (int r = 0; r < R; ++r)
      for (uint32_t j = 0; j < C.carry[r]; ++j) out_keys[C.cursor[r] - C.carry[r] + j] = S.stage[C.carry_at[r] + j];
  }
  // Buckets: pad each to a multiple of four keys with copies of its last
  // (carried) key and record its count. A bucket with no carry ends at a
  // multiple of L (or is full), already a multiple of four.
  if constexpr (kBucket) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t sl = own + r;
      if (sl >= num_slices) continue;
      const uint32_t cap_end = bucket_end(blockIdx.x, sl, Bk.cap);
      uint32_t end = min(C.cursor[r], cap_end);
      if (C.carry[r] > 0u) {
        const uint64_t last = S.stage[C.carry_at[r] + C.carry[r] - 1u];
        for (; end & 3u; ++end) out_keys[end] = last;
      }
      Bk.count[sl * gridDim.x + blockIdx.x] = end - (cap_end - Bk.cap);
    }
  }
}

// Copy of a slice (nb blocks of K words from block b0) into LDS: eight
// 16-byte loads per thread issued back to back (non-temporal: each slice is
// read once per call; 1 % faster inserts on MI355X), then the LDS stores.
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

template <uint32_t K>
__device__ __forceinline__ void load_slice_to_lds(uint4 *lds4, const uint32_t *words, uint32_t b0, uint32_t nb) {
  const u64x2 *src = reinterpret_cast<const u64x2 *>(words + (uint64_t)b0 * K);
  const uint32_t count = nb * (K / 4u);
  for (uint32_t base = 0; base < count; base += 8u * kPartThreads) {
    uint4 v[8];
#pragma unroll
    for (uint32_t u = 0; u < 8u; ++u) {
      const uint32_t i = base + u * kPartThreads + threadIdx.x;
      const u64x2 q = i < count ? __builtin_nontemporal_load(src + i) : u64x2{0ull, 0ull};
      v[u] = make_uint4((uint32_t)q.x, (uint32_t)(q.x >> 32), (uint32_t)q.y, (uint32_t)(q.y >> 32));
    }
#pragma unroll
    for (uint32_t u = 0; u < 8u; ++u) {
      const uint32_t i = base + u * kPartThreads + threadIdx.x;
      if (i < count) lds4[i] = v[u];
    }
  }
}

// Slice kernels: one lane per key, four keys per lane per step. Slice s's
// keys start 32-byte aligned (offsets are multiples of four keys), so a lane
// reads its four hashes with two 16-byte loads. Wave w takes steps of 256
// keys; lane l of a step takes keys 4l .. 4l+3. A lane whose group starts
// past the slice's last key reads the last group instead (in bounds: the
// padded run ends at a multiple of four keys), and keys at or past the
// slice's count are masked: inserts OR a zero mask; lookups write a group's
// result word in place when the group starts inside the slice and to a spare
// word past the last run otherwise. Padding hashes
// are arbitrary, so block indices are clamped into the slice before any LDS
// access.
// Index of this wave in its workgroup, as a wave-uniform (scalar) value so
// that loops over it compile to scalar branches.
__device__ __forceinline__ uint32_t wave_index() {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
}

// Hashes of one loop step for this lane: kSliceSteps groups of four keys
// (steps of 256 keys), each group index clamped to the slice's last group.
// The lookup kernel loads them through the caches, the insert kernel with the
// non-temporal hint (each the faster of the two for that kernel on MI355X).
struct SliceStep {
  uint64_t h[kSliceSteps][4];
};

template <bool kCached>
__device__ __forceinline__ void load_step(const uint64_t *__restrict__ keys, uint32_t base, uint32_t last,
                                          SliceStep &s) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (uint32_t u = 0; u < kSliceSteps; ++u) {
    const u64x2 *p = reinterpret_cast<const u64x2 *>(keys + min(base + 256u * u + 4u * lane, last));
    const u64x2 a = kCached ? p[0] : __builtin_nontemporal_load(p);
    const u64x2 b = kCached ? p[1] : __builtin_nontemporal_load(p + 1);
    s.h[u][0] = a.x;
    s.h[u][1] = a.y;
    s.h[u][2] = b.x;
    s.h[u][3] = b.y;
  }
}

// OR the masks of one step's keys into the slice in LDS: K/2 64-bit ORs per
// key in a per-block rotated pair order (fewer LDS bank conflicts: on MI355X
// the kernel takes 277 instead of 330 us for 1e8 keys into 128 MiB).
template <uint32_t K>
__device__ __forceinline__ void insert_step(const SliceStep &s, uint32_t base, uint32_t ns, uint32_t num_blocks,
                                            uint32_t b0, uint32_t nb, unsigned long long *lds2) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (uint32_t u = 0; u < kSliceSteps; ++u) {
    const uint32_t at = base + 256u * u + 4u * lane;
#pragma unroll
    for (uint32_t k = 0; k < 4u; ++k) {
      const uint64_t h = s.h[u][k];
      const uint32_t x = (uint32_t)h;
      const uint32_t bl = min(block_of((uint32_t)(h >> 32), num_blocks) - b0, nb - 1u);
      const uint32_t one = at + k < ns ? 1u : 0u;
      lds_or_key<K>(lds2, bl, x, one);
    }
  }
}

// Test one step's keys against the slice in LDS (K/4 16-byte reads per key)
// and write one result word (four result bytes) per group.
template <uint32_t K>
__device__ __forceinline__ void lookup_step(const SliceStep &s, uint32_t base, uint32_t ns, uint32_t num_blocks,
                                            uint32_t b0, uint32_t nb, const uint4 *lds4, uint32_t begin,
                                            uint32_t spare, uint32_t *__restrict__ res4) {
  constexpr uint32_t V = K / 4u;  // 16-byte pieces per block
  const uint32_t lane = lane_id();
#pragma unroll
  for (uint32_t u = 0; u < kSliceSteps; ++u) {
    const uint32_t at = base + 256u * u + 4u * lane;
    uint4 w[4][V];
#pragma unroll
    for (uint32_t k = 0; k < 4u; ++k) {
      const uint32_t bl = min(block_of((uint32_t)(s.h[u][k] >> 32), num_blocks) - b0, nb - 1u);
#pragma unroll
      for (uint32_t q = 0; q < V; ++q) w[k][q] = lds4[V * bl + q];
    }
    uint32_t r = 0;
#pragma unroll
    for (uint32_t k = 0; k < 4u; ++k) {
      const uint32_t x = (uint32_t)s.h[u][k];
      uint32_t t = 1u;
#pragma unroll
      for (uint32_t q = 0; q < V; ++q)
        t &= (w[k][q].x >> bit_of(seed_k(4u * q), x)) & (w[k][q].y >> bit_of(seed_k(4u * q + 1u), x)) &
             (w[k][q].z >> bit_of(seed_k(4u * q + 2u), x)) & (w[k][q].w >> bit_of(seed_k(4u * q + 3u), x));
      r |= (t & 1u) << (8u * k);
    }
    res4[at < ns ? (begin + at) / 4u : spare] = r;
  }
}

// Steps alternate between two register sets, so the next step's hashes are
// in flight while this step is processed and need no register copies. Both
// halves of an iteration always run (a step past the slice's keys is all
// masked), so there is no branch the compiler could sink the prefetch into;
// the scheduling barriers keep it above the step. Loads past the slice are
// clamped, so the prefetch never leaves it.
#define SBBF_SLICE_LOOP(STEP)                                               \
  do {                                                                      \
    constexpr uint32_t stride = waves * 256u * kSliceSteps;                 \
    uint32_t base = wave_index() * 256u * kSliceSteps;                      \
    const uint32_t steps = base < ns ? (ns - base + stride - 1u) / stride : 0u; \
    SliceStep sa, sb;                                                       \
    load_step<kCachedKeys>(keys, base, last, sa);                           \
    for (uint32_t it = 0; it < steps; it += 2u) {                           \
      load_step<kCachedKeys>(keys, base + stride, last, sb);                \
      __builtin_amdgcn_sched_barrier(0);                                    \
      STEP(sa, base);                                                       \
      base += stride;                                                       \
      load_step<kCachedKeys>(keys, base + stride, last, sa);                \
      __builtin_amdgcn_sched_barrier(0);                                    \
      STEP(sb, base);                                                       \
      base += stride;                                                       \
    }                                                                       \
  } while (0)

// K: 32-bit words per block (8 for the method, 4 or 16 for the variants).
template <uint32_t K>
__global__ void __launch_bounds__(kPartThreads)
part_slice_insert_kernel(const uint64_t *__restrict__ part, const uint32_t *__restrict__ offsets,
                         const uint32_t *__restrict__ tot, uint32_t *__restrict__ words, uint32_t num_blocks,
                         uint32_t slice_shift, uint32_t slice_base) {
  extern __shared__ uint4 lds4[];
  unsigned long long *lds2 = reinterpret_cast<unsigned long long *>(lds4);
  const uint32_t slice = blockIdx.x;
  const uint32_t ns = tot[slice];
  if (ns == 0) return;  // whole workgroup: the slice is unchanged
  const uint32_t b0 = (slice_base + slice) << slice_shift;
  const uint32_t nb = min(1u << slice_shift, num_blocks - b0);
  load_slice_to_lds<K>(lds4, words, b0, nb);
  __syncthreads();

  const uint64_t *keys = part + offsets[slice];
  const uint32_t last = ((ns + 3u) & ~3u) - 4u;
  constexpr uint32_t waves = kPartThreads / kWave;
  constexpr bool kCachedKeys = false;
#define SBBF_INSERT_STEP(S, BASE) insert_step<K>(S, BASE, ns, num_blocks, b0, nb, lds2)
  SBBF_SLICE_LOOP(SBBF_INSERT_STEP);
#undef SBBF_INSERT_STEP
  __syncthreads();
  uint4 *dst4 = reinterpret_cast<uint4 *>(words + (uint64_t)b0 * K);
  for (uint32_t i = threadIdx.x; i < nb * (K / 4u); i += kPartThreads) dst4[i] = lds4[i];
}

// Records of one loop step of a bucketed slice: as load_step, over the
// slice's buckets laid end to end (prefix[g]: keys in the buckets before
// bucket g; counts are multiples of four, so a group of four keys lies in one
// bucket). A group at position v finds its bucket from the coarse map
// (map[m]: the bucket holding position m << map_shift; map[m + 1] bounds the
// search from above), then a binary search over that range, usually of one
// or two buckets. part points at the slice's first bucket.
constexpr uint32_t kMaxBucketGroups = 1024;  // scatter workgroups of a bucketed insert
constexpr uint32_t kBucketMap = 4096;        // coarse map entries

__device__ __forceinline__ void load_step_buckets(const uint64_t *__restrict__ part, uint32_t cap,
                                                  const uint32_t *prefix, const uint16_t *map, uint32_t map_shift,
                                                  uint32_t base, uint32_t last, SliceStep &s) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (uint32_t u = 0; u < kSliceSteps; ++u) {
    const uint32_t v = min(base + 256u * u + 4u * lane, last);
    const uint32_t m = v >> map_shift;
    uint32_t lo = map[m], hi = map[m + 1u];
    while (lo < hi) {  // largest g in [lo, hi] with prefix[g] <= v
      const uint32_t mid = (lo + hi + 1u) >> 1;
      if (prefix[mid] <= v)
        lo = mid;
      else
        hi = mid - 1u;
    }
    const u64x2 *p = reinterpret_cast<const u64x2 *>(part + (uint64_t)lo * cap + (v - prefix[lo]));
    const u64x2 a = __builtin_nontemporal_load(p);
    const u64x2 b = __builtin_nontemporal_load(p + 1);
    s.h[u][0] = a.x;
    s.h[u][1] = a.y;
    s.h[u][2] = b.x;
    s.h[u][3] = b.y;
  }
}

// Slice insert over the fixed-capacity buckets of a count-free partition
// (one bucket per scatter workgroup): the slice in LDS, then the buckets' key
// counts scanned into a prefix and a coarse map after it, then the slice
// loop over the buckets as one sequence.
template <uint32_t K>
__global__ void __launch_bounds__(kPartThreads)
part_bucket_insert_kernel(const uint64_t *__restrict__ part, const uint32_t *__restrict__ counts, uint32_t groups,
                          uint32_t cap, uint32_t *__restrict__ words, uint32_t num_blocks, uint32_t slice_shift) {
  extern __shared__ uint4 lds4[];
  unsigned long long *lds2 = reinterpret_cast<unsigned long long *>(lds4);
  const uint32_t slice = blockIdx.x;
  const uint32_t b0 = slice << slice_shift;
  const uint32_t nb = min(1u << slice_shift, num_blocks - b0);
  // after the largest slice: prefix [kMaxBucketGroups + 1], map [kBucketMap + 1], wsum [16]
  uint32_t *prefix = reinterpret_cast<uint32_t *>(lds4 + (((size_t)1 << slice_shift) * K) / 4u);
  uint16_t *map = reinterpret_cast<uint16_t *>(prefix + kMaxBucketGroups + 1u);
  uint32_t *wsum = prefix + kMaxBucketGroups + 1u + (kBucketMap + 2u) / 2u;
  const uint32_t *my_counts = counts + (uint64_t)slice * groups;
  uint32_t ns;
  const uint32_t cnt = threadIdx.x < groups ? my_counts[threadIdx.x] : 0u;
  // The slice's loads are issued before the scan and the map are built (a
  // slice is at most 128 KiB: eight 16-byte pieces per thread) and stored to
  // LDS after.
  static_assert(8u * kPartThreads * 16u >= (128u << 10), "one round of loads holds a slice");
  const u64x2 *src = reinterpret_cast<const u64x2 *>(words + (uint64_t)b0 * K);
  const uint32_t count4 = nb * (K / 4u);
  u64x2 q[8];
#pragma unroll
  for (uint32_t u = 0; u < 8u; ++u) {
    const uint32_t i = u * kPartThreads + threadIdx.x;
    q[u] = i < count4 ? __builtin_nontemporal_load(src + i) : u64x2{0ull, 0ull};
  }
  uint32_t start;
  {
    const uint32_t c[1] = {cnt};
    start = block_scan_owned<1>(c, wsum, &ns);
  }
  if (ns == 0) return;  // whole workgroup: the slice is unchanged
  // Smallest map_shift >= 6 with at most kBucketMap map entries.
  uint32_t map_shift = 6;
  while (((ns - 1u) >> map_shift) + 1u > kBucketMap) ++map_shift;
  const uint32_t entries = ((ns - 1u) >> map_shift) + 1u;
  if (threadIdx.x < groups) {
    prefix[threadIdx.x] = start;
    // map entries whose position lies in this (non-empty) bucket
    for (uint32_t m = (uint32_t)(((uint64_t)start + (1u << map_shift) - 1u) >> map_shift);
         ((uint64_t)m << map_shift) < (uint64_t)start + cnt; ++m)
      map[m] = (uint16_t)threadIdx.x;
  }
  if (threadIdx.x == 0) map[entries] = (uint16_t)(groups - 1u);  // upper bound for the last entry
#pragma unroll
  for (uint32_t u = 0; u < 8u; ++u) {
    const uint32_t i = u * kPartThreads + threadIdx.x;
    if (i < count4) lds4[i] = make_uint4((uint32_t)q[u].x, (uint32_t)(q[u].x >> 32), (uint32_t)q[u].y,
                                         (uint32_t)(q[u].y >> 32));
  }
  __syncthreads();

  const uint64_t *part_slice = part + (uint64_t)slice * groups * cap;
  const uint32_t last = ns - 4u;  // counts are multiples of four
  constexpr uint32_t waves = kPartThreads / kWave;
  constexpr uint32_t stride = waves * 256u * kSliceSteps;
  uint32_t base = wave_index() * 256u * kSliceSteps;
  const uint32_t steps = base < ns ? (ns - base + stride - 1u) / stride : 0u;
  SliceStep sa, sb;
  load_step_buckets(part_slice, cap, prefix, map, map_shift, base, last, sa);
  for (uint32_t it = 0; it < steps; it += 2u) {
    load_step_buckets(part_slice, cap, prefix, map, map_shift, base + stride, last, sb);
    __builtin_amdgcn_sched_barrier(0);
    insert_step<K>(sa, base, ns, num_blocks, b0, nb, lds2);
    base += stride;
    load_step_buckets(part_slice, cap, prefix, map, map_shift, base + stride, last, sa);
    __builtin_amdgcn_sched_barrier(0);
    insert_step<K>(sb, base, ns, num_blocks, b0, nb, lds2);
    base += stride;
  }
  __syncthreads();
  uint4 *dst4 = reinterpret_cast<uint4 *>(words + (uint64_t)b0 * K);
  for (uint32_t i = threadIdx.x; i < nb * (K / 4u); i += kPartThreads) dst4[i] = lds4[i];
}

// Keys that found their bucket full, inserted with global atomics after the
// slice inserts (ovf_n of them; usually none).
template <uint32_t K>
__global__ void __launch_bounds__(256)
part_overflow_insert_kernel(const uint64_t *__restrict__ ovf, const uint32_t *__restrict__ ovf_n, uint32_t ovf_cap,
                            uint32_t *__restrict__ words, uint32_t num_blocks) {
  const uint32_t n = min(*ovf_n, ovf_cap);
  for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
    const uint64_t h = ovf[i];
    const uint32_t x = (uint32_t)h;
    uint32_t *blk = words + (uint64_t)block_of((uint32_t)(h >> 32), num_blocks) * K;
#pragma unroll
    for (uint32_t w = 0; w < K; ++w)
      __hip_atomic_fetch_or(blk + w, 1u << bit_of(seed_k(w), x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <uint32_t K>
__global__ void __launch_bounds__(kPartThreads)
part_slice_lookup_kernel(const uint64_t *__restrict__ part, const uint32_t *__restrict__ offsets,
                         const uint32_t *__restrict__ tot, const uint32_t *__restrict__ words, uint32_t num_blocks,
                         uint32_t slice_shift, uint32_t slice_base, uint8_t *__restrict__ res) {
  extern __shared__ uint4 lds4[];
  const uint32_t slice = blockIdx.x;
  const uint32_t ns = tot[slice];
  if (ns == 0) return;  // whole workgroup
  const uint32_t b0 = (slice_base + slice) << slice_shift;
  const uint32_t nb = min(1u << slice_shift, num_blocks - b0);
  load_slice_to_lds<K>(lds4, words, b0, nb);
  __syncthreads();

  const uint32_t begin = offsets[slice];
  const uint64_t *keys = part + begin;
  uint32_t *res4 = reinterpret_cast<uint32_t *>(res);  // begin and the padded total are multiples of 4
  // Lanes whose group starts past the slice write their word to the spare
  // word after the last slice's run (never read), so stores need no branch.
  const uint32_t spare = offsets[gridDim.x] / 4u;
  const uint32_t last = ((ns + 3u) & ~3u) - 4u;
  constexpr uint32_t waves = kPartThreads / kWave;
  constexpr bool kCachedKeys = true;
#define SBBF_LOOKUP_STEP(S, BASE) lookup_step<K>(S, BASE, ns, num_blocks, b0, nb, lds4, begin, spare, res4)
  SBBF_SLICE_LOOP(SBBF_LOOKUP_STEP);
#undef SBBF_LOOKUP_STEP
}
#undef SBBF_SLICE_LOOP

// Workgroup g restores input order for chunk g: it copies the chunk's result
// run of every slice (res[offsets[s] + start[g][s] ...], hist[g][s] bytes)
// into LDS end to end in slice order, then writes out[i] = lds[pos[i]] for
// the chunk, as bytes or packed bits (LSB-first).
template <bool kBits>
__global__ void __launch_bounds__(kPartThreads, 8)  // 8 waves per SIMD: two workgroups per CU
part_unpermute_kernel(const uint16_t *__restrict__ pos, const uint8_t *__restrict__ res,
                      const uint32_t *__restrict__ offsets, const uint32_t *__restrict__ start,
                      const uint32_t *__restrict__ hist_rows, uint32_t num_slices, uint32_t n, uint32_t chunk,
                      uint8_t *__restrict__ out8, uint32_t *__restrict__ out_bits) {
  extern __shared__ uint32_t usmem[];
  uint32_t *local = usmem;                                 // [num_slices] run start among the chunk's results
  uint32_t *src = local + num_slices;                      // [num_slices] run start in res (byte index)
  uint32_t *wsum = src + num_slices;                       // [16]
  uint8_t *vals = reinterpret_cast<uint8_t *>(wsum + 16);  // [chunk]
  const uint32_t *row = hist_rows + (uint64_t)blockIdx.x * num_slices;
  const uint32_t *my_start = start + (uint64_t)blockIdx.x * num_slices;
  {
    uint32_t c[4], at[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t s = threadIdx.x * 4u + r;
      c[r] = s < num_slices ? row[s] : 0u;
      at[r] = s < num_slices ? offsets[s] + my_start[s] : 0u;
    }
    uint32_t run = block_scan_owned<4>(c, wsum);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t s = threadIdx.x * 4u + r;
      if (s < num_slices) {
        local[s] = run;
        src[s] = at[r];
      }
      run += c[r];
    }
  }
  __syncthreads();
  // Phase 1: each group of 16 lanes copies the runs of slices q, q + 64, ...
  // with aligned 8-byte loads and byte stores into LDS. The first 128 bytes
  // of four runs are loaded back to back; the rest of a longer run (rare:
  // runs average one result per block of the slice) follows in a loop. res
  // has at least 8 bytes of padding after its last byte, so the last word
  // of a run is always inside the workspace.
  uint32_t b, e;
  chunk_range(blockIdx.x, chunk, n, &b, &e);
  const uint32_t chunk_keys = e - b;
  const uint64_t *res8 = reinterpret_cast<const uint64_t *>(res);
  const uint32_t lane16 = threadIdx.x & 15u;
  constexpr uint32_t kGroups = kPartThreads / 16u;
  constexpr uint32_t kBatch = 4;
  auto put = [&](uint64_t v, uint32_t w, uint32_t from, uint32_t len, uint8_t *dst) {
#pragma unroll
    for (uint32_t by = 0; by < 8u; ++by) {
      const uint32_t at = w * 8u + by;  // byte index into res
      if (at >= from && at < from + len) dst[at - from] = (uint8_t)(v >> (8u * by));
    }
  };
  for (uint32_t sl0 = threadIdx.x >> 4; sl0 < num_slices; sl0 += kBatch * kGroups) {
    uint64_t v[kBatch];
    uint32_t from[kBatch], len[kBatch], w[kBatch];
#pragma unroll
    for (uint32_t u = 0; u < kBatch; ++u) {
      const uint32_t sl = sl0 + u * kGroups;
      const bool ok = sl < num_slices;
      from[u] = ok ? src[sl] : 0u;
      len[u] = ok ? (sl + 1u < num_slices ? local[sl + 1u] : chunk_keys) - local[sl] : 0u;
      w[u] = (from[u] >> 3) + lane16;
      v[u] = w[u] < ((from[u] + len[u] + 7u) >> 3) ? res8[w[u]] : 0ull;
    }
#pragma unroll
    for (uint32_t u = 0; u < kBatch; ++u) {
      const uint32_t sl = sl0 + u * kGroups;
      if (sl >= num_slices) continue;
      uint8_t *dst = vals + local[sl];
      const uint32_t w_end = (from[u] + len[u] + 7u) >> 3;
      if (w[u] < w_end) put(v[u], w[u], from[u], len[u], dst);
      for (uint32_t ww = w[u] + 16u; ww < w_end; ww += 16u) put(res8[ww], ww, from[u], len[u], dst);
    }
  }
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63u;
  if constexpr (!kBits) {
    // Phase 2 (bytes): four consecutive positions per thread and step, four
    // steps per iteration; b is a multiple of 4.
    const bool aligned4 = ((uintptr_t)out8 & 3u) == 0;
    constexpr uint32_t kStep = 4u * kPartThreads;
    for (uint32_t i0 = b + 4u * threadIdx.x; i0 < e; i0 += 4u * kStep) {
      uint2 p2[4];
#pragma unroll
      for (uint32_t u = 0; u < 4u; ++u) {
        const uint32_t i = i0 + u * kStep;
        p2[u] = i + 4u <= e ? *reinterpret_cast<const uint2 *>(pos + i) : make_uint2(0u, 0u);
      }
#pragma unroll
      for (uint32_t u = 0; u < 4u; ++u) {
        const uint32_t i = i0 + u * kStep;
        if (i + 4u <= e) {
          const uint32_t word = (uint32_t)vals[p2[u].x & 0xffffu] | ((uint32_t)vals[p2[u].x >> 16] << 8) |
                                ((uint32_t)vals[p2[u].y & 0xffffu] << 16) | ((uint32_t)vals[p2[u].y >> 16] << 24);
          if (aligned4) {
            *reinterpret_cast<uint32_t *>(out8 + i) = word;
          } else {
            for (uint32_t k = 0; k < 4u; ++k) out8[i + k] = (uint8_t)(word >> (8u * k));
          }
        } else {
          for (uint32_t k = i; k < e; ++k) out8[k] = vals[pos[k]];
        }
      }
    }
  } else {
    // Phase 2 (bits): a wave takes 256 positions per step, four consecutive
    // ones per lane (one 8-byte load of positions), as a nibble; lanes 8w ..
    // 8w+7 OR their nibbles into the word of positions i0 + 32w .. +31, which
    // lane 8w stores. i0 is a multiple of 256 (chunks start at multiples of
    // the 7,168-key tile), so words are whole; positions at or past e give 0
    // bits, and a word is stored only when it starts before e.
    constexpr uint32_t kWaveSpan = 256u;
    const uint32_t wave = threadIdx.x >> 6;
    for (uint32_t i0 = b + wave * kWaveSpan; i0 < e; i0 += (kPartThreads / 64u) * kWaveSpan) {
      const uint32_t i = i0 + 4u * lane;
      uint32_t nib = 0;
      if (i + 4u <= e) {
        const uint2 p2 = *reinterpret_cast<const uint2 *>(pos + i);
        nib = (uint32_t)(vals[p2.x & 0xffffu] != 0) | ((uint32_t)(vals[p2.x >> 16] != 0) << 1) |
              ((uint32_t)(vals[p2.y & 0xffffu] != 0) << 2) | ((uint32_t)(vals[p2.y >> 16] != 0) << 3);
      } else {
        for (uint32_t k = 0; k < 4u; ++k)
          if (i + k < e) nib |= (uint32_t)(vals[pos[i + k]] != 0) << k;
      }
      uint32_t w = nib << (4u * (lane & 7u));
      w |= (uint32_t)__shfl_xor((int)w, 1);
      w |= (uint32_t)__shfl_xor((int)w, 2);
      w |= (uint32_t)__shfl_xor((int)w, 4);
      const uint32_t start = i0 + 32u * (lane >> 3);
      if ((lane & 7u) == 0 && start < e) out_bits[start / 32u] = w;
    }
  }
}

// Workspace sections (each 256-byte aligned): hist[G][P], start[G][P],
// blocksum[RB][P], tot[P], offsets[P + 1] (u32), keys (u64) and, for
// lookups, pos[n] (u16) and res (u8). Keys and results are laid out with
// every slice's run padded to a multiple of four, at most n + 3P entries.
struct PartitionLayout {
  uint32_t *hist, *start, *blocksum, *tot, *offsets;
  uint64_t *keys;
  uint16_t *pos;
  uint8_t *res;
  uint64_t bytes;
  uint32_t scatter_groups;  // lookups: scatter workgroups to spread the chunks over
};

uint32_t row_blocks(uint32_t groups) { return (groups + kScanRows - 1u) / kScanRows; }

PartitionLayout layout(void *workspace, uint64_t n, uint32_t num_slices, uint32_t groups, bool lookup) {
  auto up = [](uint64_t v) { return (v + 255u) & ~(uint64_t)255u; };
  char *base = static_cast<char *>(workspace);
  const uint64_t padded = n + 3u * (uint64_t)num_slices;
  uint64_t off = 0;
  PartitionLayout L{};
  L.hist = reinterpret_cast<uint32_t *>(base + off);
  off += up((uint64_t)groups * num_slices * 4u);
  L.start = reinterpret_cast<uint32_t *>(base + off);
  off += up((uint64_t)groups * num_slices * 4u);
  L.blocksum = reinterpret_cast<uint32_t *>(base + off);
  off += up((uint64_t)row_blocks(groups) * num_slices * 4u);
  L.tot = reinterpret_cast<uint32_t *>(base + off);
  off += up((uint64_t)num_slices * 4u);
  L.offsets = reinterpret_cast<uint32_t *>(base + off);
  off += up(((uint64_t)num_slices + 1u) * 4u);
  L.keys = reinterpret_cast<uint64_t *>(base + off);
  off += up(padded * 8u);
  if (lookup) {
    L.pos = reinterpret_cast<uint16_t *>(base + off);
    off += up(n * 2u);
    L.res = reinterpret_cast<uint8_t *>(base + off);
    off += up(padded + 8u);  // 8 bytes of padding for the unpermute kernel's word loads
  }
  L.bytes = off;
  return L;
}

// Chunking of n keys over about max_groups partitioning workgroups: chunk is
// a multiple of the scatter tile, at most kLookupChunk keys for lookups (so
// there may be more groups than max_groups), and every group gets a
// non-empty chunk. When lookups need more chunks than max_groups (the
// workgroups the count and unpermute kernels keep resident, two per compute
// unit), the tiles per chunk (5 to the most that fit) minimise rounds x
// (chunk length + a tile of fixed work per chunk): e.g. 2e8 keys take 8-tile
// chunks (3,488, seven full rounds of 512) rather than 9-tile ones (3,101, a
// seventh round almost empty).
void chunking(uint64_t n, uint32_t max_groups, bool lookup, uint32_t *chunk, uint32_t *groups) {
  const uint64_t tiles = (n + kTile - 1) / kTile;
  const uint64_t g0 = tiles < max_groups ? (tiles ? tiles : 1) : max_groups;
  uint64_t tiles_per = (tiles + g0 - 1) / g0;
  if (lookup && tiles_per * kTile > kLookupChunk) {
    const uint64_t slots = max_groups ? max_groups : 1u;
    uint64_t best = kLookupChunk / kTile, best_cost = UINT64_MAX;
    for (uint64_t tp = kLookupChunk / kTile; tp >= 5u; --tp) {
      const uint64_t g = (tiles + tp - 1u) / tp;
      // rounds x (chunk length + one tile for each chunk's fixed work: its
      // count row, the unpermute's scan over the slices)
      const uint64_t cost = (g + slots - 1u) / slots * (tp + 1u);
      if (cost < best_cost) {
        best_cost = cost;
        best = tp;
      }
    }
    tiles_per = best;
  }
  *chunk = (uint32_t)(tiles_per * kTile);
  *groups = (uint32_t)((n + *chunk - 1) / *chunk);
  if (*groups == 0) *groups = 1;
}

template <bool kWithPos, int R, uint32_t L, bool kBucket = false>
hipError_t launch_scatter(const uint64_t *hashes, uint32_t n, uint32_t chunk, uint32_t groups, uint32_t num_blocks,
                          uint32_t slice_shift, uint32_t slice_base, uint32_t num_slices, uint32_t keys,
                          const PartitionLayout &L_, hipStream_t stream, const Buckets &Bk = Buckets{}) {
  const size_t lds = scatter_lds_bytes(num_slices, kWithPos, L, R);
  // Several chunks per workgroup (lookups cut the batch finer than inserts):
  // about two workgroups per compute unit.
  const uint32_t per = kWithPos ? (groups + L_.scatter_groups - 1u) / L_.scatter_groups : 1u;
  const uint32_t grid = (groups + per - 1u) / per;
  (void)hipFuncSetAttribute((const void *)part_scatter_kernel<kWithPos, R, L, kBucket>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  (void)hipGetLastError();
  hipLaunchKernelGGL((part_scatter_kernel<kWithPos, R, L, kBucket>), dim3(grid), dim3(kScatterThreads), lds, stream,
                     hashes, n, chunk, per, num_blocks, slice_shift, slice_base, num_slices, L_.offsets, L_.start,
                     L_.hist, keys, L_.keys, kWithPos ? L_.pos : nullptr, Bk);
  return hipGetLastError();
}

// Slices per owning thread: the smallest power of two R with R * threads >= P.
// With one slice per thread, runs are written in aligned groups of
// kScatterGroup keys (the incomplete tail carried to the next tile); with two,
// in groups of four keys (32 bytes, as much carry as the LDS holds: 5 % faster
// than no carry at 256 MiB on MI355X); with four, key by key.
template <bool kWithPos>
hipError_t launch_scatter_r(const uint64_t *hashes, uint32_t n, uint32_t chunk, uint32_t groups,
                            uint32_t num_blocks, uint32_t slice_shift, uint32_t slice_base, uint32_t num_slices,
                            uint32_t keys, const PartitionLayout &L, hipStream_t stream) {
  if (num_slices <= kScatterThreads)
    return launch_scatter<kWithPos, 1, kScatterGroup>(hashes, n, chunk, groups, num_blocks, slice_shift, slice_base,
                                                      num_slices, keys, L, stream);
  if (num_slices <= 2u * kScatterThreads)
    return launch_scatter<kWithPos, 2, 4>(hashes, n, chunk, groups, num_blocks, slice_shift, slice_base, num_slices,
                                          keys, L, stream);
  static_assert(4u * kScatterThreads >= kMaxSlices, "four slices per thread cover every filter");
  return launch_scatter<kWithPos, 4, 1>(hashes, n, chunk, groups, num_blocks, slice_shift, slice_base, num_slices,
                                        keys, L, stream);
}

// Count, scan and scatter of n keys that all lie in the num_slices slices
// from slice_base (of 2^slice_shift blocks each).
hipError_t partition(const uint64_t *hashes, uint32_t n, uint32_t num_blocks, uint32_t slice_shift,
                     uint32_t slice_base, uint32_t num_slices, uint32_t chunk, uint32_t groups,
                     const PartitionLayout &L, bool with_pos, uint32_t keys, hipStream_t stream) {
  hipError_t e;
  const dim3 blk(kPartThreads);
  // Dynamic LDS above the default needs the per-kernel limit raised; an error
  // here shows up at launch.
  (void)hipFuncSetAttribute((const void *)part_count_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(num_slices * 4u));
  (void)hipGetLastError();
  hipLaunchKernelGGL(part_count_kernel, dim3(groups), blk, num_slices * 4u, stream, hashes, n, chunk, num_blocks,
                     slice_shift, slice_base, num_slices, keys, L.hist);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const dim3 scan_grid((num_slices + kScanCols - 1) / kScanCols, row_blocks(groups));
  if (scan_grid.y > 1) {  // one row block needs no carries
    hipLaunchKernelGGL(part_colsum_kernel, scan_grid, blk, 0, stream, L.hist, groups, num_slices, L.blocksum);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(part_colscan_kernel, scan_grid, blk, 0, stream, L.hist, groups, num_slices, L.blocksum, L.start,
                     L.tot);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(part_offsets_kernel, dim3(1), blk, 0, stream, L.tot, num_slices, L.offsets);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (with_pos)
    return launch_scatter_r<true>(hashes, n, chunk, groups, num_blocks, slice_shift, slice_base, num_slices, keys, L,
                                  stream);
  return launch_scatter_r<false>(hashes, n, chunk, groups, num_blocks, slice_shift, slice_base, num_slices, keys, L,
                                 stream);
}

uint32_t slices_of(uint32_t num_blocks, uint32_t slice_shift) {
  return (uint32_t)(((uint64_t)num_blocks + (1u << slice_shift) - 1u) >> slice_shift);
}

// Slice insert for K-word blocks: the slice (2^slice_shift blocks of 4K
// bytes) in dynamic LDS.
template <uint32_t K>
hipError_t launch_slice_insert(const PartitionLayout &L, uint32_t num_slices, uint32_t *words, uint32_t num_blocks,
                               uint32_t slice_shift, uint32_t slice_base, hipStream_t stream) {
  const size_t lds_bytes = ((size_t)1 << slice_shift) * 4u * K;
  (void)hipFuncSetAttribute((const void *)part_slice_insert_kernel<K>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds_bytes);
  (void)hipGetLastError();
  hipLaunchKernelGGL(part_slice_insert_kernel<K>, dim3(num_slices), dim3(kPartThreads), lds_bytes, stream, L.keys,
                     L.offsets, L.tot, words, num_blocks, slice_shift, slice_base);
  return hipGetLastError();
}

template <uint32_t K>
hipError_t launch_slice_lookup(const PartitionLayout &L, uint32_t num_slices, const uint32_t *words,
                               uint32_t num_blocks, uint32_t slice_shift, uint32_t slice_base, hipStream_t stream) {
  const size_t lds_bytes = ((size_t)1 << slice_shift) * 4u * K;
  (void)hipFuncSetAttribute((const void *)part_slice_lookup_kernel<K>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds_bytes);
  (void)hipGetLastError();
  hipLaunchKernelGGL(part_slice_lookup_kernel<K>, dim3(num_slices), dim3(kPartThreads), lds_bytes, stream, L.keys,
                     L.offsets, L.tot, words, num_blocks, slice_shift, slice_base, L.res);
  return hipGetLastError();
}

// Results of a partition (in partitioned order, L.res) back to input order.
hipError_t unpermute(const PartitionLayout &L, uint32_t num_slices, uint32_t n, uint32_t chunk, uint32_t groups,
                     uint8_t *out8, uint32_t *out_bits, hipStream_t stream) {
  const size_t u_lds = (size_t)num_slices * 8u + 64u + chunk;
  (void)hipFuncSetAttribute((const void *)part_unpermute_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)u_lds);
  (void)hipFuncSetAttribute((const void *)part_unpermute_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)u_lds);
  (void)hipGetLastError();
  if (out_bits)
    hipLaunchKernelGGL(part_unpermute_kernel<true>, dim3(groups), dim3(kPartThreads), u_lds, stream, L.pos, L.res,
                       L.offsets, L.start, L.hist, num_slices, n, chunk, nullptr, out_bits);
  else
    hipLaunchKernelGGL(part_unpermute_kernel<false>, dim3(groups), dim3(kPartThreads), u_lds, stream, L.pos, L.res,
                       L.offsets, L.start, L.hist, num_slices, n, chunk, out8, nullptr);
  return hipGetLastError();
}

// Count-free insert partition (fixed-capacity buckets, struct Buckets): for
// one-level inserts into at most 2 * kScatterThreads slices (runs carried in
// groups of four or eight keys), with at most kMaxBucketGroups scatter
// workgroups and every bucket position below 2^32. It skips the count and
// scan kernels (one read of the batch) at the price of bucket room (the
// expected keys per bucket plus eight standard deviations and 32 keys) and an
// overflow list as long as the batch.
struct BucketPlan {
  uint32_t chunk, groups, cap;
  uint64_t count_off, ovfn_off, ovf_off, keys_off, bytes;
};

bool bucket_plan(uint64_t n, uint32_t num_slices, uint32_t max_groups, BucketPlan *bp) {
  if (n == 0 || num_slices > 2u * kScatterThreads) return false;
  chunking(n, max_groups, false, &bp->chunk, &bp->groups);
  if (bp->groups > kMaxBucketGroups) return false;
  // Keys of one chunk per slice: a slice holds at most 1 / (slices - 1) of
  // the blocks (all but the last are whole).
  const double mean = (double)bp->chunk / (double)(num_slices > 1u ? num_slices - 1u : 1u);
  const uint64_t cap = ((uint64_t)(mean + 8.0 * std::sqrt(mean) + 32.0) + 7u) & ~(uint64_t)7u;
  const uint64_t positions = (uint64_t)bp->groups * num_slices * cap;
  if (positions >= (1ull << 32)) return false;
  bp->cap = (uint32_t)cap;
  auto up = [](uint64_t v) { return (v + 255u) & ~(uint64_t)255u; };
  uint64_t off = 0;
  bp->count_off = off;
  off += up((uint64_t)bp->groups * num_slices * 4u);
  bp->ovfn_off = off;
  off += 256u;
  bp->ovf_off = off;
  off += up(n * 8u);
  bp->keys_off = off;
  off += up(positions * 8u);
  bp->bytes = off;
  return true;
}

template <uint32_t K>
hipError_t launch_bucket_insert(const uint64_t *part, const uint32_t *counts, const BucketPlan &bp,
                                uint32_t num_slices, uint32_t *words, uint32_t num_blocks, uint32_t slice_shift,
                                hipStream_t stream) {
  const size_t lds_bytes =
      ((size_t)1 << slice_shift) * 4u * K + (kMaxBucketGroups + 1u + (kBucketMap + 2u) / 2u + 16u) * 4u;
  (void)hipFuncSetAttribute((const void *)part_bucket_insert_kernel<K>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds_bytes);
  (void)hipGetLastError();
  hipLaunchKernelGGL(part_bucket_insert_kernel<K>, dim3(num_slices), dim3(kPartThreads), lds_bytes, stream, part,
                     counts, bp.groups, bp.cap, words, num_blocks, slice_shift);
  return hipGetLastError();
}

template <uint32_t K>
hipError_t launch_overflow_insert(const Buckets &Bk, uint32_t *words, uint32_t num_blocks, hipStream_t stream) {
  hipLaunchKernelGGL(part_overflow_insert_kernel<K>, dim3(256), dim3(256), 0, stream, Bk.ovf, Bk.ovf_n, Bk.ovf_cap,
                     words, num_blocks);
  return hipGetLastError();
}

hipError_t insert_buckets(const uint64_t *hashes, uint32_t n, uint32_t *words, uint32_t num_blocks,
                          uint32_t slice_shift, uint32_t num_slices, void *workspace, const BucketPlan &bp,
                          uint32_t keys, hipStream_t stream, uint32_t lanes) {
  char *base = static_cast<char *>(workspace);
  const Buckets Bk{bp.cap, reinterpret_cast<uint32_t *>(base + bp.count_off),
                   reinterpret_cast<uint64_t *>(base + bp.ovf_off), reinterpret_cast<uint32_t *>(base + bp.ovfn_off),
                   n};
  hipError_t e = launch_fill(Bk.ovf_n, 1u, 0u, stream);  // a fill kernel, not a memset (graph capture)
  if (e != hipSuccess) return e;
  PartitionLayout L{};
  L.keys = reinterpret_cast<uint64_t *>(base + bp.keys_off);
  L.scatter_groups = bp.groups;
  if (num_slices <= kScatterThreads)
    e = launch_scatter<false, 1, kScatterGroup, true>(hashes, n, bp.chunk, bp.groups, num_blocks, slice_shift, 0u,
                                                       num_slices, keys, L, stream, Bk);
  else
    e = launch_scatter<false, 2, 4, true>(hashes, n, bp.chunk, bp.groups, num_blocks, slice_shift, 0u, num_slices,
                                          keys, L, stream, Bk);
  if (e != hipSuccess) return e;
  if (lanes == 4) {
    e = launch_bucket_insert<4>(L.keys, Bk.count, bp, num_slices, words, num_blocks, slice_shift, stream);
    return e != hipSuccess ? e : launch_overflow_insert<4>(Bk, words, num_blocks, stream);
  }
  if (lanes == 16) {
    e = launch_bucket_insert<16>(L.keys, Bk.count, bp, num_slices, words, num_blocks, slice_shift, stream);
    return e != hipSuccess ? e : launch_overflow_insert<16>(Bk, words, num_blocks, stream);
  }
  e = launch_bucket_insert<8>(L.keys, Bk.count, bp, num_slices, words, num_blocks, slice_shift, stream);
  return e != hipSuccess ? e : launch_overflow_insert<8>(Bk, words, num_blocks, stream);
}

// One level: the n keys all lie in the num_slices slices from slice_base.
hipError_t insert_level(const uint64_t *hashes, uint32_t n, uint32_t *words, uint32_t num_blocks, uint32_t slice_shift,
                        uint32_t slice_base, uint32_t num_slices, void *workspace, uint32_t max_groups, uint32_t keys,
                        hipStream_t stream, uint32_t lanes) {
  uint32_t chunk, groups;
  chunking(n, max_groups, false, &chunk, &groups);
  PartitionLayout L = layout(workspace, n, num_slices, groups, false);
  L.scatter_groups = groups;
  hipError_t e =
      partition(hashes, n, num_blocks, slice_shift, slice_base, num_slices, chunk, groups, L, false, keys, stream);
  if (e != hipSuccess) return e;
  if (lanes == 4) return launch_slice_insert<4>(L, num_slices, words, num_blocks, slice_shift, slice_base, stream);
  if (lanes == 16) return launch_slice_insert<16>(L, num_slices, words, num_blocks, slice_shift, slice_base, stream);
  return launch_slice_insert<8>(L, num_slices, words, num_blocks, slice_shift, slice_base, stream);
}

hipError_t lookup_level(const uint64_t *hashes, uint32_t n, const uint32_t *words, uint32_t num_blocks,
                        uint32_t slice_shift, uint32_t slice_base, uint32_t num_slices, void *workspace,
                        uint32_t max_groups, uint8_t *out8, uint32_t *out_bits, uint32_t keys, hipStream_t stream,
                        uint32_t lanes) {
  uint32_t chunk, groups;
  chunking(n, max_groups, true, &chunk, &groups);
  PartitionLayout L = layout(workspace, n, num_slices, groups, true);
  L.scatter_groups = max_groups ? max_groups : 1u;
  hipError_t e =
      partition(hashes, n, num_blocks, slice_shift, slice_base, num_slices, chunk, groups, L, true, keys, stream);
  if (e != hipSuccess) return e;
  if (lanes == 4)
    e = launch_slice_lookup<4>(L, num_slices, words, num_blocks, slice_shift, slice_base, stream);
  else if (lanes == 16)
    e = launch_slice_lookup<16>(L, num_slices, words, num_blocks, slice_shift, slice_base, stream);
  else
    e = launch_slice_lookup<8>(L, num_slices, words, num_blocks, slice_shift, slice_base, stream);
  if (e != hipSuccess) return e;
  return unpermute(L, num_slices, n, chunk, groups, out8, out_bits, stream);
}

// Two levels, for filters of more than kOneLevelSlices slices: level 1
// partitions the keys by group of kGroupSlices consecutive slices (one slice
// per scatter thread, so level 2 writes whole 64-byte groups; at most 2,048
// groups: a filter has at most 2^21 slices), then each group's keys,
// contiguous in the level-1 output, take the one-level path with that
// group's first slice as slice_base. Launching level 2 needs each group's key
// count, so the host waits for level 1 once.
constexpr uint32_t kGroupShift = 10;
constexpr uint32_t kGroupSlices = 1u << kGroupShift;
constexpr uint32_t kOneLevelSlices = kMaxSlices;
static_assert(kGroupSlices == kScatterThreads, "a level-2 group has one slice per scatter thread");
static_assert((2u << 20) / kGroupSlices <= kMaxSlices, "level 1 takes every filter's groups");

struct TwoLevel {
  uint32_t groups;           // level-1 "slices": groups of kMaxSlices slices
  uint32_t chunk, chunks;    // level-1 chunking
  PartitionLayout L1;
  void *level2;              // workspace of the level-2 calls
};

TwoLevel two_level_plan(void *workspace, uint64_t n, uint32_t num_slices, uint32_t max_groups, bool lookup) {
  TwoLevel t;
  t.groups = (num_slices + kGroupSlices - 1u) >> kGroupShift;
  chunking(n, max_groups, lookup, &t.chunk, &t.chunks);
  t.L1 = layout(workspace, n, t.groups, t.chunks, lookup);
  t.L1.scatter_groups = lookup ? (max_groups ? max_groups : 1u) : t.chunks;
  t.level2 = static_cast<char *>(workspace) + t.L1.bytes;
  return t;
}

// Level-1 slice offsets and totals, read back to the host (waits for the stream).
hipError_t group_counts(const TwoLevel &t, std::vector<uint32_t> *offsets, std::vector<uint32_t> *tot,
                        hipStream_t stream) {
  offsets->resize(t.groups + 1u);
  tot->resize(t.groups);
  hipError_t e = hipMemcpyAsync(offsets->data(), t.L1.offsets, (t.groups + 1u) * 4u, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(tot->data(), t.L1.tot, t.groups * 4u, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  return e;
}

}  // namespace

uint32_t partition_max_slices() { return 2u << 20; }
uint32_t partition_level_slices() { return kOneLevelSlices; }
uint32_t partition_group_slices() { return kGroupSlices; }
uint64_t partition_max_keys() { return 1ull << 31; }

uint64_t partition_workspace_bytes(uint64_t n, uint32_t num_slices, uint32_t max_groups, bool lookup) {
  uint32_t chunk, groups;
  chunking(n, max_groups, lookup, &chunk, &groups);
  if (num_slices <= kOneLevelSlices) {
    const uint64_t counted = layout(nullptr, n, num_slices, groups, lookup).bytes;
    BucketPlan bp;
    if (!lookup && bucket_plan(n, num_slices, max_groups, &bp)) return std::max(counted, bp.bytes);
    return counted;
  }
  // level 1, then level 2 for at most all n keys in one group
  const uint32_t g = (num_slices + kGroupSlices - 1u) >> kGroupShift;
  return layout(nullptr, n, g, groups, lookup).bytes + partition_workspace_bytes(n, kGroupSlices, max_groups, lookup);
}

hipError_t launch_insert_partitioned(const uint64_t *hashes, uint64_t n, uint32_t *words, uint32_t num_blocks,
                                     uint32_t slice_shift, void *workspace, uint32_t max_groups, uint32_t keys,
                                     hipStream_t stream, uint32_t lanes) {
  if (n == 0) return hipSuccess;
  if (lanes != 4 && lanes != 8 && lanes != 16) return hipErrorInvalidValue;
  const uint32_t num_slices = slices_of(num_blocks, slice_shift);
  if (num_slices > partition_max_slices() || n > partition_max_keys()) return hipErrorInvalidValue;
  if (num_slices <= kOneLevelSlices) {
    BucketPlan bp;
    // (the bucketed slice insert loads a slice of at most 128 KiB in one round)
    if (((uint64_t)4u * lanes << slice_shift) <= (128u << 10) && bucket_plan(n, num_slices, max_groups, &bp))
      return insert_buckets(hashes, (uint32_t)n, words, num_blocks, slice_shift, num_slices, workspace, bp, keys,
                            stream, lanes);
    return insert_level(hashes, (uint32_t)n, words, num_blocks, slice_shift, 0u, num_slices, workspace, max_groups,
                        keys, stream, lanes);
  }
  TwoLevel t = two_level_plan(workspace, n, num_slices, max_groups, false);
  hipError_t e = partition(hashes, (uint32_t)n, num_blocks, slice_shift + kGroupShift, 0u, t.groups, t.chunk,
                           t.chunks, t.L1, false, keys, stream);
  std::vector<uint32_t> off, tot;
  if (e == hipSuccess) e = group_counts(t, &off, &tot, stream);
  for (uint32_t g = 0; g < t.groups && e == hipSuccess; ++g) {
    if (tot[g] == 0) continue;
    const uint32_t base = g << kGroupShift;
    // level-1 output holds hashes (keys were hashed there)
    e = insert_level(t.L1.keys + off[g], tot[g], words, num_blocks, slice_shift, base,
                     std::min(kGroupSlices, num_slices - base), t.level2, max_groups, 0u, stream, lanes);
  }
  return e;
}

hipError_t launch_lookup_partitioned(const uint64_t *hashes, uint64_t n, const uint32_t *words, uint32_t num_blocks,
                                     uint32_t slice_shift, void *workspace, uint32_t max_groups, uint8_t *out8,
                                     uint32_t *out_bits, uint32_t keys, hipStream_t stream, uint32_t lanes) {
  if (n == 0) return hipSuccess;
  if (lanes != 4 && lanes != 8 && lanes != 16) return hipErrorInvalidValue;
  const uint32_t num_slices = slices_of(num_blocks, slice_shift);
  if (num_slices > partition_max_slices() || n > partition_max_keys()) return hipErrorInvalidValue;
  if (num_slices <= kOneLevelSlices)
    return lookup_level(hashes, (uint32_t)n, words, num_blocks, slice_shift, 0u, num_slices, workspace, max_groups,
                        out8, out_bits, keys, stream, lanes);
  TwoLevel t = two_level_plan(workspace, n, num_slices, max_groups, true);
  hipError_t e = partition(hashes, (uint32_t)n, num_blocks, slice_shift + kGroupShift, 0u, t.groups, t.chunk,
                           t.chunks, t.L1, true, keys, stream);
  std::vector<uint32_t> off, tot;
  if (e == hipSuccess) e = group_counts(t, &off, &tot, stream);
  // Each group's results go, one byte per key, to its run of the level-1
  // results (level-1 partitioned order), which level 1 then unpermutes.
  for (uint32_t g = 0; g < t.groups && e == hipSuccess; ++g) {
    if (tot[g] == 0) continue;
    const uint32_t base = g << kGroupShift;
    e = lookup_level(t.L1.keys + off[g], tot[g], words, num_blocks, slice_shift, base,
                     std::min(kGroupSlices, num_slices - base), t.level2, max_groups, t.L1.res + off[g], nullptr, 0u,
                     stream, lanes);
  }
  if (e != hipSuccess) return e;
  return unpermute(t.L1, t.groups, (uint32_t)n, t.chunk, t.chunks, out8, out_bits, stream);
}

}  // namespace sbbf
