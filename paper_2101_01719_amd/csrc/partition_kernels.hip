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
//   offsets   offsets[s] = sum of tot[< s], each rounded up to a multiple of
//             four keys for inserts (32 bytes) and of 32 for lookups (whole
//             words of the result bitmap)
//   scatter   workgroup g walks chunk g in tiles, sorts each tile by slice in
//             LDS and writes each slice's run with consecutive lanes at the
//             slice cursor offsets[s] + start[g][s] + (keys already written);
//             for lookups it also records pos[i], where key i's result sits
//             among the chunk's results
//   slice     one workgroup per slice loads the slice into LDS; insert ORs the
//             slice's keys into it and stores it back with plain stores,
//             lookup tests the slice's keys against it and writes one result
//             bit per key in partitioned order
//   unpermute lookups only: a workgroup takes up to eight consecutive chunks,
//             gathers each chunk's results into an LDS bitmap (the runs of
//             consecutive chunks in one slice are adjacent, so each slice's
//             span is read once) and writes out[i] = result[pos[i]]
//
// Lookups into at most 2,048 slices skip count, colsum, colscan and offsets
// (a read of the batch): scatter workgroup w writes its keys of slice s into
// a bucket of fixed room, its chunks' runs one after another, and key i's
// result position in its chunk is s * room + (its rank in the chunk's run),
// so no prefix over the chunk is needed; the slice lookup walks a slice's
// buckets, and the unpermute copies each run into its slot. Keys past a
// run's room go to an overflow list that a gather pass looks up last
// (skewed batches stay exact, only slower). Inserts into at most 2,048
// slices likewise write fixed-room buckets without a count (overflowing keys
// inserted with global atomics).
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
constexpr uint32_t kScatterPer = 7;        // keys per thread per scatter tile (lookups, counted inserts)
constexpr uint32_t kScatterGroup = 8;      // keys per aligned group written by the scatter (64 bytes)
constexpr uint32_t kTile = kScatterThreads * kScatterPer;
// Keys per thread per tile of the bucketed insert scatter: one more than the
// lookup scatter (which needs the registers for its positions), so fewer
// barriers per key.
constexpr uint32_t kInsertPer = 8;
constexpr uint32_t kInsertTile = kScatterThreads * kInsertPer;
constexpr uint32_t kScanRows = 256;    // rows per colsum/colscan workgroup (16 segments of 16)
constexpr uint32_t kScanCols = 64;     // columns per colsum/colscan workgroup
constexpr uint32_t kSliceSteps = 2;    // 256-key steps per wave per slice-loop iteration
// Counted lookup chunks are at most this many keys so that positions fit 16
// bits (and a chunk's result bits, 8 KiB, one slot of the unpermute's LDS).
constexpr uint32_t kLookupChunk = 65536u;
// Counted lookup runs are padded to multiples of this many keys: a run's
// results are whole 32-bit words of the result bitmap.
constexpr uint32_t kLookupAlign = 32u;
// Most lookup chunks one unpermute workgroup restores (their result runs in
// a slice are adjacent, so it reads each slice's runs as one span).
constexpr uint32_t kUnpermuteChunks = 8u;
// LDS of one bucketed-lookup unpermute workgroup (two per compute unit).
constexpr size_t kUnpermuteLds = 78u << 10;

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

// One workgroup: offsets[s] = sum of round(tot[< s]) with every run rounded
// up to a multiple of `align` keys (a power of two: 4 for inserts, so a slice
// kernel reads a run with 16-byte loads; 32 for lookups, so a run's results
// fill whole 32-bit words of the result bitmap); offsets[num_slices] is the
// padded total. Thread t owns slices 4t .. 4t+3 (num_slices <= 4096).
__global__ void __launch_bounds__(kPartThreads)
part_offsets_kernel(const uint32_t *__restrict__ tot, uint32_t num_slices, uint32_t align,
                    uint32_t *__restrict__ offsets) {
  __shared__ uint32_t wsum[16];
  uint32_t c[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const uint32_t s = threadIdx.x * 4u + r;
    c[r] = s < num_slices ? (tot[s] + align - 1u) & ~(align - 1u) : 0u;
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
// over from the previous tile, so its size is (tile keys) + (L - 1) * (slices),
// slices = R * kScatterThreads; a tile is per keys of each thread.
constexpr uint32_t stage_keys(uint32_t L, uint32_t R, uint32_t per) {
  return per * kScatterThreads + (L - 1u) * R * kScatterThreads;
}

constexpr size_t scatter_lds_bytes(uint32_t num_slices, bool with_pos, uint32_t L, uint32_t R,
                                   uint32_t per = kScatterPer) {
  return (size_t)stage_keys(L, R, per) * 8u + (size_t)num_slices * (with_pos ? 20u : 16u) + 80u;
}

struct ScatterLds {
  uint64_t *stage;  // [stage_keys(L, R, per)] keys sorted by slice
  uint2 *info;      // [P] staged position k < info.y of slice s goes to k + info.x
  uint32_t *hist;   // [P] keys per slice in the tile (ranks come from it)
  uint32_t *sbase;  // [P] staged position of the tile's first key of slice s
  uint32_t *pdelta; // [P] (lookups) chunk result position of staged position k is k + pdelta[s]
  // [P] (bucketed lookups, in place of sbase and pdelta) (sbase, low 16 bits
  // of pdelta | the rank from which the tile's keys of slice s overflow << 16)
  uint2 *sp;
  uint32_t *wsum;   // [16]
  uint32_t *spilled;  // [1] (bucketed lookups) some slice's run reached its limit in this tile
};

// Hashes of tile t0 for this thread: index t0 + t * kScatterThreads + thread,
// clamped to the chunk's last key so loads never branch. Lookups load them
// through the caches and inserts with the non-temporal hint: measured on
// MI355X at 1e8 inserts and 2e8 lookups into 128 MiB, that order is 6 %
// faster for the lookup scatter (and its slice kernel) and 5 % faster for
// the insert scatter than the other.
template <bool kCached, uint32_t P>
__device__ __forceinline__ void load_tile(const uint64_t *__restrict__ hashes, uint32_t t0, uint32_t e,
                                          uint64_t (&h)[P]) {
  constexpr uint32_t kLoad = kCached ? (uint32_t)SBBF_HASH_LOAD_CACHED : 0u;
#pragma unroll
  for (uint32_t t = 0; t < P; ++t) {
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
  // Bucketed lookups: where the current chunk's run must end (its result
  // slots and the bucket's room). pbase = s * room + (the chunk's keys of the
  // slice so far) and cursor = (the run's start) + the same count, so the
  // run's start is cursor - (pbase - s * room).
  uint32_t limit[R];
};

// Fixed-capacity buckets of the count-free insert partition. Scatter
// workgroup g (of G = gridDim.x) writes its keys of slice s to bucket
// s * G + g (a slice's buckets are adjacent), which holds up to cap keys (a
// multiple of 8) from position (s * G + g) * cap; count[s * G + g] is the
// bucket's key count rounded up to a multiple of four (padded with copies of
// its last key: a key inserted twice sets the same bits). Keys that find their
// bucket full go to ovf (ovf_n of them, at most ovf_cap), which a
// global-atomic pass inserts afterwards.
//
// Lookups (count-free lookup partition) use the same buckets, in which each
// chunk of the workgroup's range continues the previous chunk's run. A key's
// result position in its chunk is s * room + (its rank among the chunk's keys
// of slice s), so positions need no count pass; a run keeps at most `room`
// keys and stops at the bucket's end, and the keys past either limit go to
// ovf_idx (their batch indices; a gather pass looks them up after the
// unpermute). runs[c * P + s] = (first position, keys kept) of chunk c's run
// in slice s.
struct Buckets {
  uint32_t cap;
  uint32_t *count;
  uint64_t *ovf;
  uint32_t *ovf_n;
  uint32_t ovf_cap;
  uint32_t room;
  uint32_t *ovf_idx;
  uint2 *runs;
};

// End (exclusive) of scatter workgroup g's bucket of slice s.
__device__ __forceinline__ uint32_t bucket_end(uint32_t g, uint32_t s, uint32_t cap) {
  return (s * gridDim.x + g + 1u) * cap;
}

// Bucketed lookups, at a chunk boundary: record the finished chunk's runs
// (prev, unless ~0u) and start the next chunk's runs where they ended (after
// a spill, at the run's limit: no keys are carried then), each allowed
// min(room, bucket room left) keys, result positions from s * room.
template <int R>
__device__ __forceinline__ void look_bucket_chunk(SliceCursor<R> &C, uint32_t num_slices, const Buckets &Bk,
                                                  uint32_t prev) {
  const uint32_t own = threadIdx.x * R;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t sl = own + r;
    if (sl >= num_slices) continue;
    const uint32_t end = min(C.cursor[r], C.limit[r]);
    if (prev != ~0u) {
      const uint32_t run_start = C.cursor[r] - (C.pbase[r] - sl * Bk.room);
      Bk.runs[(uint64_t)prev * num_slices + sl] = make_uint2(run_start, end - run_start);
    }
    C.cursor[r] = end;
    C.limit[r] = end + min(Bk.room, bucket_end(blockIdx.x, sl, Bk.cap) - end);
    C.pbase[r] = sl * Bk.room;
  }
}

// One tile of the scatter: rank every key within its slice (LDS atomics),
// scan the slice counts (plus carried keys), stage the keys sorted by slice
// behind each slice's carried keys, and write every complete, aligned group
// of L keys with consecutive lanes; the incomplete tail of each slice's run
// stays in the stage as the next tile's carry. kFull: the whole tile is
// inside the chunk (no per-key guards).
template <bool kWithPos, int R, uint32_t L, bool kBucket, bool kFull, uint32_t P>
__device__ __forceinline__ void scatter_tile(uint64_t (&h)[P], uint32_t t0, uint32_t e,
                                             const uint32_t *__restrict__ new_chunk_hist, uint32_t new_chunk,
                                             uint32_t num_blocks,
                                             uint32_t slice_shift, uint32_t slice_base, uint32_t num_slices,
                                             uint32_t keys,
                                             const ScatterLds &S, SliceCursor<R> &C, uint64_t *__restrict__ out_keys,
                                             uint16_t *__restrict__ out_pos, const Buckets &Bk) {
  // Keys are hashed here, where the prefetched tile is first used.
  if (keys) {
#pragma unroll
    for (uint32_t t = 0; t < P; ++t) h[t] = key_hash(h[t]);
  }
  static_assert(L == 1u || R <= 2, "carried groups need at most two slices per thread");
  static_assert(!kBucket || L >= 4u, "buckets are written with carried groups");
  constexpr uint32_t kCarryMax = L > 1u ? L - 1u : 1u;
  const uint32_t own = threadIdx.x * R;
  if constexpr (kWithPos && kBucket) {
    // First tile of a new chunk (new_chunk is uniform): close the previous
    // chunk's runs.
    if (new_chunk != ~0u) look_bucket_chunk<R>(C, num_slices, Bk, new_chunk - 1u);
  } else if constexpr (kWithPos) {
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
  uint32_t s[P], rank[P];
#pragma unroll
  for (uint32_t t = 0; t < P; ++t) {
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
      // (bucketed lookups keep the carried keys' staged position only in
      // info[s].y, written with them: one register less per slice)
      const uint32_t cat = kWithPos && kBucket ? (C.carry[r] ? S.info[sl].y : 0u) : C.carry_at[r];
#pragma unroll
      for (uint32_t j = 0; j < kCarryMax; ++j) carried[r][j] = j < C.carry[r] ? S.stage[cat + j] : 0ull;
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
      const uint32_t cap_end = kWithPos ? C.limit[r] : bucket_end(blockIdx.x, sl, Bk.cap);
      spill = end > cap_end;
      if (spill) aligned = cap_end;
      if constexpr (kWithPos)
        if (spill) *S.spilled = 1u;
    }
    const uint32_t wlen = aligned > first ? aligned - first : 0u;  // keys written by this tile
    if (sl < num_slices) {
      S.info[sl] = make_uint2(first - run, run + wlen);
      const uint32_t sb = run + C.carry[r];
      if constexpr (kWithPos && kBucket) {
        // keys of rank >= limit - cursor (none if the run is already full)
        // are past the run's limit
        const uint32_t rlim = C.limit[r] > C.cursor[r] ? C.limit[r] - C.cursor[r] : 0u;
        S.sp[sl] = make_uint2(sb, ((C.pbase[r] - sb) & 0xffffu) | (rlim << 16));
      } else {
        S.sbase[sl] = sb;
        if constexpr (kWithPos) S.pdelta[sl] = C.pbase[r] - sb;
      }
    }
    C.carry[r] = spill ? 0u : m[r] - wlen;
    if constexpr (!(kWithPos && kBucket)) C.carry_at[r] = run + wlen;
    C.cursor[r] = end;
    C.pbase[r] += c[r];
    run += m[r];
  }
  lds_barrier();
#pragma unroll
  for (uint32_t t = 0; t < P; ++t) {
    const uint32_t i = t0 + t * kScatterThreads + threadIdx.x;
    if (kFull || i < e) {
      // Positions are read back only by the unpermute kernel, after the
      // slice phase: stored non-temporally (3 % faster lookups on MI355X).
      if constexpr (kWithPos && kBucket) {
        const uint2 sp = S.sp[s[t]];
        const uint32_t k = sp.x + rank[t];
        S.stage[k] = h[t];
        // (the low 16 bits: k + pdelta; rewritten below if the key is past
        // its run's limit)
        __builtin_nontemporal_store((uint16_t)(k + sp.y), out_pos + i);
      } else {
        const uint32_t k = S.sbase[s[t]] + rank[t];
        S.stage[k] = h[t];
        if constexpr (kWithPos) __builtin_nontemporal_store((uint16_t)(k + S.pdelta[s[t]]), out_pos + i);
      }
    }
  }
  if constexpr (kWithPos && kBucket) {
    // Some run reached its limit in this tile (rare; a uniform branch): the
    // keys of rank >= the slice's limit go to the overflow pass's list, with
    // any position of their chunk (the overflow pass rewrites their results).
    if (*S.spilled) {
#pragma unroll
      for (uint32_t t = 0; t < P; ++t) {
        const uint32_t i = t0 + t * kScatterThreads + threadIdx.x;
        if ((kFull || i < e) && rank[t] >= (S.sp[s[t]].y >> 16)) {
          const uint32_t o = __hip_atomic_fetch_add(Bk.ovf_n, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (o < Bk.ovf_cap) Bk.ovf_idx[o] = i;
          __builtin_nontemporal_store((uint16_t)(s[t] * Bk.room), out_pos + i);
        }
      }
    }
  }
  lds_barrier();
  // (every thread has read the flag: cleared for the next tile, whose
  // spills are recorded after two more barriers)
  if constexpr (kWithPos && kBucket)
    if (threadIdx.x == 0) *S.spilled = 0u;
#pragma unroll
  for (uint32_t t = 0; t < P + (L - 1u) * R; ++t) {
    const uint32_t k = t * kScatterThreads + threadIdx.x;
    if ((L == 1u && kFull) || k < total) {
      const uint64_t key = S.stage[k];
      const uint32_t sl = local_slice(key, num_blocks, slice_shift, slice_base, num_slices);
      const uint2 in = S.info[sl];
      if (L == 1u || k < in.y) {
        out_keys[k + in.x] = key;
      } else if constexpr (kBucket && !kWithPos) {
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

// Workgroup g partitions chunks g * chunks_per_group onwards. For lookups it
// also writes, for every key i of a chunk, the 16-bit position of its result
// inside the chunk's own results, which is what the unpermute kernel reads
// back from LDS: counted, the chunk's runs of all slices laid end to end in
// slice order; bucketed, slot s of room positions for slice s.
template <bool kWithPos, int R, uint32_t L, bool kBucket, uint32_t P>
__global__ void __launch_bounds__(kScatterThreads)
part_scatter_kernel(const uint64_t *__restrict__ hashes, uint32_t n, uint32_t chunk, uint32_t chunks_per_group,
                    uint32_t num_blocks, uint32_t slice_shift, uint32_t slice_base, uint32_t num_slices,
                    const uint32_t *__restrict__ offsets, const uint32_t *__restrict__ start,
                    const uint32_t *__restrict__ hist_rows, uint32_t keys, uint64_t *__restrict__ out_keys,
                    uint16_t *__restrict__ out_pos, Buckets Bk) {
  extern __shared__ unsigned long long smem[];
  ScatterLds S;
  S.stage = reinterpret_cast<uint64_t *>(smem);
  S.info = reinterpret_cast<uint2 *>(S.stage + stage_keys(L, R, P));
  S.hist = reinterpret_cast<uint32_t *>(S.info + num_slices);
  S.sbase = S.hist + num_slices;
  S.pdelta = S.sbase + num_slices;
  S.wsum = kWithPos ? S.pdelta + num_slices : S.pdelta;
  if constexpr (kWithPos && kBucket) {  // info [P], sp [P] (8-byte aligned), hist [P], wsum
    S.sp = S.info + num_slices;
    S.hist = reinterpret_cast<uint32_t *>(S.sp + num_slices);
    S.wsum = S.hist + num_slices;
  }
  S.spilled = S.wsum + 16;
  if (threadIdx.x == 0) *S.spilled = 0u;  // (ordered before its first use by the barrier below)

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
  const uint32_t *my_hist = kWithPos && !kBucket ? hist_rows + (uint64_t)u0 * num_slices : nullptr;
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
    C.limit[r] = C.cursor[r];
    c[r] = kWithPos && !kBucket && sl < num_slices ? my_hist[sl] : 0u;
    if (sl < num_slices) S.hist[sl] = 0u;
  }
  if constexpr (kWithPos && kBucket) {
    look_bucket_chunk<R>(C, num_slices, Bk, ~0u);
  } else if constexpr (kWithPos) {
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
  constexpr uint32_t kT = P * kScatterThreads;
  const uint32_t nfull = (e - b) / kT;
  uint64_t ha[P], hb[P];
  load_tile<kWithPos, P>(hashes, b, e, ha);
  uint32_t t0 = b, k = 0;
#define SBBF_SCATTER_TILE(FULL, H)                                                                            \
  scatter_tile<kWithPos, R, L, kBucket, FULL, P>(                                                              \
      H, t0, e,                                                                                               \
      kWithPos && !kBucket && t0 != b && t0 % chunk == 0u ? hist_rows + (uint64_t)(t0 / chunk) * num_slices  \
                                                          : nullptr,                                         \
      kWithPos && kBucket && t0 != b && t0 % chunk == 0u ? t0 / chunk : ~0u, num_blocks, slice_shift,         \
      slice_base, num_slices, keys, S, C, out_keys, out_pos, Bk)
  for (; k + 2u <= nfull; k += 2u) {
    load_tile<kWithPos, P>(hashes, t0 + kT, e, hb);
    SBBF_SCATTER_TILE(true, ha);
    t0 += kT;
    load_tile<kWithPos, P>(hashes, t0 + kT, e, ha);
    SBBF_SCATTER_TILE(true, hb);
    t0 += kT;
  }
  if (k < nfull) {
    load_tile<kWithPos, P>(hashes, t0 + kT, e, hb);
    SBBF_SCATTER_TILE(true, ha);
    t0 += kT;
    if (t0 < e) SBBF_SCATTER_TILE(false, hb);
  } else if (t0 < e) {
    SBBF_SCATTER_TILE(false, ha);
  }
#undef SBBF_SCATTER_TILE
  // The last incomplete group of every slice: its keys are still in the
  // stage (nothing rewrites it after the last tile's staging barrier).
  if constexpr (L > 1u) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (C.carry[r] == 0u) continue;
      const uint32_t cat = kWithPos && kBucket ? S.info[own + r].y : C.carry_at[r];
      for (uint32_t j = 0; j < C.carry[r]; ++j) out_keys[C.cursor[r] - C.carry[r] + j] = S.stage[cat + j];
    }
  }
  // Bucketed lookups: the last chunk's runs, and each bucket's key count.
  if constexpr (kBucket && kWithPos) {
    look_bucket_chunk<R>(C, num_slices, Bk, (e - 1u) / chunk);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t sl = own + r;
      if (sl < num_slices)
        Bk.count[sl * gridDim.x + blockIdx.x] = C.cursor[r] - (bucket_end(blockIdx.x, sl, Bk.cap) - Bk.cap);
    }
  }
  // Bucketed inserts: pad each bucket to a multiple of four keys with copies
  // of its last (carried) key and record its count. A bucket with no carry
  // ends at a multiple of L (or is full), already a multiple of four.
  if constexpr (kBucket && !kWithPos) {
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
// slice's count are masked: inserts OR a zero mask; lookups give them 0
// bits in the slice's result words (a run starts at a multiple of 32 keys,
// so its words are its own). Padding hashes
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
// key in the lane's rotated pair order o (fewer LDS bank conflicts than one
// fixed order). kMaskTail: keys at or past ns OR nothing; without it they
// are copies of the slice's last keys (clamped loads of whole, padded
// groups), whose bits are set already.
template <uint32_t K, bool kMaskTail>
__device__ __forceinline__ void insert_step(const SliceStep &s, uint32_t base, uint32_t ns, uint32_t num_blocks,
                                            uint32_t b0, uint32_t nb, unsigned long long *lds2,
                                            const OrOrder<K> &o) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (uint32_t u = 0; u < kSliceSteps; ++u) {
    const uint32_t at = base + 256u * u + 4u * lane;
#pragma unroll
    for (uint32_t k = 0; k < 4u; ++k) {
      const uint64_t h = s.h[u][k];
      const uint32_t x = (uint32_t)h;
      const uint32_t bl = min(block_of((uint32_t)(h >> 32), num_blocks) - b0, nb - 1u);
      const uint32_t one = !kMaskTail || at + k < ns ? 1u : 0u;
      lds_or_key<K>(lds2, bl, x, one, o);
    }
  }
}

// Test one step's keys against the slice in LDS (K/4 16-byte reads per key)
// and write their results as bits: lane l's four keys give a nibble, lanes
// 8m .. 8m+7 OR theirs into the word of keys base + 32m .. +31 (three DPP
// moves), which lane 8m stores when that word starts inside the slice.
// begin and base are multiples of 32, so words are whole; keys at or past ns
// give 0 bits.
template <uint32_t K>
__device__ __forceinline__ void lookup_step(const SliceStep &s, uint32_t base, uint32_t ns, uint32_t num_blocks,
                                            uint32_t b0, uint32_t nb, const uint4 *lds4, uint32_t begin,
                                            uint32_t *__restrict__ res32) {
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
      r |= (at + k < ns ? t & 1u : 0u) << k;
    }
    uint32_t word = r << (4u * (lane & 7u));
    word = or_over_eights(word);
    const uint32_t first = base + 256u * u + 32u * (lane >> 3);
    if ((lane & 7u) == 0u && first < ns) res32[(begin + first) / 32u] = word;
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
  const OrOrder<K> order = or_order<K>(lane_id());
#define SBBF_INSERT_STEP(S, BASE) insert_step<K, true>(S, BASE, ns, num_blocks, b0, nb, lds2, order)
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
  const OrOrder<K> order = or_order<K>(lane_id());
  SliceStep sa, sb;
  load_step_buckets(part_slice, cap, prefix, map, map_shift, base, last, sa);
  for (uint32_t it = 0; it < steps; it += 2u) {
    load_step_buckets(part_slice, cap, prefix, map, map_shift, base + stride, last, sb);
    __builtin_amdgcn_sched_barrier(0);
    insert_step<K, false>(sa, base, ns, num_blocks, b0, nb, lds2, order);
    base += stride;
    load_step_buckets(part_slice, cap, prefix, map, map_shift, base + stride, last, sa);
    __builtin_amdgcn_sched_barrier(0);
    insert_step<K, false>(sb, base, ns, num_blocks, b0, nb, lds2, order);
    base += stride;
  }
  __syncthreads();
  uint4 *dst4 = reinterpret_cast<uint4 *>(words + (uint64_t)b0 * K);
  for (uint32_t i = threadIdx.x; i < nb * (K / 4u); i += kPartThreads) dst4[i] = lds4[i];
}

// Bucketed lookups: a slice's buckets are walked as one sequence of 32-key
// words, each bucket taking ceil(keys / 32) of them (wprefix[g]: words before
// bucket g; the coarse map over words as for inserts), so that every result
// word belongs to one bucket: the word of bucket g's keys 32o .. 32o+31 is
// word (slice * G + g) * cap / 32 + o of the result bitmap (cap is a multiple
// of 32). One step of a lane: four keys of a word per 256-position step, how
// many of them are the bucket's (the rest are arbitrary bytes of its room,
// read in bounds and masked) and the result word they belong to.
struct BucketLookStep {
  uint64_t h[kSliceSteps][4];
  uint32_t valid[kSliceSteps];
  uint32_t dw[kSliceSteps];
};

__device__ __forceinline__ void load_step_look_buckets(const uint64_t *__restrict__ part, uint32_t cap,
                                                       const uint32_t *wprefix, const uint32_t *fill,
                                                       const uint16_t *map, uint32_t map_shift, uint32_t base,
                                                       uint32_t ns, uint32_t dw0, BucketLookStep &s) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (uint32_t u = 0; u < kSliceSteps; ++u) {
    const uint32_t v0 = base + 256u * u + 4u * lane;
    const uint32_t v = min(v0, ns - 4u);
    const uint32_t w = v >> 5;
    const uint32_t m = w >> map_shift;
    uint32_t lo = map[m], hi = map[m + 1u];
    while (lo < hi) {  // largest g in [lo, hi] with wprefix[g] <= w
      const uint32_t mid = (lo + hi + 1u) >> 1;
      if (wprefix[mid] <= w)
        lo = mid;
      else
        hi = mid - 1u;
    }
    const uint32_t o = w - wprefix[lo];
    const uint32_t slot = 32u * o + (v & 31u);
    const uint32_t f = fill[lo];
    s.valid[u] = v0 < ns && f > slot ? min(4u, f - slot) : 0u;
    s.dw[u] = dw0 + lo * (cap / 32u) + o;
    const u64x2 *p = reinterpret_cast<const u64x2 *>(part + (uint64_t)lo * cap + slot);
    const u64x2 a = p[0];  // through the caches, as the counted slice lookup
    const u64x2 b = p[1];
    s.h[u][0] = a.x;
    s.h[u][1] = a.y;
    s.h[u][2] = b.x;
    s.h[u][3] = b.y;
  }
}

template <uint32_t K>
__device__ __forceinline__ void bucket_lookup_step(const BucketLookStep &s, uint32_t base, uint32_t ns,
                                                   uint32_t num_blocks, uint32_t b0, uint32_t nb, const uint4 *lds4,
                                                   uint32_t *__restrict__ res32) {
  constexpr uint32_t V = K / 4u;
  const uint32_t lane = lane_id();
#pragma unroll
  for (uint32_t u = 0; u < kSliceSteps; ++u) {
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
      r |= (t & 1u) << k;
    }
    r &= (1u << s.valid[u]) - 1u;  // the step's keys of the bucket (0 to 4)
    uint32_t word = r << (4u * (lane & 7u));
    word = or_over_eights(word);
    const uint32_t first = base + 256u * u + 32u * (lane >> 3);
    if ((lane & 7u) == 0u && first < ns) res32[s.dw[u]] = word;
  }
}

// Slice lookup over the buckets of a count-free lookup partition: the slice
// in LDS, the buckets' word counts scanned into a prefix and a coarse map
// after it, then the slice loop over the words of all buckets.
template <uint32_t K>
__global__ void __launch_bounds__(kPartThreads)
part_bucket_lookup_kernel(const uint64_t *__restrict__ part, const uint32_t *__restrict__ counts, uint32_t groups,
                          uint32_t cap, const uint32_t *__restrict__ words, uint32_t num_blocks, uint32_t slice_shift,
                          uint32_t slice_base, uint32_t *__restrict__ res32) {
  extern __shared__ uint4 lds4[];
  const uint32_t slice = blockIdx.x;
  const uint32_t b0 = (slice_base + slice) << slice_shift;
  const uint32_t nb = min(1u << slice_shift, num_blocks - b0);
  // after the largest slice: wprefix [kMaxBucketGroups + 1], fill [kMaxBucketGroups],
  // map [kBucketMap + 1], wsum [16]
  uint32_t *wprefix = reinterpret_cast<uint32_t *>(lds4 + (((size_t)1 << slice_shift) * K) / 4u);
  uint32_t *fill = wprefix + kMaxBucketGroups + 1u;
  uint16_t *map = reinterpret_cast<uint16_t *>(fill + kMaxBucketGroups);
  uint32_t *wsum = fill + kMaxBucketGroups + (kBucketMap + 2u) / 2u;
  const uint32_t cnt = threadIdx.x < groups ? counts[(uint64_t)slice * groups + threadIdx.x] : 0u;
  const u64x2 *src = reinterpret_cast<const u64x2 *>(words + (uint64_t)b0 * K);
  const uint32_t count4 = nb * (K / 4u);
  u64x2 q[8];
#pragma unroll
  for (uint32_t u = 0; u < 8u; ++u) {
    const uint32_t i = u * kPartThreads + threadIdx.x;
    q[u] = i < count4 ? __builtin_nontemporal_load(src + i) : u64x2{0ull, 0ull};
  }
  uint32_t start, nw;
  {
    const uint32_t c[1] = {(cnt + 31u) / 32u};
    start = block_scan_owned<1>(c, wsum, &nw);
  }
  if (nw == 0) return;  // whole workgroup: no keys in this slice
  uint32_t map_shift = 0;
  while (((nw - 1u) >> map_shift) + 1u > kBucketMap) ++map_shift;
  const uint32_t entries = ((nw - 1u) >> map_shift) + 1u;
  if (threadIdx.x < groups) {
    wprefix[threadIdx.x] = start;
    fill[threadIdx.x] = cnt;
    const uint32_t wc = (cnt + 31u) / 32u;
    for (uint32_t m = (start + (1u << map_shift) - 1u) >> map_shift; (m << map_shift) < start + wc; ++m)
      map[m] = (uint16_t)threadIdx.x;
  }
  if (threadIdx.x == 0) map[entries] = (uint16_t)(groups - 1u);
#pragma unroll
  for (uint32_t u = 0; u < 8u; ++u) {
    const uint32_t i = u * kPartThreads + threadIdx.x;
    if (i < count4) lds4[i] = make_uint4((uint32_t)q[u].x, (uint32_t)(q[u].x >> 32), (uint32_t)q[u].y,
                                         (uint32_t)(q[u].y >> 32));
  }
  __syncthreads();

  const uint64_t *part_slice = part + (uint64_t)slice * groups * cap;
  const uint32_t dw0 = (uint32_t)(((uint64_t)slice * groups * cap) / 32u);
  const uint32_t ns = 32u * nw;
  constexpr uint32_t waves = kPartThreads / kWave;
  constexpr uint32_t stride = waves * 256u * kSliceSteps;
  uint32_t base = wave_index() * 256u * kSliceSteps;
  const uint32_t steps = base < ns ? (ns - base + stride - 1u) / stride : 0u;
  BucketLookStep sa, sb;
  load_step_look_buckets(part_slice, cap, wprefix, fill, map, map_shift, base, ns, dw0, sa);
  for (uint32_t it = 0; it < steps; it += 2u) {
    load_step_look_buckets(part_slice, cap, wprefix, fill, map, map_shift, base + stride, ns, dw0, sb);
    __builtin_amdgcn_sched_barrier(0);
    bucket_lookup_step<K>(sa, base, ns, num_blocks, b0, nb, lds4, res32);
    base += stride;
    load_step_look_buckets(part_slice, cap, wprefix, fill, map, map_shift, base + stride, ns, dw0, sa);
    __builtin_amdgcn_sched_barrier(0);
    bucket_lookup_step<K>(sb, base, ns, num_blocks, b0, nb, lds4, res32);
    base += stride;
  }
}

// Bucketed lookups whose run was full: each key looked up directly in the
// filter (a gather), its result stored over what the unpermute wrote (bits:
// one atomic set or clear per key, the unpermute having written whole words).
template <uint32_t K>
__global__ void __launch_bounds__(256)
part_overflow_lookup_kernel(const uint64_t *__restrict__ hashes, uint32_t keys, const uint32_t *__restrict__ ovf_idx,
                            const uint32_t *__restrict__ ovf_n, uint32_t ovf_cap, const uint32_t *__restrict__ words,
                            uint32_t num_blocks, uint8_t *__restrict__ out8, uint32_t *__restrict__ out_bits) {
  const uint32_t n = min(*ovf_n, ovf_cap);
  for (uint32_t j = blockIdx.x * 256u + threadIdx.x; j < n; j += gridDim.x * 256u) {
    const uint32_t i = ovf_idx[j];
    uint64_t h = hashes[i];
    if (keys) h = key_hash(h);
    const uint32_t x = (uint32_t)h;
    const uint32_t *blk = words + (uint64_t)block_of((uint32_t)(h >> 32), num_blocks) * K;
    uint32_t t = 1u;
#pragma unroll
    for (uint32_t w = 0; w < K; ++w) t &= blk[w] >> bit_of(seed_k(w), x);
    t &= 1u;
    if (out8) {
      out8[i] = (uint8_t)t;
    } else if (t) {
      __hip_atomic_fetch_or(out_bits + i / 32u, 1u << (i & 31u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __hip_atomic_fetch_and(out_bits + i / 32u, ~(1u << (i & 31u)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
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
                         uint32_t slice_shift, uint32_t slice_base, uint32_t *__restrict__ res32) {
  extern __shared__ uint4 lds4[];
  const uint32_t slice = blockIdx.x;
  const uint32_t ns = tot[slice];
  if (ns == 0) return;  // whole workgroup
  const uint32_t b0 = (slice_base + slice) << slice_shift;
  const uint32_t nb = min(1u << slice_shift, num_blocks - b0);
  load_slice_to_lds<K>(lds4, words, b0, nb);
  __syncthreads();

  const uint32_t begin = offsets[slice];  // a multiple of 32
  const uint64_t *keys = part + begin;
  const uint32_t last = ((ns + 3u) & ~3u) - 4u;
  constexpr uint32_t waves = kPartThreads / kWave;
  constexpr bool kCachedKeys = true;
#define SBBF_LOOKUP_STEP(S, BASE) lookup_step<K>(S, BASE, ns, num_blocks, b0, nb, lds4, begin, res32)
  SBBF_SLICE_LOOP(SBBF_LOOKUP_STEP);
#undef SBBF_LOOKUP_STEP
}
#undef SBBF_SLICE_LOOP

// Copy `len` bits of the result bitmap res32, from bit `from`, into the LDS
// bitmap dst from bit `to` (LDS ORs: a destination word can hold the ends of
// two runs). res32 has two words of padding after its last bit, so the word
// after a piece's first word can always be read.
__device__ __forceinline__ void copy_bits(const uint32_t *__restrict__ res32, uint32_t from, uint32_t len,
                                          uint32_t *dst, uint32_t to) {
  for (uint32_t i = 0; i < len; i += 32u) {
    const uint32_t nbits = min(32u, len - i);
    const uint32_t src = from + i, sw = src >> 5, ss = src & 31u;
    const uint32_t w0 = res32[sw], w1 = res32[sw + 1u];
    uint32_t v = ss ? (w0 >> ss) | (w1 << (32u - ss)) : w0;
    if (nbits < 32u) v &= (1u << nbits) - 1u;
    const uint32_t d = to + i, dw = d >> 5, ds = d & 31u;
    if (v) {
      __hip_atomic_fetch_or(dst + dw, v << ds, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (ds && ds + nbits > 32u)
        __hip_atomic_fetch_or(dst + dw + 1u, v >> (32u - ds), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
}

// Output phase of the unpermute kernels. A workgroup's chunks c0 .. c0 + nc
// - 1 are the consecutive keys [b, e); chunk c0 + j's results are bitmap j
// of `maps` (map_words words each) in LDS, and key i takes bit pos[i] of its
// chunk's bitmap; written as bytes or packed bits (LSB-first). Positions are
// read kUnpermuteIter steps at a time, the next iteration's loads issued
// before this one's results are written; the first iteration's are issued by
// unpermute_load before the kernel fills its bitmaps.
constexpr uint32_t kUnpermuteIter = 4u;

struct UnpermuteRange {
  uint32_t b, e;
};

__device__ __forceinline__ UnpermuteRange unpermute_range(uint32_t c0, uint32_t nc, uint32_t chunk, uint32_t n) {
  const uint32_t b = c0 * chunk;
  return UnpermuteRange{b, min(b + nc * chunk, n)};
}

// Bytes: thread t takes keys i0 + 4t + u * 4T .. +3 (T threads, u <
// kUnpermuteIter) of an iteration; bits: wave w takes the 256-key spans i0 +
// 256w + u * 256W (W waves), four keys per lane. i0 starts at b.
template <bool kBits>
__device__ __forceinline__ uint32_t unpermute_first(const UnpermuteRange &r) {
  return kBits ? r.b + (threadIdx.x >> 6) * 256u + 4u * (threadIdx.x & 63u) : r.b + 4u * threadIdx.x;
}

__device__ __forceinline__ void unpermute_load(const uint16_t *__restrict__ pos, uint32_t i, uint32_t e,
                                               uint2 (&p2)[kUnpermuteIter]) {
  constexpr uint32_t kStep = 4u * kPartThreads;  // keys per step, either layout
#pragma unroll
  for (uint32_t u = 0; u < kUnpermuteIter; ++u) {
    const uint32_t k = i + u * kStep;
    p2[u] = k + 4u <= e ? *reinterpret_cast<const uint2 *>(pos + k) : make_uint2(0u, 0u);
  }
}

template <bool kBits>
__device__ __forceinline__ void unpermute_write(const uint32_t *maps, uint32_t map_words,
                                                const uint16_t *__restrict__ pos, const UnpermuteRange &r,
                                                uint32_t chunk, uint2 (&cur)[kUnpermuteIter],
                                                uint8_t *__restrict__ out8, uint32_t *__restrict__ out_bits) {
  constexpr uint32_t kStep = 4u * kPartThreads;
  const uint32_t b = r.b, e = r.e;
  // the bitmap of key i's chunk (four keys of a thread, or a wave's span of
  // 256, lie in one chunk: chunks are multiples of 256 keys)
  auto bitmap = [&](uint32_t i) {
    const uint32_t x = i - b;
    uint32_t j = 0;
#pragma unroll
    for (uint32_t u = 1; u < kUnpermuteChunks; ++u) j += x >= u * chunk ? 1u : 0u;
    return maps + j * map_words;
  };
  auto bit = [](const uint32_t *vals, uint32_t p) { return (vals[p >> 5] >> (p & 31u)) & 1u; };
  const uint32_t lane = threadIdx.x & 63u;
  const bool aligned4 = ((uintptr_t)out8 & 3u) == 0;
  // (bits: the loop test is on the wave's span start, wave-uniform)
  for (uint32_t i0 = unpermute_first<kBits>(r); i0 - (kBits ? 4u * lane : 0u) < e; i0 += kUnpermuteIter * kStep) {
    uint2 nxt[kUnpermuteIter];
    unpermute_load(pos, i0 + kUnpermuteIter * kStep, e, nxt);
#pragma unroll
    for (uint32_t u = 0; u < kUnpermuteIter; ++u) {
      const uint32_t i = i0 + u * kStep;
      if constexpr (!kBits) {
        if (i + 4u <= e) {
          const uint32_t *vals = bitmap(i);
          const uint32_t word = bit(vals, cur[u].x & 0xffffu) | (bit(vals, cur[u].x >> 16) << 8) |
                                (bit(vals, cur[u].y & 0xffffu) << 16) | (bit(vals, cur[u].y >> 16) << 24);
          if (aligned4) {
            *reinterpret_cast<uint32_t *>(out8 + i) = word;
          } else {
            for (uint32_t k = 0; k < 4u; ++k) out8[i + k] = (uint8_t)(word >> (8u * k));
          }
        } else {
          for (uint32_t k = i; k < e; ++k) out8[k] = (uint8_t)bit(bitmap(k), pos[k]);
        }
      } else {
        // Lanes 8w .. 8w+7 OR their nibbles into the word of keys span +
        // 32w .. +31, which lane 8w stores when it starts before e (the span
        // starts at a multiple of 256, so words are whole; keys at or past e
        // give 0 bits).
        const uint32_t span = i - 4u * lane;
        if (span < e) {  // wave-uniform
          const uint32_t *vals = bitmap(span);
          uint32_t nib = 0;
          if (i + 4u <= e) {
            nib = bit(vals, cur[u].x & 0xffffu) | (bit(vals, cur[u].x >> 16) << 1) |
                  (bit(vals, cur[u].y & 0xffffu) << 2) | (bit(vals, cur[u].y >> 16) << 3);
          } else {
            for (uint32_t k = 0; k < 4u; ++k)
              if (i + k < e) nib |= bit(vals, pos[i + k]) << k;
          }
          uint32_t w = nib << (4u * (lane & 7u));
          w = or_over_eights(w);
          const uint32_t first = span + 32u * (lane >> 3);
          if ((lane & 7u) == 0 && first < e) out_bits[first / 32u] = w;
        }
      }
    }
#pragma unroll
    for (uint32_t u = 0; u < kUnpermuteIter; ++u) cur[u] = nxt[u];
  }
}

// Workgroup w restores input order for chunks c0 .. c0 + per - 1 (c0 =
// w * per, per at most kUnpermuteChunks). The results are a bitmap in partitioned order:
// chunk c's results in slice s are bits [offsets[s] + start[c][s], ...
// + hist[c][s]), so the runs of consecutive chunks in one slice are adjacent
// and the workgroup reads each slice's span of runs once (a few words where
// the byte results of one chunk's run took as many 128-byte lines). Pass j
// (chunk c0 + j): the chunk's slice counts are scanned into each run's place
// among the chunk's results, and the thread owning slice s copies the run's
// bits into chunk j's LDS bitmap there. Then every chunk writes out[i] =
// bit pos[i] of its bitmap for its keys, as bytes or packed bits (LSB-first).
template <bool kBits>
__global__ void __launch_bounds__(kPartThreads, 8)  // 8 waves per SIMD: two workgroups per CU
part_unpermute_kernel(const uint16_t *__restrict__ pos, const uint32_t *__restrict__ res32,
                      const uint32_t *__restrict__ offsets, const uint32_t *__restrict__ start,
                      const uint32_t *__restrict__ hist_rows, uint32_t num_slices, uint32_t n, uint32_t chunk,
                      uint32_t groups, uint32_t per, uint8_t *__restrict__ out8, uint32_t *__restrict__ out_bits) {
  extern __shared__ uint32_t usmem[];
  uint32_t *wsum = usmem;        // [2][16]: the scans of consecutive passes alternate
  uint32_t *maps = usmem + 32;   // [per][chunk / 32] result bits of each chunk
  const uint32_t map_words = chunk / 32u;  // chunk is a multiple of the 7,168-key tile
  const uint32_t c0 = blockIdx.x * per;
  const uint32_t nc = min(per, groups - c0);
  const UnpermuteRange ur = unpermute_range(c0, nc, chunk, n);
  uint2 first[kUnpermuteIter];
  unpermute_load(pos, unpermute_first<kBits>(ur), ur.e, first);
  for (uint32_t i = threadIdx.x; i < nc * map_words; i += kPartThreads) maps[i] = 0u;
  // Thread t owns slices t * R .. t * R + R - 1; cursor: the bit where its
  // slice's run of the current chunk starts.
  constexpr uint32_t R = kMaxSlices / kPartThreads;
  uint32_t cursor[R];
#pragma unroll
  for (uint32_t r = 0; r < R; ++r) {
    const uint32_t sl = threadIdx.x * R + r;
    cursor[r] = sl < num_slices ? offsets[sl] + start[(uint64_t)c0 * num_slices + sl] : 0u;
  }
  // Slice counts of chunk j in c[], of chunk j + 1 loaded during pass j.
  auto load_row = [&](uint32_t j, uint32_t (&c)[R]) {
    const uint32_t *row = hist_rows + (uint64_t)(c0 + j) * num_slices;
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
      const uint32_t sl = threadIdx.x * R + r;
      c[r] = sl < num_slices && j < nc ? row[sl] : 0u;
    }
  };
  uint32_t c[R], next[R];
  load_row(0, c);
  __syncthreads();
  for (uint32_t j = 0; j < nc; ++j) {
    load_row(j + 1u, next);
    // place of the run among chunk j's results
    uint32_t at = block_scan_owned<R, kPartThreads>(c, wsum + 16u * (j & 1u));
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
      if (c[r]) copy_bits(res32, cursor[r], c[r], maps + j * map_words, at);
      at += c[r];
      cursor[r] += c[r];
    }
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) c[r] = next[r];
  }
  __syncthreads();
  unpermute_write<kBits>(maps, map_words, pos, ur, chunk, first, out8, out_bits);
}

// Unpermute of a count-free lookup partition. Scatter workgroup g's chunks
// (per_s of them from g * per_s) are split among upw = ceil(per_s / per_u)
// workgroups of at most per_u consecutive chunks, so the runs of a workgroup's
// chunks in one slice follow each other in one bucket: runs[c][s] = (first
// bit, length) in the result bitmap res32, contiguous for consecutive chunks
// c of one scatter workgroup. Chunk j's LDS bitmap holds num_slices slots of
// room = 2^room_shift bits (at least 32: whole words), slot s the bits of its
// run in slice s and zeros after them. First a thread per slice reads its
// runs (coalesced rows) into the slice's record: the word of the first run's
// first bit and each run's bit offset from it (16-bit); then the slots are
// filled slice by slice, so the lanes of a wave read one or two windows of a
// few words of res32 rather than a line per lane.
template <bool kBits>
__global__ void __launch_bounds__(kPartThreads, 8)  // 8 waves per SIMD: two workgroups per CU
part_unpermute_buckets_kernel(const uint16_t *__restrict__ pos, const uint32_t *__restrict__ res32,
                              const uint2 *__restrict__ runs, uint32_t num_slices, uint32_t room_shift, uint32_t n,
                              uint32_t chunk, uint32_t groups, uint32_t per_s, uint32_t per_u,
                              uint8_t *__restrict__ out8, uint32_t *__restrict__ out_bits) {
  extern __shared__ uint32_t usmem[];
  const uint32_t upw = (per_s + per_u - 1u) / per_u;
  const uint32_t sg = blockIdx.x / upw, part = blockIdx.x - sg * upw;
  const uint32_t c0 = sg * per_s + part * per_u;
  if (c0 >= groups) return;  // whole workgroup (the last scatter workgroup may have fewer chunks)
  const uint32_t nc = min(min(per_u, per_s - part * per_u), groups - c0);
  const uint32_t slot_shift = room_shift - 5u;  // words per slot: 2^slot_shift
  const uint32_t map_words = num_slices << slot_shift;
  uint32_t *maps = usmem;                            // [per_u][map_words]
  uint32_t *first_word = maps + per_u * map_words;   // [num_slices]
  uint16_t *pre = reinterpret_cast<uint16_t *>(first_word + num_slices);  // [num_slices][per_u + 1]
  const uint32_t rec = per_u + 1u;
  const UnpermuteRange ur = unpermute_range(c0, nc, chunk, n);
  uint2 first[kUnpermuteIter];
  unpermute_load(pos, unpermute_first<kBits>(ur), ur.e, first);
  for (uint32_t sl = threadIdx.x; sl < num_slices; sl += kPartThreads) {
    uint32_t len[kUnpermuteChunks];
    uint32_t s0 = 0;
#pragma unroll
    for (uint32_t j = 0; j < kUnpermuteChunks; ++j) {
      len[j] = 0u;
      if (j < nc) {
        const uint2 r = runs[(uint64_t)(c0 + j) * num_slices + sl];
        if (j == 0) s0 = r.x;
        len[j] = r.y;
      }
    }
    uint32_t at = s0 & 31u;
#pragma unroll
    for (uint32_t j = 0; j < kUnpermuteChunks; ++j) {
      if (j < nc) {
        pre[sl * rec + j] = (uint16_t)at;
        at += len[j];
      }
    }
    pre[sl * rec + nc] = (uint16_t)at;
    first_word[sl] = s0 >> 5;
  }
  __syncthreads();
  const uint32_t per_slice = nc << slot_shift;  // words of one slice's slots over the chunks
  const uint32_t total = num_slices * per_slice;
  constexpr uint32_t kIn = 4u;
  for (uint32_t x0 = threadIdx.x; x0 < total; x0 += kIn * kPartThreads) {
    uint32_t v[kIn], dst[kIn];
#pragma unroll
    for (uint32_t u = 0; u < kIn; ++u) {
      const uint32_t x = x0 + u * kPartThreads;
      v[u] = 0u;
      dst[u] = ~0u;
      if (x < total) {
        const uint32_t sl = x / per_slice, r = x - sl * per_slice;
        const uint32_t j = r >> slot_shift, w = r & ((1u << slot_shift) - 1u);
        dst[u] = j * map_words + (sl << slot_shift) + w;
        const uint32_t a = pre[sl * rec + j] + 32u * w, end = pre[sl * rec + j + 1u];
        if (a < end) {
          const uint32_t sw = first_word[sl] + (a >> 5), ss = a & 31u;
          const uint32_t nbits = min(32u, end - a);
          uint32_t wd = res32[sw];
          if (ss) wd = (wd >> ss) | (res32[sw + 1u] << (32u - ss));
          v[u] = nbits < 32u ? wd & ((1u << nbits) - 1u) : wd;
        }
      }
    }
#pragma unroll
    for (uint32_t u = 0; u < kIn; ++u)
      if (dst[u] != ~0u) maps[dst[u]] = v[u];
  }
  __syncthreads();
  unpermute_write<kBits>(maps, map_words, pos, ur, chunk, first, out8, out_bits);
}

// Workspace sections (each 256-byte aligned): hist[G][P], start[G][P],
// blocksum[RB][P], tot[P], offsets[P + 1] (u32), keys (u64) and, for
// lookups, pos[n] (u16) and res (a bitmap of 32-bit words). Keys and results
// are laid out with every slice's run padded to a multiple of four keys for
// inserts (at most n + 3P entries) and of kLookupAlign for lookups (at most
// n + 31P).
struct PartitionLayout {
  uint32_t *hist, *start, *blocksum, *tot, *offsets;
  uint64_t *keys;
  uint16_t *pos;
  uint32_t *res;
  uint64_t bytes;
  uint32_t scatter_groups;  // lookups: scatter workgroups to spread the chunks over
};

uint32_t row_blocks(uint32_t groups) { return (groups + kScanRows - 1u) / kScanRows; }

PartitionLayout layout(void *workspace, uint64_t n, uint32_t num_slices, uint32_t groups, bool lookup) {
  auto up = [](uint64_t v) { return (v + 255u) & ~(uint64_t)255u; };
  char *base = static_cast<char *>(workspace);
  const uint64_t padded = n + (lookup ? kLookupAlign - 1u : 3u) * (uint64_t)num_slices;
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
    L.res = reinterpret_cast<uint32_t *>(base + off);
    // two words of padding: the unpermute kernel reads the word after each
    // piece's first
    off += up(((padded + 31u) / 32u + 2u) * 4u);
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
void chunking(uint64_t n, uint32_t max_groups, bool lookup, uint32_t *chunk, uint32_t *groups,
              uint32_t tile = kTile) {
  const uint64_t tiles = (n + tile - 1) / tile;
  const uint64_t g0 = tiles < max_groups ? (tiles ? tiles : 1) : max_groups;
  uint64_t tiles_per = (tiles + g0 - 1) / g0;
  if (lookup && tiles_per * tile > kLookupChunk) {
    const uint64_t slots = max_groups ? max_groups : 1u;
    uint64_t best = kLookupChunk / tile, best_cost = UINT64_MAX;
    for (uint64_t tp = kLookupChunk / tile; tp >= 5u; --tp) {
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
  *chunk = (uint32_t)(tiles_per * tile);
  *groups = (uint32_t)((n + *chunk - 1) / *chunk);
  if (*groups == 0) *groups = 1;
}

template <bool kWithPos, int R, uint32_t L, bool kBucket = false, uint32_t P = kScatterPer>
hipError_t launch_scatter(const uint64_t *hashes, uint32_t n, uint32_t chunk, uint32_t groups, uint32_t num_blocks,
                          uint32_t slice_shift, uint32_t slice_base, uint32_t num_slices, uint32_t keys,
                          const PartitionLayout &L_, hipStream_t stream, const Buckets &Bk = Buckets{}) {
  const size_t lds = scatter_lds_bytes(num_slices, kWithPos, L, R, P);
  // Several chunks per workgroup (lookups cut the batch finer than inserts):
  // about two workgroups per compute unit.
  const uint32_t per = kWithPos ? (groups + L_.scatter_groups - 1u) / L_.scatter_groups : 1u;
  const uint32_t grid = (groups + per - 1u) / per;
  (void)hipFuncSetAttribute((const void *)part_scatter_kernel<kWithPos, R, L, kBucket, P>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  (void)hipGetLastError();
  hipLaunchKernelGGL((part_scatter_kernel<kWithPos, R, L, kBucket, P>), dim3(grid), dim3(kScatterThreads), lds, stream,
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
  hipLaunchKernelGGL(part_offsets_kernel, dim3(1), blk, 0, stream, L.tot, num_slices, with_pos ? kLookupAlign : 4u,
                     L.offsets);
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

// Results of a partition (in partitioned order, L.res) back to input order:
// per chunks per workgroup, enough to fill `slots` workgroups (at most
// kUnpermuteChunks).
hipError_t unpermute(const PartitionLayout &L, uint32_t num_slices, uint32_t n, uint32_t chunk, uint32_t groups,
                     uint32_t slots, uint8_t *out8, uint32_t *out_bits, hipStream_t stream) {
  if (slots == 0) slots = 1;
  const uint32_t per = std::max(1u, std::min(kUnpermuteChunks, (groups + slots - 1u) / slots));
  const uint32_t grid = (groups + per - 1u) / per;
  const size_t u_lds = 128u + (size_t)per * (chunk / 8u);
  (void)hipFuncSetAttribute((const void *)part_unpermute_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)u_lds);
  (void)hipFuncSetAttribute((const void *)part_unpermute_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)u_lds);
  (void)hipGetLastError();
  if (out_bits)
    hipLaunchKernelGGL(part_unpermute_kernel<true>, dim3(grid), dim3(kPartThreads), u_lds, stream, L.pos, L.res,
                       L.offsets, L.start, L.hist, num_slices, n, chunk, groups, per, nullptr, out_bits);
  else
    hipLaunchKernelGGL(part_unpermute_kernel<false>, dim3(grid), dim3(kPartThreads), u_lds, stream, L.pos, L.res,
                       L.offsets, L.start, L.hist, num_slices, n, chunk, groups, per, out8, nullptr);
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
  chunking(n, max_groups, false, &bp->chunk, &bp->groups, kInsertTile);
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
    e = launch_scatter<false, 1, kScatterGroup, true, kInsertPer>(hashes, n, bp.chunk, bp.groups, num_blocks,
                                                                   slice_shift, 0u, num_slices, keys, L, stream, Bk);
  else
    e = launch_scatter<false, 2, 4, true, kInsertPer>(hashes, n, bp.chunk, bp.groups, num_blocks, slice_shift, 0u,
                                                      num_slices, keys, L, stream, Bk);
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

// Count-free lookup partition (struct Buckets, lookup side): for one-level
// lookups into at most 2 * kScatterThreads slices. Results are placed by
// position in slots of `room` bits per (chunk, slice), room the largest
// power of two from 32 to 4,096 with slices * room <= 2^16 (16-bit
// positions); a chunk is
// the most tiles (at most nine) whose expected run in one slice, plus six
// standard deviations, fits a slot. Each scatter workgroup takes `per`
// consecutive chunks into its buckets, of room for their expected keys plus
// eight standard deviations and 32 keys, rounded up to 32 (whole result
// words). It skips the count and scan kernels (one read of the batch).
struct LookPlan {
  uint32_t chunk, groups;  // lookup chunks
  uint32_t sgroups, per;   // scatter workgroups (buckets per slice), chunks per scatter workgroup
  uint32_t cap, room;
  uint64_t runs_off, count_off, ovfn_off, ovf_off, pos_off, keys_off, res_off, bytes;
};

bool look_plan(uint64_t n, uint32_t num_slices, uint32_t max_groups, LookPlan *lp) {
  if (n == 0 || n > UINT32_MAX || num_slices == 0 || num_slices > 2u * kScatterThreads) return false;
  // room: a power of two (the unpermute splits positions by shifts) of at
  // most 4,096 (the unpermute keeps run offsets over eight chunks in 16 bits)
  uint32_t room = 4096u;
  while (room > 32u && (uint64_t)room * num_slices > 65536u) room >>= 1;
  if ((uint64_t)room * num_slices > 65536u) return false;
  // a slice holds at most 1 / (slices - 1) of the blocks (all but the last are whole)
  const double share = 1.0 / (double)(num_slices > 1u ? num_slices - 1u : 1u);
  uint32_t tiles = 9u;
  for (; tiles > 0u; --tiles) {
    const double mean = tiles * (double)kTile * share;
    if (mean + 6.0 * std::sqrt(mean) + 1.0 <= (double)room) break;
  }
  if (tiles == 0u) return false;
  lp->room = room;
  lp->chunk = tiles * kTile;
  lp->groups = (uint32_t)((n + lp->chunk - 1u) / lp->chunk);
  // Scatter workgroups: half the partition workgroups (the default of two
  // per compute unit gives one per unit, the scatter kernel's residency):
  // fewer, larger buckets than with two per unit, so less room per word walk
  // in the slice kernel (lookup call 1.59 -> 1.56 ms at 2e8 keys on MI355X).
  const uint32_t slots = std::max(1u, std::min(max_groups / 2u, kMaxBucketGroups));
  lp->per = (lp->groups + slots - 1u) / slots;
  lp->sgroups = (lp->groups + lp->per - 1u) / lp->per;
  const double mean = (double)lp->per * lp->chunk * share;
  const uint64_t cap = ((uint64_t)(mean + 8.0 * std::sqrt(mean) + 32.0) + 31u) & ~(uint64_t)31u;
  const uint64_t positions = (uint64_t)lp->sgroups * num_slices * cap;
  if (positions >= (1ull << 32) - 64u) return false;
  lp->cap = (uint32_t)cap;
  auto up = [](uint64_t v) { return (v + 255u) & ~(uint64_t)255u; };
  uint64_t off = 0;
  lp->runs_off = off;
  off += up((uint64_t)lp->groups * num_slices * 8u);
  lp->count_off = off;
  off += up((uint64_t)lp->sgroups * num_slices * 4u);
  lp->ovfn_off = off;
  off += 256u;
  lp->ovf_off = off;
  off += up(n * 4u);
  lp->pos_off = off;
  off += up(n * 2u);
  lp->keys_off = off;
  off += up(positions * 8u);
  lp->res_off = off;
  off += up((positions / 32u + 2u) * 4u);  // two words of padding for the unpermute's word pairs
  lp->bytes = off;
  return true;
}

// LDS of a count-free unpermute workgroup of per_u chunks: the bitmaps and
// the slice records (a word and per_u + 1 16-bit offsets per slice).
size_t look_unpermute_lds(uint32_t per_u, uint32_t num_slices, uint32_t room) {
  return ((size_t)per_u * num_slices * (room / 8u) + (size_t)num_slices * 4u + (size_t)num_slices * (per_u + 1u) * 2u +
          3u) & ~(size_t)3u;
}

// Chunks per count-free unpermute workgroup: at most kUnpermuteChunks of one
// scatter workgroup's, as many as fit kUnpermuteLds bytes of LDS, so that two
// workgroups share a compute unit.
uint32_t look_unpermute_chunks(const LookPlan &lp, uint32_t num_slices) {
  uint32_t per_u = std::min(kUnpermuteChunks, lp.per);
  while (per_u > 1u && look_unpermute_lds(per_u, num_slices, lp.room) > kUnpermuteLds) --per_u;
  return per_u;
}

template <uint32_t K>
hipError_t launch_bucket_lookup(const uint64_t *part, const uint32_t *counts, const LookPlan &lp,
                                uint32_t num_slices, const uint32_t *words, uint32_t num_blocks, uint32_t slice_shift,
                                uint32_t slice_base, uint32_t *res32, hipStream_t stream) {
  const size_t lds_bytes = ((size_t)1 << slice_shift) * 4u * K +
                           (2u * kMaxBucketGroups + 1u + (kBucketMap + 2u) / 2u + 16u) * 4u;
  (void)hipFuncSetAttribute((const void *)part_bucket_lookup_kernel<K>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds_bytes);
  (void)hipGetLastError();
  hipLaunchKernelGGL(part_bucket_lookup_kernel<K>, dim3(num_slices), dim3(kPartThreads), lds_bytes, stream, part,
                     counts, lp.sgroups, lp.cap, words, num_blocks, slice_shift, slice_base, res32);
  return hipGetLastError();
}

template <uint32_t K>
hipError_t launch_overflow_lookup(const uint64_t *hashes, uint32_t keys, const Buckets &Bk, const uint32_t *words,
                                  uint32_t num_blocks, uint8_t *out8, uint32_t *out_bits, hipStream_t stream) {
  hipLaunchKernelGGL(part_overflow_lookup_kernel<K>, dim3(256), dim3(256), 0, stream, hashes, keys, Bk.ovf_idx,
                     Bk.ovf_n, Bk.ovf_cap, words, num_blocks, out8, out_bits);
  return hipGetLastError();
}

template <int R, uint32_t L>
hipError_t launch_look_scatter(const uint64_t *hashes, uint32_t n, const LookPlan &lp, uint32_t num_blocks,
                               uint32_t slice_shift, uint32_t slice_base, uint32_t num_slices, uint32_t keys,
                               uint64_t *part, uint16_t *pos, const Buckets &Bk, hipStream_t stream) {
  const size_t lds = scatter_lds_bytes(num_slices, true, L, R);
  (void)hipFuncSetAttribute((const void *)part_scatter_kernel<true, R, L, true, kScatterPer>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  (void)hipGetLastError();
  hipLaunchKernelGGL((part_scatter_kernel<true, R, L, true, kScatterPer>), dim3(lp.sgroups), dim3(kScatterThreads), lds,
                     stream,
                     hashes, n, lp.chunk, lp.per, num_blocks, slice_shift, slice_base, num_slices, nullptr, nullptr,
                     nullptr, keys, part, pos, Bk);
  return hipGetLastError();
}

// Count-free lookup: scatter into buckets (positions, runs, bucket counts,
// overflow list), slice lookups over the buckets, unpermute by run, then the
// overflowing keys.
hipError_t lookup_buckets(const uint64_t *hashes, uint32_t n, const uint32_t *words, uint32_t num_blocks,
                          uint32_t slice_shift, uint32_t slice_base, uint32_t num_slices, void *workspace,
                          const LookPlan &lp, uint32_t slots, uint8_t *out8, uint32_t *out_bits, uint32_t keys,
                          hipStream_t stream, uint32_t lanes) {
  char *base = static_cast<char *>(workspace);
  Buckets Bk{};
  Bk.cap = lp.cap;
  Bk.count = reinterpret_cast<uint32_t *>(base + lp.count_off);
  Bk.ovf_n = reinterpret_cast<uint32_t *>(base + lp.ovfn_off);
  Bk.ovf_cap = n;
  Bk.room = lp.room;
  Bk.ovf_idx = reinterpret_cast<uint32_t *>(base + lp.ovf_off);
  Bk.runs = reinterpret_cast<uint2 *>(base + lp.runs_off);
  uint16_t *pos = reinterpret_cast<uint16_t *>(base + lp.pos_off);
  uint64_t *part = reinterpret_cast<uint64_t *>(base + lp.keys_off);
  uint32_t *res32 = reinterpret_cast<uint32_t *>(base + lp.res_off);
  hipError_t e = launch_fill(Bk.ovf_n, 1u, 0u, stream);  // a fill kernel, not a memset (graph capture)
  if (e != hipSuccess) return e;
  if (num_slices <= kScatterThreads)
    e = launch_look_scatter<1, kScatterGroup>(hashes, n, lp, num_blocks, slice_shift, slice_base, num_slices, keys,
                                              part, pos, Bk, stream);
  else
    e = launch_look_scatter<2, 4>(hashes, n, lp, num_blocks, slice_shift, slice_base, num_slices, keys, part, pos,
                                  Bk, stream);
  if (e != hipSuccess) return e;
  if (lanes == 4)
    e = launch_bucket_lookup<4>(part, Bk.count, lp, num_slices, words, num_blocks, slice_shift, slice_base, res32,
                                stream);
  else if (lanes == 16)
    e = launch_bucket_lookup<16>(part, Bk.count, lp, num_slices, words, num_blocks, slice_shift, slice_base, res32,
                                 stream);
  else
    e = launch_bucket_lookup<8>(part, Bk.count, lp, num_slices, words, num_blocks, slice_shift, slice_base, res32,
                                stream);
  if (e != hipSuccess) return e;
  const uint32_t per_u = look_unpermute_chunks(lp, num_slices);
  const uint32_t upw = (lp.per + per_u - 1u) / per_u;
  const uint32_t grid = lp.sgroups * upw;
  const size_t u_lds = look_unpermute_lds(per_u, num_slices, lp.room);
  uint32_t room_shift = 5;
  while ((1u << room_shift) < lp.room) ++room_shift;
  (void)slots;
  if (out_bits) {
    (void)hipFuncSetAttribute((const void *)part_unpermute_buckets_kernel<true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)u_lds);
    (void)hipGetLastError();
    hipLaunchKernelGGL(part_unpermute_buckets_kernel<true>, dim3(grid), dim3(kPartThreads), u_lds, stream, pos, res32,
                       Bk.runs, num_slices, room_shift, n, lp.chunk, lp.groups, lp.per, per_u, nullptr, out_bits);
  } else {
    (void)hipFuncSetAttribute((const void *)part_unpermute_buckets_kernel<false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)u_lds);
    (void)hipGetLastError();
    hipLaunchKernelGGL(part_unpermute_buckets_kernel<false>, dim3(grid), dim3(kPartThreads), u_lds, stream, pos,
                       res32, Bk.runs, num_slices, room_shift, n, lp.chunk, lp.groups, lp.per, per_u, out8, nullptr);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (lanes == 4) return launch_overflow_lookup<4>(hashes, keys, Bk, words, num_blocks, out8, out_bits, stream);
  if (lanes == 16) return launch_overflow_lookup<16>(hashes, keys, Bk, words, num_blocks, out8, out_bits, stream);
  return launch_overflow_lookup<8>(hashes, keys, Bk, words, num_blocks, out8, out_bits, stream);
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
  LookPlan lp;
  if (look_plan(n, num_slices, max_groups, &lp))
    return lookup_buckets(hashes, n, words, num_blocks, slice_shift, slice_base, num_slices, workspace, lp,
                          max_groups, out8, out_bits, keys, stream, lanes);
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
  return unpermute(L, num_slices, n, chunk, groups, max_groups, out8, out_bits, stream);
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
    LookPlan lp;
    if (lookup && look_plan(n, num_slices, max_groups, &lp)) return std::max(counted, lp.bytes);
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
  // Each group's results go, one bit per key, to its run of the level-1
  // results (level-1 partitioned order; runs start at multiples of 32 keys,
  // so at whole words), which level 1 then unpermutes.
  for (uint32_t g = 0; g < t.groups && e == hipSuccess; ++g) {
    if (tot[g] == 0) continue;
    const uint32_t base = g << kGroupShift;
    e = lookup_level(t.L1.keys + off[g], tot[g], words, num_blocks, slice_shift, base,
                     std::min(kGroupSlices, num_slices - base), t.level2, max_groups, nullptr,
                     t.L1.res + off[g] / 32u, 0u, stream, lanes);
  }
  if (e != hipSuccess) return e;
  return unpermute(t.L1, t.groups, (uint32_t)n, t.chunk, t.chunks, max_groups, out8, out_bits, stream);
}

}  // namespace sbbf
