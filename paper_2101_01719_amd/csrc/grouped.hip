// Grouped launches: inserts into and lookups in many filters of uneven sizes
// in one launch (a HIP graph of three or four kernels), instead of one launch
// per filter per operation.
//
// Every filter runs the same method as the single-filter path; the group only
// changes how work is spread over the device:
//
//   partition  for every filter larger than the LDS threshold (cut into at
//           most 1,024 slices of 2^slice_shift blocks), one workgroup per chunk
//           of 7,168 of its insert keys sorts the chunk by slice in LDS and
//           appends one run per slice to that slice's run list, taking the
//           room from the filter's region of a key array with one device
//           atomic per run (key order inside a slice does not matter: a
//           filter is the OR of all masks).
//   insert  one persistent kernel over (filter, slice) tiles, largest first,
//           from one atomic queue. The workgroup of a tile loads its slice into
//           LDS, ORs in the masks of its keys and stores the slice back with
//           plain stores. A filter within the LDS threshold is one tile that
//           streams the filter's keys; a partitioned slice reads only its runs;
//           a filter with more slices than that streams all of its keys for
//           every slice and ORs those that fall in it.
//   lookup  one persistent kernel over (filter, key range) tiles with the
//           8-lane gather of the single-filter lookup. Tiles sit in eight
//           queues, one per XCD (workgroups are dispatched to the XCDs round
//           robin, so workgroup w starts on queue w % 8); all tiles of a filter
//           go to one queue so its blocks stay in that XCD's L2. A workgroup
//           whose queue is empty takes tiles from the other queues.
//           Filters of at most lookup_lds_slices LDS slices are looked up by
//           a second persistent kernel first (same queue scheme): the workgroup
//           of a tile holds the tile's keys in registers and passes over the
//           filter one slice at a time, loading the slice into LDS (the next
//           slice's loads in flight during the pass) and testing the keys that
//           fall in it; results go out in input order from registers.
//
// The plan (tiles, queues, filter table) lives in device memory and is built
// on the host from the per-filter key counts.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"
#include "sbbf_device.h"

namespace sbbf {
namespace {

constexpr int kQueues = 8;  // XCDs of the device (lookup queues)
constexpr uint32_t kInsertThreads = 1024;
constexpr uint32_t kPartPer = 7;                             // keys per thread of a partition chunk
constexpr uint32_t kPartChunk = kInsertThreads * kPartPer;   // keys per partition chunk
constexpr uint32_t kMaxLocalSlices = kInsertThreads;         // slices of one partitioned filter
constexpr uint32_t kRunBatch = kInsertThreads;               // runs staged in LDS at a time
constexpr uint32_t kStreamTile = 0xFFFFFFFFu;                // tile that streams its filter's keys
// LDS lookups: workgroups of T = 256, 512 or 1,024 threads hold 16 keys per
// thread and pass over slices of 4T blocks (128 T bytes: eight 16-byte loads
// per thread), so smaller workgroups share a compute unit's LDS.
constexpr uint32_t kLdsLookPer = 16;                         // keys per thread of an LDS lookup tile
constexpr uint32_t kLdsLookLoads = 8;                        // 16-byte slice loads per thread
// LDS of the partition kernel: stage [kPartChunk] u64, delta [kMaxLocalSlices]
// u64, hist and loff [kMaxLocalSlices] u32, wsum [16].
constexpr size_t kPartLds = (size_t)kPartChunk * 8u + (size_t)kMaxLocalSlices * 16u + 64u;
// LDS after an insert tile's slice words: run prefix [kRunBatch + 1] u32,
// run offsets [kRunBatch] u64, wsum [16].
constexpr size_t kRunLds = (size_t)kRunBatch * 12u + 4u + 64u + 4u;

struct GFilter {
  uint32_t *words;
  uint32_t num_blocks;
  uint32_t pad;
};

struct GInsTile {
  uint32_t filter;
  uint32_t b0;     // first block of the tile's slice
  uint32_t nb;     // blocks in the slice
  uint32_t slice;  // global id of a partitioned filter's slice, or kStreamTile
};

// A filter whose insert keys are partitioned by slice before the insert tiles
// run: each slice's keys end up as runs in the partitioned key array.
struct GPart {
  uint64_t base;        // first index of its keys in the partitioned key array
  uint32_t filter;
  uint32_t slice_base;  // global id of its first slice
  uint32_t nslices;
  uint32_t shift;       // slice = block >> shift
};

struct GChunk {
  uint32_t k;     // the chunk's place in its filter: keys k * kPartChunk .. of the call
  uint32_t part;
};

struct GRun {
  uint64_t start;  // first key in the partitioned key array
  uint32_t count;
  uint32_t pad;
};

struct GSlice {
  uint32_t run_off;  // first entry of its run list
  uint32_t run_cap;  // entries (one per chunk of its filter)
};

struct GLookTile {
  uint64_t begin;  // first key, relative to the filter's first lookup key of the call
  uint32_t count;  // keys in the tile at the filter's planned capacity (fewer when the call has fewer)
  uint32_t filter;
};

// Device-side plan: pointers into one allocation (part_keys is a second one).
struct GPlanDev {
  const GFilter *filters;
  const uint64_t *ins_off;   // [F + 1] the call's insert key ranges (device memory)
  const uint64_t *look_off;  // [F + 1] the call's lookup key ranges (device memory)
  const uint64_t *ins_cap;   // [F] planned insert keys per filter (the most one call may bring)
  const uint64_t *look_cap;  // [F] planned lookup keys per filter
  uint32_t *bad;             // lowest filter whose call range broke its capacity, else 0xFFFFFFFF
  const GInsTile *ins_tiles; // [n_ins_tiles]
  const GLookTile *look_tiles;
  const uint32_t *queue_begin;  // [kQueues + 1] tile ranges per queue
  const GLookTile *lds_tiles;   // LDS lookup tiles, at most 16 keys per thread each
  const uint32_t *lds_queue_begin;  // [kQueues + 1]
  uint32_t *counters;           // [1 + 2 * kQueues]: insert queue, lookup queues, LDS lookup queues
  const GPart *parts;           // [n_parts]
  const GChunk *chunks;         // [n_chunks]
  const GSlice *slices;         // [n_slices]
  GRun *runs;                   // run lists, GSlice::run_off / run_cap
  uint32_t *nruns;              // [n_slices] runs written so far
  unsigned long long *tops;     // [n_parts] next free index of each part's region
  uint64_t *part_keys;          // partitioned insert keys
  uint32_t n_ins_tiles;
  uint32_t n_parts;
  uint32_t n_slices;
  uint32_t pad;
};

// Keys of filter f in this call, from the call's offsets: off[f + 1] - off[f],
// at most the planned capacity cap[f]. A decreasing range or a count above
// the capacity is recorded (the lowest such filter, in *bad) and clamped, so
// no kernel touches more keys of a filter than were planned for it.
__device__ __forceinline__ uint64_t call_range(const uint64_t *off, const uint64_t *cap, uint32_t f, uint32_t *bad,
                                               uint64_t *begin) {
  const uint64_t b = off[f], e = off[f + 1], c = cap[f];
  uint64_t n = e > b ? e - b : 0u;
  if (e < b || n > c) {
    __hip_atomic_fetch_min(bad, f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    n = n < c ? n : c;
  }
  *begin = b;
  return n;
}

// ---- insert -----------------------------------------------------------------

// OR the mask of one key into the slice [b0, b0 + nb) of a filter of B blocks
// held in LDS (four 64-bit words per block; pairs in the lane's rotated
// order o). A key outside the slice, or an invalid lane, ORs a zero mask into
// block 0.
__device__ __forceinline__ void or_key(unsigned long long *lds2, uint64_t h, bool valid, uint32_t B, uint32_t b0,
                                       uint32_t nb, const OrOrder<8> &o) {
  const uint32_t rel = block_of((uint32_t)(h >> 32), B) - b0;
  const bool in = valid && rel < nb;
  lds_or_key<8>(lds2, in ? rel : 0u, (uint32_t)h, in ? 1u : 0u, o);
}

// Partition of one chunk of a partitioned filter's insert keys by slice: rank
// every key within its slice (LDS atomics), scan the counts, take room for
// each slice's run from the filter's region (one device atomic per slice of
// the chunk), record the run in the slice's run list, stage the keys sorted
// by slice in LDS and write the runs with consecutive lanes. Key order inside
// a slice is irrelevant (a filter is the OR of all masks).
__global__ void __launch_bounds__(kInsertThreads)
grouped_part_kernel(GPlanDev plan, const uint64_t *__restrict__ hashes) {
  extern __shared__ unsigned long long psm[];
  uint64_t *stage = reinterpret_cast<uint64_t *>(psm);  // [kPartChunk]
  unsigned long long *delta = psm + kPartChunk;         // [kMaxLocalSlices]
  uint32_t *hist = reinterpret_cast<uint32_t *>(delta + kMaxLocalSlices);
  uint32_t *loff = hist + kMaxLocalSlices;
  uint32_t *wsum = loff + kMaxLocalSlices;
  const GChunk ch = plan.chunks[blockIdx.x];
  const GPart pt = plan.parts[ch.part];
  const uint32_t B = plan.filters[pt.filter].num_blocks;
  uint64_t kb;
  const uint64_t nf = call_range(plan.ins_off, plan.ins_cap, pt.filter, plan.bad, &kb);
  const uint64_t first = (uint64_t)ch.k * kPartChunk;
  if (first >= nf) return;  // this call brings the filter fewer keys (the whole workgroup leaves)
  const uint32_t ns = pt.nslices, n = (uint32_t)min((uint64_t)kPartChunk, nf - first);
  const uint64_t *src = hashes + kb + first;
  if (threadIdx.x < ns) hist[threadIdx.x] = 0u;
  uint64_t h[kPartPer];
#pragma unroll
  for (uint32_t t = 0; t < kPartPer; ++t) {
    const uint32_t i = t * kInsertThreads + threadIdx.x;
    h[t] = load_hash<0>(src + (i < n ? i : n - 1u));
  }
  __syncthreads();
  uint32_t s[kPartPer], rank[kPartPer];
#pragma unroll
  for (uint32_t t = 0; t < kPartPer; ++t) {
    const uint32_t i = t * kInsertThreads + threadIdx.x;
    s[t] = block_of((uint32_t)(h[t] >> 32), B) >> pt.shift;
    rank[t] = __hip_atomic_fetch_add(hist + s[t], i < n ? 1u : 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __syncthreads();
  const uint32_t c[1] = {threadIdx.x < ns ? hist[threadIdx.x] : 0u};
  const uint32_t run = block_scan_owned<1, kInsertThreads>(c, wsum);
  if (threadIdx.x < ns) {
    loff[threadIdx.x] = run;
    if (c[0] > 0u) {
      const unsigned long long at = __hip_atomic_fetch_add(plan.tops + ch.part, (unsigned long long)c[0],
                                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint32_t slice = pt.slice_base + threadIdx.x;
      const uint32_t k = __hip_atomic_fetch_add(plan.nruns + slice, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      plan.runs[plan.slices[slice].run_off + k] = GRun{at, c[0], 0u};
      delta[threadIdx.x] = at - run;
    }
  }
  __syncthreads();
#pragma unroll
  for (uint32_t t = 0; t < kPartPer; ++t) {
    const uint32_t i = t * kInsertThreads + threadIdx.x;
    if (i < n) stage[loff[s[t]] + rank[t]] = h[t];
  }
  __syncthreads();
#pragma unroll
  for (uint32_t t = 0; t < kPartPer; ++t) {
    const uint32_t k = t * kInsertThreads + threadIdx.x;
    if (k < n) {
      const uint64_t key = stage[k];
      plan.part_keys[k + delta[block_of((uint32_t)(key >> 32), B) >> pt.shift]] = key;
    }
  }
}

// Insert tiles, taken from one queue: the workgroup loads its slice into LDS,
// ORs in the masks of its keys and stores the slice back with plain stores.
// A stream tile reads all insert keys of its filter and ORs those that fall
// in the slice (a whole small filter, or a slice of a filter with more slices
// than one partition chunk can sort); a partitioned tile reads exactly its
// slice's runs, handled as one sequence of keys.
__global__ void __launch_bounds__(kInsertThreads)
grouped_insert_kernel(GPlanDev plan, const uint64_t *__restrict__ hashes, uint32_t words_lds_bytes) {
  extern __shared__ uint4 lds4[];
  unsigned long long *lds2 = reinterpret_cast<unsigned long long *>(lds4);
  uint32_t *pre = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(lds4) + words_lds_bytes);  // [kRunBatch + 1]
  unsigned long long *off = reinterpret_cast<unsigned long long *>(pre + kRunBatch + 2u);           // [kRunBatch]
  uint32_t *wsum = reinterpret_cast<uint32_t *>(off + kRunBatch);                                   // [16]
  __shared__ uint32_t tile_id;
  const uint32_t lane = lane_id();
  const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const OrOrder<8> order = or_order<8>(lane);
  constexpr uint32_t waves = kInsertThreads / kWave;
  constexpr uint32_t U = 4;
  constexpr uint32_t kStep = 64u * U;

  for (;;) {
    if (threadIdx.x == 0)
      tile_id = __hip_atomic_fetch_add(plan.counters, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const uint32_t t = tile_id;
    __syncthreads();  // every thread has read tile_id before it is overwritten
    if (t >= plan.n_ins_tiles) break;
    const GInsTile tile = plan.ins_tiles[t];
    const GFilter flt = plan.filters[tile.filter];
    // Keys of the tile in this call: a stream tile's filter range, or a
    // partitioned slice's runs. A tile with none leaves its slice untouched.
    uint64_t kb = 0;
    uint32_t n = 0, nr = 0;
    if (tile.slice == kStreamTile)
      n = (uint32_t)call_range(plan.ins_off, plan.ins_cap, tile.filter, plan.bad, &kb);
    else
      nr = plan.nruns[tile.slice];
    if (n == 0 && nr == 0) continue;
    const uint4 *src4 = reinterpret_cast<const uint4 *>(flt.words + (uint64_t)tile.b0 * 8u);
    for (uint32_t i = threadIdx.x; i < tile.nb * 2u; i += kInsertThreads) lds4[i] = src4[i];
    __syncthreads();
    if (tile.slice == kStreamTile) {
      const uint64_t *keys = hashes + kb;
      for (uint32_t base = wave * kStep; base < n; base += waves * kStep) {
        uint64_t hv[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
          const uint32_t i = base + 64u * u + lane;
          hv[u] = load_hash<0>(keys + (i < n ? i : n - 1u));
        }
#pragma unroll
        for (uint32_t u = 0; u < U; ++u)
          or_key(lds2, hv[u], base + 64u * u + lane < n, flt.num_blocks, tile.b0, tile.nb, order);
      }
    } else {
      const GRun *runs = plan.runs + plan.slices[tile.slice].run_off;
      for (uint32_t r0 = 0; r0 < nr; r0 += kRunBatch) {
        // Runs r0 .. r0 + m - 1 as one sequence: pre[k] is where run k starts
        // in it and key j of the sequence is part_keys[off[k] + j].
        const uint32_t m = min(kRunBatch, nr - r0);
        const uint32_t k = threadIdx.x;
        const GRun rn = k < m ? runs[r0 + k] : GRun{0ull, 0u, 0u};
        const uint32_t cnt[1] = {rn.count};
        uint32_t total;
        const uint32_t at = block_scan_owned<1, kInsertThreads>(cnt, wsum, &total);
        if (k < m) {
          pre[k] = at;
          off[k] = rn.start - at;
        }
        if (k == 0) pre[m] = total;
        __syncthreads();
        uint32_t rw = 0;  // run of the wave's first key (wave-uniform)
        for (uint32_t base = wave * kStep; base < total; base += waves * kStep) {
          while (pre[rw + 1u] <= base) ++rw;
          uint64_t hv[U];
#pragma unroll
          for (uint32_t u = 0; u < U; ++u) {
            const uint32_t j = min(base + 64u * u + lane, total - 1u);
            uint32_t r = rw;
            while (pre[r + 1u] <= j) ++r;
            hv[u] = load_hash<0>(plan.part_keys + off[r] + j);
          }
#pragma unroll
          for (uint32_t u = 0; u < U; ++u)
            or_key(lds2, hv[u], base + 64u * u + lane < total, flt.num_blocks, tile.b0, tile.nb, order);
        }
        __syncthreads();  // pre and off are rewritten by the next batch
      }
    }
    __syncthreads();
    uint4 *dst4 = reinterpret_cast<uint4 *>(flt.words + (uint64_t)tile.b0 * 8u);
    for (uint32_t i = threadIdx.x; i < tile.nb * 2u; i += kInsertThreads) dst4[i] = lds4[i];
    __syncthreads();  // LDS is reused by the next tile
  }
}

// ---- lookup -----------------------------------------------------------------

template <int U>
__global__ void __launch_bounds__(256)
grouped_lookup_kernel(GPlanDev plan, const uint64_t *__restrict__ hashes, uint8_t *__restrict__ out) {
  __shared__ uint32_t tile_id;
  const uint32_t lane = lane_id();
  const uint32_t j = lane & 7u;
  const uint32_t group = lane & ~7u;
  const uint32_t seed = seed_of_word(j);
  const uint32_t waves = blockDim.x / kWave;
  const uint32_t wave = threadIdx.x / kWave;
  constexpr uint32_t kChunk = 64u * U;
  const uint32_t home = blockIdx.x % kQueues;

  for (uint32_t qi = 0; qi < kQueues; ++qi) {
    const uint32_t queue = (home + qi) % kQueues;
    const uint32_t qb = plan.queue_begin[queue];
    const uint32_t qn = plan.queue_begin[queue + 1] - qb;
    for (;;) {
      if (threadIdx.x == 0)
        tile_id = __hip_atomic_fetch_add(plan.counters + 1 + queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
      const uint32_t t = tile_id;
      __syncthreads();
      if (t >= qn) break;
      const GLookTile tile = plan.look_tiles[qb + t];
      uint64_t lb;
      const uint64_t nf = call_range(plan.look_off, plan.look_cap, tile.filter, plan.bad, &lb);
      if (tile.begin >= nf) continue;  // past the filter's keys in this call
      const GFilter flt = plan.filters[tile.filter];
      const uint64_t *keys = hashes + lb + tile.begin;
      uint8_t *res = out + lb + tile.begin;
      const uint32_t n = (uint32_t)min((uint64_t)tile.count, nf - tile.begin);
      for (uint32_t base = wave * kChunk; base < n; base += waves * kChunk) {
        uint32_t blk[U], lo[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t i = base + 64u * u + lane;
          const uint64_t h = load_hash<0>(keys + (i < n ? i : n - 1u));
          lo[u] = (uint32_t)h;
          blk[u] = block_of((uint32_t)(h >> 32), flt.num_blocks);
        }
        uint32_t word[U][8], bit[U][8];
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
          for (int p = 0; p < 8; ++p) {
            const uint32_t b = lane_read(blk[u], group + p);
            bit[u][p] = bit_of(seed, lane_read(lo[u], group + p));
            word[u][p] = flt.words[(uint64_t)b * 8u + j];
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          uint64_t r = 0;
#pragma unroll
          for (int p = 0; p < 8; ++p) r |= fold_pass(ballot((word[u][p] >> bit[u][p]) & 1u), p);
          const uint32_t i = base + 64u * u + lane;
          if (i < n) res[i] = (uint8_t)((r >> lane) & 1u);
        }
      }
    }
  }
}

// LDS lookup tiles (filters of few slices). A tile's keys stay in registers,
// kLdsLookPer per thread (key p of thread t is key p * T + t); the workgroup
// of T threads passes over the filter's slices of 2^slice_shift <= 4T blocks: the
// slice is stored into LDS from registers, the next slice's loads are issued,
// and every key whose block lies in the slice reads its block (two 16-byte
// LDS reads) and tests its eight bits. After the last slice each thread writes
// its keys' result bytes. Lanes past the tile repeat its last key and write
// nothing.
template <uint32_t T>
__global__ void __launch_bounds__(T, 4)  // 4 waves per SIMD: 1,024 threads per compute unit
grouped_lds_lookup_kernel(GPlanDev plan, const uint64_t *__restrict__ hashes, uint8_t *__restrict__ out,
                          uint32_t slice_shift) {
  extern __shared__ uint4 lds4[];
  __shared__ uint32_t tile_id;
  constexpr uint32_t kLoads = kLdsLookLoads;  // 16-byte loads per thread per slice (slices of at most 4T blocks)
  const uint32_t home = blockIdx.x % kQueues;
  const uint32_t S = 1u << slice_shift;
  for (uint32_t qi = 0; qi < kQueues; ++qi) {
    const uint32_t queue = (home + qi) % kQueues;
    const uint32_t qb = plan.lds_queue_begin[queue];
    const uint32_t qn = plan.lds_queue_begin[queue + 1] - qb;
    for (;;) {
      if (threadIdx.x == 0)
        tile_id = __hip_atomic_fetch_add(plan.counters + 1 + kQueues + queue, 1u, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
      const uint32_t t = tile_id;
      __syncthreads();
      if (t >= qn) break;
      const GLookTile tile = plan.lds_tiles[qb + t];
      uint64_t lb;
      const uint64_t nf = call_range(plan.look_off, plan.look_cap, tile.filter, plan.bad, &lb);
      if (tile.begin >= nf) continue;  // past the filter's keys in this call
      const GFilter flt = plan.filters[tile.filter];
      const uint32_t B = flt.num_blocks, n = (uint32_t)min((uint64_t)tile.count, nf - tile.begin);
      const uint64_t *keys = hashes + lb + tile.begin;
      const uint4 *src4 = reinterpret_cast<const uint4 *>(flt.words);
      // Per key: its block, and its eight bit indices packed five bits each
      // (words 0..5 in ia, 6 and 7 in ib), computed once for all passes.
      uint32_t blk[kLdsLookPer], ia[kLdsLookPer], ib[kLdsLookPer];
#pragma unroll
      for (uint32_t p = 0; p < kLdsLookPer; ++p) {
        const uint32_t i = p * T + threadIdx.x;
        const uint64_t h = load_hash<0>(keys + (i < n ? i : n - 1u));
        const uint32_t x = (uint32_t)h;
        blk[p] = block_of((uint32_t)(h >> 32), B);
        ia[p] = bit_of(kSeed0, x) | (bit_of(kSeed1, x) << 5) | (bit_of(kSeed2, x) << 10) |
                (bit_of(kSeed3, x) << 15) | (bit_of(kSeed4, x) << 20) | (bit_of(kSeed5, x) << 25);
        ib[p] = bit_of(kSeed6, x) | (bit_of(kSeed7, x) << 5);
      }
      uint4 q[kLoads];
      uint32_t count4 = min(S, B) * 2u;  // 16-byte pieces of the slice in flight
#pragma unroll
      for (uint32_t u = 0; u < kLoads; ++u) {
        const uint32_t i = u * T + threadIdx.x;
        q[u] = i < count4 ? src4[i] : make_uint4(0u, 0u, 0u, 0u);
      }
      uint32_t res = 0;
      for (uint32_t b0 = 0;; b0 += S) {  // ends after the slice that holds block B - 1
        const uint32_t nb = min(S, B - b0);
        __syncthreads();  // the previous pass (or tile) has finished reading LDS
#pragma unroll
        for (uint32_t u = 0; u < kLoads; ++u) {
          const uint32_t i = u * T + threadIdx.x;
          if (i < count4) lds4[i] = q[u];
        }
        __syncthreads();
        if (B - b0 > S) {  // the next slice's loads, in flight during this pass
          count4 = min(S, B - b0 - S) * 2u;
          const uint4 *nxt = src4 + (uint64_t)(b0 + S) * 2u;
#pragma unroll
          for (uint32_t u = 0; u < kLoads; ++u) {
            const uint32_t i = u * T + threadIdx.x;
            q[u] = i < count4 ? nxt[i] : make_uint4(0u, 0u, 0u, 0u);
          }
        }
        // Four keys at a time: their eight LDS reads in flight together (the
        // scheduling barrier keeps later keys' reads from being hoisted, which
        // would need more registers than a thread has).
#pragma unroll
        for (uint32_t p0 = 0; p0 < kLdsLookPer; p0 += 4u) {
#pragma unroll
          for (uint32_t p = p0; p < p0 + 4u; ++p) {
            const uint32_t rel = blk[p] - b0;
            if (rel < nb) {
              const uint4 w0 = lds4[2u * rel], w1 = lds4[2u * rel + 1u];
              uint32_t a = ia[p], b = ib[p];
              // Opaque to the optimizer: the shift amounts below are then
              // extracted in each pass instead of hoisted out of the slice
              // loop (16 keys x 8 amounts would not fit in registers).
              asm volatile("" : "+v"(a), "+v"(b));
              const uint32_t ok = (w0.x >> (a & 31u)) & (w0.y >> ((a >> 5) & 31u)) & (w0.z >> ((a >> 10) & 31u)) &
                                  (w0.w >> ((a >> 15) & 31u)) & (w1.x >> ((a >> 20) & 31u)) &
                                  (w1.y >> ((a >> 25) & 31u)) & (w1.z >> (b & 31u)) & (w1.w >> ((b >> 5) & 31u)) & 1u;
              res |= ok << p;
            }
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        if (B - b0 <= S) break;
      }
      uint8_t *dst = out + lb + tile.begin;
#pragma unroll
      for (uint32_t p = 0; p < kLdsLookPer; ++p) {
        const uint32_t i = p * T + threadIdx.x;
        if (i < n) dst[i] = (uint8_t)((res >> p) & 1u);
      }
    }
  }
}

// Resets the queue counters, and for the insert phase each part's region
// cursor and each slice's run count (a kernel rather than memsets so the
// graph holds kernel nodes only). what: 1 insert phase, 2 lookup phase.
__global__ void grouped_reset_kernel(GPlanDev plan, uint32_t what) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (what & 1u) {
    if (i == 0) plan.counters[0] = 0u;
    if (i < plan.n_parts) plan.tops[i] = plan.parts[i].base;
    if (i < plan.n_slices) plan.nruns[i] = 0u;
  }
  if ((what & 2u) && i < 2u * (uint32_t)kQueues) plan.counters[1 + i] = 0u;
}

// Order-sensitive 64-bit digest of device words, for comparing autotune
// candidates: sum over i of mix(i, w[i]) with 64-bit wrap-around.
__global__ void digest_kernel(const uint32_t *__restrict__ words, uint64_t n, unsigned long long *acc) {
  unsigned long long s = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    unsigned long long z = ((unsigned long long)i << 32) ^ words[i];
    z = (z ^ (z >> 31)) * 0x7fb5d329728ea185ull;
    z = (z ^ (z >> 27)) * 0x81dadef4bc2dd44dull;
    s += z ^ (z >> 33);
  }
  __hip_atomic_fetch_add(acc, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void fill_kernel_u32(uint32_t *p, uint32_t n) {
  if (threadIdx.x < n) p[threadIdx.x] = 0u;
}

__global__ void digest_chain_kernel(unsigned long long *acc, unsigned long long f) {
  unsigned long long z = acc[0] + f * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  acc[0] = z ^ (z >> 31);
}

__global__ void digest_tail_kernel(const uint8_t *p, uint32_t n, unsigned long long *acc) {
  if (threadIdx.x == 0) {
    unsigned long long v = 0;
    for (uint32_t i = 0; i < n; ++i) v = (v << 8) | p[i];
    acc[0] += (v + 1) * 0xff51afd7ed558ccdull;
  }
}

}  // namespace

// ---- host side ------------------------------------------------------------------

struct GroupedPlanHost {
  std::vector<uint64_t> ins_cap, look_cap;  // planned keys per filter
  std::vector<uint64_t> ins_off, look_off;  // host offsets of a fixed-shape plan (empty for a capacity plan)
  bool capacity = false;                     // key ranges come from device offsets at every run
  uint64_t ins_total = 0, look_total = 0;    // sums of the capacities
  sbbf_grouped_config cfg;
  bool planned = false;
  uint32_t n_ins_tiles = 0, n_look_tiles = 0, n_chunks = 0, n_lds_tiles = 0;
  size_t insert_lds = 0;   // LDS of the largest insert slice
  size_t lds_look_bytes = 0;   // LDS of the LDS lookup kernel (its largest slice)
  uint32_t lds_look_shift = 0; // log2 blocks per LDS lookup slice
  void *dev = nullptr;     // device allocation holding the plan tables
  void *keys = nullptr;    // device allocation of the partitioned insert keys
  GPlanDev pd{};
  // graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t n_reset = nullptr, n_part = nullptr, n_ins = nullptr, n_look_lds = nullptr, n_look = nullptr;
  const void *g_ins = nullptr, *g_look = nullptr;
  void *g_out = nullptr;
  const void *g_ins_off = nullptr, *g_look_off = nullptr;
};

}  // namespace sbbf

struct sbbf_group {
  std::vector<sbbf_filter *> filters;
  int device = 0;
  sbbf::GroupedPlanHost plan;
  uint64_t plans = 0, graph_builds = 0, graph_updates = 0;  // host work done for this group
};

namespace sbbf {

void free_plan(GroupedPlanHost &p) {
  // Queued runs may still read the plan tables or use the graph.
  if (p.exec || p.dev) (void)hipDeviceSynchronize();
  if (p.exec) (void)hipGraphExecDestroy(p.exec);
  if (p.graph) (void)hipGraphDestroy(p.graph);
  if (p.dev) (void)hipFree(p.dev);
  if (p.keys) (void)hipFree(p.keys);
  p.exec = nullptr;
  p.graph = nullptr;
  p.dev = nullptr;
  p.keys = nullptr;
  p.n_part = nullptr;
  p.n_look_lds = nullptr;
  p.planned = false;
  p.g_ins = p.g_look = nullptr;
  p.g_out = nullptr;
  p.g_ins_off = p.g_look_off = nullptr;
}

sbbf_grouped_config default_config(const sbbf_device_info &info) {
  sbbf_grouped_config c;
  memset(&c, 0, sizeof(c));
  // Gather lookups: the shape the autotuner picks for the 2,048-filter
  // workload on MI355X (4,096-key tiles, four 64-key chunks in flight per
  // wave, four 256-thread workgroups per CU).
  c.lookup_tile_keys = 4096;
  c.lookup_threads = 256;
  c.lookup_unroll = 4;
  c.lookup_blocks_per_cu = 4;
  c.insert_slice_shift = 12;
  while (c.insert_slice_shift > 6 && ((uint64_t)32u << c.insert_slice_shift) > info.lds_per_block) --c.insert_slice_shift;
  c.insert_lds_bytes = (uint64_t)32u << c.insert_slice_shift;
  c.xcd_queues = 1;
  // Measured on MI355X (2,048 filters of 1e3..1e6 keys, 4 lookups per
  // insert): filters of up to four 128 KiB slices from LDS, the rest by the
  // gather, 7.3 ms for the lookup phase against 7.9 with the gather alone.
  c.lookup_lds_slices = 4;
  c.lookup_lds_threads = 1024;
  return c;
}

// Blocks per LDS lookup slice: four per thread of the workgroup (eight
// 16-byte loads per thread), or the largest power of two whose words fit one
// workgroup's LDS.
static uint32_t lds_look_shift(uint32_t threads, const sbbf_device_info &info) {
  uint32_t sh = 0;
  while ((1u << (sh + 1u)) <= threads * (kLdsLookLoads / 2u)) ++sh;
  while (sh > 0 && ((uint64_t)32u << sh) > info.lds_per_block) --sh;
  return sh;
}

sbbf_status check_config(const sbbf_grouped_config &c, const sbbf_device_info &info) {
  if (c.lookup_tile_keys < 64 || c.lookup_tile_keys % 64) return set_error(SBBF_EINVAL, "lookup_tile_keys must be a multiple of 64");
  if (c.lookup_threads < 64 || c.lookup_threads > 256 || c.lookup_threads % 64)
    return set_error(SBBF_EINVAL, "lookup_threads must be 64, 128, 192 or 256");
  if (c.lookup_unroll != 1 && c.lookup_unroll != 2 && c.lookup_unroll != 4)
    return set_error(SBBF_EINVAL, "lookup_unroll must be 1, 2 or 4");
  if (c.lookup_blocks_per_cu < 1 || c.lookup_blocks_per_cu > 64) return set_error(SBBF_EINVAL, "lookup_blocks_per_cu out of range");
  if (c.insert_slice_shift < 6 || ((uint64_t)32u << c.insert_slice_shift) > info.lds_per_block)
    return set_error(SBBF_EINVAL, "insert slice must fit one workgroup's LDS");
  if (c.insert_lds_bytes > info.lds_per_block) return set_error(SBBF_EINVAL, "insert_lds_bytes exceeds the LDS per workgroup");
  if (c.lookup_lds_threads != 256 && c.lookup_lds_threads != 512 && c.lookup_lds_threads != 1024)
    return set_error(SBBF_EINVAL, "lookup_lds_threads must be 256, 512 or 1024");
  return SBBF_OK;
}

hipError_t launch_lookup_any(int unroll, dim3 g, dim3 b, hipStream_t s, const GPlanDev &pd, const uint64_t *h, uint8_t *out) {
  switch (unroll) {
    case 1: hipLaunchKernelGGL(grouped_lookup_kernel<1>, g, b, 0, s, pd, h, out); break;
    case 2: hipLaunchKernelGGL(grouped_lookup_kernel<2>, g, b, 0, s, pd, h, out); break;
    default: hipLaunchKernelGGL(grouped_lookup_kernel<4>, g, b, 0, s, pd, h, out); break;
  }
  return hipGetLastError();
}

hipError_t launch_lds_lookup(uint32_t threads, dim3 g, size_t lds, hipStream_t s, const GPlanDev &pd,
                             const uint64_t *h, uint8_t *out, uint32_t shift) {
  switch (threads) {
    case 256: hipLaunchKernelGGL(grouped_lds_lookup_kernel<256>, g, dim3(256), lds, s, pd, h, out, shift); break;
    case 512: hipLaunchKernelGGL(grouped_lds_lookup_kernel<512>, g, dim3(512), lds, s, pd, h, out, shift); break;
    default: hipLaunchKernelGGL(grouped_lds_lookup_kernel<1024>, g, dim3(1024), lds, s, pd, h, out, shift); break;
  }
  return hipGetLastError();
}

const void *lds_lookup_func(uint32_t threads) {
  switch (threads) {
    case 256: return (const void *)grouped_lds_lookup_kernel<256>;
    case 512: return (const void *)grouped_lds_lookup_kernel<512>;
    default: return (const void *)grouped_lds_lookup_kernel<1024>;
  }
}

const void *lookup_func(int unroll) {
  switch (unroll) {
    case 1: return (const void *)grouped_lookup_kernel<1>;
    case 2: return (const void *)grouped_lookup_kernel<2>;
    default: return (const void *)grouped_lookup_kernel<4>;
  }
}

// Dynamic LDS of the insert kernel: the largest slice, then the run staging.
static size_t insert_kernel_lds(const GroupedPlanHost &p) { return ((p.insert_lds + 31u) & ~(size_t)31u) + kRunLds; }

static dim3 reset_grid(const GroupedPlanHost &p) {
  const uint32_t n = std::max<uint32_t>({(uint32_t)kQueues, p.pd.n_parts, p.pd.n_slices, 1u});
  return dim3((n + 255u) / 256u);
}

// Build tiles and queues for the group from per-filter capacities (keys
// inserted and looked up per call, at most) and copy them to the device.
// Tiles are relative to each filter's key ranges, which the kernels read from
// device offsets when they run: the plan's own copy of host offsets for a
// fixed-shape plan (ins_off and look_off given), the caller's per-call
// offsets for a capacity plan (both NULL).
sbbf_status grouped_build_plan(sbbf_group *g, const uint64_t *ins_cap, const uint64_t *look_cap,
                               const uint64_t *ins_off, const uint64_t *look_off, const sbbf_grouped_config &cfg,
                               const sbbf_device_info &info) {
  GroupedPlanHost &p = g->plan;
  free_plan(p);
  const uint32_t F = (uint32_t)g->filters.size();
  p.ins_cap.assign(ins_cap, ins_cap + F);
  p.look_cap.assign(look_cap, look_cap + F);
  p.capacity = ins_off == nullptr;
  if (p.capacity) {
    p.ins_off.clear();
    p.look_off.clear();
  } else {
    p.ins_off.assign(ins_off, ins_off + F + 1);
    p.look_off.assign(look_off, look_off + F + 1);
  }
  p.ins_total = p.look_total = 0;
  for (uint32_t f = 0; f < F; ++f) {
    if (p.ins_cap[f] > 0xFFFFFFFFull)
      return set_error(SBBF_EUNSUPPORTED, "a filter takes at most 2^32 - 1 insert keys per grouped call");
    p.ins_total += p.ins_cap[f];
    p.look_total += p.look_cap[f];
    if (p.ins_total < p.ins_cap[f] || p.look_total < p.look_cap[f])
      return set_error(SBBF_EINVAL, "key capacities overflow 64 bits");
  }
  ++g->plans;
  p.cfg = cfg;

  // Insert tiles. A filter that fits insert_lds_bytes is one stream tile. A
  // larger one is cut into slices of S blocks; with at most kMaxLocalSlices
  // slices its keys are partitioned by slice (chunks of kPartChunk keys, one
  // run per slice and chunk) and each slice is a partitioned tile, else each
  // slice is a stream tile.
  struct Cost {
    uint64_t cost;
    GInsTile t;
  };
  std::vector<Cost> ins;
  std::vector<GPart> parts;
  std::vector<std::vector<GChunk>> part_chunks;
  std::vector<GSlice> slices;
  uint64_t part_keys = 0, run_total = 0;
  size_t max_lds = 32;
  const uint32_t S = 1u << cfg.insert_slice_shift;
  for (uint32_t f = 0; f < F; ++f) {
    const uint64_t n = p.ins_cap[f];
    if (n == 0) continue;
    const uint32_t B = g->filters[f]->num_blocks;
    if ((uint64_t)B * 32u <= cfg.insert_lds_bytes) {
      ins.push_back({n, {f, 0u, B, kStreamTile}});
      max_lds = std::max(max_lds, (size_t)B * 32u);
      continue;
    }
    const uint32_t ns = (uint32_t)(((uint64_t)B + S - 1u) / S);
    const bool partition = ns <= kMaxLocalSlices;
    if (partition) {
      const uint32_t pi = (uint32_t)parts.size();
      const uint32_t n_chunks = (uint32_t)((n + kPartChunk - 1u) / kPartChunk);
      parts.push_back({part_keys, f, (uint32_t)slices.size(), ns, cfg.insert_slice_shift});
      part_chunks.emplace_back();
      for (uint32_t k = 0; k < n_chunks; ++k) part_chunks.back().push_back({k, pi});
      part_keys += n;
      for (uint32_t k = 0; k < ns; ++k) {
        slices.push_back({(uint32_t)run_total, n_chunks});
        run_total += n_chunks;
      }
    }
    for (uint32_t k = 0; k < ns; ++k) {
      const uint64_t b0 = (uint64_t)k * S;
      const uint32_t nb = (uint32_t)std::min<uint64_t>(S, B - b0);
      if (partition)
        ins.push_back({(n + ns - 1u) / ns, {f, (uint32_t)b0, nb, parts.back().slice_base + k}});
      else
        ins.push_back({n, {f, (uint32_t)b0, nb, kStreamTile}});
      max_lds = std::max(max_lds, (size_t)nb * 32u);
    }
  }
  if (run_total > 0xFFFFFFFFull) return set_error(SBBF_EUNSUPPORTED, "too many insert keys in partitioned filters");
  std::stable_sort(ins.begin(), ins.end(), [](const Cost &a, const Cost &b) { return a.cost > b.cost; });
  p.n_ins_tiles = (uint32_t)ins.size();
  p.insert_lds = max_lds;
  // Chunks of different filters interleaved, so that workgroups running at
  // the same time mostly take room from different filters' regions.
  std::vector<GChunk> chunks;
  for (size_t k = 0;; ++k) {
    bool any = false;
    for (auto &pc : part_chunks)
      if (k < pc.size()) {
        chunks.push_back(pc[k]);
        any = true;
      }
    if (!any) break;
  }
  p.n_chunks = (uint32_t)chunks.size();

  // Lookup tiles, filters assigned to queues greedily by work (largest first).
  std::vector<uint32_t> order(F);
  std::iota(order.begin(), order.end(), 0u);
  std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return p.look_cap[a] > p.look_cap[b]; });
  // Filters of at most lookup_lds_slices LDS slices take LDS tiles (their own
  // queues, balanced separately), the rest gather tiles.
  const int nq = cfg.xcd_queues ? kQueues : 1;
  p.lds_look_shift = lds_look_shift(cfg.lookup_lds_threads, info);
  std::vector<std::vector<GLookTile>> qt(kQueues), qlds(kQueues);
  std::vector<uint64_t> load(kQueues, 0), load_lds(kQueues, 0);
  uint32_t lds_max_blocks = 0;
  for (uint32_t f : order) {
    const uint64_t n = p.look_cap[f];
    if (n == 0) continue;
    const uint32_t B = g->filters[f]->num_blocks;
    const uint64_t nsl = ((uint64_t)B + (1u << p.lds_look_shift) - 1u) >> p.lds_look_shift;
    const bool lds = nsl <= cfg.lookup_lds_slices;
    std::vector<uint64_t> &ld = lds ? load_lds : load;
    int best = 0;
    for (int k = 1; k < nq; ++k)
      if (ld[k] < ld[best]) best = k;
    ld[best] += n;
    const uint32_t tk = lds ? kLdsLookPer * cfg.lookup_lds_threads : cfg.lookup_tile_keys;
    for (uint64_t at = 0; at < n; at += tk) {
      const uint32_t c = (uint32_t)std::min<uint64_t>(tk, n - at);
      (lds ? qlds : qt)[best].push_back({at, c, f});
    }
    if (lds) lds_max_blocks = std::max(lds_max_blocks, std::min(B, 1u << p.lds_look_shift));
  }
  auto concat = [](const std::vector<std::vector<GLookTile>> &q, std::vector<uint32_t> &begin,
                   std::vector<GLookTile> &all) {
    begin.assign(kQueues + 1, 0);
    for (int k = 0; k < kQueues; ++k) {
      begin[k] = (uint32_t)all.size();
      all.insert(all.end(), q[k].begin(), q[k].end());
    }
    begin[kQueues] = (uint32_t)all.size();
  };
  std::vector<uint32_t> qbegin, qbegin_lds;
  std::vector<GLookTile> look, look_lds;
  concat(qt, qbegin, look);
  concat(qlds, qbegin_lds, look_lds);
  p.n_look_tiles = (uint32_t)look.size();
  p.n_lds_tiles = (uint32_t)look_lds.size();
  p.lds_look_bytes = (size_t)lds_max_blocks * 32u;

  std::vector<GFilter> ft(F);
  for (uint32_t f = 0; f < F; ++f) ft[f] = {g->filters[f]->words, g->filters[f]->num_blocks, 0u};

  // One device allocation: filters | ins_off | look_off | ins_cap | look_cap |
  // bad | ins tiles | look tiles | queue_begin | LDS look tiles | LDS
  // queue_begin | counters | parts | chunks | slices | runs | nruns | tops;
  // the partitioned keys are a second one.
  auto up = [](size_t v) { return (v + 255u) & ~(size_t)255u; };
  auto at_least1 = [](size_t v) { return std::max<size_t>(1, v); };
  const size_t o_f = 0;
  const size_t o_io = o_f + up(F * sizeof(GFilter));
  const size_t o_lo = o_io + up((F + 1) * sizeof(uint64_t));
  const size_t o_ic = o_lo + up((F + 1) * sizeof(uint64_t));
  const size_t o_lc = o_ic + up(F * sizeof(uint64_t));
  const size_t o_bad = o_lc + up(F * sizeof(uint64_t));
  const size_t o_it = o_bad + up(sizeof(uint32_t));
  const size_t o_lt = o_it + up(at_least1(ins.size()) * sizeof(GInsTile));
  const size_t o_qb = o_lt + up(at_least1(look.size()) * sizeof(GLookTile));
  const size_t o_ll = o_qb + up((kQueues + 1) * sizeof(uint32_t));
  const size_t o_lq = o_ll + up(at_least1(look_lds.size()) * sizeof(GLookTile));
  const size_t o_c = o_lq + up((kQueues + 1) * sizeof(uint32_t));
  const size_t o_pt = o_c + up((1 + 2 * kQueues) * sizeof(uint32_t));
  const size_t o_ch = o_pt + up(at_least1(parts.size()) * sizeof(GPart));
  const size_t o_sl = o_ch + up(at_least1(chunks.size()) * sizeof(GChunk));
  const size_t o_rn = o_sl + up(at_least1(slices.size()) * sizeof(GSlice));
  const size_t o_nr = o_rn + up(at_least1(run_total) * sizeof(GRun));
  const size_t o_tp = o_nr + up(at_least1(slices.size()) * sizeof(uint32_t));
  const size_t total = o_tp + up(at_least1(parts.size()) * sizeof(unsigned long long));
  std::vector<char> host(o_rn, 0);  // runs, nruns and tops are written on the device
  memcpy(host.data() + o_f, ft.data(), F * sizeof(GFilter));
  if (!p.capacity) {
    memcpy(host.data() + o_io, p.ins_off.data(), (F + 1) * sizeof(uint64_t));
    memcpy(host.data() + o_lo, p.look_off.data(), (F + 1) * sizeof(uint64_t));
  }
  memcpy(host.data() + o_ic, p.ins_cap.data(), F * sizeof(uint64_t));
  memcpy(host.data() + o_lc, p.look_cap.data(), F * sizeof(uint64_t));
  const uint32_t no_bad = 0xFFFFFFFFu;
  memcpy(host.data() + o_bad, &no_bad, sizeof(no_bad));
  for (size_t i = 0; i < ins.size(); ++i) memcpy(host.data() + o_it + i * sizeof(GInsTile), &ins[i].t, sizeof(GInsTile));
  if (!look.empty()) memcpy(host.data() + o_lt, look.data(), look.size() * sizeof(GLookTile));
  memcpy(host.data() + o_qb, qbegin.data(), (kQueues + 1) * sizeof(uint32_t));
  if (!look_lds.empty()) memcpy(host.data() + o_ll, look_lds.data(), look_lds.size() * sizeof(GLookTile));
  memcpy(host.data() + o_lq, qbegin_lds.data(), (kQueues + 1) * sizeof(uint32_t));
  if (!parts.empty()) memcpy(host.data() + o_pt, parts.data(), parts.size() * sizeof(GPart));
  if (!chunks.empty()) memcpy(host.data() + o_ch, chunks.data(), chunks.size() * sizeof(GChunk));
  if (!slices.empty()) memcpy(host.data() + o_sl, slices.data(), slices.size() * sizeof(GSlice));
  hipError_t e = dev_malloc(&p.dev, total);
  if (e != hipSuccess) return hip_error(e, "hipMalloc(grouped plan)");
  e = hipMemcpy(p.dev, host.data(), o_rn, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_error(e, "hipMemcpy(grouped plan)");
  if (part_keys) {
    e = dev_malloc(&p.keys, part_keys * sizeof(uint64_t));
    if (e != hipSuccess) return hip_error(e, "hipMalloc(grouped partitioned keys)");
  }
  char *d = static_cast<char *>(p.dev);
  p.pd.filters = reinterpret_cast<const GFilter *>(d + o_f);
  // A capacity plan's kernels take the offsets of each run instead.
  p.pd.ins_off = p.capacity ? nullptr : reinterpret_cast<const uint64_t *>(d + o_io);
  p.pd.look_off = p.capacity ? nullptr : reinterpret_cast<const uint64_t *>(d + o_lo);
  p.pd.ins_cap = reinterpret_cast<const uint64_t *>(d + o_ic);
  p.pd.look_cap = reinterpret_cast<const uint64_t *>(d + o_lc);
  p.pd.bad = reinterpret_cast<uint32_t *>(d + o_bad);
  p.pd.ins_tiles = reinterpret_cast<const GInsTile *>(d + o_it);
  p.pd.look_tiles = reinterpret_cast<const GLookTile *>(d + o_lt);
  p.pd.queue_begin = reinterpret_cast<const uint32_t *>(d + o_qb);
  p.pd.lds_tiles = reinterpret_cast<const GLookTile *>(d + o_ll);
  p.pd.lds_queue_begin = reinterpret_cast<const uint32_t *>(d + o_lq);
  p.pd.counters = reinterpret_cast<uint32_t *>(d + o_c);
  p.pd.parts = reinterpret_cast<const GPart *>(d + o_pt);
  p.pd.chunks = reinterpret_cast<const GChunk *>(d + o_ch);
  p.pd.slices = reinterpret_cast<const GSlice *>(d + o_sl);
  p.pd.runs = reinterpret_cast<GRun *>(d + o_rn);
  p.pd.nruns = reinterpret_cast<uint32_t *>(d + o_nr);
  p.pd.tops = reinterpret_cast<unsigned long long *>(d + o_tp);
  p.pd.part_keys = static_cast<uint64_t *>(p.keys);
  p.pd.n_ins_tiles = p.n_ins_tiles;
  p.pd.n_parts = (uint32_t)parts.size();
  p.pd.n_slices = (uint32_t)slices.size();
  // The kernels' dynamic LDS limit is a property of the function, shared by
  // every group: it is raised to the device's maximum, never lowered to this
  // plan's need, so that planning another group cannot break this one's graph.
  (void)hipFuncSetAttribute((const void *)grouped_insert_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)info.lds_per_block);
  (void)hipFuncSetAttribute((const void *)grouped_part_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)info.lds_per_block);
  for (uint32_t t : {256u, 512u, 1024u})
    (void)hipFuncSetAttribute(lds_lookup_func(t), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)info.lds_per_block);
  (void)hipGetLastError();
  p.planned = true;
  return SBBF_OK;
}

static dim3 insert_grid(const sbbf_device_info &info, const GroupedPlanHost &p) {
  return dim3(std::max(1u, std::min<uint32_t>(p.n_ins_tiles, (uint32_t)info.compute_units)));
}

static dim3 lookup_grid(const sbbf_device_info &info, const GroupedPlanHost &p) {
  const uint32_t want = (uint32_t)info.compute_units * p.cfg.lookup_blocks_per_cu;
  return dim3(std::max<uint32_t>(kQueues, std::min<uint32_t>(want, std::max<uint32_t>(p.n_look_tiles, kQueues))));
}

// As many LDS lookup workgroups per compute unit as its LDS holds, up to
// 1,024 threads (16 waves: each thread needs 128 registers), or fewer
// workgroups when there are fewer tiles.
static dim3 lds_lookup_grid(const sbbf_device_info &info, const GroupedPlanHost &p) {
  const uint64_t per_cu_lds = std::max<uint64_t>(1, info.lds_per_cu / std::max<size_t>(p.lds_look_bytes, 1));
  const uint64_t per_cu = std::max<uint64_t>(1, std::min<uint64_t>(per_cu_lds, 1024u / p.cfg.lookup_lds_threads));
  const uint64_t want = (uint64_t)info.compute_units * per_cu;
  return dim3((uint32_t)std::max<uint64_t>(kQueues, std::min<uint64_t>(want, p.n_lds_tiles)));
}

static uint32_t insert_words_lds(const GroupedPlanHost &p) { return (uint32_t)((p.insert_lds + 31u) & ~(size_t)31u); }

sbbf_status grouped_insert_phase(sbbf_group *g, const uint64_t *d_ins, hipStream_t s, const sbbf_device_info &info) {
  GroupedPlanHost &p = g->plan;
  hipLaunchKernelGGL(grouped_reset_kernel, reset_grid(p), dim3(256), 0, s, p.pd, 1u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, "grouped reset");
  if (p.n_chunks) {
    hipLaunchKernelGGL(grouped_part_kernel, dim3(p.n_chunks), dim3(kInsertThreads), kPartLds, s, p.pd, d_ins);
    if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "grouped partition");
  }
  if (p.n_ins_tiles == 0) return SBBF_OK;
  hipLaunchKernelGGL(grouped_insert_kernel, insert_grid(info, p), dim3(kInsertThreads), insert_kernel_lds(p), s, p.pd,
                     d_ins, insert_words_lds(p));
  return hip_error(hipGetLastError(), "grouped insert");
}

sbbf_status grouped_lookup_phase(sbbf_group *g, const uint64_t *d_look, uint8_t *d_out, hipStream_t s,
                                 const sbbf_device_info &info) {
  GroupedPlanHost &p = g->plan;
  hipLaunchKernelGGL(grouped_reset_kernel, reset_grid(p), dim3(256), 0, s, p.pd, 2u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, "grouped reset");
  if (p.n_lds_tiles) {
    e = launch_lds_lookup(p.cfg.lookup_lds_threads, lds_lookup_grid(info, p), p.lds_look_bytes, s, p.pd, d_look,
                          d_out, p.lds_look_shift);
    if (e != hipSuccess) return hip_error(e, "grouped LDS lookup");
  }
  if (p.n_look_tiles == 0) return SBBF_OK;
  return hip_error(launch_lookup_any(p.cfg.lookup_unroll, lookup_grid(info, p), dim3(p.cfg.lookup_threads), s, p.pd,
                                     d_look, d_out),
                   "grouped lookup");
}

// The graph: reset -> partition (when the group has partitioned filters) ->
// insert -> lookup (kernel nodes only). Kernel parameters are copied into the
// graph when a node is added or updated.
static sbbf_status set_insert_nodes(GroupedPlanHost &p, const uint64_t *d_ins, const sbbf_device_info &info,
                                    bool add) {
  hipKernelNodeParams kp;
  memset(&kp, 0, sizeof(kp));
  hipError_t e;
  const uint64_t *ins_arg = d_ins;
  hipGraphNode_t prev = p.n_reset;
  if (p.n_chunks) {
    void *part_args[] = {(void *)&p.pd, (void *)&ins_arg};
    kp.func = (void *)grouped_part_kernel;
    kp.gridDim = dim3(p.n_chunks);
    kp.blockDim = dim3(kInsertThreads);
    kp.sharedMemBytes = (unsigned)kPartLds;
    kp.kernelParams = part_args;
    e = add ? hipGraphAddKernelNode(&p.n_part, p.graph, &prev, 1, &kp) : hipGraphExecKernelNodeSetParams(p.exec, p.n_part, &kp);
    if (e != hipSuccess) return hip_error(e, "graph node (partition)");
    prev = p.n_part;
  }
  uint32_t words_lds = insert_words_lds(p);
  void *ins_args[] = {(void *)&p.pd, (void *)&ins_arg, (void *)&words_lds};
  kp.func = (void *)grouped_insert_kernel;
  kp.gridDim = insert_grid(info, p);
  kp.blockDim = dim3(kInsertThreads);
  kp.sharedMemBytes = (unsigned)insert_kernel_lds(p);
  kp.kernelParams = ins_args;
  e = add ? hipGraphAddKernelNode(&p.n_ins, p.graph, &prev, 1, &kp) : hipGraphExecKernelNodeSetParams(p.exec, p.n_ins, &kp);
  if (e != hipSuccess) return hip_error(e, "graph node (insert)");
  return SBBF_OK;
}

// The lookup nodes: the LDS lookup (when the plan has LDS tiles), then the
// gather lookup, in sequence after the insert node.
static sbbf_status set_lookup_node(GroupedPlanHost &p, const uint64_t *d_look, uint8_t *d_out,
                                   const sbbf_device_info &info, bool add) {
  hipKernelNodeParams kp;
  memset(&kp, 0, sizeof(kp));
  const uint64_t *look_arg = d_look;
  uint8_t *out_arg = d_out;
  hipGraphNode_t prev = p.n_ins;
  hipError_t e;
  if (p.n_lds_tiles) {
    uint32_t shift = p.lds_look_shift;
    void *lds_args[] = {(void *)&p.pd, (void *)&look_arg, (void *)&out_arg, (void *)&shift};
    kp.func = const_cast<void *>(lds_lookup_func(p.cfg.lookup_lds_threads));
    kp.gridDim = lds_lookup_grid(info, p);
    kp.blockDim = dim3(p.cfg.lookup_lds_threads);
    kp.sharedMemBytes = (unsigned)p.lds_look_bytes;
    kp.kernelParams = lds_args;
    e = add ? hipGraphAddKernelNode(&p.n_look_lds, p.graph, &prev, 1, &kp)
            : hipGraphExecKernelNodeSetParams(p.exec, p.n_look_lds, &kp);
    if (e != hipSuccess) return hip_error(e, "graph node (LDS lookup)");
    prev = p.n_look_lds;
  }
  void *look_args[] = {(void *)&p.pd, (void *)&look_arg, (void *)&out_arg};
  kp.func = (void *)lookup_func(p.cfg.lookup_unroll);
  kp.gridDim = lookup_grid(info, p);
  kp.blockDim = dim3(p.cfg.lookup_threads);
  kp.sharedMemBytes = 0;
  kp.kernelParams = look_args;
  e = add ? hipGraphAddKernelNode(&p.n_look, p.graph, &prev, 1, &kp)
          : hipGraphExecKernelNodeSetParams(p.exec, p.n_look, &kp);
  return e == hipSuccess ? SBBF_OK : hip_error(e, "graph node (lookup)");
}

static sbbf_status build_graph(sbbf_group *g, const uint64_t *d_ins, const uint64_t *d_look, uint8_t *d_out,
                               const sbbf_device_info &info) {
  GroupedPlanHost &p = g->plan;
  hipError_t e = hipGraphCreate(&p.graph, 0);
  if (e != hipSuccess) return hip_error(e, "hipGraphCreate");
  uint32_t what = 3u;
  void *reset_args[] = {(void *)&p.pd, (void *)&what};
  hipKernelNodeParams kp;
  memset(&kp, 0, sizeof(kp));
  kp.func = (void *)grouped_reset_kernel;
  kp.gridDim = reset_grid(p);
  kp.blockDim = dim3(256);
  kp.kernelParams = reset_args;
  e = hipGraphAddKernelNode(&p.n_reset, p.graph, nullptr, 0, &kp);
  if (e != hipSuccess) return hip_error(e, "hipGraphAddKernelNode(reset)");
  sbbf_status st = set_insert_nodes(p, d_ins, info, true);
  if (st != SBBF_OK) return st;
  if ((st = set_lookup_node(p, d_look, d_out, info, true)) != SBBF_OK) return st;
  e = hipGraphInstantiate(&p.exec, p.graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_error(e, "hipGraphInstantiate");
  p.g_ins = d_ins;
  p.g_look = d_look;
  p.g_out = d_out;
  p.g_ins_off = p.pd.ins_off;
  p.g_look_off = p.pd.look_off;
  ++g->graph_builds;
  return SBBF_OK;
}

static sbbf_status update_graph(sbbf_group *g, const uint64_t *d_ins, const uint64_t *d_look, uint8_t *d_out,
                                const sbbf_device_info &info) {
  GroupedPlanHost &p = g->plan;
  sbbf_status st = set_insert_nodes(p, d_ins, info, false);
  if (st != SBBF_OK) return st;
  if ((st = set_lookup_node(p, d_look, d_out, info, false)) != SBBF_OK) return st;
  p.g_ins = d_ins;
  p.g_look = d_look;
  p.g_out = d_out;
  p.g_ins_off = p.pd.ins_off;
  p.g_look_off = p.pd.look_off;
  ++g->graph_updates;
  return SBBF_OK;
}

// One graph launch. A capacity plan takes the run's device offsets; the
// graph's kernel nodes hold them (and the data pointers) as arguments and are
// updated only when a pointer changes, never re-planned: new counts in the
// same offset buffers need no host work at all.
sbbf_status grouped_run_graph(sbbf_group *g, const uint64_t *d_ins, const uint64_t *d_look, uint8_t *d_out,
                              hipStream_t s, const sbbf_device_info &info, const uint64_t *d_ins_off = nullptr,
                              const uint64_t *d_look_off = nullptr) {
  GroupedPlanHost &p = g->plan;
  if (p.capacity) {
    p.pd.ins_off = d_ins_off;
    p.pd.look_off = d_look_off;
  }
  sbbf_status st = SBBF_OK;
  if (!p.exec) {
    st = build_graph(g, d_ins, d_look, d_out, info);
  } else if (p.g_ins != d_ins || p.g_look != d_look || p.g_out != d_out || p.g_ins_off != p.pd.ins_off ||
             p.g_look_off != p.pd.look_off) {
    st = update_graph(g, d_ins, d_look, d_out, info);
  }
  if (st != SBBF_OK) return st;
  return hip_error(hipGraphLaunch(p.exec, s), "hipGraphLaunch(grouped)");
}

static void digest_launch(const uint32_t *words, uint64_t n, unsigned long long *acc, hipStream_t s) {
  if (n == 0) return;
  const uint64_t want = (n + 255) / 256;
  hipLaunchKernelGGL(digest_kernel, dim3((uint32_t)std::min<uint64_t>(want, 1024)), dim3(256), 0, s, words, n, acc);
}

// Digest of all filters (in group order) and of the planned lookup outputs.
static sbbf_status group_digest(sbbf_group *g, const uint8_t *d_out, hipStream_t s, uint64_t *digest) {
  unsigned long long *acc = nullptr;
  hipError_t e = dev_malloc_async((void **)&acc, sizeof(unsigned long long) * 2, s);
  if (e != hipSuccess) return hip_error(e, "hipMallocAsync(digest)");
  hipLaunchKernelGGL(fill_kernel_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t *>(acc), 4u);
  unsigned long long h = 0x243f6a8885a308d3ull;
  for (size_t f = 0; f < g->filters.size(); ++f) {
    digest_launch(g->filters[f]->words, (uint64_t)g->filters[f]->num_blocks * 8u, acc, s);
    // Chain filters so that swapping two equal-sized filters changes the digest.
    hipLaunchKernelGGL(digest_chain_kernel, dim3(1), dim3(1), 0, s, acc, (unsigned long long)f);
  }
  const uint64_t nl = g->plan.look_off.empty() ? 0 : g->plan.look_off.back();  // 0 for a capacity plan
  if (d_out && nl) {
    // Bytes are digested as 32-bit words plus the ragged tail.
    digest_launch(reinterpret_cast<const uint32_t *>(d_out), nl / 4, acc + 1, s);
    if (nl % 4) {
      hipLaunchKernelGGL(digest_tail_kernel, dim3(1), dim3(64), 0, s, d_out + (nl / 4) * 4, (uint32_t)(nl % 4), acc + 1);
    }
  }
  unsigned long long hostv[2] = {0, 0};
  e = hipMemcpyAsync(hostv, acc, sizeof(hostv), hipMemcpyDeviceToHost, s);
  hipError_t e2 = hipFreeAsync(acc, s);
  hipError_t e3 = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_error(e, "hipMemcpyAsync(digest)");
  if (e2 != hipSuccess) return hip_error(e2, "hipFreeAsync(digest)");
  if (e3 != hipSuccess) return hip_error(e3, "hipStreamSynchronize(digest)");
  *digest = hostv[0] * 0x9e3779b97f4a7c15ull ^ hostv[1] ^ h;
  return SBBF_OK;
}

}  // namespace sbbf

// ---- C ABI -----------------------------------------------------------------------

using namespace sbbf;

namespace {

// Cache key of an autotune result: device, ROCm runtime, and the batch shape
// (filter count, total keys, largest filter) in powers of two.
std::string tune_key(const sbbf_device_info &info, const sbbf_group *g) {
  int rt = 0;
  (void)hipRuntimeGetVersion(&rt);
  uint64_t ins = g->plan.ins_total, look = g->plan.look_total;
  uint32_t maxb = 0;
  for (auto *f : g->filters) maxb = std::max(maxb, f->num_blocks);
  auto lg = [](uint64_t v) { int k = 0; while (v > 1) { v >>= 1; ++k; } return k; };
  char buf[256];
  snprintf(buf, sizeof(buf), "%s|cu%d|hip%d|F%zu|ins2^%d|look2^%d|maxb2^%d", info.arch, info.compute_units, rt,
           g->filters.size(), lg(ins), lg(look), lg(maxb));
  for (char *c = buf; *c; ++c)
    if (*c == ' ') *c = '_';
  return buf;
}

bool cache_lookup(const char *path, const std::string &key, sbbf_grouped_config *cfg) {
  FILE *fp = fopen(path, "r");
  if (!fp) return false;
  char line[512];
  bool found = false;
  while (fgets(line, sizeof(line), fp)) {
    char k[256];
    sbbf_grouped_config c;
    unsigned long long lds = 0;
    memset(&c, 0, sizeof(c));
    if (sscanf(line, "%255s %u %u %u %u %u %u %llu %u %u", k, &c.lookup_tile_keys, &c.lookup_threads,
               &c.lookup_unroll, &c.lookup_blocks_per_cu, &c.insert_slice_shift, &c.xcd_queues, &lds,
               &c.lookup_lds_slices, &c.lookup_lds_threads) == 10 &&
        key == k) {
      c.insert_lds_bytes = lds;
      *cfg = c;  // the last matching line wins
      found = true;
    }
  }
  fclose(fp);
  return found;
}

void cache_store(const char *path, const std::string &key, const sbbf_grouped_config &c) {
  FILE *fp = fopen(path, "a");
  if (!fp) return;
  fprintf(fp, "%s %u %u %u %u %u %u %llu %u %u\n", key.c_str(), c.lookup_tile_keys, c.lookup_threads,
          c.lookup_unroll, c.lookup_blocks_per_cu, c.insert_slice_shift, c.xcd_queues,
          (unsigned long long)c.insert_lds_bytes, c.lookup_lds_slices, c.lookup_lds_threads);
  fclose(fp);
}

sbbf_status need_plan(const sbbf_group *g) {
  if (!g) return set_error(SBBF_EINVAL, "group is NULL");
  if (!g->plan.planned) return set_error(SBBF_EINVAL, "group has no plan (call sbbf_grouped_plan)");
  return SBBF_OK;
}

// Entry points that take no offsets need a plan made from host offsets.
sbbf_status need_fixed_plan(const sbbf_group *g) {
  sbbf_status st = need_plan(g);
  if (st != SBBF_OK) return st;
  if (g->plan.capacity)
    return set_error(SBBF_EINVAL, "the group has a capacity plan: its runs take device offsets "
                                  "(sbbf_grouped_run_offsets)");
  return SBBF_OK;
}

sbbf_status check_io(const sbbf_group *g, const uint64_t *d_ins, const uint64_t *d_look, const uint8_t *d_out) {
  const uint64_t ni = g->plan.ins_total, nl = g->plan.look_total;
  if (ni && (!d_ins || ((uintptr_t)d_ins & 7))) return set_error(SBBF_EINVAL, "d_ins is NULL or not 8-byte aligned");
  if (nl && (!d_look || ((uintptr_t)d_look & 7))) return set_error(SBBF_EINVAL, "d_look is NULL or not 8-byte aligned");
  if (nl && !d_out) return set_error(SBBF_EINVAL, "d_out is NULL");
  return SBBF_OK;
}

}  // namespace

extern "C" {

sbbf_status sbbf_grouped_default_config(sbbf_grouped_config *out) {
  if (!out) return set_error(SBBF_EINVAL, "out is NULL");
  sbbf_status st;
  const sbbf_device_info *info = current_device_info(&st);
  if (!info) return st;
  *out = default_config(*info);
  return SBBF_OK;
}

sbbf_status sbbf_grouped_create(sbbf_filter *const *filters, uint32_t num_filters, sbbf_group **out) {
  if (!out) return set_error(SBBF_EINVAL, "out is NULL");
  *out = nullptr;
  if (num_filters == 0 || !filters) return set_error(SBBF_EINVAL, "a group needs at least one filter");
  for (uint32_t f = 0; f < num_filters; ++f) {
    if (!filters[f]) return set_error(SBBF_EINVAL, "filter " + std::to_string(f) + " is NULL");
    if (filters[f]->lanes != 8)
      return set_error(SBBF_EUNSUPPORTED, "filter " + std::to_string(f) + " is a block variant; groups take "
                                          "eight-word blocks only");
  }
  // The filters' memory must not overlap: a slice of a filter is loaded,
  // updated and stored back whole by one workgroup, so two entries over the
  // same words would lose each other's inserts.
  {
    std::vector<std::pair<uintptr_t, uintptr_t>> span(num_filters);
    for (uint32_t f = 0; f < num_filters; ++f) {
      const uintptr_t b = reinterpret_cast<uintptr_t>(filters[f]->words);
      span[f] = {b, b + (uintptr_t)filters[f]->num_blocks * 32u};
    }
    std::sort(span.begin(), span.end());
    for (uint32_t f = 1; f < num_filters; ++f)
      if (span[f].first < span[f - 1].second)
        return set_error(SBBF_EINVAL, "filters of a group must not share memory (each filter appears once)");
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "hipGetDevice");
  sbbf_group *g = new (std::nothrow) sbbf_group();
  if (!g) return set_error(SBBF_ENOMEM, "group allocation failed");
  g->filters.assign(filters, filters + num_filters);
  g->device = dev;
  *out = g;
  return SBBF_OK;
}

sbbf_status sbbf_grouped_destroy(sbbf_group *g) {
  if (!g) return set_error(SBBF_EINVAL, "group is NULL");
  free_plan(g->plan);
  delete g;
  return SBBF_OK;
}

sbbf_status sbbf_grouped_plan(sbbf_group *g, const uint64_t *h_ins_offsets, const uint64_t *h_look_offsets,
                              const sbbf_grouped_config *cfg) {
  if (!g || !h_ins_offsets || !h_look_offsets) return set_error(SBBF_EINVAL, "group or offsets is NULL");
  sbbf_status st;
  const sbbf_device_info *info = current_device_info(&st);
  if (!info) return st;
  const sbbf_grouped_config c = cfg ? *cfg : default_config(*info);
  if ((st = check_config(c, *info)) != SBBF_OK) return st;
  const size_t F = g->filters.size();
  std::vector<uint64_t> ic(F), lc(F);
  for (size_t f = 0; f < F; ++f) {
    if (h_ins_offsets[f + 1] < h_ins_offsets[f] || h_look_offsets[f + 1] < h_look_offsets[f])
      return set_error(SBBF_EINVAL, "offsets must be non-decreasing");
    ic[f] = h_ins_offsets[f + 1] - h_ins_offsets[f];
    lc[f] = h_look_offsets[f + 1] - h_look_offsets[f];
  }
  return grouped_build_plan(g, ic.data(), lc.data(), h_ins_offsets, h_look_offsets, c, *info);
}

sbbf_status sbbf_grouped_plan_capacity(sbbf_group *g, const uint64_t *h_ins_cap, const uint64_t *h_look_cap,
                                       const sbbf_grouped_config *cfg) {
  if (!g || !h_ins_cap || !h_look_cap) return set_error(SBBF_EINVAL, "group or capacities is NULL");
  sbbf_status st;
  const sbbf_device_info *info = current_device_info(&st);
  if (!info) return st;
  const sbbf_grouped_config c = cfg ? *cfg : default_config(*info);
  if ((st = check_config(c, *info)) != SBBF_OK) return st;
  return grouped_build_plan(g, h_ins_cap, h_look_cap, nullptr, nullptr, c, *info);
}

sbbf_status sbbf_grouped_run_offsets(sbbf_group *g, const uint64_t *d_ins, const uint64_t *d_ins_offsets,
                                     const uint64_t *d_look, const uint64_t *d_look_offsets, uint8_t *d_out,
                                     sbbf_stream s) {
  sbbf_status st = need_plan(g);
  if (st != SBBF_OK || (st = check_io(g, d_ins, d_look, d_out)) != SBBF_OK) return st;
  if (!g->plan.capacity)
    return set_error(SBBF_EINVAL, "the group's plan has fixed offsets (use sbbf_grouped_run, or plan with "
                                  "sbbf_grouped_plan_capacity)");
  if (!d_ins_offsets || !d_look_offsets || ((uintptr_t)d_ins_offsets & 7) || ((uintptr_t)d_look_offsets & 7))
    return set_error(SBBF_EINVAL, "d_ins_offsets and d_look_offsets must be 8-byte aligned device pointers");
  const sbbf_device_info *info = current_device_info(&st);
  if (!info) return st;
  return grouped_run_graph(g, d_ins, d_look, d_out, (hipStream_t)s, *info, d_ins_offsets, d_look_offsets);
}

sbbf_status sbbf_grouped_check(sbbf_group *g, sbbf_stream s, uint32_t *first_bad) {
  sbbf_status st = need_plan(g);
  if (st != SBBF_OK) return st;
  uint32_t bad = 0xFFFFFFFFu;
  hipStream_t stream = (hipStream_t)s;
  hipError_t e = hipMemcpyAsync(&bad, g->plan.pd.bad, sizeof(bad), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_error(e, "sbbf_grouped_check");
  if (first_bad) *first_bad = bad;
  if (bad == 0xFFFFFFFFu) return SBBF_OK;
  e = launch_fill(g->plan.pd.bad, 1, 0xFFFFFFFFu, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_error(e, "sbbf_grouped_check (reset)");
  return set_error(SBBF_EINVAL, "filter " + std::to_string(bad) + " had a key range above its planned capacity "
                                "(or decreasing offsets) in a run; its keys past the capacity were not processed");
}

sbbf_status sbbf_grouped_counters(const sbbf_group *g, uint64_t *plans, uint64_t *graph_builds,
                                  uint64_t *graph_updates) {
  if (!g) return set_error(SBBF_EINVAL, "group is NULL");
  if (plans) *plans = g->plans;
  if (graph_builds) *graph_builds = g->graph_builds;
  if (graph_updates) *graph_updates = g->graph_updates;
  return SBBF_OK;
}

sbbf_status sbbf_grouped_get_config(const sbbf_group *g, sbbf_grouped_config *out) {
  sbbf_status st = need_plan(g);
  if (st != SBBF_OK) return st;
  if (!out) return set_error(SBBF_EINVAL, "out is NULL");
  *out = g->plan.cfg;
  return SBBF_OK;
}

sbbf_status sbbf_grouped_run(sbbf_group *g, const uint64_t *d_ins, const uint64_t *d_look, uint8_t *d_out,
                             sbbf_stream s) {
  sbbf_status st = need_fixed_plan(g);
  if (st != SBBF_OK || (st = check_io(g, d_ins, d_look, d_out)) != SBBF_OK) return st;
  const sbbf_device_info *info = current_device_info(&st);
  if (!info) return st;
  return grouped_run_graph(g, d_ins, d_look, d_out, (hipStream_t)s, *info);
}

sbbf_status sbbf_grouped_insert(sbbf_group *g, const uint64_t *d_ins, sbbf_stream s) {
  sbbf_status st = need_fixed_plan(g);
  if (st != SBBF_OK) return st;
  if (g->plan.ins_total && (!d_ins || ((uintptr_t)d_ins & 7)))
    return set_error(SBBF_EINVAL, "d_ins is NULL or not 8-byte aligned");
  const sbbf_device_info *info = current_device_info(&st);
  if (!info) return st;
  return grouped_insert_phase(g, d_ins, (hipStream_t)s, *info);
}

sbbf_status sbbf_grouped_lookup(sbbf_group *g, const uint64_t *d_look, uint8_t *d_out, sbbf_stream s) {
  sbbf_status st = need_fixed_plan(g);
  if (st != SBBF_OK) return st;
  const uint64_t nl = g->plan.look_total;
  if (nl && (!d_look || ((uintptr_t)d_look & 7) || !d_out))
    return set_error(SBBF_EINVAL, "d_look or d_out is NULL, or d_look is not 8-byte aligned");
  const sbbf_device_info *info = current_device_info(&st);
  if (!info) return st;
  return grouped_lookup_phase(g, d_look, d_out, (hipStream_t)s, *info);
}

sbbf_status sbbf_grouped_run_per_filter(sbbf_group *g, const uint64_t *d_ins, const uint64_t *d_look,
                                        uint8_t *d_out, sbbf_stream s) {
  sbbf_status st = need_fixed_plan(g);
  if (st != SBBF_OK || (st = check_io(g, d_ins, d_look, d_out)) != SBBF_OK) return st;
  const auto &io = g->plan.ins_off, &lo = g->plan.look_off;
  // The library's own choice per call, as a caller of plain launches gets it.
  for (size_t f = 0; f < g->filters.size(); ++f) {
    st = sbbf_insert_batch_ex(g->filters[f], d_ins + io[f], io[f + 1] - io[f], nullptr, s);
    if (st != SBBF_OK) return st;
  }
  for (size_t f = 0; f < g->filters.size(); ++f) {
    st = sbbf_lookup_batch_ex(g->filters[f], d_look + lo[f], lo[f + 1] - lo[f], d_out + lo[f], nullptr, nullptr, s);
    if (st != SBBF_OK) return st;
  }
  return SBBF_OK;
}

sbbf_status sbbf_grouped_digest(sbbf_group *g, const uint8_t *d_out, sbbf_stream s, uint64_t *digest) {
  if (!g || !digest) return set_error(SBBF_EINVAL, "group or digest is NULL");
  if (d_out && (!g->plan.planned || g->plan.capacity))
    return set_error(SBBF_EINVAL, "an output digest needs a plan made from host offsets");
  return group_digest(g, d_out, (hipStream_t)s, digest);
}

sbbf_status sbbf_grouped_autotune(sbbf_group *g, const uint64_t *d_ins, const uint64_t *d_look, uint8_t *d_out,
                                  uint32_t reps, const char *cache_path, int force, sbbf_grouped_config *best) {
  sbbf_status st = need_fixed_plan(g);
  if (st != SBBF_OK || (st = check_io(g, d_ins, d_look, d_out)) != SBBF_OK) return st;
  const sbbf_device_info *info = current_device_info(&st);
  if (!info) return st;
  const std::string key = tune_key(*info, g);
  const std::vector<uint64_t> ins_off = g->plan.ins_off, look_off = g->plan.look_off;
  const std::vector<uint64_t> ins_cap = g->plan.ins_cap, look_cap = g->plan.look_cap;
  if (cache_path && !force) {
    sbbf_grouped_config c;
    if (cache_lookup(cache_path, key, &c) && check_config(c, *info) == SBBF_OK) {
      if ((st = grouped_build_plan(g, ins_cap.data(), look_cap.data(), ins_off.data(), look_off.data(), c, *info)) != SBBF_OK) return st;
      if (best) *best = c;
      return SBBF_OK;
    }
  }
  if (reps == 0) reps = 5;
  // The inputs come from the caller's streams; wait for them.
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_error(e, "hipDeviceSynchronize(autotune)");
  hipStream_t s = nullptr;
  e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_error(e, "hipStreamCreate(autotune)");
  // Snapshot the filters so every candidate starts from the same contents.
  uint64_t total = 0;
  for (auto *f : g->filters) total += (uint64_t)f->num_blocks * 32u;
  char *snap = nullptr;
  e = dev_malloc((void **)&snap, total);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(s);
    return hip_error(e, "hipMalloc(autotune snapshot)");
  }
  auto copy_all = [&](bool save) {
    uint64_t at = 0;
    for (auto *f : g->filters) {
      const size_t b = (size_t)f->num_blocks * 32u;
      if (save)
        (void)hipMemcpyAsync(snap + at, f->words, b, hipMemcpyDeviceToDevice, s);
      else
        (void)hipMemcpyAsync(f->words, snap + at, b, hipMemcpyDeviceToDevice, s);
      at += b;
    }
  };
  copy_all(true);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);

  // Coordinate descent from the defaults over each parameter's candidate values.
  sbbf_grouped_config cur = default_config(*info);
  std::vector<std::pair<int, std::vector<uint64_t>>> axes = {
      {0, {4096, 16384, 65536}},  // lookup_tile_keys
      {1, {64, 128, 256}},        // lookup_threads
      {2, {1, 2, 4}},             // lookup_unroll
      {3, {2, 4, 8, 16}},         // lookup_blocks_per_cu
      {5, {0, 1}},                // xcd_queues
      {6, {16384, 65536, (uint64_t)32u << cur.insert_slice_shift}},  // insert_lds_bytes
      {7, {0, 1, 2, 4, 8, 16}},   // lookup_lds_slices
      {8, {256, 512, 1024}},      // lookup_lds_threads
  };
  auto with = [](sbbf_grouped_config c, int axis, uint64_t v) {
    switch (axis) {
      case 0: c.lookup_tile_keys = (uint32_t)v; break;
      case 1: c.lookup_threads = (uint32_t)v; break;
      case 2: c.lookup_unroll = (uint32_t)v; break;
      case 3: c.lookup_blocks_per_cu = (uint32_t)v; break;
      case 5: c.xcd_queues = (uint32_t)v; break;
      case 6: c.insert_lds_bytes = v; break;
      case 7: c.lookup_lds_slices = (uint32_t)v; break;
      case 8: c.lookup_lds_threads = (uint32_t)v; break;
    }
    return c;
  };
  bool have_ref = false;
  uint64_t ref_digest = 0;
  float best_ms = 1e30f;
  sbbf_grouped_config best_cfg = cur;
  auto measure = [&](const sbbf_grouped_config &c, float *ms) -> sbbf_status {
    sbbf_status r = grouped_build_plan(g, ins_cap.data(), look_cap.data(), ins_off.data(), look_off.data(), c, *info);
    if (r != SBBF_OK) return r;
    std::vector<float> t;
    for (uint32_t k = 0; k <= reps; ++k) {
      copy_all(false);
      (void)hipEventRecord(e0, s);
      r = grouped_run_graph(g, d_ins, d_look, d_out, s, *info);
      if (r != SBBF_OK) return r;
      (void)hipEventRecord(e1, s);
      hipError_t es = hipEventSynchronize(e1);
      if (es != hipSuccess) return hip_error(es, "autotune run");
      float v = 0;
      (void)hipEventElapsedTime(&v, e0, e1);
      if (k > 0) t.push_back(v);  // the first run warms up
    }
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    uint64_t dg = 0;
    if ((r = group_digest(g, d_out, s, &dg)) != SBBF_OK) return r;
    if (!have_ref) {
      ref_digest = dg;
      have_ref = true;
    } else if (dg != ref_digest) {
      return set_error(SBBF_EDEVICE, "autotune candidate produced different results");
    }
    return SBBF_OK;
  };
  float ms = 0;
  st = measure(cur, &ms);
  if (st == SBBF_OK) {
    best_ms = ms;
    best_cfg = cur;
    for (int sweep = 0; sweep < 2 && st == SBBF_OK; ++sweep) {
      for (auto &ax : axes) {
        for (uint64_t v : ax.second) {
          sbbf_grouped_config c = with(best_cfg, ax.first, v);
          if (memcmp(&c, &best_cfg, sizeof(c)) == 0 || check_config(c, *info) != SBBF_OK) continue;
          if ((st = measure(c, &ms)) != SBBF_OK) break;
          if (ms < best_ms) {
            best_ms = ms;
            best_cfg = c;
          }
        }
        if (st != SBBF_OK) break;
      }
    }
  }
  copy_all(false);  // leave the filters as they were
  hipError_t es = hipStreamSynchronize(s);
  (void)hipFree(snap);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  if (st != SBBF_OK) return st;
  if (es != hipSuccess) return hip_error(es, "autotune synchronise");
  if ((st = grouped_build_plan(g, ins_cap.data(), look_cap.data(), ins_off.data(), look_off.data(), best_cfg, *info)) != SBBF_OK) return st;
  if (cache_path) cache_store(cache_path, key, best_cfg);
  if (best) *best = best_cfg;
  return SBBF_OK;
}

}  // extern "C"
