// Partitioned insert and lookup: filters larger than one workgroup's LDS
// processed slice by slice, with streaming memory traffic only.
//
// The filter is cut into slices of S = 2^slice_shift consecutive blocks (a
// slice fits one workgroup's LDS). Block selection is monotone in the high
// half of the hash, so every key belongs to exactly one slice. The batch is
// cut into G contiguous chunks, one per partitioning workgroup. Kernels:
//
//   count     workgroup g counts the keys of chunk g per slice -> hist[g][s]
//   colscan   start[g][s] = sum of hist[< g][s]; tot[s] = sum over g
//   offsets   offsets[s] = sum of tot[< s]: where slice s begins
//   scatter   workgroup g walks chunk g in tiles, sorts each tile by slice in
//             LDS and writes each slice's run with consecutive lanes at the
//             slice cursor offsets[s] + start[g][s] + (keys already written);
//             for lookups it also records pos[i], where key i went
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
// pure and return to input order through pos. Positions are 32-bit: one
// launch handles fewer than 2^32 keys (the C ABI splits larger batches).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"
#include "sbbf_device.h"

namespace sbbf {
namespace {

constexpr uint32_t kPartThreads = 1024;                          // count, scan, slice and unpermute kernels
constexpr uint32_t kScatterThreads = 512;
constexpr uint32_t kScatterPerThread = 8;
constexpr uint32_t kTile = kScatterThreads * kScatterPerThread;  // keys per scatter tile
constexpr int kSliceUnroll = 8;                                  // 64-key chunks per wave per iteration
constexpr uint32_t kColsPerScanBlock = 64;
// Lookup chunks are at most this many keys so that one chunk's result bytes
// fit one workgroup's LDS in the unpermute kernel.
constexpr uint32_t kLookupChunk = 128u * 1024u;

__device__ __forceinline__ uint32_t slice_of(uint64_t h, uint32_t num_blocks, uint32_t slice_shift) {
  return block_of((uint32_t)(h >> 32), num_blocks) >> slice_shift;
}

// Exclusive prefix sum of in[0..count) into out[0..count) by the whole
// workgroup (blockDim.x a multiple of 64, at most 1024). `wsum` holds 16
// words of LDS scratch. Contains barriers: every thread must call it.
__device__ void block_exclusive_scan(const uint32_t *in, uint32_t *out, uint32_t count, uint32_t *wsum) {
  const uint32_t per = (count + blockDim.x - 1) / blockDim.x;
  const uint32_t b = threadIdx.x * per;
  const uint32_t e = min(b + per, count);
  uint32_t sum = 0;
  for (uint32_t i = b; i < e; ++i) sum += in[i];
  const uint32_t lane = threadIdx.x & 63u;
  uint32_t x = sum;  // inclusive scan over the wave
  for (uint32_t d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x < 64) {
    const uint32_t nw = blockDim.x >> 6;
    const uint32_t v = threadIdx.x < nw ? wsum[threadIdx.x] : 0u;
    uint32_t z = v;
    for (uint32_t d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(z, d, 64);
      if (lane >= d) z += y;
    }
    if (threadIdx.x < nw) wsum[threadIdx.x] = z - v;  // exclusive over waves
  }
  __syncthreads();
  uint32_t run = wsum[threadIdx.x >> 6] + x - sum;
  for (uint32_t i = b; i < e; ++i) {
    out[i] = run;
    run += in[i];
  }
  __syncthreads();
}

__device__ __forceinline__ void chunk_range(uint32_t g, uint32_t chunk, uint32_t n, uint32_t *b, uint32_t *e) {
  const uint64_t lo = (uint64_t)g * chunk;
  *b = (uint32_t)min<uint64_t>(lo, n);
  *e = (uint32_t)min<uint64_t>(lo + chunk, n);
}

__global__ void __launch_bounds__(kPartThreads)
part_count_kernel(const uint64_t *__restrict__ hashes, uint32_t n, uint32_t chunk, uint32_t num_blocks,
                  uint32_t slice_shift, uint32_t num_slices, uint32_t *__restrict__ hist_out) {
  extern __shared__ uint32_t hist[];
  for (uint32_t i = threadIdx.x; i < num_slices; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  uint32_t b, e;
  chunk_range(blockIdx.x, chunk, n, &b, &e);
  for (uint32_t i = b + threadIdx.x; i < e; i += blockDim.x) {
    const uint32_t s = slice_of(load_hash<0>(hashes + i), num_blocks, slice_shift);
    __hip_atomic_fetch_add(hist + s, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __syncthreads();
  uint32_t *row = hist_out + (uint64_t)blockIdx.x * num_slices;
  for (uint32_t i = threadIdx.x; i < num_slices; i += blockDim.x) row[i] = hist[i];
}

// Column prefix sums of hist[groups][num_slices]. A workgroup handles 64
// columns with 16 threads per column, each summing a contiguous run of rows.
__global__ void __launch_bounds__(kPartThreads)
part_colscan_kernel(const uint32_t *__restrict__ hist, uint32_t groups, uint32_t num_slices,
                    uint32_t *__restrict__ start, uint32_t *__restrict__ tot) {
  __shared__ uint32_t seg_sum[kPartThreads / kColsPerScanBlock][kColsPerScanBlock];
  constexpr uint32_t kSegs = kPartThreads / kColsPerScanBlock;
  const uint32_t c = threadIdx.x % kColsPerScanBlock;
  const uint32_t seg = threadIdx.x / kColsPerScanBlock;
  const uint32_t col = blockIdx.x * kColsPerScanBlock + c;
  const uint32_t rows = (groups + kSegs - 1) / kSegs;
  const uint32_t r0 = min(seg * rows, groups);
  const uint32_t r1 = min(r0 + rows, groups);
  uint32_t sum = 0;
  if (col < num_slices)
    for (uint32_t r = r0; r < r1; ++r) sum += hist[(uint64_t)r * num_slices + col];
  seg_sum[seg][c] = sum;
  __syncthreads();
  uint32_t run = 0;
  for (uint32_t k = 0; k < seg; ++k) run += seg_sum[k][c];
  if (col < num_slices) {
    for (uint32_t r = r0; r < r1; ++r) {
      start[(uint64_t)r * num_slices + col] = run;
      run += hist[(uint64_t)r * num_slices + col];
    }
    if (seg == kSegs - 1) tot[col] = run;
  }
}

// One workgroup: offsets[s] = sum of tot[< s]; offsets[num_slices] = total.
__global__ void __launch_bounds__(kPartThreads)
part_offsets_kernel(const uint32_t *__restrict__ tot, uint32_t num_slices, uint32_t *__restrict__ offsets) {
  __shared__ uint32_t wsum[16];
  // block_exclusive_scan reads `in` from any memory; offsets[] is the output.
  block_exclusive_scan(tot, offsets, num_slices, wsum);
  if (threadIdx.x == 0) offsets[num_slices] = offsets[num_slices - 1] + tot[num_slices - 1];
}

constexpr size_t scatter_lds_bytes(uint32_t num_slices) {
  return (size_t)kTile * 8u + (size_t)kTile * 2u + (size_t)num_slices * 16u + 64u;
}

// Workgroup g partitions chunk g. For lookups it also writes, for every key i
// of the chunk, its position inside the chunk's own results (the chunk's runs
// of all slices laid end to end in slice order), which is what the unpermute
// kernel reads back from LDS.
template <bool kWithPos>
__global__ void __launch_bounds__(kScatterThreads)
part_scatter_kernel(const uint64_t *__restrict__ hashes, uint32_t n, uint32_t chunk, uint32_t num_blocks,
                    uint32_t slice_shift, uint32_t num_slices, const uint32_t *__restrict__ offsets,
                    const uint32_t *__restrict__ start, const uint32_t *__restrict__ hist_rows,
                    uint64_t *__restrict__ out_keys, uint32_t *__restrict__ out_pos) {
  extern __shared__ unsigned long long smem[];
  unsigned long long *stage_keys = smem;                                    // [kTile]
  uint16_t *stage_slice = reinterpret_cast<uint16_t *>(stage_keys + kTile);  // [kTile]
  uint32_t *cursor = reinterpret_cast<uint32_t *>(stage_slice + kTile);      // [num_slices]
  uint32_t *hist = cursor + num_slices;                                      // [num_slices]
  uint32_t *loff = hist + num_slices;                                        // [num_slices]
  uint32_t *local = loff + num_slices;                                       // [num_slices] (lookups)
  uint32_t *wsum = local + num_slices;                                       // [16]

  const uint32_t *my_start = start + (uint64_t)blockIdx.x * num_slices;
  for (uint32_t i = threadIdx.x; i < num_slices; i += blockDim.x) cursor[i] = offsets[i] + my_start[i];
  if constexpr (kWithPos) {
    // local[s]: where slice s's run starts among this chunk's results; then
    // turned into local[s] - (first cursor of s), so that a key's position in
    // the chunk's results is local[s] + cursor[s] + rank.
    block_exclusive_scan(hist_rows + (uint64_t)blockIdx.x * num_slices, local, num_slices, wsum);
    for (uint32_t i = threadIdx.x; i < num_slices; i += blockDim.x) local[i] -= cursor[i];
  }
  uint32_t b, e;
  chunk_range(blockIdx.x, chunk, n, &b, &e);
  // Indices past the chunk are clamped to its last key so loads never branch;
  // such lanes add 0 to the histogram and write nothing.
  uint64_t h[kScatterPerThread];
#pragma unroll
  for (uint32_t t = 0; t < kScatterPerThread; ++t) {
    const uint32_t i = b + t * blockDim.x + threadIdx.x;
    h[t] = load_hash<0>(hashes + (i < e ? i : e - 1u));
  }
  for (uint32_t tile0 = b; tile0 < e; tile0 += kTile) {
    for (uint32_t i = threadIdx.x; i < num_slices; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    uint32_t s[kScatterPerThread], rank[kScatterPerThread];
#pragma unroll
    for (uint32_t t = 0; t < kScatterPerThread; ++t) {
      const uint32_t i = tile0 + t * blockDim.x + threadIdx.x;
      s[t] = slice_of(h[t], num_blocks, slice_shift);
      rank[t] = __hip_atomic_fetch_add(hist + s[t], i < e ? 1u : 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    // Load the next tile now, so the loads overlap the scan, staging and writes.
    uint64_t next[kScatterPerThread];
#pragma unroll
    for (uint32_t t = 0; t < kScatterPerThread; ++t) {
      const uint32_t i = tile0 + kTile + t * blockDim.x + threadIdx.x;
      next[t] = load_hash<0>(hashes + (i < e ? i : e - 1u));
    }
    __syncthreads();
    block_exclusive_scan(hist, loff, num_slices, wsum);
#pragma unroll
    for (uint32_t t = 0; t < kScatterPerThread; ++t) {
      const uint32_t i = tile0 + t * blockDim.x + threadIdx.x;
      if (i < e) {
        const uint32_t k = loff[s[t]] + rank[t];
        stage_keys[k] = h[t];
        stage_slice[k] = (uint16_t)s[t];
        if constexpr (kWithPos) out_pos[i] = local[s[t]] + cursor[s[t]] + rank[t];
      }
    }
    __syncthreads();
    const uint32_t count = min(kTile, e - tile0);
    uint32_t sl[kScatterPerThread];
    unsigned long long key[kScatterPerThread];
#pragma unroll
    for (uint32_t t = 0; t < kScatterPerThread; ++t) {
      const uint32_t k = t * blockDim.x + threadIdx.x;
      sl[t] = k < count ? stage_slice[k] : 0u;
      key[t] = stage_keys[k];
    }
#pragma unroll
    for (uint32_t t = 0; t < kScatterPerThread; ++t) {
      const uint32_t k = t * blockDim.x + threadIdx.x;
      const uint32_t dst = cursor[sl[t]] + (k - loff[sl[t]]);
      if (k < count) out_keys[dst] = key[t];
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < num_slices; i += blockDim.x) cursor[i] += hist[i];
    // (the barrier at the top of the next tile orders these updates)
#pragma unroll
    for (uint32_t t = 0; t < kScatterPerThread; ++t) h[t] = next[t];
  }
}

__device__ __forceinline__ void load_slice_to_lds(uint4 *lds4, const uint32_t *words, uint32_t b0, uint32_t nb) {
  const uint4 *src4 = reinterpret_cast<const uint4 *>(words + (uint64_t)b0 * 8u);
  for (uint32_t i = threadIdx.x; i < nb * 2u; i += blockDim.x) lds4[i] = src4[i];
}

// Slice kernels use four lanes per key: lane l owns words 2q and 2q+1
// (q = l % 4) of the block as one 64-bit LDS word. In pass p (0..3) the four
// lanes of group g (lanes 4g..4g+3) take key 4g + p of a 64-key chunk and
// load its hash directly (the four lanes read the same address), so a chunk
// needs four loads and four 64-bit LDS operations per lane. Lanes past the
// slice's last key load that last key instead (a real key of the slice, so
// every LDS index stays in range); inserting it again changes nothing, and
// lookup results of those lanes are not written. This keeps the loops free of
// branches so all loads, then all LDS accesses, are issued back to back.
template <int U>
__device__ __forceinline__ void load_pass_hashes(const uint64_t *__restrict__ keys, uint32_t n, uint32_t base,
                                                 uint32_t group4, uint64_t (&h)[U][4]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const uint32_t i = base + 64u * u + group4 + p;
      h[u][p] = load_hash<0>(keys + (i < n ? i : n - 1u));
    }
  }
}

template <int U>
__global__ void __launch_bounds__(kPartThreads)
part_slice_insert_kernel(const uint64_t *__restrict__ part, const uint32_t *__restrict__ offsets,
                         uint32_t *__restrict__ words, uint32_t num_blocks, uint32_t slice_shift) {
  extern __shared__ uint4 lds4[];
  unsigned long long *lds2 = reinterpret_cast<unsigned long long *>(lds4);
  const uint32_t slice = blockIdx.x;
  const uint32_t b0 = slice << slice_shift;
  const uint32_t nb = min(1u << slice_shift, num_blocks - b0);
  load_slice_to_lds(lds4, words, b0, nb);
  __syncthreads();

  const uint32_t begin = offsets[slice];
  const uint32_t n = offsets[slice + 1] - begin;
  const uint64_t *keys = part + begin;
  const uint32_t lane = lane_id();
  const uint32_t q = lane & 3u;
  const uint32_t group4 = lane & ~3u;
  const uint32_t seed_lo = seed_of_word(2u * q);
  const uint32_t seed_hi = seed_of_word(2u * q + 1u);
  const uint32_t waves = blockDim.x / kWave;
  constexpr uint32_t kChunk = 64u * U;
  for (uint32_t base = (threadIdx.x / kWave) * kChunk; base < n; base += waves * kChunk) {
    uint64_t h[U][4];
    load_pass_hashes<U>(keys, n, base, group4, h);
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const uint32_t b = block_of((uint32_t)(h[u][p] >> 32), num_blocks) - b0;
        const uint32_t x = (uint32_t)h[u][p];
        const unsigned long long m = (unsigned long long)(1u << bit_of(seed_lo, x)) |
                                     ((unsigned long long)(1u << bit_of(seed_hi, x)) << 32);
        __hip_atomic_fetch_or(lds2 + b * 4u + q, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  }
  __syncthreads();
  uint4 *dst4 = reinterpret_cast<uint4 *>(words + (uint64_t)b0 * 8u);
  for (uint32_t i = threadIdx.x; i < nb * 2u; i += blockDim.x) dst4[i] = lds4[i];
}

template <int U>
__global__ void __launch_bounds__(kPartThreads)
part_slice_lookup_kernel(const uint64_t *__restrict__ part, const uint32_t *__restrict__ offsets,
                         const uint32_t *__restrict__ words, uint32_t num_blocks, uint32_t slice_shift,
                         uint8_t *__restrict__ res) {
  extern __shared__ uint4 lds4[];
  const unsigned long long *lds2 = reinterpret_cast<const unsigned long long *>(lds4);
  const uint32_t slice = blockIdx.x;
  const uint32_t b0 = slice << slice_shift;
  const uint32_t nb = min(1u << slice_shift, num_blocks - b0);
  load_slice_to_lds(lds4, words, b0, nb);
  __syncthreads();

  const uint32_t begin = offsets[slice];
  const uint32_t n = offsets[slice + 1] - begin;
  const uint64_t *keys = part + begin;
  uint8_t *out = res + begin;
  const uint32_t lane = lane_id();
  const uint32_t q = lane & 3u;
  const uint32_t group4 = lane & ~3u;
  const uint32_t seed_lo = seed_of_word(2u * q);
  const uint32_t seed_hi = seed_of_word(2u * q + 1u);
  const uint32_t waves = blockDim.x / kWave;
  constexpr uint32_t kChunk = 64u * U;
  for (uint32_t base = (threadIdx.x / kWave) * kChunk; base < n; base += waves * kChunk) {
    uint64_t h[U][4];
    load_pass_hashes<U>(keys, n, base, group4, h);
    unsigned long long w[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int p = 0; p < 4; ++p) w[u][p] = lds2[(block_of((uint32_t)(h[u][p] >> 32), num_blocks) - b0) * 4u + q];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      uint64_t r = 0;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const uint32_t x = (uint32_t)h[u][p];
        const uint32_t hit = (uint32_t)(w[u][p] >> bit_of(seed_lo, x)) & (uint32_t)(w[u][p] >> (32u + bit_of(seed_hi, x))) & 1u;
        // Byte g of ballot p holds (in its bits 4g..4g+3) the four tests of key 4g + p.
        const uint64_t m = ballot(hit != 0u);
        uint64_t t = m & (m >> 2);
        t &= t >> 1;
        r |= (t & 0x1111111111111111ull) << p;
      }
      const uint32_t i = base + 64u * u + lane;
      if (i < n) out[i] = (uint8_t)((r >> lane) & 1u);
    }
  }
}

// Workgroup g restores input order for chunk g: it copies the chunk's result
// run of every slice (res[offsets[s] + start[g][s] ...], hist[g][s] bytes)
// into LDS end to end in slice order, then writes out[i] = lds[pos[i]] for
// the chunk, as bytes or packed bits (LSB-first).
template <bool kBits>
__global__ void __launch_bounds__(kPartThreads)
part_unpermute_kernel(const uint32_t *__restrict__ pos, const uint8_t *__restrict__ res,
                      const uint32_t *__restrict__ offsets, const uint32_t *__restrict__ start,
                      const uint32_t *__restrict__ hist_rows, uint32_t num_slices, uint32_t n, uint32_t chunk,
                      uint8_t *__restrict__ out8, uint32_t *__restrict__ out_bits) {
  extern __shared__ uint32_t usmem[];
  uint32_t *local = usmem;                                 // [num_slices]
  uint32_t *wsum = local + num_slices;                     // [16]
  uint8_t *vals = reinterpret_cast<uint8_t *>(wsum + 16);  // [chunk]
  const uint32_t *row = hist_rows + (uint64_t)blockIdx.x * num_slices;
  const uint32_t *my_start = start + (uint64_t)blockIdx.x * num_slices;
  block_exclusive_scan(row, local, num_slices, wsum);
  // Phase 1: thread t copies the runs of slices t, t + blockDim.x, ... with
  // aligned 4-byte loads (res has at least 4 bytes of padding after its last
  // byte, so the last word of a run is always inside the workspace).
  for (uint32_t sl = threadIdx.x; sl < num_slices; sl += blockDim.x) {
    const uint32_t len = row[sl];
    const uint32_t src = offsets[sl] + my_start[sl];  // byte index into res
    uint8_t *dst = vals + local[sl];
    const uint32_t w_begin = src >> 2, w_end = (src + len + 3u) >> 2;
    const uint32_t *res4 = reinterpret_cast<const uint32_t *>(res);
    for (uint32_t w0 = w_begin; w0 < w_end; w0 += 8u) {
      uint32_t v[8];
#pragma unroll
      for (uint32_t k = 0; k < 8u; ++k) v[k] = w0 + k < w_end ? res4[w0 + k] : 0u;
#pragma unroll
      for (uint32_t k = 0; k < 8u; ++k) {
#pragma unroll
        for (uint32_t by = 0; by < 4u; ++by) {
          const uint32_t at = (w0 + k) * 4u + by;  // byte index into res
          if (at >= src && at < src + len) dst[at - src] = (uint8_t)(v[k] >> (8u * by));
        }
      }
    }
  }
  __syncthreads();
  uint32_t b, e;
  chunk_range(blockIdx.x, chunk, n, &b, &e);
  const uint32_t lane = threadIdx.x & 63u;
  if constexpr (!kBits) {
    // Phase 2 (bytes): four consecutive positions per thread; b is a multiple of 4.
    const bool aligned4 = ((uintptr_t)out8 & 3u) == 0;
    for (uint32_t i = b + 4u * threadIdx.x; i < e; i += 4u * blockDim.x) {
      if (i + 4u <= e) {
        const uint4 p4 = *reinterpret_cast<const uint4 *>(pos + i);
        const uint32_t word = (uint32_t)vals[p4.x] | ((uint32_t)vals[p4.y] << 8) | ((uint32_t)vals[p4.z] << 16) |
                              ((uint32_t)vals[p4.w] << 24);
        if (aligned4) {
          *reinterpret_cast<uint32_t *>(out8 + i) = word;
        } else {
          for (uint32_t k = 0; k < 4u; ++k) out8[i + k] = (uint8_t)(word >> (8u * k));
        }
      } else {
        for (uint32_t k = i; k < e; ++k) out8[k] = vals[pos[k]];
      }
    }
  } else {
    // Phase 2 (bits): one position per lane. i0 is wave-uniform (chunks start
    // at multiples of 64), so every lane of a wave runs the same iterations
    // and the ballot sees the whole wave.
    for (uint32_t i0 = b + (threadIdx.x & ~63u); i0 < e; i0 += blockDim.x) {
      const uint32_t i = i0 + lane;
      const uint8_t r = i < e ? vals[pos[i]] : (uint8_t)0;
      const uint64_t m = ballot(r != 0);
      if (lane == 0) out_bits[i0 / 32u] = (uint32_t)m;
      if (lane == 1 && n - i0 > 32u) out_bits[i0 / 32u + 1u] = (uint32_t)(m >> 32);
    }
  }
}

// Workspace sections (each 256-byte aligned): hist[G][P], start[G][P], tot[P],
// offsets[P + 1] (u32), keys[n] (u64) and, for lookups, pos[n] (u32), res[n] (u8).
struct PartitionLayout {
  uint32_t *hist, *start, *tot, *offsets;
  uint64_t *keys;
  uint32_t *pos;
  uint8_t *res;
  uint64_t bytes;
};

PartitionLayout layout(void *workspace, uint64_t n, uint32_t num_slices, uint32_t groups, bool lookup) {
  auto up = [](uint64_t v) { return (v + 255u) & ~(uint64_t)255u; };
  char *base = static_cast<char *>(workspace);
  uint64_t off = 0;
  PartitionLayout L{};
  L.hist = reinterpret_cast<uint32_t *>(base + off);
  off += up((uint64_t)groups * num_slices * 4u);
  L.start = reinterpret_cast<uint32_t *>(base + off);
  off += up((uint64_t)groups * num_slices * 4u);
  L.tot = reinterpret_cast<uint32_t *>(base + off);
  off += up((uint64_t)num_slices * 4u);
  L.offsets = reinterpret_cast<uint32_t *>(base + off);
  off += up(((uint64_t)num_slices + 1u) * 4u);
  L.keys = reinterpret_cast<uint64_t *>(base + off);
  off += up(n * 8u);
  if (lookup) {
    L.pos = reinterpret_cast<uint32_t *>(base + off);
    off += up(n * 4u);
    L.res = reinterpret_cast<uint8_t *>(base + off);
    off += up(n + 4u);  // 4 bytes of padding for the unpermute kernel's word loads
  }
  L.bytes = off;
  return L;
}

// Chunking of n keys over about max_groups partitioning workgroups: chunk is
// a multiple of the scatter tile, at most kLookupChunk keys for lookups (so
// there may be more groups than max_groups), and every group gets a
// non-empty chunk.
void chunking(uint64_t n, uint32_t max_groups, bool lookup, uint32_t *chunk, uint32_t *groups) {
  const uint64_t tiles = (n + kTile - 1) / kTile;
  const uint64_t g0 = tiles < max_groups ? (tiles ? tiles : 1) : max_groups;
  uint64_t tiles_per = (tiles + g0 - 1) / g0;
  if (lookup && tiles_per * kTile > kLookupChunk) tiles_per = kLookupChunk / kTile;
  *chunk = (uint32_t)(tiles_per * kTile);
  *groups = (uint32_t)((n + *chunk - 1) / *chunk);
  if (*groups == 0) *groups = 1;
}

hipError_t partition(const uint64_t *hashes, uint32_t n, uint32_t num_blocks, uint32_t slice_shift,
                     uint32_t num_slices, uint32_t chunk, uint32_t groups, const PartitionLayout &L, bool with_pos,
                     hipStream_t stream) {
  hipError_t e;
  const dim3 blk(kPartThreads);
  const size_t sc_lds = scatter_lds_bytes(num_slices);
  // Dynamic LDS above the default needs the per-kernel limit raised; an error
  // here shows up at launch.
  (void)hipFuncSetAttribute((const void *)part_count_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(num_slices * 4u));
  (void)hipFuncSetAttribute((const void *)part_scatter_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sc_lds);
  (void)hipFuncSetAttribute((const void *)part_scatter_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sc_lds);
  (void)hipGetLastError();
  hipLaunchKernelGGL(part_count_kernel, dim3(groups), blk, num_slices * 4u, stream, hashes, n, chunk, num_blocks,
                     slice_shift, num_slices, L.hist);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(part_colscan_kernel, dim3((num_slices + kColsPerScanBlock - 1) / kColsPerScanBlock), blk, 0,
                     stream, L.hist, groups, num_slices, L.start, L.tot);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(part_offsets_kernel, dim3(1), blk, 0, stream, L.tot, num_slices, L.offsets);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const dim3 sblk(kScatterThreads);
  if (with_pos)
    hipLaunchKernelGGL(part_scatter_kernel<true>, dim3(groups), sblk, sc_lds, stream, hashes, n, chunk, num_blocks,
                       slice_shift, num_slices, L.offsets, L.start, L.hist, L.keys, L.pos);
  else
    hipLaunchKernelGGL(part_scatter_kernel<false>, dim3(groups), sblk, sc_lds, stream, hashes, n, chunk, num_blocks,
                       slice_shift, num_slices, L.offsets, L.start, L.hist, L.keys, nullptr);
  return hipGetLastError();
}

uint32_t slices_of(uint32_t num_blocks, uint32_t slice_shift) {
  return (uint32_t)(((uint64_t)num_blocks + (1u << slice_shift) - 1u) >> slice_shift);
}

}  // namespace

uint32_t partition_max_slices() { return 4096; }
uint64_t partition_max_keys() { return 1ull << 31; }

uint64_t partition_workspace_bytes(uint64_t n, uint32_t num_slices, uint32_t max_groups, bool lookup) {
  uint32_t chunk, groups;
  chunking(n, max_groups, lookup, &chunk, &groups);
  return layout(nullptr, n, num_slices, groups, lookup).bytes;
}

hipError_t launch_insert_partitioned(const uint64_t *hashes, uint64_t n, uint32_t *words, uint32_t num_blocks,
                                     uint32_t slice_shift, void *workspace, uint32_t max_groups,
                                     hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const uint32_t num_slices = slices_of(num_blocks, slice_shift);
  if (num_slices > partition_max_slices() || n > partition_max_keys()) return hipErrorInvalidValue;
  uint32_t chunk, groups;
  chunking(n, max_groups, false, &chunk, &groups);
  const PartitionLayout L = layout(workspace, n, num_slices, groups, false);
  hipError_t e = partition(hashes, (uint32_t)n, num_blocks, slice_shift, num_slices, chunk, groups, L, false, stream);
  if (e != hipSuccess) return e;
  const size_t lds_bytes = ((size_t)1 << slice_shift) * 32u;
  (void)hipFuncSetAttribute((const void *)part_slice_insert_kernel<kSliceUnroll>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  (void)hipGetLastError();
  hipLaunchKernelGGL(part_slice_insert_kernel<kSliceUnroll>, dim3(num_slices), dim3(kPartThreads), lds_bytes, stream,
                     L.keys, L.offsets, words, num_blocks, slice_shift);
  return hipGetLastError();
}

hipError_t launch_lookup_partitioned(const uint64_t *hashes, uint64_t n, const uint32_t *words, uint32_t num_blocks,
                                     uint32_t slice_shift, void *workspace, uint32_t max_groups, uint8_t *out8,
                                     uint32_t *out_bits, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const uint32_t num_slices = slices_of(num_blocks, slice_shift);
  if (num_slices > partition_max_slices() || n > partition_max_keys()) return hipErrorInvalidValue;
  uint32_t chunk, groups;
  chunking(n, max_groups, true, &chunk, &groups);
  const PartitionLayout L = layout(workspace, n, num_slices, groups, true);
  hipError_t e = partition(hashes, (uint32_t)n, num_blocks, slice_shift, num_slices, chunk, groups, L, true, stream);
  if (e != hipSuccess) return e;
  const size_t lds_bytes = ((size_t)1 << slice_shift) * 32u;
  (void)hipFuncSetAttribute((const void *)part_slice_lookup_kernel<kSliceUnroll>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  (void)hipGetLastError();
  hipLaunchKernelGGL(part_slice_lookup_kernel<kSliceUnroll>, dim3(num_slices), dim3(kPartThreads), lds_bytes, stream,
                     L.keys, L.offsets, words, num_blocks, slice_shift, L.res);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t u_lds = (size_t)num_slices * 4u + 64u + chunk;
  (void)hipFuncSetAttribute((const void *)part_unpermute_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)u_lds);
  (void)hipFuncSetAttribute((const void *)part_unpermute_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)u_lds);
  (void)hipGetLastError();
  if (out_bits)
    hipLaunchKernelGGL(part_unpermute_kernel<true>, dim3(groups), dim3(kPartThreads), u_lds, stream, L.pos, L.res,
                       L.offsets, L.start, L.hist, num_slices, (uint32_t)n, chunk, nullptr, out_bits);
  else
    hipLaunchKernelGGL(part_unpermute_kernel<false>, dim3(groups), dim3(kPartThreads), u_lds, stream, L.pos, L.res,
                       L.offsets, L.start, L.hist, num_slices, (uint32_t)n, chunk, out8, nullptr);
  return hipGetLastError();
}

}  // namespace sbbf
