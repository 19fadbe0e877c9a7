// Partitioned insert: inserts into a filter larger than one workgroup's LDS
// without global atomics.
//
// The filter is cut into slices of S = 2^slice_shift consecutive blocks (a
// slice fits one workgroup's LDS). Because block selection is monotone in the
// high half of the hash, every key belongs to exactly one slice. Four kernels:
//
//   count    per-slice key counts (LDS histogram per workgroup, merged with
//            one global atomic add per non-empty bin)
//   scan     exclusive prefix sum of the counts -> slice offsets and cursors
//   scatter  each workgroup bins a tile of keys in LDS, claims a contiguous
//            range per slice with one atomic add, and writes the keys there
//            (runs of keys of one slice are written together)
//   slice    one workgroup per slice: load the slice into LDS, OR every key
//            of the slice into it, store the slice back with plain stores
//
// The final filter is the OR of all masks, so the order of keys inside a
// slice (which the atomic cursor makes arbitrary) does not affect it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"
#include "sbbf_device.h"

namespace sbbf {
namespace {

constexpr uint32_t kPartThreads = 1024;
constexpr uint32_t kScatterPerThread = 8;  // keys per thread per scatter tile

__device__ __forceinline__ uint32_t slice_of(uint64_t h, uint32_t num_blocks, uint32_t slice_shift) {
  return block_of((uint32_t)(h >> 32), num_blocks) >> slice_shift;
}

__global__ void __launch_bounds__(kPartThreads)
part_count_kernel(const uint64_t *__restrict__ hashes, uint64_t n, uint32_t num_blocks, uint32_t slice_shift,
                  uint32_t num_slices, unsigned long long *__restrict__ counts) {
  extern __shared__ uint32_t hist[];
  for (uint32_t i = threadIdx.x; i < num_slices; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint32_t s = slice_of(load_hash<0>(hashes + i), num_blocks, slice_shift);
    __hip_atomic_fetch_add(hist + s, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < num_slices; i += blockDim.x) {
    const uint32_t c = hist[i];
    if (c) __hip_atomic_fetch_add(counts + i, (unsigned long long)c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One workgroup of kPartThreads threads: offsets[s] = sum of counts[< s],
// offsets[num_slices] = total; cursors[s] = offsets[s].
__global__ void __launch_bounds__(kPartThreads)
part_scan_kernel(const unsigned long long *__restrict__ counts, uint32_t num_slices,
                 unsigned long long *__restrict__ offsets, unsigned long long *__restrict__ cursors) {
  __shared__ unsigned long long partial[kPartThreads];
  const uint32_t per = (num_slices + blockDim.x - 1) / blockDim.x;
  const uint32_t b = threadIdx.x * per;
  const uint32_t e = min(b + per, num_slices);
  unsigned long long sum = 0;
  for (uint32_t i = b; i < e; ++i) sum += counts[i];
  partial[threadIdx.x] = sum;
  __syncthreads();
  // Hillis-Steele inclusive scan over the per-thread sums.
  for (uint32_t d = 1; d < blockDim.x; d <<= 1) {
    const unsigned long long v = threadIdx.x >= d ? partial[threadIdx.x - d] : 0ull;
    __syncthreads();
    partial[threadIdx.x] += v;
    __syncthreads();
  }
  unsigned long long run = partial[threadIdx.x] - sum;  // exclusive
  for (uint32_t i = b; i < e; ++i) {
    offsets[i] = run;
    cursors[i] = run;
    run += counts[i];
  }
  if (threadIdx.x == blockDim.x - 1) offsets[num_slices] = partial[threadIdx.x];
}

__global__ void __launch_bounds__(kPartThreads)
part_scatter_kernel(const uint64_t *__restrict__ hashes, uint64_t n, uint32_t num_blocks, uint32_t slice_shift,
                    uint32_t num_slices, unsigned long long *__restrict__ cursors, uint64_t *__restrict__ out) {
  extern __shared__ unsigned long long smem[];
  unsigned long long *base = smem;                                  // [num_slices]
  uint32_t *hist = reinterpret_cast<uint32_t *>(smem + num_slices);  // [num_slices]
  const uint64_t tile_keys = (uint64_t)blockDim.x * kScatterPerThread;
  for (uint64_t tile = blockIdx.x; tile * tile_keys < n; tile += gridDim.x) {
    for (uint32_t i = threadIdx.x; i < num_slices; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    uint64_t h[kScatterPerThread];
    uint32_t s[kScatterPerThread], rank[kScatterPerThread];
#pragma unroll
    for (uint32_t t = 0; t < kScatterPerThread; ++t) {
      const uint64_t i = tile * tile_keys + (uint64_t)t * blockDim.x + threadIdx.x;
      h[t] = i < n ? load_hash<0>(hashes + i) : 0ull;
      s[t] = slice_of(h[t], num_blocks, slice_shift);
      rank[t] = i < n ? __hip_atomic_fetch_add(hist + s[t], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)
                      : 0u;
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < num_slices; i += blockDim.x) {
      const uint32_t c = hist[i];
      if (c)
        base[i] = __hip_atomic_fetch_add(cursors + i, (unsigned long long)c, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
#pragma unroll
    for (uint32_t t = 0; t < kScatterPerThread; ++t) {
      const uint64_t i = tile * tile_keys + (uint64_t)t * blockDim.x + threadIdx.x;
      if (i < n) out[base[s[t]] + rank[t]] = h[t];
    }
    __syncthreads();
  }
}

// One workgroup per slice. Waves take 64-key chunks of the slice's key range
// with the same 8-lane layout as the other inserts.
template <int U>
__global__ void __launch_bounds__(kPartThreads)
part_slice_insert_kernel(const uint64_t *__restrict__ part, const unsigned long long *__restrict__ offsets,
                         uint32_t *__restrict__ words, uint32_t num_blocks, uint32_t slice_shift) {
  extern __shared__ uint4 lds4[];
  uint32_t *lds = reinterpret_cast<uint32_t *>(lds4);
  const uint32_t slice = blockIdx.x;
  const uint32_t b0 = slice << slice_shift;
  const uint32_t nb = min(1u << slice_shift, num_blocks - b0);
  const uint4 *src4 = reinterpret_cast<const uint4 *>(words + (uint64_t)b0 * 8u);
  for (uint32_t i = threadIdx.x; i < nb * 2u; i += blockDim.x) lds4[i] = src4[i];
  __syncthreads();

  const uint64_t begin = offsets[slice];
  const uint64_t n = offsets[slice + 1] - begin;
  const uint64_t *hashes = part + begin;
  const uint32_t lane = lane_id();
  const uint32_t j = lane & 7u;
  const uint32_t group = lane & ~7u;
  const uint32_t seed = seed_of_word(j);
  const uint32_t waves = blockDim.x / kWave;
  constexpr uint64_t kChunk = (uint64_t)kWave * U;
  for (uint64_t base = (uint64_t)(threadIdx.x / kWave) * kChunk; base < n; base += (uint64_t)waves * kChunk) {
    uint32_t blk[U], lo[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t i = base + (uint64_t)(kWave * u) + lane;
      const uint64_t h = i < n ? load_hash<0>(hashes + i) : 0ull;  // tail lanes: values never used
      lo[u] = (uint32_t)h;
      blk[u] = block_of((uint32_t)(h >> 32), num_blocks) - b0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const uint32_t b = lane_read(blk[u], group + p);
        const uint32_t x = lane_read(lo[u], group + p);
        const uint64_t key = base + (uint64_t)(kWave * u) + group + p;
        if (key < n) {
          __hip_atomic_fetch_or(lds + b * 8u + j, 1u << bit_of(seed, x), __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
    }
  }
  __syncthreads();
  uint4 *dst4 = reinterpret_cast<uint4 *>(words + (uint64_t)b0 * 8u);
  for (uint32_t i = threadIdx.x; i < nb * 2u; i += blockDim.x) dst4[i] = lds4[i];
}

}  // namespace

uint64_t partition_workspace_bytes(uint64_t n, uint32_t num_slices) {
  // counts[P], offsets[P + 1], cursors[P] (u64 each), then the keys (8 B each),
  // every section 256-byte aligned.
  auto up = [](uint64_t v) { return (v + 255u) & ~(uint64_t)255u; };
  return up((uint64_t)num_slices * 8u) + up(((uint64_t)num_slices + 1u) * 8u) + up((uint64_t)num_slices * 8u) +
         up(n * 8u);
}

hipError_t launch_insert_partitioned(const uint64_t *hashes, uint64_t n, uint32_t *words, uint32_t num_blocks,
                                     uint32_t slice_shift, void *workspace, uint32_t grid, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const uint32_t num_slices = (uint32_t)(((uint64_t)num_blocks + (1u << slice_shift) - 1u) >> slice_shift);
  auto up = [](uint64_t v) { return (v + 255u) & ~(uint64_t)255u; };
  char *ws = static_cast<char *>(workspace);
  auto *counts = reinterpret_cast<unsigned long long *>(ws);
  ws += up((uint64_t)num_slices * 8u);
  auto *offsets = reinterpret_cast<unsigned long long *>(ws);
  ws += up(((uint64_t)num_slices + 1u) * 8u);
  auto *cursors = reinterpret_cast<unsigned long long *>(ws);
  ws += up((uint64_t)num_slices * 8u);
  auto *keys = reinterpret_cast<uint64_t *>(ws);

  hipError_t e = launch_fill(reinterpret_cast<uint32_t *>(counts), (uint64_t)num_slices * 2u, 0u, stream);
  if (e != hipSuccess) return e;
  const dim3 blk(kPartThreads);
  // Dynamic LDS above the 64 KiB default needs the per-kernel limit raised;
  // an error here shows up at launch.
  (void)hipFuncSetAttribute((const void *)part_count_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(num_slices * 4u));
  (void)hipFuncSetAttribute((const void *)part_scatter_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(num_slices * 12u));
  (void)hipGetLastError();
  hipLaunchKernelGGL(part_count_kernel, dim3(grid), blk, num_slices * 4u, stream, hashes, n, num_blocks, slice_shift,
                     num_slices, counts);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(part_scan_kernel, dim3(1), blk, 0, stream, counts, num_slices, offsets, cursors);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(part_scatter_kernel, dim3(grid), blk, (size_t)num_slices * 12u, stream, hashes, n, num_blocks,
                     slice_shift, num_slices, cursors, keys);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t lds_bytes = ((size_t)1 << slice_shift) * 32u;
  (void)hipFuncSetAttribute((const void *)part_slice_insert_kernel<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds_bytes);
  (void)hipGetLastError();
  hipLaunchKernelGGL(part_slice_insert_kernel<2>, dim3(num_slices), blk, lds_bytes, stream, keys, offsets, words,
                     num_blocks, slice_shift);
  return hipGetLastError();
}

}  // namespace sbbf
