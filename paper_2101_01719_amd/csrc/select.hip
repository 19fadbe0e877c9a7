// Lookup with stream compaction: the ascending indices of the keys a filter
// reports present. The lookup itself is any lookup strategy writing the
// packed result bitmap; these kernels turn the bitmap into indices.
//
//   count  one workgroup per tile of kTileKeys keys: set bits of its words
//   scan   one workgroup: exclusive prefix of the tile counts, and the total
//   emit   one workgroup per tile: each thread takes one word,
//          the workgroup scans their bit counts, writes its indices into LDS
//          in order and copies them out with consecutive lanes
//
// Indices are 32-bit: one call takes fewer than 2^32 keys.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"
#include "sbbf_device.h"

namespace sbbf {
namespace {

constexpr uint32_t kSelThreads = 256;
constexpr uint32_t kWordsPerThread = 1;
constexpr uint32_t kTileWords = kSelThreads * kWordsPerThread;  // 256 words
constexpr uint32_t kTileKeys = kTileWords * 32u;                 // 8,192 keys
constexpr uint32_t kScanThreads = 1024;

__global__ void __launch_bounds__(kSelThreads)
select_count_kernel(const uint32_t *__restrict__ bits, uint64_t nwords, uint32_t *__restrict__ counts) {
  __shared__ uint32_t wsum[16];
  const uint64_t w0 = (uint64_t)blockIdx.x * kTileWords + (uint64_t)threadIdx.x * kWordsPerThread;
  uint32_t c = 0;
#pragma unroll
  for (uint32_t k = 0; k < kWordsPerThread; ++k) c += w0 + k < nwords ? __popc(bits[w0 + k]) : 0u;
  const uint32_t cs[1] = {c};
  uint32_t total;
  (void)block_scan_owned<1, kSelThreads>(cs, wsum, &total);
  if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

// One workgroup: offsets[t] = sum of counts[< t]; *total = sum of all. Thread
// i owns tiles [i * per, (i + 1) * per).
__global__ void __launch_bounds__(kScanThreads)
select_scan_kernel(const uint32_t *__restrict__ counts, uint32_t ntiles, uint32_t *__restrict__ offsets,
                   unsigned long long *__restrict__ total) {
  __shared__ uint32_t wsum[16];
  const uint32_t per = (ntiles + kScanThreads - 1u) / kScanThreads;
  const uint32_t b = min(threadIdx.x * per, ntiles), e = min(b + per, ntiles);
  uint32_t s = 0;
  for (uint32_t t = b; t < e; ++t) s += counts[t];
  const uint32_t cs[1] = {s};
  uint32_t all;
  uint32_t run = block_scan_owned<1, kScanThreads>(cs, wsum, &all);
  for (uint32_t t = b; t < e; ++t) {
    offsets[t] = run;
    run += counts[t];
  }
  if (threadIdx.x == 0) *total = all;
}

__global__ void __launch_bounds__(kSelThreads)
select_emit_kernel(const uint32_t *__restrict__ bits, uint64_t nwords, const uint32_t *__restrict__ offsets,
                   uint32_t *__restrict__ indices) {
  __shared__ uint32_t wsum[16];
  __shared__ uint32_t staged[kTileKeys];
  const uint64_t tile_w0 = (uint64_t)blockIdx.x * kTileWords;
  const uint64_t w0 = tile_w0 + (uint64_t)threadIdx.x * kWordsPerThread;
  uint32_t word[kWordsPerThread];
  uint32_t c = 0;
#pragma unroll
  for (uint32_t k = 0; k < kWordsPerThread; ++k) {
    word[k] = w0 + k < nwords ? bits[w0 + k] : 0u;
    c += __popc(word[k]);
  }
  const uint32_t cs[1] = {c};
  uint32_t total;
  uint32_t at = block_scan_owned<1, kSelThreads>(cs, wsum, &total);
  const uint32_t key0 = (uint32_t)(w0 * 32u);
#pragma unroll
  for (uint32_t k = 0; k < kWordsPerThread; ++k) {
    uint32_t m = word[k];
    while (m) {
      const uint32_t b = __ffs(m) - 1u;
      m &= m - 1u;
      staged[at++] = key0 + 32u * k + b;
    }
  }
  __syncthreads();
  uint32_t *dst = indices + offsets[blockIdx.x];
  for (uint32_t i = threadIdx.x; i < total; i += kSelThreads) dst[i] = staged[i];
}

}  // namespace

uint64_t select_workspace_bytes(uint64_t n) {
  const uint64_t words = (n + 31u) / 32u;
  const uint64_t tiles = (n + kTileKeys - 1u) / kTileKeys;
  return ((words * 4u + 255u) & ~(uint64_t)255u) + 2u * ((tiles * 4u + 255u) & ~(uint64_t)255u);
}

uint32_t *select_bits(void *workspace) { return static_cast<uint32_t *>(workspace); }

hipError_t launch_select(uint64_t n, void *workspace, uint32_t *indices, unsigned long long *count,
                         hipStream_t stream) {
  const uint64_t words = (n + 31u) / 32u;
  const uint32_t tiles = (uint32_t)((n + kTileKeys - 1u) / kTileKeys);
  char *base = static_cast<char *>(workspace);
  const uint32_t *bits = reinterpret_cast<const uint32_t *>(base);
  uint32_t *counts = reinterpret_cast<uint32_t *>(base + ((words * 4u + 255u) & ~(uint64_t)255u));
  uint32_t *offsets = counts + (((uint64_t)tiles * 4u + 255u) & ~(uint64_t)255u) / 4u;
  hipError_t e;
  hipLaunchKernelGGL(select_count_kernel, dim3(tiles), dim3(kSelThreads), 0, stream, bits, words, counts);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(select_scan_kernel, dim3(1), dim3(kScanThreads), 0, stream, counts, tiles, offsets, count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(select_emit_kernel, dim3(tiles), dim3(kSelThreads), 0, stream, bits, words, offsets, indices);
  return hipGetLastError();
}

}  // namespace sbbf
