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

#include <mutex>
#include <vector>

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

// Workspace: the bitmap (ceil(n / 32) words), then the tile counts and the
// tile offsets, each padded to 256 bytes.
constexpr uint64_t workspace_bytes(uint64_t n) {
  return ((((n + 31u) / 32u) * 4u + 255u) & ~(uint64_t)255u) +
         2u * (((n + kTileKeys - 1u) / kTileKeys * 4u + 255u) & ~(uint64_t)255u);
}

// The allocation-free select keeps its workspace in a static device array
// sized for at most kNoAllocMaxKeys keys per call: 32 MiB of bitmap and
// 2 x 128 KiB of tile tables. Every GPU the library runs on holds its own copy
// until the process ends. In host code `scratch` names a host-side stand-in,
// not device memory: only the address hipGetSymbolAddress returns for the
// current device is ever passed to kernels or copies.
constexpr uint64_t kNoAllocMaxKeys = 1ull << 28;
constexpr uint64_t kScratchBytes = workspace_bytes(kNoAllocMaxKeys);
static_assert(kScratchBytes == 33816576ull, "allocation-free select workspace size");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on the current device, looked up once per
// device on its first call (with that device current) and kept.
void *scratch_on_current_device(sbbf_status *st) {
  static std::mutex mu;
  static std::vector<void *> addr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *st = hip_error(e, "hipGetDevice");
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *st = hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(select scratch)");
      return nullptr;
    }
    addr[dev] = p;
  }
  *st = SBBF_OK;
  return addr[dev];
}

}  // namespace

uint64_t select_workspace_bytes(uint64_t n) { return workspace_bytes(n); }

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

// ---- C ABI -------------------------------------------------------------------

using namespace sbbf;

extern "C" sbbf_status sbbf_lookup_select_noalloc(const sbbf_filter *f, const uint64_t *d_hashes, size_t n,
                                                  uint32_t *d_indices, uint64_t *d_count, const sbbf_launch *cfg,
                                                  sbbf_stream s) {
  if (!f) return set_error(SBBF_EINVAL, "filter is NULL");
  if (!d_count) return set_error(SBBF_EINVAL, "d_count is NULL");
  if ((uintptr_t)d_count & 7u) return set_error(SBBF_EINVAL, "d_count must be 8-byte aligned");
  if ((uint64_t)n > kNoAllocMaxKeys)
    return set_error(SBBF_EINVAL, "sbbf_lookup_select_noalloc takes at most 2^28 keys per call (its static "
                                  "workspace holds " + std::to_string(kScratchBytes) + " bytes); got " +
                                      std::to_string((unsigned long long)n));
  if (n > 0) {
    if (!d_hashes) return set_error(SBBF_EINVAL, "d_hashes is NULL");
    if ((uintptr_t)d_hashes & 7u) return set_error(SBBF_EINVAL, "d_hashes must be 8-byte aligned");
    if (!d_indices) return set_error(SBBF_EINVAL, "d_indices is NULL");
    if ((uintptr_t)d_indices & 3u) return set_error(SBBF_EINVAL, "d_indices is not aligned to 4");
  }
  sbbf_launch c = cfg ? *cfg : sbbf_launch{0, 0, 0, 0, 0};
  if (c.strategy == SBBF_LOOKUP_AUTO) c.strategy = SBBF_LOOKUP_GATHER;
  if (c.strategy != SBBF_LOOKUP_GATHER)
    return set_error(SBBF_EUNSUPPORTED, "sbbf_lookup_select_noalloc takes the gather lookup only (the "
                                        "partitioned lookup allocates a workspace)");
  hipStream_t stream = (hipStream_t)s;
  if (n == 0) return hip_error(launch_fill(reinterpret_cast<uint32_t *>(d_count), 2, 0u, stream), "select count");
  sbbf_status st;
  void *ws = scratch_on_current_device(&st);
  if (!ws) return st;
  // The lookup writes every word of the bitmap and the select kernels write
  // every tile count and offset they read, so nothing needs clearing.
  st = sbbf_lookup_batch_ex(f, d_hashes, n, nullptr, select_bits(ws), &c, s);
  if (st != SBBF_OK) return st;
  return hip_error(launch_select(n, ws, d_indices, reinterpret_cast<unsigned long long *>(d_count), stream),
                   "select");
}
