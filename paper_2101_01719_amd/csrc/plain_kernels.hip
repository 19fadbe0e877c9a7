// Plain (single filter) insert and lookup kernels for gfx950, plus the
// measurement kernels that share their access pattern.
//
// Insert and lookup follow the paper's appendix routines applied to a batch:
// block selection, the eight-word mask, then an OR into (insert) or a test of
// (lookup) the selected 256-bit block. The batch is spread over waves with a
// grid-stride loop over 64-key chunks; each wave keeps `U` chunks in flight so
// that 8U independent 32-byte block accesses are outstanding per wave.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"
#include "sbbf_device.h"

namespace sbbf {
namespace {

struct WaveCursor {
  uint64_t first;   // first chunk index of this wave
  uint64_t stride;  // chunks between successive iterations
};

__device__ __forceinline__ WaveCursor wave_cursor() {
  const uint64_t waves_per_block = blockDim.x / kWave;
  const uint64_t wave = (uint64_t)blockIdx.x * waves_per_block + (threadIdx.x / kWave);
  return {wave, (uint64_t)gridDim.x * waves_per_block};
}

// Stage U chunks of 64 hashes starting at key `base`: block index and low half
// of the hash held by each lane. Keys at or past n become hash 0 (block 0,
// always in range); their results are discarded by the callers.
template <int U>
__device__ __forceinline__ void stage(const uint64_t *__restrict__ hashes, uint64_t n, uint64_t base,
                                      uint32_t num_blocks, uint32_t lane, uint32_t (&blk)[U], uint32_t (&lo)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint64_t i = base + (uint64_t)(kWave * u) + lane;
    const uint64_t h = i < n ? load_hash(hashes + i) : 0ull;
    lo[u] = (uint32_t)h;
    blk[u] = block_of((uint32_t)(h >> 32), num_blocks);
  }
}

// ---- lookup -----------------------------------------------------------------

template <int U, bool kBits>
__global__ void __launch_bounds__(1024)
lookup_kernel(const uint64_t *__restrict__ hashes, uint64_t n, const uint32_t *__restrict__ words,
              uint32_t num_blocks, uint8_t *__restrict__ out8, uint32_t *__restrict__ out_bits) {
  const uint32_t lane = lane_id();
  const uint32_t j = lane & 7u;       // word of the block owned by this lane
  const uint32_t group = lane & ~7u;  // first lane of this lane's 8-lane group
  const uint32_t seed = seed_of_word(j);
  const WaveCursor wc = wave_cursor();
  constexpr uint64_t kChunk = (uint64_t)kWave * U;

  for (uint64_t base = wc.first * kChunk; base < n; base += wc.stride * kChunk) {
    uint32_t blk[U], lo[U];
    stage<U>(hashes, n, base, num_blocks, lane, blk, lo);

    // Issue every block read of the U chunks before testing any of them.
    uint32_t word[U][8], bit[U][8];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const uint32_t b = lane_read(blk[u], group + p);
        const uint32_t x = lane_read(lo[u], group + p);
        bit[u][p] = bit_of(seed, x);
        word[u][p] = words[(uint64_t)b * 8u + j];
      }
    }

#pragma unroll
    for (int u = 0; u < U; ++u) {
      uint64_t r = 0;
#pragma unroll
      for (int p = 0; p < 8; ++p) r |= fold_pass(ballot((word[u][p] >> bit[u][p]) & 1u), p);
      const uint64_t i0 = base + (uint64_t)(kWave * u);
      if (i0 >= n) break;
      if constexpr (!kBits) {
        if (i0 + lane < n) out8[i0 + lane] = (uint8_t)((r >> lane) & 1u);
      } else {
        const uint64_t left = n - i0;
        if (left < 64) r &= (1ull << left) - 1ull;
        const uint64_t w0 = i0 / 32;  // i0 is a multiple of 64
        if (lane == 0) out_bits[w0] = (uint32_t)r;
        if (lane == 1 && left > 32) out_bits[w0 + 1] = (uint32_t)(r >> 32);
      }
    }
  }
}

// ---- insert: 32-bit global atomics, one key per 8 lanes ---------------------

template <int U>
__global__ void __launch_bounds__(1024)
insert_atomic32_kernel(const uint64_t *__restrict__ hashes, uint64_t n, uint32_t *__restrict__ words,
                       uint32_t num_blocks) {
  const uint32_t lane = lane_id();
  const uint32_t j = lane & 7u;
  const uint32_t group = lane & ~7u;
  const uint32_t seed = seed_of_word(j);
  const WaveCursor wc = wave_cursor();
  constexpr uint64_t kChunk = (uint64_t)kWave * U;

  for (uint64_t base = wc.first * kChunk; base < n; base += wc.stride * kChunk) {
    uint32_t blk[U], lo[U];
    stage<U>(hashes, n, base, num_blocks, lane, blk, lo);
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const uint32_t b = lane_read(blk[u], group + p);
        const uint32_t x = lane_read(lo[u], group + p);
        const uint64_t key = base + (uint64_t)(kWave * u) + group + p;
        if (key < n) {
          __hip_atomic_fetch_or(words + (uint64_t)b * 8u + j, 1u << bit_of(seed, x), __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
  }
}

// ---- insert: 64-bit global atomics, one key per 4 lanes ---------------------
// Lane l handles words 2q and 2q+1 (q = l % 4) of the key of lane 4g + p in
// pass p (g = l / 4), so a pass covers 16 keys and four passes a chunk.

template <int U>
__global__ void __launch_bounds__(1024)
insert_atomic64_kernel(const uint64_t *__restrict__ hashes, uint64_t n, uint32_t *__restrict__ words,
                       uint32_t num_blocks) {
  const uint32_t lane = lane_id();
  const uint32_t q = lane & 3u;
  const uint32_t group = lane & ~3u;
  const uint32_t seed_lo = seed_of_word(2u * q);
  const uint32_t seed_hi = seed_of_word(2u * q + 1u);
  unsigned long long *pairs = reinterpret_cast<unsigned long long *>(words);
  const WaveCursor wc = wave_cursor();
  constexpr uint64_t kChunk = (uint64_t)kWave * U;

  for (uint64_t base = wc.first * kChunk; base < n; base += wc.stride * kChunk) {
    uint32_t blk[U], lo[U];
    stage<U>(hashes, n, base, num_blocks, lane, blk, lo);
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const uint32_t b = lane_read(blk[u], group + p);
        const uint32_t x = lane_read(lo[u], group + p);
        const uint64_t key = base + (uint64_t)(kWave * u) + group + p;
        if (key < n) {
          const unsigned long long m = (unsigned long long)(1u << bit_of(seed_lo, x)) |
                                       ((unsigned long long)(1u << bit_of(seed_hi, x)) << 32);
          __hip_atomic_fetch_or(pairs + (uint64_t)b * 4u + q, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
  }
}

// ---- insert: LDS-private copies -----------------------------------------------
// The whole filter (8 * num_blocks words) lives in this workgroup's LDS. With
// one workgroup it starts from the filter's current contents and is stored
// back with plain stores (the workgroup is the only writer). With several,
// each starts from zero, ORs its share of the keys, and ORs its non-zero
// 64-bit word pairs into the filter with global atomics.

template <int U>
__global__ void __launch_bounds__(1024)
insert_lds_kernel(const uint64_t *__restrict__ hashes, uint64_t n, uint32_t *__restrict__ words,
                  uint32_t num_blocks) {
  extern __shared__ uint4 lds4[];
  uint32_t *lds = reinterpret_cast<uint32_t *>(lds4);
  const uint32_t n_vec4 = num_blocks * 2u;  // 32 bytes per block = 2 x uint4
  const bool owner = gridDim.x == 1;
  const uint4 *src4 = reinterpret_cast<const uint4 *>(words);
  for (uint32_t i = threadIdx.x; i < n_vec4; i += blockDim.x) lds4[i] = owner ? src4[i] : make_uint4(0, 0, 0, 0);
  __syncthreads();

  const uint32_t lane = lane_id();
  const uint32_t j = lane & 7u;
  const uint32_t group = lane & ~7u;
  const uint32_t seed = seed_of_word(j);
  const WaveCursor wc = wave_cursor();
  constexpr uint64_t kChunk = (uint64_t)kWave * U;
  for (uint64_t base = wc.first * kChunk; base < n; base += wc.stride * kChunk) {
    uint32_t blk[U], lo[U];
    stage<U>(hashes, n, base, num_blocks, lane, blk, lo);
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

  if (owner) {
    uint4 *dst4 = reinterpret_cast<uint4 *>(words);
    for (uint32_t i = threadIdx.x; i < n_vec4; i += blockDim.x) dst4[i] = lds4[i];
  } else {
    const unsigned long long *lds2 = reinterpret_cast<const unsigned long long *>(lds4);
    unsigned long long *pairs = reinterpret_cast<unsigned long long *>(words);
    for (uint32_t i = threadIdx.x; i < num_blocks * 4u; i += blockDim.x) {
      const unsigned long long v = lds2[i];
      if (v) __hip_atomic_fetch_or(pairs + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---- fill -------------------------------------------------------------------------

__global__ void __launch_bounds__(256) fill_kernel(uint32_t *__restrict__ words, uint64_t num_words, uint32_t value) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t n4 = num_words / 4;
  uint4 *w4 = reinterpret_cast<uint4 *>(words);
  const uint4 v = make_uint4(value, value, value, value);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) w4[i] = v;
  for (uint64_t i = n4 * 4 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < num_words; i += stride)
    words[i] = value;
}

// ---- measurement kernels ------------------------------------------------------------
// Same staging and block addressing as lookup/insert, without the mask.

template <int U>
__global__ void __launch_bounds__(1024)
bench_gather_kernel(const uint64_t *__restrict__ hashes, uint64_t n, const uint32_t *__restrict__ buf,
                    uint32_t num_blocks, uint8_t *__restrict__ out8) {
  const uint32_t lane = lane_id();
  const uint32_t j = lane & 7u;
  const uint32_t group = lane & ~7u;
  const WaveCursor wc = wave_cursor();
  constexpr uint64_t kChunk = (uint64_t)kWave * U;
  for (uint64_t base = wc.first * kChunk; base < n; base += wc.stride * kChunk) {
    uint32_t blk[U], lo[U];
    stage<U>(hashes, n, base, num_blocks, lane, blk, lo);
    uint32_t word[U][8];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int p = 0; p < 8; ++p) word[u][p] = buf[(uint64_t)lane_read(blk[u], group + p) * 8u + j];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      uint64_t any = 0;
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const uint64_t m = ballot(word[u][p] != 0u);
        uint64_t t = m | (m >> 4);
        t |= t >> 2;
        t |= t >> 1;
        any |= (t & 0x0101010101010101ull) << p;
      }
      const uint64_t i0 = base + (uint64_t)(kWave * u);
      if (i0 + lane < n) out8[i0 + lane] = (uint8_t)((any >> lane) & 1u);
    }
  }
}

template <int U, bool kWide>
__global__ void __launch_bounds__(1024)
bench_atomic_kernel(const uint64_t *__restrict__ hashes, uint64_t n, uint32_t *__restrict__ buf,
                    uint32_t num_blocks) {
  const uint32_t lane = lane_id();
  const WaveCursor wc = wave_cursor();
  constexpr uint64_t kChunk = (uint64_t)kWave * U;
  constexpr uint32_t kLanes = kWide ? 4u : 8u;
  const uint32_t part = lane & (kLanes - 1u);
  const uint32_t group = lane & ~(kLanes - 1u);
  for (uint64_t base = wc.first * kChunk; base < n; base += wc.stride * kChunk) {
    uint32_t blk[U], lo[U];
    stage<U>(hashes, n, base, num_blocks, lane, blk, lo);
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (uint32_t p = 0; p < kLanes; ++p) {
        const uint32_t b = lane_read(blk[u], group + p);
        const uint64_t key = base + (uint64_t)(kWave * u) + group + p;
        if (key < n) {
          if constexpr (kWide) {
            unsigned long long *pairs = reinterpret_cast<unsigned long long *>(buf);
            __hip_atomic_fetch_or(pairs + (uint64_t)b * 4u + part, 0x0000000100000001ull << (part * 2u),
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          } else {
            __hip_atomic_fetch_or(buf + (uint64_t)b * 8u + part, 1u << part, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
    }
  }
}

template <int U>
__global__ void __launch_bounds__(1024)
bench_stream_kernel(const uint64_t *__restrict__ hashes, uint64_t n, uint8_t *__restrict__ out8) {
  const uint32_t lane = lane_id();
  const WaveCursor wc = wave_cursor();
  constexpr uint64_t kChunk = (uint64_t)kWave * U;
  for (uint64_t base = wc.first * kChunk; base < n; base += wc.stride * kChunk) {
    uint64_t h[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t i = base + (uint64_t)(kWave * u) + lane;
      h[u] = i < n ? load_hash(hashes + i) : 0ull;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t i = base + (uint64_t)(kWave * u) + lane;
      if (i < n) out8[i] = (uint8_t)(__popcll(h[u]) & 1);
    }
  }
}

// ---- dispatch helpers ---------------------------------------------------------------

#define SBBF_DISPATCH_UNROLL4(U, CALL) \
  switch (U) {                        \
    case 1: CALL(1); break;           \
    case 2: CALL(2); break;           \
    case 4: CALL(4); break;           \
    default: return hipErrorInvalidValue; \
  }

#define SBBF_DISPATCH_UNROLL(U, CALL) \
  switch (U) {                        \
    case 1: CALL(1); break;           \
    case 2: CALL(2); break;           \
    case 4: CALL(4); break;           \
    case 8: CALL(8); break;           \
    default: return hipErrorInvalidValue; \
  }

}  // namespace

hipError_t launch_lookup(const uint64_t *hashes, uint64_t n, const uint32_t *words, uint32_t num_blocks,
                         uint8_t *out8, uint32_t *out_bits, const Shape &s, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  if (s.unroll > 4) return hipErrorInvalidValue;  // eight chunks in flight exceed the register file
  const dim3 g(s.grid), b(s.threads);
#define CALL(U)                                                                                            \
  if (out_bits)                                                                                            \
    hipLaunchKernelGGL((lookup_kernel<U, true>), g, b, 0, stream, hashes, n, words, num_blocks, nullptr,   \
                       out_bits);                                                                          \
  else                                                                                                     \
    hipLaunchKernelGGL((lookup_kernel<U, false>), g, b, 0, stream, hashes, n, words, num_blocks, out8,     \
                       nullptr);
  SBBF_DISPATCH_UNROLL4(s.unroll, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_insert_atomic32(const uint64_t *hashes, uint64_t n, uint32_t *words, uint32_t num_blocks,
                                  const Shape &s, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const dim3 g(s.grid), b(s.threads);
#define CALL(U) hipLaunchKernelGGL((insert_atomic32_kernel<U>), g, b, 0, stream, hashes, n, words, num_blocks);
  SBBF_DISPATCH_UNROLL(s.unroll, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_insert_atomic64(const uint64_t *hashes, uint64_t n, uint32_t *words, uint32_t num_blocks,
                                  const Shape &s, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const dim3 g(s.grid), b(s.threads);
#define CALL(U) hipLaunchKernelGGL((insert_atomic64_kernel<U>), g, b, 0, stream, hashes, n, words, num_blocks);
  SBBF_DISPATCH_UNROLL(s.unroll, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_insert_lds(const uint64_t *hashes, uint64_t n, uint32_t *words, uint32_t num_blocks,
                             const Shape &s, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const dim3 g(s.grid), b(s.threads);
  const size_t lds_bytes = (size_t)num_blocks * 32u;
#define CALL(U)                                                                                      \
  {                                                                                                  \
    /* Raise the dynamic LDS limit; an error here shows up at launch. */                           \
    (void)hipFuncSetAttribute((const void *)insert_lds_kernel<U>,                                     \
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);            \
    (void)hipGetLastError();                                                                         \
    hipLaunchKernelGGL((insert_lds_kernel<U>), g, b, lds_bytes, stream, hashes, n, words, num_blocks); \
  }
  SBBF_DISPATCH_UNROLL(s.unroll, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_fill(uint32_t *words, uint64_t num_words, uint32_t value, hipStream_t stream) {
  if (num_words == 0) return hipSuccess;
  const uint64_t want = (num_words / 4 + 255) / 256;
  const uint32_t grid = (uint32_t)(want < 4096 ? (want ? want : 1) : 4096);
  hipLaunchKernelGGL(fill_kernel, dim3(grid), dim3(256), 0, stream, words, num_words, value);
  return hipGetLastError();
}

hipError_t launch_bench_gather(const uint32_t *buf, uint32_t num_blocks, const uint64_t *hashes, uint64_t n,
                               uint8_t *out, const Shape &s, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  if (s.unroll > 4) return hipErrorInvalidValue;
  const dim3 g(s.grid), b(s.threads);
#define CALL(U) hipLaunchKernelGGL((bench_gather_kernel<U>), g, b, 0, stream, hashes, n, buf, num_blocks, out);
  SBBF_DISPATCH_UNROLL4(s.unroll, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_bench_atomic(uint32_t *buf, uint32_t num_blocks, const uint64_t *hashes, uint64_t n, bool wide,
                               const Shape &s, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const dim3 g(s.grid), b(s.threads);
#define CALL(U)                                                                                        \
  if (wide)                                                                                            \
    hipLaunchKernelGGL((bench_atomic_kernel<U, true>), g, b, 0, stream, hashes, n, buf, num_blocks);   \
  else                                                                                                 \
    hipLaunchKernelGGL((bench_atomic_kernel<U, false>), g, b, 0, stream, hashes, n, buf, num_blocks);
  SBBF_DISPATCH_UNROLL(s.unroll, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_bench_stream(const uint64_t *hashes, uint64_t n, uint8_t *out, const Shape &s,
                               hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const dim3 g(s.grid), b(s.threads);
#define CALL(U) hipLaunchKernelGGL((bench_stream_kernel<U>), g, b, 0, stream, hashes, n, out);
  SBBF_DISPATCH_UNROLL(s.unroll, CALL)
#undef CALL
  return hipGetLastError();
}

}  // namespace sbbf
