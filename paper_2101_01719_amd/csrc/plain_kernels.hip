// Plain (single filter) insert and lookup kernels for gfx950, plus the
// measurement kernels that share their access pattern.
//
// Insert and lookup follow the paper's appendix routines applied to a batch:
// block selection, the eight-word mask, then an OR into (insert) or a test of
// (lookup) the selected 256-bit block. The batch is spread over waves with a
// grid-stride loop over 64-key chunks; each wave keeps `U` chunks in flight so
// that 8U independent 32-byte block accesses are outstanding per wave.
// `kFlags` selects cache policies only (SBBF_* flags); results never depend
// on it. `K` is the number of 32-bit words per block: 8 for the method, 4 or
// 16 for the block variants (groups of K lanes per key, K passes per chunk).
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
// of the hash held by each lane (the input is hashed first when `keys` is
// set). Keys at or past n become hash 0 (block 0, always in range); their
// results are discarded by the callers.
template <int U, uint32_t kFlags>
__device__ __forceinline__ void stage(const uint64_t *__restrict__ hashes, uint64_t n, uint64_t base,
                                      uint32_t num_blocks, uint32_t lane, uint32_t keys, uint32_t (&blk)[U],
                                      uint32_t (&lo)[U]) {
  uint64_t hv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint64_t i = base + (uint64_t)(kWave * u) + lane;
    hv[u] = i < n ? load_hash<kFlags>(hashes + i) : 0ull;
  }
  if (keys) {
#pragma unroll
    for (int u = 0; u < U; ++u) hv[u] = key_hash(hv[u]);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint64_t h = hv[u];
    lo[u] = (uint32_t)h;
    blk[u] = block_of((uint32_t)(h >> 32), num_blocks);
  }
}

// ---- lookup -----------------------------------------------------------------

// Seed of word j for K-word blocks (j < K).
template <uint32_t K>
__device__ __forceinline__ uint32_t lane_seed(uint32_t j) {
  if constexpr (K <= 8) {
    return seed_of_word(j);
  } else {
    return seed_k(j);
  }
}

template <int U, bool kBits, uint32_t kFlags, uint32_t K = 8>
__global__ void __launch_bounds__(1024)
lookup_kernel(const uint64_t *__restrict__ hashes, uint64_t n, const uint32_t *__restrict__ words,
              uint32_t num_blocks, uint8_t *__restrict__ out8, uint32_t *__restrict__ out_bits, uint32_t keys) {
  const uint32_t lane = lane_id();
  const uint32_t j = lane & (K - 1u);       // word of the block owned by this lane
  const uint32_t group = lane & ~(K - 1u);  // first lane of this lane's K-lane group
  const uint32_t seed = lane_seed<K>(j);
  const WaveCursor wc = wave_cursor();
  constexpr uint64_t kChunk = (uint64_t)kWave * U;

  for (uint64_t base = wc.first * kChunk; base < n; base += wc.stride * kChunk) {
    uint32_t blk[U], lo[U];
    stage<U, kFlags>(hashes, n, base, num_blocks, lane, keys, blk, lo);

    // Issue every block read of the U chunks before testing any of them.
    uint32_t word[U][K], bit[U][K];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (uint32_t p = 0; p < K; ++p) {
        const uint32_t b = lane_read(blk[u], group + p);
        const uint32_t x = lane_read(lo[u], group + p);
        bit[u][p] = bit_of(seed, x);
        word[u][p] = load_word<kFlags>(words + (uint64_t)b * K + j);
      }
    }

#pragma unroll
    for (int u = 0; u < U; ++u) {
      uint64_t r = 0;
#pragma unroll
      for (uint32_t p = 0; p < K; ++p) r |= fold_pass_k<K>(ballot((word[u][p] >> bit[u][p]) & 1u), p);
      const uint64_t i0 = base + (uint64_t)(kWave * u);
      if (i0 >= n) break;
      if constexpr (!kBits) {
        if (i0 + lane < n) store_result<kFlags>(out8 + i0 + lane, (uint8_t)((r >> lane) & 1u));
      } else {
        const uint64_t left = n - i0;
        if (left < 64) r &= (1ull << left) - 1ull;
        const uint64_t w0 = i0 / 32;  // i0 is a multiple of 64
        if (lane == 0) store_result<kFlags>(out_bits + w0, (uint32_t)r);
        if (lane == 1 && left > 32) store_result<kFlags>(out_bits + w0 + 1, (uint32_t)(r >> 32));
      }
    }
  }
}

// ---- insert: 32-bit global atomics, one key per 8 lanes ---------------------

template <int U, uint32_t kFlags, uint32_t K = 8>
__global__ void __launch_bounds__(1024)
insert_atomic32_kernel(const uint64_t *__restrict__ hashes, uint64_t n, uint32_t *__restrict__ words,
                       uint32_t num_blocks, uint32_t keys) {
  const uint32_t lane = lane_id();
  const uint32_t j = lane & (K - 1u);
  const uint32_t group = lane & ~(K - 1u);
  const uint32_t seed = lane_seed<K>(j);
  const WaveCursor wc = wave_cursor();
  constexpr uint64_t kChunk = (uint64_t)kWave * U;

  for (uint64_t base = wc.first * kChunk; base < n; base += wc.stride * kChunk) {
    uint32_t blk[U], lo[U];
    stage<U, kFlags>(hashes, n, base, num_blocks, lane, keys, blk, lo);
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (uint32_t p = 0; p < K; ++p) {
        const uint32_t b = lane_read(blk[u], group + p);
        const uint32_t x = lane_read(lo[u], group + p);
        const uint64_t key = base + (uint64_t)(kWave * u) + group + p;
        if (key < n) {
          __hip_atomic_fetch_or(words + (uint64_t)b * K + j, 1u << bit_of(seed, x), __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
  }
}

// ---- insert: 64-bit global atomics, one key per K/2 lanes -------------------
// With Q = K/2, lane l handles words 2q and 2q+1 (q = l % Q) of the key of
// lane Q g + p in pass p (g = l / Q), so a pass covers 64/Q keys and Q passes
// a chunk (for K = 8: 16 keys per pass, four passes).

template <int U, uint32_t kFlags, uint32_t K = 8>
__global__ void __launch_bounds__(1024)
insert_atomic64_kernel(const uint64_t *__restrict__ hashes, uint64_t n, uint32_t *__restrict__ words,
                       uint32_t num_blocks, uint32_t keys) {
  constexpr uint32_t Q = K / 2u;
  const uint32_t lane = lane_id();
  const uint32_t q = lane & (Q - 1u);
  const uint32_t group = lane & ~(Q - 1u);
  const uint32_t seed_lo = lane_seed<K>(2u * q);
  const uint32_t seed_hi = lane_seed<K>(2u * q + 1u);
  unsigned long long *pairs = reinterpret_cast<unsigned long long *>(words);
  const WaveCursor wc = wave_cursor();
  constexpr uint64_t kChunk = (uint64_t)kWave * U;

  for (uint64_t base = wc.first * kChunk; base < n; base += wc.stride * kChunk) {
    uint32_t blk[U], lo[U];
    stage<U, kFlags>(hashes, n, base, num_blocks, lane, keys, blk, lo);
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (uint32_t p = 0; p < Q; ++p) {
        const uint32_t b = lane_read(blk[u], group + p);
        const uint32_t x = lane_read(lo[u], group + p);
        const uint64_t key = base + (uint64_t)(kWave * u) + group + p;
        if (key < n) {
          const unsigned long long m = (unsigned long long)(1u << bit_of(seed_lo, x)) |
                                       ((unsigned long long)(1u << bit_of(seed_hi, x)) << 32);
          __hip_atomic_fetch_or(pairs + (uint64_t)b * Q + q, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
  }
}

// ---- insert: LDS-private copies -----------------------------------------------
// The whole filter (K * num_blocks words) lives in this workgroup's LDS. With
// one workgroup it starts from the filter's current contents and is stored
// back with plain stores (the workgroup is the only writer). With several,
// each starts from zero, ORs its share of the keys, and ORs its non-zero
// 64-bit word pairs into the filter with global atomics.

template <int U, uint32_t kFlags, uint32_t K = 8>
__global__ void __launch_bounds__(1024)
insert_lds_kernel(const uint64_t *__restrict__ hashes, uint64_t n, uint32_t *__restrict__ words,
                  uint32_t num_blocks, uint32_t keys) {
  extern __shared__ uint4 lds4[];
  uint32_t *lds = reinterpret_cast<uint32_t *>(lds4);
  const uint32_t n_vec4 = num_blocks * (K / 4u);  // 4K bytes per block = K/4 x uint4
  const bool owner = gridDim.x == 1;
  const uint4 *src4 = reinterpret_cast<const uint4 *>(words);
  for (uint32_t i = threadIdx.x; i < n_vec4; i += blockDim.x) lds4[i] = owner ? src4[i] : make_uint4(0, 0, 0, 0);
  __syncthreads();

  const uint32_t lane = lane_id();
  const uint32_t j = lane & (K - 1u);
  const uint32_t group = lane & ~(K - 1u);
  const uint32_t seed = lane_seed<K>(j);
  const WaveCursor wc = wave_cursor();
  constexpr uint64_t kChunk = (uint64_t)kWave * U;
  for (uint64_t base = wc.first * kChunk; base < n; base += wc.stride * kChunk) {
    uint32_t blk[U], lo[U];
    stage<U, kFlags>(hashes, n, base, num_blocks, lane, keys, blk, lo);
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (uint32_t p = 0; p < K; ++p) {
        const uint32_t b = lane_read(blk[u], group + p);
        const uint32_t x = lane_read(lo[u], group + p);
        const uint64_t key = base + (uint64_t)(kWave * u) + group + p;
        if (key < n) {
          __hip_atomic_fetch_or(lds + b * K + j, 1u << bit_of(seed, x), __ATOMIC_RELAXED,
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
    for (uint32_t i = threadIdx.x; i < num_blocks * (K / 2u); i += blockDim.x) {
      const unsigned long long v = lds2[i];
      if (v) __hip_atomic_fetch_or(pairs + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---- fill -------------------------------------------------------------------------

// dst |= src over whole filters (both 32-byte aligned, num_words a multiple
// of 8): 16-byte loads and stores, grid-stride.
__global__ void __launch_bounds__(256) union_kernel(uint4 *__restrict__ dst, const uint4 *__restrict__ src, uint64_t n4) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
    const uint4 a = dst[i], b = src[i];
    dst[i] = make_uint4(a.x | b.x, a.y | b.y, a.z | b.z, a.w | b.w);
  }
}

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

template <int U, uint32_t kFlags>
__global__ void __launch_bounds__(1024)
bench_gather_kernel(const uint64_t *__restrict__ hashes, uint64_t n, const uint32_t *__restrict__ buf,
                    uint32_t num_blocks, uint8_t *__restrict__ out8) {
  constexpr uint32_t keys = 0;  // measurement kernels take hashes
  const uint32_t lane = lane_id();
  const uint32_t j = lane & 7u;
  const uint32_t group = lane & ~7u;
  const WaveCursor wc = wave_cursor();
  constexpr uint64_t kChunk = (uint64_t)kWave * U;
  for (uint64_t base = wc.first * kChunk; base < n; base += wc.stride * kChunk) {
    uint32_t blk[U], lo[U];
    stage<U, kFlags>(hashes, n, base, num_blocks, lane, keys, blk, lo);
    uint32_t word[U][8];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int p = 0; p < 8; ++p)
        word[u][p] = load_word<kFlags>(buf + (uint64_t)lane_read(blk[u], group + p) * 8u + j);
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
      if (i0 + lane < n) store_result<kFlags>(out8 + i0 + lane, (uint8_t)((any >> lane) & 1u));
    }
  }
}

template <int U, bool kWide, uint32_t kFlags>
__global__ void __launch_bounds__(1024)
bench_atomic_kernel(const uint64_t *__restrict__ hashes, uint64_t n, uint32_t *__restrict__ buf,
                    uint32_t num_blocks) {
  constexpr uint32_t keys = 0;  // measurement kernels take hashes
  const uint32_t lane = lane_id();
  const WaveCursor wc = wave_cursor();
  constexpr uint64_t kChunk = (uint64_t)kWave * U;
  constexpr uint32_t kLanes = kWide ? 4u : 8u;
  const uint32_t part = lane & (kLanes - 1u);
  const uint32_t group = lane & ~(kLanes - 1u);
  for (uint64_t base = wc.first * kChunk; base < n; base += wc.stride * kChunk) {
    uint32_t blk[U], lo[U];
    stage<U, kFlags>(hashes, n, base, num_blocks, lane, keys, blk, lo);
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

template <int U, uint32_t kFlags>
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
      h[u] = i < n ? load_hash<kFlags>(hashes + i) : 0ull;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t i = base + (uint64_t)(kWave * u) + lane;
      if (i < n) store_result<kFlags>(out8 + i, (uint8_t)(__popcll(h[u]) & 1));
    }
  }
}

// ---- dispatch -------------------------------------------------------------------------
// SBBF_DISPATCH_U{4,8}(u, BODY) instantiates BODY(U) for the unroll value u;
// BODY must end in `return`.

#define SBBF_DISPATCH_U4(u, BODY)         \
  switch (u) {                            \
    case 1: { BODY(1) }                   \
    case 2: { BODY(2) }                   \
    case 4: { BODY(4) }                   \
    default: return hipErrorInvalidValue; \
  }

#define SBBF_DISPATCH_U2(u, BODY)         \
  switch (u) {                            \
    case 1: { BODY(1) }                   \
    case 2: { BODY(2) }                   \
    default: return hipErrorInvalidValue; \
  }

#define SBBF_DISPATCH_U8(u, BODY)         \
  switch (u) {                            \
    case 1: { BODY(1) }                   \
    case 2: { BODY(2) }                   \
    case 4: { BODY(4) }                   \
    case 8: { BODY(8) }                   \
    default: return hipErrorInvalidValue; \
  }

// Runs Launcher<F>::run for the flag value F equal to `flags` (0..15).
template <template <uint32_t> class Launcher, typename... Args>
hipError_t dispatch_flags(uint32_t flags, Args... args) {
  switch (flags & SBBF_FLAGS_MASK) {
    case 0: return Launcher<0>::run(args...);
    case 1: return Launcher<1>::run(args...);
    case 2: return Launcher<2>::run(args...);
    case 3: return Launcher<3>::run(args...);
    case 4: return Launcher<4>::run(args...);
    case 5: return Launcher<5>::run(args...);
    case 6: return Launcher<6>::run(args...);
    case 7: return Launcher<7>::run(args...);
    case 8: return Launcher<8>::run(args...);
    case 9: return Launcher<9>::run(args...);
    case 10: return Launcher<10>::run(args...);
    case 11: return Launcher<11>::run(args...);
    case 12: return Launcher<12>::run(args...);
    case 13: return Launcher<13>::run(args...);
    case 14: return Launcher<14>::run(args...);
    case 15: return Launcher<15>::run(args...);
  }
  return hipErrorInvalidValue;
}

template <uint32_t F>
struct LookupLauncher {
  static hipError_t run(const uint64_t *hashes, uint64_t n, const uint32_t *words, uint32_t num_blocks,
                        uint8_t *out8, uint32_t *out_bits, Shape s, hipStream_t stream) {
    const dim3 g(s.grid), b(s.threads);
#define BODY(U)                                                                                              \
  if (out_bits)                                                                                              \
    hipLaunchKernelGGL((lookup_kernel<U, true, F>), g, b, 0, stream, hashes, n, words, num_blocks, nullptr,  \
                       out_bits, s.keys);                                                                    \
  else                                                                                                       \
    hipLaunchKernelGGL((lookup_kernel<U, false, F>), g, b, 0, stream, hashes, n, words, num_blocks, out8,    \
                       nullptr, s.keys);                                                                     \
  return hipGetLastError();
    SBBF_DISPATCH_U4(s.unroll, BODY)
#undef BODY
  }
};

// Lookups in the four- and sixteen-word block variants, with the default
// cache policies. Sixteen-word blocks keep at most two chunks in flight per
// wave (32 block words per lane).
template <uint32_t K>
hipError_t run_lookup_variant(const uint64_t *hashes, uint64_t n, const uint32_t *words, uint32_t num_blocks,
                              uint8_t *out8, uint32_t *out_bits, const Shape &s, hipStream_t stream) {
  const dim3 g(s.grid), b(s.threads);
#define BODY(U)                                                                                              \
  if (out_bits)                                                                                              \
    hipLaunchKernelGGL((lookup_kernel<U, true, 0, K>), g, b, 0, stream, hashes, n, words, num_blocks, nullptr, \
                       out_bits, s.keys);                                                                    \
  else                                                                                                       \
    hipLaunchKernelGGL((lookup_kernel<U, false, 0, K>), g, b, 0, stream, hashes, n, words, num_blocks, out8,   \
                       nullptr, s.keys);                                                                     \
  return hipGetLastError();
  if constexpr (K == 16) {
    SBBF_DISPATCH_U2(s.unroll > 2 ? 2u : s.unroll, BODY)
  } else {
    SBBF_DISPATCH_U4(s.unroll, BODY)
  }
#undef BODY
}

template <uint32_t F>
struct GatherLauncher {
  static hipError_t run(const uint32_t *buf, uint32_t num_blocks, const uint64_t *hashes, uint64_t n, uint8_t *out,
                        Shape s, hipStream_t stream) {
    const dim3 g(s.grid), b(s.threads);
#define BODY(U)                                                                                              \
  hipLaunchKernelGGL((bench_gather_kernel<U, F>), g, b, 0, stream, hashes, n, buf, num_blocks, out);         \
  return hipGetLastError();
    SBBF_DISPATCH_U4(s.unroll, BODY)
#undef BODY
  }
};

// Inserts only use the hash-load flag, so each insert kernel exists in two
// cache variants (H = 0 or SBBF_HASH_LOAD_CACHED); the block variants (K = 4
// or 16 words) use the default.
template <uint32_t H, uint32_t K = 8>
hipError_t run_insert(int kind, const uint64_t *hashes, uint64_t n, uint32_t *words, uint32_t num_blocks,
                      const Shape &s, hipStream_t stream) {
  const dim3 g(s.grid), b(s.threads);
  if (kind == SBBF_INSERT_ATOMIC32) {
#define BODY(U)                                                                                       \
  hipLaunchKernelGGL((insert_atomic32_kernel<U, H, K>), g, b, 0, stream, hashes, n, words, num_blocks, s.keys); \
  return hipGetLastError();
    SBBF_DISPATCH_U8(s.unroll, BODY)
#undef BODY
  }
  if (kind == SBBF_INSERT_ATOMIC64) {
#define BODY(U)                                                                                       \
  hipLaunchKernelGGL((insert_atomic64_kernel<U, H, K>), g, b, 0, stream, hashes, n, words, num_blocks, s.keys); \
  return hipGetLastError();
    SBBF_DISPATCH_U8(s.unroll, BODY)
#undef BODY
  }
  const size_t lds_bytes = (size_t)num_blocks * 4u * K;
#define BODY(U)                                                                                              \
  /* Raise the dynamic LDS limit; an error here shows up at launch. */                                       \
  (void)hipFuncSetAttribute((const void *)insert_lds_kernel<U, H, K>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                            (int)lds_bytes);                                                                 \
  (void)hipGetLastError();                                                                                   \
  hipLaunchKernelGGL((insert_lds_kernel<U, H, K>), g, b, lds_bytes, stream, hashes, n, words, num_blocks, s.keys); \
  return hipGetLastError();
  SBBF_DISPATCH_U8(s.unroll, BODY)
#undef BODY
}

hipError_t insert_any(int kind, const uint64_t *hashes, uint64_t n, uint32_t *words, uint32_t num_blocks,
                      const Shape &s, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  if (s.lanes == 4) return run_insert<0, 4>(kind, hashes, n, words, num_blocks, s, stream);
  if (s.lanes == 16) return run_insert<0, 16>(kind, hashes, n, words, num_blocks, s, stream);
  if (s.lanes != 8) return hipErrorInvalidValue;
  if (s.flags & SBBF_HASH_LOAD_CACHED)
    return run_insert<SBBF_HASH_LOAD_CACHED>(kind, hashes, n, words, num_blocks, s, stream);
  return run_insert<0>(kind, hashes, n, words, num_blocks, s, stream);
}

}  // namespace

hipError_t launch_lookup(const uint64_t *hashes, uint64_t n, const uint32_t *words, uint32_t num_blocks,
                         uint8_t *out8, uint32_t *out_bits, const Shape &s, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  if (s.lanes == 4) return run_lookup_variant<4>(hashes, n, words, num_blocks, out8, out_bits, s, stream);
  if (s.lanes == 16) return run_lookup_variant<16>(hashes, n, words, num_blocks, out8, out_bits, s, stream);
  if (s.lanes != 8) return hipErrorInvalidValue;
  return dispatch_flags<LookupLauncher>(s.flags, hashes, n, words, num_blocks, out8, out_bits, s, stream);
}

hipError_t launch_insert_atomic32(const uint64_t *hashes, uint64_t n, uint32_t *words, uint32_t num_blocks,
                                  const Shape &s, hipStream_t stream) {
  return insert_any(SBBF_INSERT_ATOMIC32, hashes, n, words, num_blocks, s, stream);
}

hipError_t launch_insert_atomic64(const uint64_t *hashes, uint64_t n, uint32_t *words, uint32_t num_blocks,
                                  const Shape &s, hipStream_t stream) {
  return insert_any(SBBF_INSERT_ATOMIC64, hashes, n, words, num_blocks, s, stream);
}

hipError_t launch_insert_lds(const uint64_t *hashes, uint64_t n, uint32_t *words, uint32_t num_blocks,
                             const Shape &s, hipStream_t stream) {
  return insert_any(SBBF_INSERT_LDS, hashes, n, words, num_blocks, s, stream);
}

hipError_t launch_union(uint32_t *dst, const uint32_t *src, uint64_t num_words, hipStream_t stream) {
  const uint64_t n4 = num_words / 4;
  if (n4 == 0) return hipSuccess;
  const uint64_t want = (n4 + 255) / 256;
  const uint32_t grid = (uint32_t)(want < 8192 ? want : 8192);
  hipLaunchKernelGGL(union_kernel, dim3(grid), dim3(256), 0, stream, reinterpret_cast<uint4 *>(dst),
                     reinterpret_cast<const uint4 *>(src), n4);
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
  return dispatch_flags<GatherLauncher>(s.flags, buf, num_blocks, hashes, n, out, s, stream);
}

hipError_t launch_bench_atomic(uint32_t *buf, uint32_t num_blocks, const uint64_t *hashes, uint64_t n, bool wide,
                               const Shape &s, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const dim3 g(s.grid), b(s.threads);
#define BODY(U)                                                                                              \
  if (wide)                                                                                                  \
    hipLaunchKernelGGL((bench_atomic_kernel<U, true, 0>), g, b, 0, stream, hashes, n, buf, num_blocks);      \
  else                                                                                                       \
    hipLaunchKernelGGL((bench_atomic_kernel<U, false, 0>), g, b, 0, stream, hashes, n, buf, num_blocks);     \
  return hipGetLastError();
  SBBF_DISPATCH_U8(s.unroll, BODY)
#undef BODY
}

hipError_t launch_bench_stream(const uint64_t *hashes, uint64_t n, uint8_t *out, const Shape &s,
                               hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const dim3 g(s.grid), b(s.threads);
#define BODY(U)                                                                                              \
  if (s.flags & SBBF_RESULT_STORE_NT)                                                                        \
    hipLaunchKernelGGL((bench_stream_kernel<U, SBBF_RESULT_STORE_NT>), g, b, 0, stream, hashes, n, out);     \
  else                                                                                                       \
    hipLaunchKernelGGL((bench_stream_kernel<U, 0>), g, b, 0, stream, hashes, n, out);                        \
  return hipGetLastError();
  SBBF_DISPATCH_U8(s.unroll, BODY)
#undef BODY
}

}  // namespace sbbf
