// Device-side building blocks of the split block Bloom filter on gfx950.
//
// Work layout used by every kernel: a wave of 64 lanes is eight groups of
// eight lanes. A key is handled by one group, and lane j of the group owns
// word j of the key's 256-bit block, so a block access is one 32-byte piece
// of memory touched by eight neighbouring lanes. Each lane keeps the seed of
// its own word in a register.
//
// Keys are staged 64 at a time: lane l loads hash l of a 64-hash chunk
// (a coalesced 512-byte read), and in pass p (0..7) group g takes the key held
// by lane 8g + p, fetched with a cross-lane permute. After the eight passes
// the wave has handled key l in group l / 8 during pass l % 8, which is what
// lets lookups rebuild a per-lane result with scalar bit operations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sbbf.h"

namespace sbbf {

constexpr int kWave = 64;
constexpr int kLanesPerKey = 8;

// The eight odd multiply-shift seeds, in word (lane) order: word 2k uses the
// low half and word 2k+1 the high half of the k-th 64-bit constant printed in
// the paper's appendix figure (a 256-bit vector built from four 64-bit values
// on little-endian x86 holds them in that order).
constexpr uint32_t kSeed0 = 0x44974d91u;
constexpr uint32_t kSeed1 = 0x47b6137bu;
constexpr uint32_t kSeed2 = 0xa2b7289du;
constexpr uint32_t kSeed3 = 0x8824ad5bu;
constexpr uint32_t kSeed4 = 0x2df1424bu;
constexpr uint32_t kSeed5 = 0x705495c7u;
constexpr uint32_t kSeed6 = 0x5c6bfb31u;
constexpr uint32_t kSeed7 = 0x9efc4947u;

// Seed of word j (0..7); a select chain, evaluated once per kernel.
__device__ __forceinline__ uint32_t seed_of_word(uint32_t j) {
  const uint32_t a = (j & 1) ? kSeed1 : kSeed0;
  const uint32_t b = (j & 1) ? kSeed3 : kSeed2;
  const uint32_t c = (j & 1) ? kSeed5 : kSeed4;
  const uint32_t d = (j & 1) ? kSeed7 : kSeed6;
  const uint32_t ab = (j & 2) ? b : a;
  const uint32_t cd = (j & 2) ? d : c;
  return (j & 4) ? cd : ab;
}

// Block variants with K = 4 or 16 words (the paper notes that four or sixteen
// lanes would work as well as eight, and prints seeds for eight only). Four
// lanes use seeds 0..3 above. Sixteen lanes use the eight above for words
// 0..7 and these for words 8..15: the low 32 bits of the first eight outputs
// of SplitMix64 seeded with 16, each with its lowest bit set (odd, as
// multiply-shift hashing needs).
constexpr uint32_t kSeed8 = 0xba779207u;
constexpr uint32_t kSeed9 = 0xc985644bu;
constexpr uint32_t kSeed10 = 0xa4e84675u;
constexpr uint32_t kSeed11 = 0xe421c8dbu;
constexpr uint32_t kSeed12 = 0xbd38674fu;
constexpr uint32_t kSeed13 = 0x58ee486du;
constexpr uint32_t kSeed14 = 0x8ddb3387u;
constexpr uint32_t kSeed15 = 0x7ea09599u;

// Seed of word j (0..15) of a block of any variant (the first K are used).
// A select chain for run-time j, folded to a constant for a constant j.
__host__ __device__ constexpr uint32_t seed_k(uint32_t j) {
  const uint32_t lo[8] = {kSeed0, kSeed1, kSeed2, kSeed3, kSeed4, kSeed5, kSeed6, kSeed7};
  const uint32_t hi[8] = {kSeed8, kSeed9, kSeed10, kSeed11, kSeed12, kSeed13, kSeed14, kSeed15};
  uint32_t a = 0, b = 0;
  for (uint32_t i = 0; i < 8; ++i) {
    a = (j & 7u) == i ? lo[i] : a;
    b = (j & 7u) == i ? hi[i] : b;
  }
  return j < 8u ? a : b;
}

// Block of a hash: high 32 bits of hi32(h) * num_blocks (a 32x32 multiply-high).
__device__ __forceinline__ uint32_t block_of(uint32_t hash_hi, uint32_t num_blocks) {
  return __umulhi(hash_hi, num_blocks);
}

// Bit position in [0, 32) chosen for one word: top five bits of the low 32
// bits of seed * x.
__device__ __forceinline__ uint32_t bit_of(uint32_t seed, uint32_t hash_lo) {
  return (seed * hash_lo) >> 27;
}

// Order of the K/2 64-bit ORs with which lds_or_key sets a key's bits in an
// LDS block of K words (as K/2 word pairs): the i-th OR goes to pair
// p = (i + r) mod K/2 with seeds of words 2p and 2p + 1. With one key per
// lane and the pairs in a fixed order, the i-th ORs of a wave's keys all fall
// on one of eight 8-byte offsets of a 256-byte LDS bank row; with r taken from
// the lane they spread over the whole row (random blocks give the rest). OR is
// order-free, so the filter is the same either way. Built once per thread:
// choosing the seeds per key costs about 25 compare-and-selects per key.
template <uint32_t K>
struct OrOrder {
  uint32_t sa[K / 2u], sb[K / 2u], pair[K / 2u];
};

template <uint32_t K>
__device__ __forceinline__ OrOrder<K> or_order(uint32_t r) {
  constexpr uint32_t kPairs = K / 2u;
  OrOrder<K> o;
#pragma unroll
  for (uint32_t i = 0; i < kPairs; ++i) {
    const uint32_t p = (i + r) & (kPairs - 1u);
    o.sa[i] = seed_k(2u * p);
    o.sb[i] = seed_k(2u * p + 1u);
    o.pair[i] = p;
  }
  return o;
}

// OR the mask of one key (low hash half x) into block bl of a filter of K-word
// blocks held in LDS as K/2 64-bit word pairs (one = 0 ORs nothing), in the
// order o.
template <uint32_t K>
__device__ __forceinline__ void lds_or_key(unsigned long long *lds2, uint32_t bl, uint32_t x, uint32_t one,
                                           const OrOrder<K> &o) {
  constexpr uint32_t kPairs = K / 2u;
  unsigned long long *blk = lds2 + (uint64_t)bl * kPairs;
#pragma unroll
  for (uint32_t i = 0; i < kPairs; ++i)
    __hip_atomic_fetch_or(blk + o.pair[i],
                          (unsigned long long)(one << bit_of(o.sa[i], x)) |
                              ((unsigned long long)(one << bit_of(o.sb[i], x)) << 32),
                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// OR of w over each aligned group of eight lanes, in every lane of the group,
// by DPP moves (no LDS traffic): lanes exchanged within quads (xor 1, then
// xor 2), then lane i with lane 7 - i of each eight (half-row mirror).
__device__ __forceinline__ uint32_t or_over_eights(uint32_t w) {
  w |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0xb1, 0xf, 0xf, false);   // quad_perm [1,0,3,2]
  w |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0x4e, 0xf, 0xf, false);   // quad_perm [2,3,0,1]
  w |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0x141, 0xf, 0xf, false);  // row_half_mirror
  return w;
}

// Value of `v` in lane `src` (0..63) of this wave.
__device__ __forceinline__ uint32_t lane_read(uint32_t v, uint32_t src) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src << 2), (int)v);
}

// Wave-wide ballot of a predicate.
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Hash of a key, for the entry points that take keys instead of hashes: the
// 64-bit finalizer of MurmurHash3 (A. Appleby, public domain), a bijection
// on 64-bit values with full avalanche. The method hashes each key once and
// leaves the hash function open (construction paragraph); this is the
// library's choice of it.
__host__ __device__ inline uint64_t key_hash(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

// v itself, or key_hash(v) when the kernel was given keys (a uniform flag).
__device__ __forceinline__ uint64_t as_hash(uint64_t v, uint32_t keys) { return keys ? key_hash(v) : v; }

// Load of one hash. By default with the non-temporal hint: the hash arrays are
// read once and should not displace the filter from the caches.
template <uint32_t kFlags>
__device__ __forceinline__ uint64_t load_hash(const uint64_t *p) {
  if constexpr ((kFlags & SBBF_HASH_LOAD_CACHED) != 0) {
    return *p;
  } else {
    return __builtin_nontemporal_load(p);
  }
}

// Load of one filter word for a lookup, with the cache policy of the flags.
template <uint32_t kFlags>
__device__ __forceinline__ uint32_t load_word(const uint32_t *p) {
  constexpr uint32_t pol = kFlags & SBBF_FILTER_LOAD_MASK;
  if constexpr (pol == SBBF_FILTER_LOAD_NT) {
    return __builtin_nontemporal_load(p);
  } else if constexpr (pol == SBBF_FILTER_LOAD_DEVICE) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else if constexpr (pol == SBBF_FILTER_LOAD_SYSTEM) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  } else {
    return *p;
  }
}

// Store of one result value, non-temporal when the flags ask for it.
template <uint32_t kFlags, typename T>
__device__ __forceinline__ void store_result(T *p, T v) {
  if constexpr ((kFlags & SBBF_RESULT_STORE_NT) != 0) {
    __builtin_nontemporal_store(v, p);
  } else {
    *p = v;
  }
}

// From the eight ballots of one 64-key chunk (pass p holds, in byte g, the
// eight word tests of the key of lane 8g + p), build the 64-bit result mask
// whose bit l is 1 when all eight word tests of the key of lane l passed.
__device__ __forceinline__ uint64_t fold_pass(uint64_t m, int p) {
  uint64_t t = m & (m >> 4);
  t &= t >> 2;
  t &= t >> 1;
  return (t & 0x0101010101010101ull) << p;
}

// fold_pass for K-lane groups: in pass p, group g of K lanes holds the K
// word tests of the key of lane K g + p; the result bit of that key is the
// AND of the group's K bits, placed at bit K g + p.
template <uint32_t K>
__device__ __forceinline__ uint64_t fold_pass_k(uint64_t m, uint32_t p) {
  static_assert(K == 4 || K == 8 || K == 16, "four, eight or sixteen lanes");
  uint64_t t = m;
#pragma unroll
  for (uint32_t s = K / 2; s >= 1; s /= 2) t &= t >> s;
  constexpr uint64_t kFirst = K == 4 ? 0x1111111111111111ull : K == 8 ? 0x0101010101010101ull : 0x0001000100010001ull;
  return (t & kFirst) << p;
}

// Workgroup barrier that orders LDS accesses only: outstanding global loads
// and stores stay in flight across it. For workgroups whose threads share
// data through LDS only.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Inclusive prefix sum over the 64 lanes of a wave with DPP row shifts
// (Hillis-Steele inside each row of 16 lanes) and the two row broadcasts.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15 -> rows 1, 3
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31 -> rows 2, 3
  return x;
}

// Exclusive prefix over a workgroup of T threads (a multiple of 64, at most
// 1024), thread t holding the R consecutive entries t*R .. t*R+R-1 in c[]:
// returns the sum of all entries before its first (and the sum of all in
// *total). `wsum` is 16 words of LDS; contains one barrier, and wsum may be
// rewritten only after a further barrier.
template <int R, uint32_t T = 1024>
__device__ __forceinline__ uint32_t block_scan_owned(const uint32_t (&c)[R], uint32_t *wsum,
                                                     uint32_t *total = nullptr) {
  uint32_t sum = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) sum += c[r];
  const uint32_t incl = wave_inclusive_scan(sum);
  const uint32_t wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63u) == 63u) wsum[wave] = incl;
  lds_barrier();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (uint32_t w = 0; w < T / 64u; ++w) {
    const uint32_t v = wsum[w];
    before += w < wave ? v : 0u;
    all += v;
  }
  if (total) *total = all;
  return before + incl - sum;
}

}  // namespace sbbf
