/*
 * CPU oracle for split block Bloom filters (Apple, "Split block Bloom
 * filters", arXiv 2101.01719).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, obviously correct reference
 * that the GPU path is checked against. Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it. It shares no code,
 * header, table or constant with the GPU library, and the GPU library never
 * calls it.
 *
 * Plain C11, scalar, single-threaded, no intrinsics. The method is exact
 * integer arithmetic, so the oracle is its definition written out:
 *
 *   block selection  b = floor(hi32(h) * B / 2^32)      (appendix figure, block_index)
 *   lane rehash      x = lo32(h);  idx_j = (s_j * x mod 2^32) >> 27,  j = 0..7
 *                    (construction paragraph: multiply-shift hashing of the key
 *                    into [0, 32) with odd seeds; appendix figure, make_mask)
 *   insert           W[8b + j] |= 1 << idx_j for every j   (appendix figure, add_hash)
 *   lookup           present iff W[8b + j] has bit idx_j for every j
 *                    (appendix figure, find_hash)
 *
 * Filter image: B blocks of 256 bits, block b is the eight 32-bit words
 * W[8b .. 8b+7]; word j is lane j of the 256-bit block in x86 little-endian
 * lane order, so the byte image equals the appendix's __m256i array.
 *
 * Readings taken where the paper is silent or loose (each justified in the
 * accompanying design notes):
 *   - the seeds come from the four 64-bit constants of the appendix figure;
 *     a 256-bit vector initialised from four 64-bit values holds constant k
 *     in lanes 2k (low half) and 2k+1 (high half) on little-endian x86;
 *   - the rehash keeps the low 32 bits of the product before shifting (the
 *     formula in the text omits the "mod 2^32"; the 32-bit lane multiply of
 *     the listing keeps only the low half);
 *   - every index in [0, 32) is reachable (a comment in the listing says
 *     [0, 31), which contradicts the shift by 27);
 *   - the result of many inserts is the OR of their masks, independent of
 *     order and duplicates.
 */
#include <stddef.h>
#include <stdint.h>
#include <string.h>

/* The four 64-bit constants printed in the appendix figure, in print order. */
static const uint64_t kPrintedConstants[4] = {
    UINT64_C(0x47b6137b44974d91),
    UINT64_C(0x8824ad5ba2b7289d),
    UINT64_C(0x705495c72df1424b),
    UINT64_C(0x9efc49475c6bfb31),
};

/* Lane seeds: constant k fills lane 2k with its low half and lane 2k+1 with
 * its high half (little-endian lane order of a 256-bit vector). */
void sbbf_oracle_seeds(uint32_t seeds[8]) {
  for (int k = 0; k < 4; ++k) {
    seeds[2 * k] = (uint32_t)(kPrintedConstants[k] & UINT64_C(0xffffffff));
    seeds[2 * k + 1] = (uint32_t)(kPrintedConstants[k] >> 32);
  }
}

/* Block selection: multiply the high 32 bits of the hash by the block count
 * and keep the high 32 bits of the 64-bit product. Result is in [0, B). */
uint64_t sbbf_oracle_block(uint64_t hash, uint32_t num_blocks) {
  uint64_t hi = hash >> 32;
  return (hi * (uint64_t)num_blocks) >> 32;
}

/* The eight bit positions for the low 32 bits of a hash. */
void sbbf_oracle_bit_indices(uint32_t x, uint32_t idx[8]) {
  uint32_t seeds[8];
  sbbf_oracle_seeds(seeds);
  for (int j = 0; j < 8; ++j) {
    uint32_t product = (uint32_t)((uint64_t)seeds[j] * (uint64_t)x); /* mod 2^32 */
    idx[j] = product >> 27;                                           /* top 5 bits */
  }
}

/* The 256-bit mask as eight 32-bit words, exactly one bit set in each. */
void sbbf_oracle_mask(uint32_t x, uint32_t mask[8]) {
  uint32_t idx[8];
  sbbf_oracle_bit_indices(x, idx);
  for (int j = 0; j < 8; ++j) mask[j] = UINT32_C(1) << idx[j];
}

/* Insert n hashes into the filter words (8 * num_blocks uint32). */
void sbbf_oracle_insert(uint32_t *words, uint32_t num_blocks, const uint64_t *hashes, uint64_t n) {
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t b = sbbf_oracle_block(hashes[i], num_blocks);
    uint32_t mask[8];
    sbbf_oracle_mask((uint32_t)(hashes[i] & UINT64_C(0xffffffff)), mask);
    for (int j = 0; j < 8; ++j) words[8 * b + (uint64_t)j] |= mask[j];
  }
}

/* One lookup: 1 when every mask bit is set in the selected block. */
int sbbf_oracle_contains(const uint32_t *words, uint32_t num_blocks, uint64_t hash) {
  uint64_t b = sbbf_oracle_block(hash, num_blocks);
  uint32_t mask[8];
  sbbf_oracle_mask((uint32_t)(hash & UINT64_C(0xffffffff)), mask);
  for (int j = 0; j < 8; ++j) {
    if ((words[8 * b + (uint64_t)j] & mask[j]) == 0) return 0;
  }
  return 1;
}

/* Lookups as one byte per key, 0 or 1. */
void sbbf_oracle_lookup(const uint32_t *words, uint32_t num_blocks, const uint64_t *hashes, uint64_t n,
                        uint8_t *out) {
  for (uint64_t i = 0; i < n; ++i) out[i] = (uint8_t)sbbf_oracle_contains(words, num_blocks, hashes[i]);
}

/* Lookups packed LSB-first: key i is bit (i % 32) of word i / 32. The
 * ceil(n / 32) output words are fully written (unused high bits are 0). */
void sbbf_oracle_lookup_bits(const uint32_t *words, uint32_t num_blocks, const uint64_t *hashes, uint64_t n,
                             uint32_t *bits) {
  uint64_t nw = (n + 31) / 32;
  for (uint64_t w = 0; w < nw; ++w) bits[w] = 0;
  for (uint64_t i = 0; i < n; ++i) {
    if (sbbf_oracle_contains(words, num_blocks, hashes[i])) bits[i / 32] |= UINT32_C(1) << (i % 32);
  }
}

static unsigned popcount32(uint32_t v) {
  unsigned c = 0;
  while (v) {
    v &= v - 1;
    ++c;
  }
  return c;
}

/* Total number of set bits in the filter. */
uint64_t sbbf_oracle_popcount(const uint32_t *words, uint64_t num_words) {
  uint64_t c = 0;
  for (uint64_t i = 0; i < num_words; ++i) c += popcount32(words[i]);
  return c;
}

/* Estimated false-positive probability of this particular filter for a
 * uniformly random non-member hash, treating the eight lane indices as
 * independent and uniform on [0, 32): mean over blocks of the product over
 * lanes of (set bits in the lane word) / 32. fp64. */
double sbbf_oracle_conditional_fpr(const uint32_t *words, uint32_t num_blocks) {
  double sum = 0.0;
  for (uint64_t b = 0; b < num_blocks; ++b) {
    double p = 1.0;
    for (int j = 0; j < 8; ++j) p *= (double)popcount32(words[8 * b + (uint64_t)j]) / 32.0;
    sum += p;
  }
  return sum / (double)num_blocks;
}

/* For every lane j and every x in [x_begin, x_end), count how often each bit
 * index 0..31 is chosen: hist[32 * j + idx] += 1. hist is not cleared. */
void sbbf_oracle_index_histogram(uint64_t x_begin, uint64_t x_end, uint64_t hist[256]) {
  uint32_t seeds[8];
  sbbf_oracle_seeds(seeds);
  for (uint64_t x = x_begin; x < x_end; ++x) {
    for (int j = 0; j < 8; ++j) {
      uint32_t product = (uint32_t)((uint64_t)seeds[j] * x);
      hist[32 * j + (product >> 27)] += 1;
    }
  }
}

/* Number of hashes among n that map to each block: count[b] += 1. */
void sbbf_oracle_block_histogram(const uint64_t *hashes, uint64_t n, uint32_t num_blocks, uint64_t *count) {
  for (uint64_t i = 0; i < n; ++i) count[sbbf_oracle_block(hashes[i], num_blocks)] += 1;
}

/* Key hashing for the entry points that take keys (the method hashes each
 * key once and leaves the function open; the library's choice is the 64-bit
 * finalizer of MurmurHash3 by A. Appleby): out[i] = fmix64(keys[i]), where
 * fmix64 xor-shifts right by 33, multiplies by 0xff51afd7ed558ccd, xor-shifts
 * by 33, multiplies by 0xc4ceb9fe1a85ec53 and xor-shifts by 33 (mod 2^64). */
void sbbf_oracle_key_hash(const uint64_t *keys, uint64_t n, uint64_t *out) {
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t k = keys[i];
    k = k ^ (k >> 33);
    k = k * UINT64_C(0xff51afd7ed558ccd);
    k = k ^ (k >> 33);
    k = k * UINT64_C(0xc4ceb9fe1a85ec53);
    k = k ^ (k >> 33);
    out[i] = k;
  }
}

/* ---- Block variants with four or sixteen lanes ----------------------------
 *
 * The paper picks eight lanes so that a block fills one 256-bit SIMD register
 * and notes that four or sixteen lanes would work too (list of central ideas,
 * footnote). A K-lane block is K 32-bit words, W[K b .. K b + K - 1]; block
 * selection is unchanged and word j takes bit (s_j * lo32(h) mod 2^32) >> 27.
 * The paper prints seeds for eight lanes only. Readings:
 *   K = 4:  seeds 0..3 of the appendix figure (its first two constants);
 *   K = 8:  the eight seeds of the figure (the method itself);
 *   K = 16: the eight seeds of the figure, then eight more odd seeds: the low
 *           32 bits of the first eight outputs of SplitMix64 seeded with 16,
 *           each with its lowest bit set.
 */
static const uint32_t kExtraSeeds[8] = {
    UINT32_C(0xba779207), UINT32_C(0xc985644b), UINT32_C(0xa4e84675), UINT32_C(0xe421c8db),
    UINT32_C(0xbd38674f), UINT32_C(0x58ee486d), UINT32_C(0x8ddb3387), UINT32_C(0x7ea09599),
};

/* Seeds of a K-lane block in word order; returns 0, or -1 for another K. */
int sbbf_oracle_variant_seeds(uint32_t lanes, uint32_t seeds[16]) {
  if (lanes != 4 && lanes != 8 && lanes != 16) return -1;
  uint32_t paper[8];
  sbbf_oracle_seeds(paper);
  for (uint32_t j = 0; j < lanes; ++j) seeds[j] = j < 8 ? paper[j] : kExtraSeeds[j - 8];
  return 0;
}

/* The K-word mask for the low 32 bits of a hash: one bit in each word. */
void sbbf_oracle_variant_mask(uint32_t lanes, uint32_t x, uint32_t mask[16]) {
  uint32_t seeds[16];
  sbbf_oracle_variant_seeds(lanes, seeds);
  for (uint32_t j = 0; j < lanes; ++j) {
    uint32_t product = (uint32_t)((uint64_t)seeds[j] * (uint64_t)x); /* mod 2^32 */
    mask[j] = UINT32_C(1) << (product >> 27);
  }
}

/* Insert into a K-lane filter (K * num_blocks words). */
void sbbf_oracle_variant_insert(uint32_t *words, uint32_t lanes, uint32_t num_blocks, const uint64_t *hashes,
                                uint64_t n) {
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t b = sbbf_oracle_block(hashes[i], num_blocks);
    uint32_t mask[16];
    sbbf_oracle_variant_mask(lanes, (uint32_t)(hashes[i] & UINT64_C(0xffffffff)), mask);
    for (uint32_t j = 0; j < lanes; ++j) words[(uint64_t)lanes * b + j] |= mask[j];
  }
}

/* One lookup in a K-lane filter: 1 when every word holds its mask bit. */
int sbbf_oracle_variant_contains(const uint32_t *words, uint32_t lanes, uint32_t num_blocks, uint64_t hash) {
  uint64_t b = sbbf_oracle_block(hash, num_blocks);
  uint32_t mask[16];
  sbbf_oracle_variant_mask(lanes, (uint32_t)(hash & UINT64_C(0xffffffff)), mask);
  for (uint32_t j = 0; j < lanes; ++j) {
    if ((words[(uint64_t)lanes * b + j] & mask[j]) == 0) return 0;
  }
  return 1;
}

void sbbf_oracle_variant_lookup(const uint32_t *words, uint32_t lanes, uint32_t num_blocks, const uint64_t *hashes,
                                uint64_t n, uint8_t *out) {
  for (uint64_t i = 0; i < n; ++i) out[i] = (uint8_t)sbbf_oracle_variant_contains(words, lanes, num_blocks, hashes[i]);
}
