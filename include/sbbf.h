/*
 * sbbf.h — C ABI of the MI355X (gfx950) split block Bloom filter library.
 *
 * The method is the split block Bloom filter of J. Apple, "Split block Bloom
 * filters" (arXiv 2101.01719):
 *   - a filter is an array of 256-bit blocks, each split into eight 32-bit
 *     words (construction paragraph; appendix figure);
 *   - a 64-bit hash h selects block b = ((h >> 32) * num_blocks) >> 32
 *     (appendix figure, block selection);
 *   - its low 32 bits x are rehashed by eight odd-seed multiply-shift hashes,
 *     idx_j = (s_j * x mod 2^32) >> 27, one per word (construction paragraph,
 *     appendix figure, mask routine);
 *   - insert sets bit idx_j of word j of block b for every j; lookup reports
 *     present when all eight bits are set (appendix figure, insert and
 *     lookup routines). Deletion is not part of the method.
 *
 * Memory layout shared by every entry point:
 *   filter   uint32 words[8 * num_blocks] in device memory, little-endian,
 *            block-major: word j of block b at index 8 * b + j. This is the
 *            byte image of the paper's array of 256-bit vectors. 32-byte
 *            aligned.
 *   hashes   uint64 [n] in device memory, 8-byte aligned, caller-owned.
 *   results  uint8 [n] (0 or 1 per hash), or a packed bitmap uint32
 *            [ceil(n / 32)] with hash i at bit (i % 32) of word i / 32.
 *
 * Conventions:
 *   - Every call returns an sbbf_status. Argument checks are synchronous: on
 *     error nothing is enqueued and sbbf_last_error() holds a description.
 *     n == 0 is a no-op that returns SBBF_OK.
 *   - Work is enqueued on the given HIP stream (a hipStream_t passed as
 *     void*; NULL is the default stream) and completes asynchronously; a
 *     lookup sees every insert enqueued before it on the same stream. Device
 *     faults surface when the caller synchronises the stream.
 *   - Caller-owned buffers must stay valid until the stream passes the call.
 *   - Handles are not locked. Inserts into one filter that run at the same
 *     time (on several streams) are safe on the device only with the atomic
 *     strategies (SBBF_INSERT_ATOMIC32, SBBF_INSERT_ATOMIC64): the
 *     partitioned and LDS strategies read a part of the filter into LDS, OR
 *     into it and store it back whole, so another insert running at the same
 *     time into that part can lose its bits. SBBF_INSERT_AUTO may choose
 *     either kind; order such calls (one stream, or events) or name an atomic
 *     strategy. A lookup running concurrently with inserts sees some subset of
 *     them.
 *   - The filter bytes produced by any insert strategy and any launch
 *     configuration are identical: the final filter is the OR of all masks.
 */
#ifndef SBBF_H_
#define SBBF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbbf_filter sbbf_filter; /* opaque: device words + block count */
typedef struct sbbf_group sbbf_group;   /* opaque: a grouped plan over many filters */
typedef struct sbbf_server sbbf_server; /* opaque: the serving loop */
typedef void *sbbf_stream;              /* a hipStream_t; NULL = default stream */

typedef enum sbbf_status {
  SBBF_OK = 0,
  SBBF_EINVAL = 1,      /* bad argument (null pointer, size, alignment) */
  SBBF_ENOMEM = 2,      /* device or host allocation failed */
  SBBF_EDEVICE = 3,     /* a HIP call failed; sbbf_last_error() has HIP's text */
  SBBF_EBUDGET = 4,     /* the serving arena budget does not admit the request */
  SBBF_EUNSUPPORTED = 5,/* the option is not available on this device */
  SBBF_EAGAIN = 6       /* nothing to do yet (serving poll) */
} sbbf_status;

/* Insert strategies. All produce identical filter bytes. */
typedef enum sbbf_insert_strategy {
  SBBF_INSERT_AUTO = 0,     /* library choice by filter size and key count */
  SBBF_INSERT_ATOMIC32 = 1, /* one key per K lanes (K = words per block, 8 unless a
                               variant), one 32-bit global atomic OR per lane */
  SBBF_INSERT_ATOMIC64 = 2, /* one key per K/2 lanes, one 64-bit global atomic OR per lane */
  SBBF_INSERT_LDS = 3,      /* private copies of the whole filter in LDS, OR-merged;
                               only when the filter's 4 * K * num_blocks bytes fit one
                               workgroup's LDS */
  SBBF_INSERT_PARTITIONED = 4 /* keys split by filter slice (a slice fits one workgroup's
                               LDS), then one workgroup ORs each slice in LDS and stores
                               it back; no global atomics on the filter. Filters of up
                               to 2,048 slices split without counting first: each
                               partitioning workgroup fills fixed-room buckets per
                               slice, and keys that find theirs full (skewed batches)
                               are ORed with global atomics afterwards. Uses a
                               stream-ordered device workspace of about 22 bytes per
                               key (8 bytes per key with counting; batches above 2^31
                               keys are processed 2^31 at a time). Filters of more than
                               4,096 slices (above 512 MiB) are partitioned in two
                               levels (by group of 1,024 slices, then by slice), about
                               twice the workspace, and the call waits for the stream
                               once to size the second level */
} sbbf_insert_strategy;

/* Lookup strategies (the `strategy` field of sbbf_launch for lookups). All
 * give identical results. */
typedef enum sbbf_lookup_strategy {
  SBBF_LOOKUP_AUTO = 0,        /* library choice by filter size and key count */
  SBBF_LOOKUP_GATHER = 1,      /* one block read per key, K lanes per key */
  SBBF_LOOKUP_PARTITIONED = 2  /* keys split by filter slice, each slice tested from one
                                  workgroup's LDS, results returned to input order. Filters
                                  of up to 2,048 slices split without counting first: each
                                  partitioning workgroup fills fixed-room buckets per slice
                                  and keys past a run's room (skewed batches) are looked up
                                  by a gather afterwards. Uses a stream-ordered device
                                  workspace of about 15 to 20 bytes per key for batches of
                                  1e8 keys and more (more for small batches over many
                                  slices: the buckets' room; about 11 with counting; batches
                                  above 2^31 keys are processed 2^31 at a time); above 4,096
                                  slices two levels, as for inserts */
} sbbf_lookup_strategy;

/* Memory-access flags of sbbf_launch (cache policy only; results are
 * identical for every value). */
enum {
  SBBF_FILTER_LOAD_DEFAULT = 0u,  /* lookup block reads: cached at every level */
  SBBF_FILTER_LOAD_NT = 1u,       /* ... with the non-temporal hint */
  SBBF_FILTER_LOAD_DEVICE = 2u,   /* ... device-coherent (skip the per-CU cache) */
  SBBF_FILTER_LOAD_SYSTEM = 3u,   /* ... system-coherent */
  SBBF_FILTER_LOAD_MASK = 3u,
  SBBF_HASH_LOAD_CACHED = 4u,     /* hash reads without the non-temporal hint */
  SBBF_RESULT_STORE_NT = 8u,      /* lookup result writes with the non-temporal hint */
  SBBF_FLAGS_MASK = 15u
};

/* Launch shape for the plain kernels. Zero fields take library defaults. */
typedef struct sbbf_launch {
  uint32_t block_threads; /* workgroup size: 64 .. 1024, a multiple of 64 */
  uint32_t grid_blocks;   /* workgroups; for SBBF_INSERT_LDS the number of private copies */
  uint32_t unroll;        /* 64-key chunks each wave keeps in flight: 1, 2, 4 or 8 (lookup: at most 4) */
  uint32_t strategy;      /* an sbbf_insert_strategy (inserts) or sbbf_lookup_strategy (lookups) */
  uint32_t flags;         /* SBBF_* memory-access flags above; 0 = library default */
} sbbf_launch;

/* Device facts the library uses to size launches (queried once per device). */
typedef struct sbbf_device_info {
  int32_t device;
  int32_t compute_units;
  int32_t max_threads_per_block;
  int32_t warp_size;
  uint64_t lds_per_block;    /* bytes of LDS one workgroup may allocate */
  uint64_t lds_per_cu;       /* bytes of LDS per compute unit */
  uint64_t l2_bytes;
  uint64_t global_mem_bytes;
  int32_t clock_khz;
  int32_t memory_clock_khz;
  int32_t memory_bus_bits;
  char arch[64];             /* e.g. "gfx950:sramecc+:xnack-" */
} sbbf_device_info;

/* ---- library ------------------------------------------------------------ */

/* Text for a status code (static storage). */
const char *sbbf_status_string(sbbf_status s);
/* Detail of the last failing call on this host thread ("" if none). */
const char *sbbf_last_error(void);
/* Facts about the current HIP device. */
sbbf_status sbbf_device_query(sbbf_device_info *out);
/* Blocks for n keys at bits_per_key bits each: max(1, ceil(n * bits_per_key / 256)).
 * Returns 0 when the result would exceed 2^32 - 1 or bits_per_key <= 0. */
uint64_t sbbf_blocks_for(uint64_t n, double bits_per_key);
/* The paper's false-positive model (analysis section, the Poisson-sum
 * equation): F(a) = sum over i >= 0 of Poisson_a(i) * (1 - (31/32)^i)^8 for
 * a mean of a = keys_per_block distinct hashes per block; computed in double. */
double sbbf_fpr_model(double keys_per_block);
/* Sizing from a target rate by inverting that model: the smallest number of
 * blocks B >= 1 with F(n / B) <= fpr. Returns 0 (and sets sbbf_last_error)
 * when fpr is not in (0, 1) or more than 2^32 - 1 blocks would be needed.
 * The paper's useful band of rates is about 0.4 % to 19 % (introduction;
 * analysis section). */
uint64_t sbbf_blocks_for_fpr(uint64_t n, double fpr);
/* The same model and sizing for the block variants with `lanes` 32-bit words
 * per block (4, 8 or 16; the paper notes that four or sixteen lanes would
 * work as well as eight, in a footnote to its list of central ideas): the
 * exponent 8 becomes `lanes`. On a bad lane count the model returns -1 and
 * the sizing 0, and sbbf_last_error says why. */
double sbbf_fpr_model_variant(double keys_per_block, uint32_t lanes);
uint64_t sbbf_blocks_for_fpr_variant(uint64_t n, double fpr, uint32_t lanes);

/* ---- single filter --------------------------------------------------------- */

/* Allocate a zeroed filter of num_blocks 256-bit blocks (1 .. 2^32 - 1) in
 * device memory owned by the handle. */
sbbf_status sbbf_create(uint32_t num_blocks, sbbf_filter **out);
/* Wrap caller-owned device memory of 32 * num_blocks bytes (32-byte
 * aligned, e.g. a torch tensor). Not cleared; never freed by the library. */
sbbf_status sbbf_create_wrapped(void *d_words, uint32_t num_blocks, sbbf_filter **out);
/* Block variants (footnote to the paper's list of central ideas: four or
 * sixteen lanes would work too). A filter of num_blocks blocks of `lanes`
 * 32-bit words (4, 8 or 16; 8 is the method itself, as sbbf_create), so
 * 4 * lanes * num_blocks bytes, block b at byte 4 * lanes * b. Block selection
 * is unchanged; word j of a block takes bit (s_j * lo32(h) mod 2^32) >> 27.
 * The paper prints seeds for eight words only: four-word blocks use its seeds
 * 0..3; sixteen-word blocks use its eight seeds for words 0..7 and, for words
 * 8..15, 0xba779207, 0xc985644b, 0xa4e84675, 0xe421c8db, 0xbd38674f,
 * 0x58ee486d, 0x8ddb3387, 0x7ea09599 (the low 32 bits of the first eight
 * outputs of SplitMix64 seeded with 16, lowest bit set). Every single-filter
 * entry point (insert, lookup, select, keys, union, serialization, copies)
 * takes variant filters; grouped plans reject them (SBBF_EUNSUPPORTED), and
 * the memory-access flags of sbbf_launch are ignored for them. SBBF_EINVAL
 * for another lane count. */
sbbf_status sbbf_create_variant(uint32_t num_blocks, uint32_t lanes, sbbf_filter **out);
sbbf_status sbbf_create_wrapped_variant(void *d_words, uint32_t num_blocks, uint32_t lanes, sbbf_filter **out);
/* 32-bit words per block of the filter (8 unless made as a variant; 0 for NULL). */
uint32_t sbbf_lanes(const sbbf_filter *f);
/* Release the handle (and its memory when owned). Does not synchronise;
 * the caller must not destroy a filter that queued work still uses. */
sbbf_status sbbf_destroy(sbbf_filter *f);
/* Zero every word, enqueued on the stream (a kernel, no memset node). */
sbbf_status sbbf_clear(sbbf_filter *f, sbbf_stream s);
uint32_t sbbf_num_blocks(const sbbf_filter *f);
void *sbbf_device_words(const sbbf_filter *f);

/* Copy the filter's 4 * lanes * num_blocks bytes to host memory, or replace them
 * from host memory (checkpoint and restore of the byte image). Enqueued on
 * the stream; with pageable host memory the copy completes before return,
 * with pinned memory the caller synchronises before touching host_dst. */
sbbf_status sbbf_copy_words_to_host(const sbbf_filter *f, void *host_dst, sbbf_stream s);
sbbf_status sbbf_copy_words_from_host(sbbf_filter *f, const void *host_src, sbbf_stream s);

/* Union: dst |= src word by word, so dst then reports present every hash
 * inserted into either (a filter is the OR of its keys' masks: appendix
 * figure, insert routine). Both filters must have the same num_blocks and
 * lanes (SBBF_EINVAL otherwise); dst == src is a no-op. Enqueued on the stream. */
sbbf_status sbbf_union(sbbf_filter *dst, const sbbf_filter *src, sbbf_stream s);

/* Serialized form of a filter: a 32-byte header (8 bytes "SBBF256\0",
 * uint32 version 1, uint32 seed order 1 = word j uses seed j in the
 * little-endian lane order of the appendix figure's constants (then, for
 * sixteen-word blocks, the eight further seeds of sbbf_create_variant),
 * uint32 num_blocks, uint32 word size 4, uint32 words per block (8; a 0 is
 * read as 8; 4 or 16 for the variants), 4 reserved zero bytes; all
 * little-endian), then the 4 * lanes * num_blocks bytes of the filter image.
 * sbbf_serialized_bytes is the size for eight-word blocks, the _variant form
 * for any (0 for a bad lane count). */
uint64_t sbbf_serialized_bytes(uint32_t num_blocks);
uint64_t sbbf_serialized_bytes_variant(uint32_t num_blocks, uint32_t lanes);
/* Write the serialized form to host memory of at least
 * sbbf_serialized_bytes_variant(num_blocks, lanes) bytes; waits for the
 * stream (the image is the filter after all work enqueued before the call). */
sbbf_status sbbf_serialize(const sbbf_filter *f, void *host_dst, size_t capacity, sbbf_stream s);
/* A new library-owned filter from a serialized form of exactly `size` bytes.
 * SBBF_EINVAL on a bad magic, size or block count, SBBF_EUNSUPPORTED on
 * another version, word size, seed order or words per block. Synchronous. */
sbbf_status sbbf_deserialize(const void *host_src, size_t size, sbbf_filter **out);

/* The strategy SBBF_INSERT_AUTO / SBBF_LOOKUP_AUTO picks for a batch of n
 * hashes on this filter and the current device (0 on a bad argument).
 * Inserts: partitioned when n is at least two keys per block and at least
 * 4M keys (and the filter splits into at most 4,096 slices), else 32-bit
 * atomics. Lookups: the cheaper of the gather and the partitioned lookup by
 * a cost model fitted to MI355X measurements (filter size and n). */
uint32_t sbbf_auto_insert_strategy(const sbbf_filter *f, size_t n);
uint32_t sbbf_auto_lookup_strategy(const sbbf_filter *f, size_t n);

/* Insert n hashes (appendix figure, insert routine; applied to every hash). */
sbbf_status sbbf_insert_batch(sbbf_filter *f, const uint64_t *d_hashes, size_t n, sbbf_stream s);
/* As sbbf_insert_batch with an explicit strategy and launch shape (NULL = defaults). */
sbbf_status sbbf_insert_batch_ex(sbbf_filter *f, const uint64_t *d_hashes, size_t n, const sbbf_launch *cfg,
                                 sbbf_stream s);
/* Look up n hashes; d_out[i] = 1 when hash i is reported present, else 0
 * (appendix figure, lookup routine). */
sbbf_status sbbf_lookup_batch(const sbbf_filter *f, const uint64_t *d_hashes, size_t n, uint8_t *d_out,
                              sbbf_stream s);
/* As sbbf_lookup_batch, packed: bit (i % 32) of d_bits[i / 32]; all
 * ceil(n / 32) words are written, unused high bits are 0. d_bits 4-byte aligned. */
sbbf_status sbbf_lookup_batch_bits(const sbbf_filter *f, const uint64_t *d_hashes, size_t n, uint32_t *d_bits,
                                   sbbf_stream s);
/* Lookup with an explicit launch shape (NULL = defaults). Exactly one of
 * d_out and d_bits is non-NULL. */
sbbf_status sbbf_lookup_batch_ex(const sbbf_filter *f, const uint64_t *d_hashes, size_t n, uint8_t *d_out,
                                 uint32_t *d_bits, const sbbf_launch *cfg, sbbf_stream s);

/* ---- keys instead of hashes -------------------------------------------------
 * The method hashes each key once to 64 bits and leaves the hash function
 * open (construction paragraph). These entry points take 64-bit keys and
 * hash them on the device as they are loaded, with sbbf_key_hash: the 64-bit
 * finalizer of MurmurHash3 (A. Appleby), k ^= k >> 33; k *= 0xff51afd7ed558ccd;
 * k ^= k >> 33; k *= 0xc4ceb9fe1a85ec53; k ^= k >> 33 (all mod 2^64), a
 * bijection with full avalanche, so distinct keys give distinct hashes. The
 * result is identical to inserting or looking up sbbf_key_hash(key). */
uint64_t sbbf_key_hash(uint64_t key);
/* As sbbf_insert_batch_ex on the hashes of n keys (cfg NULL = defaults). */
sbbf_status sbbf_insert_keys(sbbf_filter *f, const uint64_t *d_keys, size_t n, const sbbf_launch *cfg,
                             sbbf_stream s);
/* As sbbf_lookup_batch_ex with d_out on the hashes of n keys. */
sbbf_status sbbf_lookup_keys(const sbbf_filter *f, const uint64_t *d_keys, size_t n, uint8_t *d_out,
                             const sbbf_launch *cfg, sbbf_stream s);

/* Lookup with stream compaction: writes, in ascending order, the indices i of
 * the hashes the filter reports present (appendix figure, lookup routine) to
 * d_indices[0 .. count) and count to *d_count. The paper names database
 * engines as the filter's users (introduction; the discussion after the
 * evaluation table); there a lookup decides which rows go on, and this entry
 * point returns just those rows' indices. d_indices holds room for up to n
 * indices (uint32, 4-byte aligned,
 * caller-owned); d_count is one uint64 in device memory (8-byte aligned),
 * written by the device (0 when n == 0). n < 2^32. cfg chooses the lookup
 * strategy and launch shape as for sbbf_lookup_batch_ex (NULL = defaults).
 * Uses a stream-ordered workspace of about n / 8 bytes. */
sbbf_status sbbf_lookup_select(const sbbf_filter *f, const uint64_t *d_hashes, size_t n, uint32_t *d_indices,
                               uint64_t *d_count, const sbbf_launch *cfg, sbbf_stream s);

/* Allocation-free form of sbbf_lookup_select, for callers that cannot
 * allocate device memory during the call: code under HIP graph capture,
 * tight serving loops, and harnesses that forbid hipMalloc. Same arguments,
 * results and argument checks as sbbf_lookup_select, with three differences:
 *   - the lookup is always the gather (cfg's strategy must be
 *     SBBF_LOOKUP_AUTO or SBBF_LOOKUP_GATHER; SBBF_EUNSUPPORTED for the
 *     partitioned lookup, which allocates a workspace);
 *   - the workspace (result bitmap and per-tile counts and offsets) is a
 *     static device array of 33,816,576 bytes that each GPU the library runs
 *     on holds until the process ends; no device memory is allocated or
 *     freed by the call;
 *   - n is at most 2^28 (268,435,456) keys per call; a larger n returns
 *     SBBF_EINVAL and enqueues nothing.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents: calls on one stream are ordered and safe, but calls that overlap
 * in time on one GPU (on different streams, or from different host threads)
 * race on the array and give wrong results. */
sbbf_status sbbf_lookup_select_noalloc(const sbbf_filter *f, const uint64_t *d_hashes, size_t n,
                                       uint32_t *d_indices, uint64_t *d_count, const sbbf_launch *cfg,
                                       sbbf_stream s);

/* ---- measurement kernels (same access pattern, no filter arithmetic) ------- */

/* Random 32-byte gather ceiling: for each hash, read the 32-byte block
 * ((h >> 32) * num_blocks) >> 32 of d_buf with 8 lanes and write one byte
 * (1 when the block has any non-zero word). Same launch shape as lookup. */
sbbf_status sbbf_bench_gather(const uint32_t *d_buf, uint32_t num_blocks, const uint64_t *d_hashes, size_t n,
                              uint8_t *d_out, const sbbf_launch *cfg, sbbf_stream s);
/* Random atomic-OR ceiling: for each hash, OR a fixed one-bit word into each
 * of the 8 words of its block with 32-bit global atomics (or 4 x 64-bit when
 * strategy == SBBF_INSERT_ATOMIC64). */
sbbf_status sbbf_bench_atomic(uint32_t *d_buf, uint32_t num_blocks, const uint64_t *d_hashes, size_t n,
                              const sbbf_launch *cfg, sbbf_stream s);
/* Streaming ceiling: read n uint64, write n bytes (the low byte's parity). */
sbbf_status sbbf_bench_stream(const uint64_t *d_hashes, size_t n, uint8_t *d_out, const sbbf_launch *cfg,
                              sbbf_stream s);

/* ---- grouped: many filters in one launch ----------------------------------- */
/* A group holds F filters. A run performs every filter's inserts, then every
 * filter's lookups (each filter as in the appendix figure's insert and lookup
 * routines), as one HIP graph launch of a few kernel nodes; results are
 * identical to one plain insert and one plain lookup per filter. Key ranges are
 * CSR offsets: filter f inserts d_ins[ins_off[f] .. ins_off[f+1]) and looks up
 * d_look[look_off[f] .. look_off[f+1]), writing d_out[look_off[f] ..].
 *
 * Two kinds of plan:
 *   - fixed shape (sbbf_grouped_plan): the offsets are given on the host once
 *     and every sbbf_grouped_run uses them;
 *   - capacity (sbbf_grouped_plan_capacity): the plan fixes, per filter, the
 *     most keys one run may insert and look up; every sbbf_grouped_run_offsets
 *     brings its own offsets in device memory, read by the kernels when the
 *     graph runs. Changing the counts needs no host planning and no graph
 *     rebuild (the graph is updated only when a buffer pointer changes), so a
 *     caller whose per-filter counts change on every call rewrites the offset
 *     buffers on the device and launches again. */

typedef struct sbbf_grouped_config {
  uint32_t lookup_tile_keys;     /* keys per lookup tile, a multiple of 64 */
  uint32_t lookup_threads;       /* lookup workgroup size: 64, 128, 192 or 256 */
  uint32_t lookup_unroll;        /* 64-key chunks in flight per wave: 1, 2 or 4 */
  uint32_t lookup_blocks_per_cu; /* persistent lookup workgroups per compute unit */
  uint32_t insert_slice_shift;   /* log2 blocks per insert slice (a slice fits one workgroup's LDS) */
  uint32_t xcd_queues;           /* 1: lookup tiles of a filter stay on one XCD queue; 0: one queue */
  uint64_t insert_lds_bytes;     /* filters up to this size are inserted whole by one workgroup */
  uint32_t lookup_lds_slices;    /* filters of at most this many slices of 4 * lookup_lds_threads blocks are
                                    looked up from LDS, one slice at a time, by tiles of 16 keys per thread
                                    held in registers; 0: every filter is looked up by the gather */
  uint32_t lookup_lds_threads;   /* LDS lookup workgroup size: 256, 512 or 1024 (slices of 32, 64 or 128 KiB) */
} sbbf_grouped_config;

/* Defaults for the current device. */
sbbf_status sbbf_grouped_default_config(sbbf_grouped_config *out);
/* A group over filters[0 .. num_filters) (handles are borrowed; they must outlive
 * the group). Their memory must not overlap (a filter appears once): else
 * SBBF_EINVAL. */
sbbf_status sbbf_grouped_create(sbbf_filter *const *filters, uint32_t num_filters, sbbf_group **out);
sbbf_status sbbf_grouped_destroy(sbbf_group *g);
/* Build the plan from host offsets (num_filters + 1 entries each, non-decreasing;
 * at most 2^32 - 1 insert keys per filter). cfg NULL = defaults. Synchronous. */
sbbf_status sbbf_grouped_plan(sbbf_group *g, const uint64_t *h_ins_offsets, const uint64_t *h_look_offsets,
                              const sbbf_grouped_config *cfg);
/* Build a capacity plan: h_ins_cap[f] and h_look_cap[f] (num_filters entries
 * each, host memory) are the most keys filter f inserts and looks up in one
 * run (at most 2^32 - 1 insert keys per filter). Tiles, queues and the
 * partitioned-key region are sized for these capacities; a run with fewer keys
 * skips the work it does not have. cfg NULL = defaults. Synchronous. */
sbbf_status sbbf_grouped_plan_capacity(sbbf_group *g, const uint64_t *h_ins_cap, const uint64_t *h_look_cap,
                                       const sbbf_grouped_config *cfg);
/* The configuration of the current plan. */
sbbf_status sbbf_grouped_get_config(const sbbf_group *g, sbbf_grouped_config *out);
/* Inserts, then lookups, of the planned batch as one graph launch on the stream. */
sbbf_status sbbf_grouped_run(sbbf_group *g, const uint64_t *d_ins, const uint64_t *d_look, uint8_t *d_out,
                             sbbf_stream s);
/* One run under a capacity plan: d_ins_offsets and d_look_offsets are
 * num_filters + 1 uint64 each in device memory (8-byte aligned, caller-owned),
 * read by the kernels when the run executes, so they may be written on the
 * stream just before it. Filter f inserts d_ins[d_ins_offsets[f] ..
 * d_ins_offsets[f+1]) and looks up d_look[d_look_offsets[f] ..
 * d_look_offsets[f+1]), writing d_out at the same positions. d_ins, d_look
 * and d_out must hold the ranges the offsets name. A filter whose range is
 * decreasing or longer than its capacity has only its first capacity keys
 * processed (no access beyond them); the run records the lowest such filter
 * for sbbf_grouped_check. SBBF_EINVAL on a group with a fixed-shape plan. */
sbbf_status sbbf_grouped_run_offsets(sbbf_group *g, const uint64_t *d_ins, const uint64_t *d_ins_offsets,
                                     const uint64_t *d_look, const uint64_t *d_look_offsets, uint8_t *d_out,
                                     sbbf_stream s);
/* Waits for the stream, then reports whether every run since the last check
 * kept its key ranges within the plan's capacities: SBBF_OK and *first_bad =
 * 0xFFFFFFFF if so, else SBBF_EINVAL, *first_bad = the lowest offending filter,
 * and the record is cleared. first_bad may be NULL. */
sbbf_status sbbf_grouped_check(sbbf_group *g, sbbf_stream s, uint32_t *first_bad);
/* Host work done for the group so far: plans built (autotuning builds one per
 * candidate), graphs instantiated, and graph updates (a run with different
 * buffer pointers than the graph holds). Any pointer may be NULL. */
sbbf_status sbbf_grouped_counters(const sbbf_group *g, uint64_t *plans, uint64_t *graph_builds,
                                  uint64_t *graph_updates);
/* The two phases as separate kernel launches (no graph). This, the per-filter
 * baseline, the output digest and the autotuner need a fixed-shape plan
 * (SBBF_EINVAL on a capacity plan). */
sbbf_status sbbf_grouped_insert(sbbf_group *g, const uint64_t *d_ins, sbbf_stream s);
sbbf_status sbbf_grouped_lookup(sbbf_group *g, const uint64_t *d_look, uint8_t *d_out, sbbf_stream s);
/* Baseline with the same results: one plain launch per filter per operation,
 * each with the library's default strategy (as sbbf_insert_batch and
 * sbbf_lookup_batch choose it for that filter and key count). */
sbbf_status sbbf_grouped_run_per_filter(sbbf_group *g, const uint64_t *d_ins, const uint64_t *d_look,
                                        uint8_t *d_out, sbbf_stream s);
/* 64-bit digest of every filter's words (in group order) and of d_out over the
 * planned lookups (d_out may be NULL). Synchronises the stream. */
sbbf_status sbbf_grouped_digest(sbbf_group *g, const uint8_t *d_out, sbbf_stream s, uint64_t *digest);
/* Search launch configurations for the planned batch, timing `reps` graph
 * launches per candidate. Synchronous: waits for the device first, so the
 * inputs may come from any stream. The filters are restored to their contents before
 * every candidate and after the search, so the search leaves them unchanged.
 * Every candidate must produce the same digest as the first, else
 * SBBF_EDEVICE. The best configuration is planned and returned in *best.
 * With cache_path, a stored result for this device and batch shape is used
 * instead of searching (unless force != 0), and a new result is appended. */
sbbf_status sbbf_grouped_autotune(sbbf_group *g, const uint64_t *d_ins, const uint64_t *d_look, uint8_t *d_out,
                                  uint32_t reps, const char *cache_path, int force, sbbf_grouped_config *best);

/* ---- serving: resident filters, continuous batching ------------------------ */
/* The server keeps filters resident in a device arena bounded by a byte budget
 * and queues requests (insert or lookup batches of any size, hashes and outputs
 * in device memory) per filter. Each round of its loop launches, into every
 * free step slot, one step made of the queued requests: per filter the longest
 * queue prefix of the form inserts-then-lookups, so a lookup sees exactly the
 * inserts that arrived before it on its filter, as if run alone. Steps run in
 * order on the server's stream; new requests join the next step while earlier
 * ones run. Not thread-safe: one host thread drives a server. */

typedef struct sbbf_server_config {
  uint64_t hbm_budget_bytes;   /* bytes of filters the arena admits */
  uint32_t max_inflight_steps; /* steps queued on the device at once (slots), 1..64 */
  uint32_t max_step_requests;  /* requests per step */
  uint64_t max_step_keys;      /* keys per step (a larger single request runs alone) */
  uint32_t tile_keys;          /* keys per workgroup tile, a multiple of 64 */
  uint32_t reserved;
} sbbf_server_config;

typedef struct sbbf_request {
  uint64_t arrival_ns;   /* replay: arrival time relative to the start of the replay */
  uint32_t filter_id;
  uint32_t op;           /* 0 insert, 1 lookup */
  const uint64_t *d_hashes;
  uint8_t *d_out;        /* lookups: one byte per hash */
  uint64_t n;
} sbbf_request;

typedef struct sbbf_serving_stats {
  uint64_t requests_done, keys_done, steps;
  double p50_us, p99_us, max_us; /* latency: completion seen by the host minus arrival */
  double span_s;                 /* first arrival to last completion */
  double gkeys_per_s;            /* keys_done / span_s / 1e9 */
  uint64_t arena_used_bytes, arena_reserved_bytes;
} sbbf_serving_stats;

sbbf_status sbbf_server_default_config(sbbf_server_config *out);
sbbf_status sbbf_server_create(const sbbf_server_config *cfg, sbbf_server **out);
/* Waits for queued device work, then frees everything. */
sbbf_status sbbf_server_destroy(sbbf_server *s);
/* Admit a zeroed filter of num_blocks blocks; SBBF_EBUDGET when the budget does
 * not allow it (the caller may retry after removing filters). */
sbbf_status sbbf_server_add_filter(sbbf_server *s, uint32_t num_blocks, uint32_t *filter_id);
/* Finish the filter's queued work, then release its memory and id. */
sbbf_status sbbf_server_remove_filter(sbbf_server *s, uint32_t filter_id);
sbbf_status sbbf_server_arena_usage(const sbbf_server *s, uint64_t *used_bytes, uint64_t *reserved_bytes);
/* Queue one request (arrival = now). Buffers stay caller-owned and must
 * remain valid until the request completes. */
sbbf_status sbbf_server_submit(sbbf_server *s, uint32_t filter_id, int op, const uint64_t *d_hashes, uint64_t n,
                               uint8_t *d_out, uint64_t *req_id);
/* One round of the loop: record finished steps, launch steps into free slots;
 * with wait != 0 and nothing launched, block until one step finishes. */
sbbf_status sbbf_server_pump(sbbf_server *s, int wait);
/* Run the loop until every queued request has completed. */
sbbf_status sbbf_server_drain(sbbf_server *s);
/* Completed request ids since the last poll (SBBF_EAGAIN when none). */
sbbf_status sbbf_server_poll(sbbf_server *s, uint64_t *done_ids, uint32_t cap, uint32_t *n_done);
sbbf_status sbbf_server_request_times(const sbbf_server *s, uint64_t req_id, uint64_t *arrival_ns, uint64_t *done_ns);
/* Drive a request log (sorted by arrival_ns) through the loop from this thread:
 * with realtime != 0 each request is queued when its arrival time is reached,
 * else all are due at once (queued 2,048 per round of the loop, so that steps
 * start while the rest are queued; arrival time = when queued). Returns when
 * all have completed; *first_id is the id of log[0] (ids are consecutive). */
sbbf_status sbbf_server_replay(sbbf_server *s, const sbbf_request *log, uint64_t count, int realtime,
                               uint64_t *first_id);
/* Baseline with the same results as sbbf_server_replay: waits for queued work,
 * then issues every request of the log in order as one plain call on the
 * server's stream (sbbf_insert_batch_ex with 32-bit atomics, or
 * sbbf_lookup_batch_ex with the gather) against the resident filters, with no
 * batching and no arrival times; waits for the stream and returns the wall
 * time from the first call to the end in *seconds. Filter ids must be
 * resident and ops 0 or 1 (else SBBF_EINVAL, nothing issued). Each request
 * sees exactly the requests before it, so the filters and lookup outputs equal
 * the serving loop's on the same log. */
sbbf_status sbbf_server_replay_per_request(sbbf_server *s, const sbbf_request *log, uint64_t count,
                                           double *seconds);
sbbf_status sbbf_server_stats(const sbbf_server *s, sbbf_serving_stats *out);
/* Checkpoint / restore one filter's bytes (waits for all queued work first). */
sbbf_status sbbf_server_snapshot(sbbf_server *s, uint32_t filter_id, void *host_dst);
sbbf_status sbbf_server_restore(sbbf_server *s, uint32_t filter_id, const void *host_src);

#ifdef __cplusplus
} /* extern "C" */
#endif

#endif /* SBBF_H_ */
