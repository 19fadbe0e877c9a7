// Host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "sbbf.h"

struct sbbf_filter {
  uint32_t *words;      // lanes * num_blocks uint32, 32-byte aligned device memory
  uint32_t num_blocks;  // 1 .. 2^32 - 1
  bool owned;           // memory allocated by sbbf_create
  int device;           // device current when the handle was made
  uint32_t lanes;       // 32-bit words per block: 8 (the method), or 4 or 16 (block variants)
};

namespace sbbf {

// Resolved launch shape of one plain kernel call.
struct Shape {
  uint32_t threads;  // workgroup size, multiple of 64
  uint32_t grid;     // workgroups
  uint32_t unroll;   // 64-key chunks per wave in flight (1, 2, 4, 8)
  uint32_t flags;    // SBBF_* memory-access flags
  uint32_t keys;     // 1: the input holds keys, hashed on load (key_hash)
  uint32_t lanes;    // 32-bit words per block (8, or 4 or 16 for the block variants)
};

// Allocation-failure injection, for tests of the error paths: while the
// environment variable SBBF_FAULT_INJECT is "alloc", every device, stream-
// ordered or pinned host allocation the library makes fails with
// hipErrorOutOfMemory (the call returns SBBF_ENOMEM) without being attempted.
// These wrappers are the library's only allocation calls.
bool fault_alloc();
hipError_t dev_malloc(void **p, size_t bytes);
hipError_t dev_malloc_async(void **p, size_t bytes, hipStream_t stream);
hipError_t host_malloc_mapped(void **p, size_t bytes, unsigned int flags);

// Cached device facts (per device, queried once).
const sbbf_device_info &device_info(int device);
const sbbf_device_info *current_device_info(sbbf_status *st);

// Thread-local error text and status helpers.
sbbf_status set_error(sbbf_status s, const std::string &msg);
sbbf_status hip_error(hipError_t e, const char *what);
void clear_error();

// Launch-shape resolution: fills zero fields with defaults for n keys.
sbbf_status resolve_shape(const sbbf_launch *cfg, uint64_t n, uint32_t default_unroll, Shape *out,
                          uint32_t max_unroll = 8);

// Kernel launchers (plain_kernels.hip). All are asynchronous on `stream`.
hipError_t launch_lookup(const uint64_t *hashes, uint64_t n, const uint32_t *words, uint32_t num_blocks,
                         uint8_t *out8, uint32_t *out_bits, const Shape &shape, hipStream_t stream);
hipError_t launch_insert_atomic32(const uint64_t *hashes, uint64_t n, uint32_t *words, uint32_t num_blocks,
                                  const Shape &shape, hipStream_t stream);
hipError_t launch_insert_atomic64(const uint64_t *hashes, uint64_t n, uint32_t *words, uint32_t num_blocks,
                                  const Shape &shape, hipStream_t stream);
// LDS-private insert. With shape.grid == 1 the single workgroup owns the
// filter (load, OR, plain store); with more, each workgroup ORs a zeroed
// private copy and merges its non-zero words with global atomics.
hipError_t launch_insert_lds(const uint64_t *hashes, uint64_t n, uint32_t *words, uint32_t num_blocks,
                             const Shape &shape, hipStream_t stream);
hipError_t launch_fill(uint32_t *words, uint64_t num_words, uint32_t value, hipStream_t stream);
// dst[i] |= src[i] for i < num_words (a multiple of 8; both 32-byte aligned).
hipError_t launch_union(uint32_t *dst, const uint32_t *src, uint64_t num_words, hipStream_t stream);

// Partitioned insert and lookup (partition_kernels.hip). Slices hold
// 2^slice_shift blocks (at most partition_max_slices() slices); one launch
// takes at most partition_max_keys() keys; the batch is cut into at most
// `max_groups` chunks (one partitioning workgroup each); `workspace` holds
// partition_workspace_bytes(n, slices, max_groups, lookup) bytes.
uint32_t partition_max_slices();
// Slices one level of the partition handles; filters with more take two
// levels (keys grouped by runs of this many slices first; the host waits for
// the stream once per call to size the second level).
uint32_t partition_level_slices();
uint32_t partition_group_slices();  // slices per level-2 group
uint64_t partition_max_keys();
uint64_t partition_workspace_bytes(uint64_t n, uint32_t num_slices, uint32_t max_groups, bool lookup);
// keys: the input holds keys, hashed on load (key_hash).
// lanes: 32-bit words per block (8, or 4 or 16); slices hold 2^slice_shift
// blocks of 4 * lanes bytes.
hipError_t launch_insert_partitioned(const uint64_t *hashes, uint64_t n, uint32_t *words, uint32_t num_blocks,
                                     uint32_t slice_shift, void *workspace, uint32_t max_groups, uint32_t keys,
                                     hipStream_t stream, uint32_t lanes = 8);
hipError_t launch_lookup_partitioned(const uint64_t *hashes, uint64_t n, const uint32_t *words, uint32_t num_blocks,
                                     uint32_t slice_shift, void *workspace, uint32_t max_groups, uint8_t *out8,
                                     uint32_t *out_bits, uint32_t keys, hipStream_t stream, uint32_t lanes = 8);

// Stream compaction of a lookup bitmap (select.hip): the workspace starts
// with the bitmap (ceil(n / 32) words, select_bits()) the lookup writes;
// launch_select writes the ascending indices of set bits and their count.
uint64_t select_workspace_bytes(uint64_t n);
uint32_t *select_bits(void *workspace);
hipError_t launch_select(uint64_t n, void *workspace, uint32_t *indices, unsigned long long *count,
                         hipStream_t stream);

// The grouped C ABI (sbbf_grouped_*) is implemented in grouped.hip.

hipError_t launch_bench_gather(const uint32_t *buf, uint32_t num_blocks, const uint64_t *hashes, uint64_t n,
                               uint8_t *out, const Shape &shape, hipStream_t stream);
hipError_t launch_bench_atomic(uint32_t *buf, uint32_t num_blocks, const uint64_t *hashes, uint64_t n, bool wide,
                               const Shape &shape, hipStream_t stream);
hipError_t launch_bench_stream(const uint64_t *hashes, uint64_t n, uint8_t *out, const Shape &shape,
                               hipStream_t stream);

}  // namespace sbbf
