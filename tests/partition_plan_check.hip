// Host-side check of the partition planner (no device needed): for a sweep
// of batch sizes, slice counts and workgroup counts, every plan the
// partitioned insert and lookup can choose keeps the invariants its kernels'
// indexing relies on (positions in 16 bits, bucket positions in 32 bits,
// whole result words, workspace sections large enough and disjoint, LDS
// within a compute unit's 160 KiB). Compiled together with the planner's
// source by tests/test_partition_plan.py; prints one line per violation and
// "plan check ok" at the end.
#include "../paper_2101_01719_amd/csrc/partition_kernels.hip"

#include <stdio.h>

namespace sbbf {
// The planner's translation unit launches a fill kernel defined elsewhere in
// the library; never called here.
hipError_t launch_fill(uint32_t *, uint64_t, uint32_t, hipStream_t) { return hipErrorNotSupported; }
}  // namespace sbbf

static int fails = 0;
static unsigned long long checks = 0;
#define CHECK(c, ...)                                                       \
  do {                                                                      \
    ++checks;                                                               \
    if (!(c)) {                                                             \
      if (++fails <= 40) {                                                  \
        fprintf(stderr, "violated: %s (", #c);                              \
        fprintf(stderr, __VA_ARGS__);                                       \
        fprintf(stderr, ")\n");                                             \
      }                                                                     \
    }                                                                       \
  } while (0)

using namespace sbbf;

static const size_t kLdsPerCu = 160u << 10;

static void check_look(uint64_t n, uint32_t P, uint32_t mg) {
  LookPlan lp;
  if (!look_plan(n, P, mg, &lp)) {
    // the library then takes the counted partition: only for one- and
    // two-slice filters (no room for a 7,168-key chunk) or more than 2,048
    CHECK(n == 0 || P > 2u * kScatterThreads || P <= 2u, "n=%llu P=%u mg=%u: no count-free plan",
          (unsigned long long)n, P, mg);
    return;
  }
  const char *fmt = "n=%llu P=%u mg=%u";
  const unsigned long long nn = n;
  CHECK(lp.room >= 32u && lp.room <= 4096u && (lp.room & (lp.room - 1u)) == 0u, fmt, nn, P, mg);
  CHECK((uint64_t)P * lp.room <= 65536u, fmt, nn, P, mg);               // 16-bit positions
  CHECK(lp.chunk % kTile == 0u && lp.chunk >= kTile && lp.chunk <= 9u * kTile, fmt, nn, P, mg);
  CHECK(lp.chunk % 256u == 0u, fmt, nn, P, mg);                         // whole output words per wave span
  CHECK((uint64_t)lp.groups == (n + lp.chunk - 1u) / lp.chunk, fmt, nn, P, mg);
  CHECK(lp.per >= 1u && lp.sgroups >= 1u && lp.sgroups <= kMaxBucketGroups, fmt, nn, P, mg);
  CHECK((uint64_t)(lp.sgroups - 1u) * lp.per < lp.groups && (uint64_t)lp.sgroups * lp.per >= lp.groups, fmt, nn, P,
        mg);                                                            // no empty scatter workgroup
  CHECK(lp.cap % 32u == 0u && lp.cap >= 32u, fmt, nn, P, mg);            // bucket words are whole
  const uint64_t positions = (uint64_t)lp.sgroups * P * lp.cap;
  CHECK(positions < (1ull << 32) - 64u, fmt, nn, P, mg);
  // workspace sections: 256-byte aligned, in order, each large enough
  const uint64_t off[] = {lp.runs_off, lp.count_off, lp.ovfn_off, lp.ovf_off, lp.pos_off, lp.keys_off, lp.res_off,
                          lp.bytes};
  const uint64_t need[] = {(uint64_t)lp.groups * P * 8u, (uint64_t)lp.sgroups * P * 4u, 4u, n * 4u, n * 2u,
                           positions * 8u, (positions / 32u + 2u) * 4u};
  for (int k = 0; k < 7; ++k) {
    CHECK(off[k] % 256u == 0u, fmt, nn, P, mg);
    CHECK(off[k + 1] >= off[k] + need[k], "section %d: n=%llu P=%u mg=%u", k, nn, P, mg);
  }
  CHECK(partition_workspace_bytes(n, P, mg, true) >= lp.bytes, fmt, nn, P, mg);
  // unpermute workgroups: chunks of one scatter workgroup, LDS for two per CU,
  // 16-bit run offsets
  const uint32_t per_u = look_unpermute_chunks(lp, P);
  CHECK(per_u >= 1u && per_u <= kUnpermuteChunks && per_u <= lp.per, fmt, nn, P, mg);
  const size_t u_lds = look_unpermute_lds(per_u, P, lp.room);
  CHECK(u_lds <= kUnpermuteLds && 2u * u_lds <= kLdsPerCu, fmt, nn, P, mg);
  CHECK(31u + (uint64_t)per_u * lp.room <= 65535u, fmt, nn, P, mg);
  // scatter and slice-kernel LDS
  const uint32_t R = P <= kScatterThreads ? 1u : 2u, L = R == 1u ? kScatterGroup : 4u;
  CHECK(scatter_lds_bytes(P, true, L, R) <= kLdsPerCu, fmt, nn, P, mg);
  for (uint32_t K : {4u, 8u, 16u}) {
    const size_t slice = 131072u;  // the largest slice the library makes
    CHECK(slice + (2u * kMaxBucketGroups + 1u + (kBucketMap + 2u) / 2u + 16u) * 4u <= kLdsPerCu, "K=%u", K);
  }
}

static void check_insert_buckets(uint64_t n, uint32_t P, uint32_t mg) {
  BucketPlan bp;
  if (!bucket_plan(n, P, mg, &bp)) return;  // the counted insert partition then
  const unsigned long long nn = n;
  CHECK(bp.groups >= 1u && bp.groups <= kMaxBucketGroups && bp.chunk % kInsertTile == 0u, "ins n=%llu P=%u mg=%u", nn, P,
        mg);
  CHECK((uint64_t)bp.groups * bp.chunk >= n && (uint64_t)(bp.groups - 1u) * bp.chunk < n, "ins n=%llu", nn);
  CHECK(bp.cap % 8u == 0u && bp.cap >= 32u, "ins cap n=%llu P=%u", nn, P);   // whole 64-byte groups
  const uint64_t positions = (uint64_t)bp.groups * P * bp.cap;
  CHECK(positions < (1ull << 32), "ins positions n=%llu P=%u mg=%u", nn, P, mg);
  const uint64_t off[] = {bp.count_off, bp.ovfn_off, bp.ovf_off, bp.keys_off, bp.bytes};
  const uint64_t need[] = {(uint64_t)bp.groups * P * 4u, 4u, n * 8u, positions * 8u};
  for (int k = 0; k < 4; ++k) {
    CHECK(off[k] % 256u == 0u, "ins n=%llu", nn);
    CHECK(off[k + 1] >= off[k] + need[k], "ins section %d: n=%llu P=%u mg=%u", k, nn, P, mg);
  }
  CHECK(partition_workspace_bytes(n, P, mg, false) >= bp.bytes, "ins ws n=%llu P=%u", nn, P);
  const uint32_t R = P <= kScatterThreads ? 1u : 2u, L = R == 1u ? kScatterGroup : 4u;
  CHECK(scatter_lds_bytes(P, false, L, R, kInsertPer) <= kLdsPerCu, "ins scatter LDS P=%u", P);
}

static void check_counted(uint64_t n, uint32_t P, uint32_t mg) {
  uint32_t chunk, groups;
  chunking(n, mg, true, &chunk, &groups);
  const unsigned long long nn = n;
  CHECK(chunk % kTile == 0u && chunk <= kLookupChunk, "counted n=%llu P=%u mg=%u", nn, P, mg);
  CHECK((uint64_t)groups * chunk >= n && (uint64_t)(groups - 1u) * chunk < (n ? n : 1u), "counted n=%llu", nn);
  const PartitionLayout L = layout(nullptr, n, P, groups, true);
  CHECK(L.bytes >= n * 2u + (n + 31ull * P) * 8u, "counted n=%llu P=%u", nn, P);
  const uint32_t R = kMaxSlices / kPartThreads;
  CHECK(P <= R * kPartThreads, "P=%u", P);
  CHECK(scatter_lds_bytes(P, true, P <= kScatterThreads ? kScatterGroup : (P <= 2u * kScatterThreads ? 4u : 1u),
                          P <= kScatterThreads ? 1u : (P <= 2u * kScatterThreads ? 2u : 4u)) <= kLdsPerCu,
        "counted scatter LDS P=%u", P);
}

int main() {
  const uint64_t ns[] = {1, 3, 4, 5, 255, 256, 257, 7167, 7168, 7169, 28671, 28672, 28673, 43008, 100000, 1000003,
                         12345678, 100000000, 200000000, 1ull << 31};
  const uint32_t Ps[] = {1, 2, 3, 4, 5, 17, 40, 64, 255, 256, 257, 300, 301, 511, 512, 513, 1000, 1023, 1024, 1025,
                         1536, 1537, 2047, 2048, 2049, 4096};
  const uint32_t mgs[] = {1, 2, 3, 7, 64, 100, 256, 512, 1023, 1024, 2048};
  for (uint64_t n : ns)
    for (uint32_t P : Ps)
      for (uint32_t mg : mgs) {
        check_look(n, P, mg);
        check_insert_buckets(n, P, mg);
        if (P <= kMaxSlices) check_counted(n, P, mg);
      }
  if (fails) {
    fprintf(stderr, "%d of %llu checks failed\n", fails, checks);
    return 1;
  }
  printf("plan check ok: %llu checks\n", checks);
  return 0;
}
