// C ABI of the library: handles, argument checks, launch-shape defaults and
// dispatch to the kernels. Every public function is declared in sbbf.h.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "sbbf_device.h"
#include "sbbf.h"

namespace sbbf {
namespace {

thread_local std::string t_last_error;

// Indexed by device id. A deque: growing it for a new device keeps the entries
// other threads already hold references to in place; an entry is written once,
// under the lock, before it is marked valid, and never changes after.
std::mutex g_info_mu;
std::deque<sbbf_device_info> g_info;
std::deque<bool> g_info_valid;

// Default launch shape: 256-thread workgroups and enough of them to give every
// compute unit 8 workgroups (32 waves) when the batch is large enough; the
// grid-stride loop covers the rest.
constexpr uint32_t kDefaultThreads = 256;
constexpr uint32_t kDefaultBlocksPerCU = 8;

bool aligned(const void *p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

}  // namespace

sbbf_status set_error(sbbf_status s, const std::string &msg) {
  t_last_error = msg;
  return s;
}

sbbf_status hip_error(hipError_t e, const char *what) {
  if (e == hipSuccess) return SBBF_OK;
  std::string m = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  return set_error(e == hipErrorOutOfMemory ? SBBF_ENOMEM : SBBF_EDEVICE, m);
}

void clear_error() { t_last_error.clear(); }

bool fault_alloc() {
  const char *v = getenv("SBBF_FAULT_INJECT");
  return v != nullptr && strcmp(v, "alloc") == 0;
}

hipError_t dev_malloc(void **p, size_t bytes) { return fault_alloc() ? hipErrorOutOfMemory : hipMalloc(p, bytes); }

hipError_t dev_malloc_async(void **p, size_t bytes, hipStream_t stream) {
  return fault_alloc() ? hipErrorOutOfMemory : hipMallocAsync(p, bytes, stream);
}

hipError_t host_malloc_mapped(void **p, size_t bytes, unsigned int flags) {
  return fault_alloc() ? hipErrorOutOfMemory : hipHostMalloc(p, bytes, flags);
}

const sbbf_device_info &device_info(int device) {
  std::lock_guard<std::mutex> lock(g_info_mu);
  if ((int)g_info.size() <= device) {
    g_info.resize(device + 1);
    g_info_valid.resize(device + 1, false);
  }
  if (!g_info_valid[device]) {
    sbbf_device_info info;
    memset(&info, 0, sizeof(info));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
      info.device = device;
      info.compute_units = prop.multiProcessorCount;
      info.max_threads_per_block = prop.maxThreadsPerBlock;
      info.warp_size = prop.warpSize;
      info.lds_per_block = prop.sharedMemPerBlock;
      info.lds_per_cu = prop.maxSharedMemoryPerMultiProcessor;
      info.l2_bytes = (uint64_t)prop.l2CacheSize;
      info.global_mem_bytes = prop.totalGlobalMem;
      info.clock_khz = prop.clockRate;
      info.memory_clock_khz = prop.memoryClockRate;
      info.memory_bus_bits = prop.memoryBusWidth;
      snprintf(info.arch, sizeof(info.arch), "%s", prop.gcnArchName);
      g_info[device] = info;
      g_info_valid[device] = true;
    } else {
      (void)hipGetLastError();
      static const sbbf_device_info kNone{};  // zeros; callers check compute_units
      return kNone;
    }
  }
  return g_info[device];
}

const sbbf_device_info *current_device_info(sbbf_status *st) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *st = hip_error(e, "hipGetDevice");
    return nullptr;
  }
  const sbbf_device_info &info = device_info(dev);
  if (info.compute_units <= 0) {
    *st = set_error(SBBF_EDEVICE, "hipGetDeviceProperties failed");
    return nullptr;
  }
  *st = SBBF_OK;
  return &info;
}

sbbf_status resolve_shape(const sbbf_launch *cfg, uint64_t n, uint32_t default_unroll, Shape *out,
                          uint32_t max_unroll) {
  sbbf_status st;
  const sbbf_device_info *info = current_device_info(&st);
  if (!info) return st;
  uint32_t threads = cfg && cfg->block_threads ? cfg->block_threads : kDefaultThreads;
  uint32_t unroll = cfg && cfg->unroll ? cfg->unroll : default_unroll;
  if (threads < 64 || threads > 1024 || threads % 64 != 0)
    return set_error(SBBF_EINVAL, "block_threads must be a multiple of 64 in [64, 1024]");
  if (unroll != 1 && unroll != 2 && unroll != 4 && unroll != 8)
    return set_error(SBBF_EINVAL, "unroll must be 1, 2, 4 or 8");
  if (unroll > max_unroll)
    return set_error(SBBF_EINVAL, "unroll must be at most " + std::to_string(max_unroll) + " for this kernel");
  uint32_t grid = cfg ? cfg->grid_blocks : 0;
  if (grid == 0) {
    const uint64_t keys_per_block = (uint64_t)(threads / 64) * 64u * unroll;
    const uint64_t need = (n + keys_per_block - 1) / keys_per_block;
    const uint64_t cap = (uint64_t)info->compute_units * kDefaultBlocksPerCU * (kDefaultThreads / 64) / (threads / 64);
    grid = (uint32_t)(need < cap ? (need ? need : 1) : cap);
  }
  const uint32_t flags = cfg ? cfg->flags : 0u;
  if (flags & ~(uint32_t)SBBF_FLAGS_MASK) return set_error(SBBF_EINVAL, "unknown flag bits");
  out->threads = threads;
  out->grid = grid;
  out->unroll = unroll;
  out->flags = flags;
  out->keys = 0;
  out->lanes = 8;
  return SBBF_OK;
}

}  // namespace sbbf

using namespace sbbf;

extern "C" {

const char *sbbf_status_string(sbbf_status s) {
  // A C caller may pass any integer; its bits are read as one, since loading
  // an enumerator outside the enumeration's values is undefined in C++.
  int v;
  memcpy(&v, &s, sizeof(v));
  switch (v) {
    case SBBF_OK: return "ok";
    case SBBF_EINVAL: return "invalid argument";
    case SBBF_ENOMEM: return "out of memory";
    case SBBF_EDEVICE: return "device error";
    case SBBF_EBUDGET: return "over budget";
    case SBBF_EUNSUPPORTED: return "unsupported";
    case SBBF_EAGAIN: return "try again";
  }
  return "unknown status";
}

const char *sbbf_last_error(void) { return t_last_error.c_str(); }

sbbf_status sbbf_device_query(sbbf_device_info *out) {
  if (!out) return set_error(SBBF_EINVAL, "out is NULL");
  sbbf_status st;
  const sbbf_device_info *info = current_device_info(&st);
  if (!info) return st;
  *out = *info;
  return SBBF_OK;
}

uint64_t sbbf_blocks_for(uint64_t n, double bits_per_key) {
  if (!(bits_per_key > 0.0) || !std::isfinite(bits_per_key)) return 0;
  const long double bits = (long double)n * (long double)bits_per_key;
  const long double blocks = std::ceil(bits / 256.0L);
  if (blocks > 4294967295.0L) return 0;
  return blocks < 1.0L ? 1 : (uint64_t)blocks;
}

static bool valid_lanes(uint32_t lanes) { return lanes == 4 || lanes == 8 || lanes == 16; }

// Bytes of a filter: num_blocks blocks of `lanes` 32-bit words.
static uint64_t filter_bytes(uint32_t num_blocks, uint32_t lanes) { return (uint64_t)num_blocks * 4u * lanes; }
static uint64_t filter_bytes(const sbbf_filter *f) { return filter_bytes(f->num_blocks, f->lanes); }

sbbf_status sbbf_create(uint32_t num_blocks, sbbf_filter **out) { return sbbf_create_variant(num_blocks, 8, out); }

sbbf_status sbbf_create_variant(uint32_t num_blocks, uint32_t lanes, sbbf_filter **out) {
  if (!out) return set_error(SBBF_EINVAL, "out is NULL");
  *out = nullptr;
  if (num_blocks == 0) return set_error(SBBF_EINVAL, "num_blocks must be >= 1");
  if (!valid_lanes(lanes)) return set_error(SBBF_EINVAL, "lanes must be 4, 8 or 16");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "hipGetDevice");
  void *p = nullptr;
  const size_t bytes = (size_t)filter_bytes(num_blocks, lanes);
  e = dev_malloc(&p, bytes);
  if (e != hipSuccess) return hip_error(e, "hipMalloc(filter)");
  e = hipMemset(p, 0, bytes);
  if (e != hipSuccess) {
    (void)hipFree(p);
    return hip_error(e, "hipMemset(filter)");
  }
  sbbf_filter *f = new (std::nothrow) sbbf_filter{static_cast<uint32_t *>(p), num_blocks, true, dev, lanes};
  if (!f) {
    (void)hipFree(p);
    return set_error(SBBF_ENOMEM, "handle allocation failed");
  }
  *out = f;
  return SBBF_OK;
}

sbbf_status sbbf_create_wrapped(void *d_words, uint32_t num_blocks, sbbf_filter **out) {
  return sbbf_create_wrapped_variant(d_words, num_blocks, 8, out);
}

sbbf_status sbbf_create_wrapped_variant(void *d_words, uint32_t num_blocks, uint32_t lanes, sbbf_filter **out) {
  if (!out) return set_error(SBBF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!d_words) return set_error(SBBF_EINVAL, "d_words is NULL");
  if (num_blocks == 0) return set_error(SBBF_EINVAL, "num_blocks must be >= 1");
  if (!valid_lanes(lanes)) return set_error(SBBF_EINVAL, "lanes must be 4, 8 or 16");
  if (!aligned(d_words, 32)) return set_error(SBBF_EINVAL, "filter memory must be 32-byte aligned");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "hipGetDevice");
  sbbf_filter *f = new (std::nothrow) sbbf_filter{static_cast<uint32_t *>(d_words), num_blocks, false, dev, lanes};
  if (!f) return set_error(SBBF_ENOMEM, "handle allocation failed");
  *out = f;
  return SBBF_OK;
}

sbbf_status sbbf_destroy(sbbf_filter *f) {
  if (!f) return set_error(SBBF_EINVAL, "filter is NULL");
  sbbf_status st = SBBF_OK;
  if (f->owned) {
    hipError_t e = hipFree(f->words);
    if (e != hipSuccess) st = hip_error(e, "hipFree(filter)");
  }
  delete f;
  return st;
}

sbbf_status sbbf_clear(sbbf_filter *f, sbbf_stream s) {
  if (!f) return set_error(SBBF_EINVAL, "filter is NULL");
  return hip_error(launch_fill(f->words, (uint64_t)f->num_blocks * f->lanes, 0u, (hipStream_t)s), "clear");
}

uint32_t sbbf_num_blocks(const sbbf_filter *f) { return f ? f->num_blocks : 0; }

uint32_t sbbf_lanes(const sbbf_filter *f) { return f ? f->lanes : 0; }

// ---- sizing from a target false-positive rate, union, serialization --------

// False-positive model of the analysis section: a block holding i hashes has
// a given bit of a lane set with probability 1 - (31/32)^i, and a non-member
// is reported present when all eight of its lane bits are set; with block
// loads Poisson(a) distributed, F(a) = sum over i of Poisson_a(i) times
// (1 - (31/32)^i)^8. Summed in double over i within 40 sqrt(a) + 50 of a,
// outside which the Poisson weight is far below double resolution.
static double fpr_of_load(double a, uint32_t lanes = 8) {
  if (!(a > 0.0)) return 0.0;
  // 1 - F(a) is at most K * E[(31/32)^i] = K * exp(-a / 32) under the Poisson
  // load, below fp64's resolution of 1 from about 2,000 keys per block. Far
  // above that the sum is not formed: its index would stop advancing in fp64
  // (and an infinite load would never end the loop).
  if (a > 1e6) return 1.0;
  const double w = 40.0 * std::sqrt(a) + 50.0;
  const double lo = std::max(1.0, std::floor(a - w)), hi = std::ceil(a + w);
  const double la = std::log(a), l = std::log(31.0 / 32.0);
  double s = 0.0;
  for (double i = lo; i <= hi; i += 1.0) {
    const double p = std::exp(-a + i * la - std::lgamma(i + 1.0));
    const double q = -std::expm1(i * l);  // 1 - (31/32)^i
    const double q2 = q * q, q4 = q2 * q2, q8 = q4 * q4;
    // all `lanes` bits of a non-member set: q^lanes
    s += p * (lanes == 8 ? q8 : lanes == 4 ? q4 : q8 * q8);
  }
  return s;
}

double sbbf_fpr_model(double keys_per_block) { return fpr_of_load(keys_per_block); }

double sbbf_fpr_model_variant(double keys_per_block, uint32_t lanes) {
  if (!valid_lanes(lanes)) {
    set_error(SBBF_EINVAL, "lanes must be 4, 8 or 16");
    return -1.0;
  }
  return fpr_of_load(keys_per_block, lanes);
}

uint64_t sbbf_blocks_for_fpr(uint64_t n, double fpr) { return sbbf_blocks_for_fpr_variant(n, fpr, 8); }

uint64_t sbbf_blocks_for_fpr_variant(uint64_t n, double fpr, uint32_t lanes) {
  if (!valid_lanes(lanes)) {
    set_error(SBBF_EINVAL, "lanes must be 4, 8 or 16");
    return 0;
  }
  if (!(fpr > 0.0 && fpr < 1.0)) {
    set_error(SBBF_EINVAL, "fpr must be in (0, 1)");
    return 0;
  }
  if (n == 0) return 1;
  const uint64_t max_b = 0xFFFFFFFFull;
  if (fpr_of_load((double)n / (double)max_b, lanes) > fpr) {
    set_error(SBBF_EINVAL, "the target rate needs more than 2^32 - 1 blocks for this many keys");
    return 0;
  }
  if (fpr_of_load((double)n, lanes) <= fpr) return 1;
  uint64_t lo = 1, hi = max_b;  // F(n / lo) > fpr >= F(n / hi); F grows with the load
  while (hi - lo > 1) {
    const uint64_t mid = lo + (hi - lo) / 2;
    if (fpr_of_load((double)n / (double)mid, lanes) <= fpr)
      hi = mid;
    else
      lo = mid;
  }
  return hi;
}

sbbf_status sbbf_union(sbbf_filter *dst, const sbbf_filter *src, sbbf_stream s) {
  if (!dst || !src) return set_error(SBBF_EINVAL, "filter is NULL");
  if (dst->num_blocks != src->num_blocks) return set_error(SBBF_EINVAL, "filters differ in num_blocks");
  if (dst->lanes != src->lanes) return set_error(SBBF_EINVAL, "filters differ in lanes per block");
  if (dst->words == src->words) return SBBF_OK;
  return hip_error(launch_union(dst->words, src->words, (uint64_t)dst->num_blocks * dst->lanes, (hipStream_t)s),
                   "union");
}

namespace {
// Serialized filter: a 32-byte header, then the filter's byte image.
struct SerialHeader {
  char magic[8];        // "SBBF256" and a zero byte
  uint32_t version;     // 1
  uint32_t seed_order;  // 1: word j uses seed j of the little-endian lane order of the appendix figure's constants
                        //    (sixteen-word blocks: then the eight SplitMix64-derived seeds)
  uint32_t num_blocks;
  uint32_t word_bytes;  // 4
  uint32_t lanes;       // words per block: 8 (0 is read as 8), 4 or 16
  uint32_t reserved;    // 0
};
static_assert(sizeof(SerialHeader) == 32, "header is 32 bytes");
const char kMagic[8] = {'S', 'B', 'B', 'F', '2', '5', '6', '\0'};
}  // namespace

uint64_t sbbf_serialized_bytes(uint32_t num_blocks) { return 32u + (uint64_t)num_blocks * 32u; }

uint64_t sbbf_serialized_bytes_variant(uint32_t num_blocks, uint32_t lanes) {
  return valid_lanes(lanes) ? 32u + filter_bytes(num_blocks, lanes) : 0u;
}

sbbf_status sbbf_serialize(const sbbf_filter *f, void *host_dst, size_t capacity, sbbf_stream s) {
  if (!f || !host_dst) return set_error(SBBF_EINVAL, "filter or host_dst is NULL");
  if (capacity < 32u + filter_bytes(f)) return set_error(SBBF_EINVAL, "host_dst is too small");
  SerialHeader h;
  memcpy(h.magic, kMagic, 8);
  h.version = 1;
  h.seed_order = 1;
  h.num_blocks = f->num_blocks;
  h.word_bytes = 4;
  h.lanes = f->lanes;
  h.reserved = 0;
  memcpy(host_dst, &h, sizeof(h));
  hipError_t e = hipMemcpyAsync(static_cast<char *>(host_dst) + sizeof(h), f->words, (size_t)filter_bytes(f),
                                hipMemcpyDeviceToHost, (hipStream_t)s);
  if (e != hipSuccess) return hip_error(e, "hipMemcpyAsync(serialize)");
  return hip_error(hipStreamSynchronize((hipStream_t)s), "hipStreamSynchronize(serialize)");
}

sbbf_status sbbf_deserialize(const void *host_src, size_t size, sbbf_filter **out) {
  if (!host_src || !out) return set_error(SBBF_EINVAL, "host_src or out is NULL");
  if (size < sizeof(SerialHeader)) return set_error(SBBF_EINVAL, "too short for a header");
  SerialHeader h;
  memcpy(&h, host_src, sizeof(h));
  if (memcmp(h.magic, kMagic, 8) != 0) return set_error(SBBF_EINVAL, "not a serialized filter (magic)");
  if (h.version != 1 || h.word_bytes != 4) return set_error(SBBF_EUNSUPPORTED, "unsupported format version");
  if (h.seed_order != 1) return set_error(SBBF_EUNSUPPORTED, "filter written with another seed order");
  if (h.num_blocks == 0) return set_error(SBBF_EINVAL, "num_blocks is 0");
  const uint32_t lanes = h.lanes == 0 ? 8u : h.lanes;
  if (!valid_lanes(lanes) || h.reserved != 0) return set_error(SBBF_EUNSUPPORTED, "unsupported block layout");
  if (size != 32u + filter_bytes(h.num_blocks, lanes))
    return set_error(SBBF_EINVAL, "size does not match num_blocks and lanes");
  sbbf_filter *f = nullptr;
  sbbf_status st = sbbf_create_variant(h.num_blocks, lanes, &f);
  if (st != SBBF_OK) return st;
  hipError_t e = hipMemcpy(f->words, static_cast<const char *>(host_src) + sizeof(h), (size_t)filter_bytes(f),
                           hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    sbbf_destroy(f);
    return hip_error(e, "hipMemcpy(deserialize)");
  }
  *out = f;
  return SBBF_OK;
}

sbbf_status sbbf_copy_words_to_host(const sbbf_filter *f, void *host_dst, sbbf_stream s) {
  if (!f || !host_dst) return set_error(SBBF_EINVAL, "filter or host_dst is NULL");
  return hip_error(hipMemcpyAsync(host_dst, f->words, (size_t)filter_bytes(f), hipMemcpyDeviceToHost,
                                  (hipStream_t)s),
                   "hipMemcpyAsync(filter to host)");
}

sbbf_status sbbf_copy_words_from_host(sbbf_filter *f, const void *host_src, sbbf_stream s) {
  if (!f || !host_src) return set_error(SBBF_EINVAL, "filter or host_src is NULL");
  return hip_error(hipMemcpyAsync(f->words, host_src, (size_t)filter_bytes(f), hipMemcpyHostToDevice,
                                  (hipStream_t)s),
                   "hipMemcpyAsync(filter from host)");
}

void *sbbf_device_words(const sbbf_filter *f) { return f ? f->words : nullptr; }

static sbbf_status check_batch(const sbbf_filter *f, const void *d_hashes, size_t n, const void *d_out,
                               const char *out_name, uintptr_t out_align) {
  if (!f) return set_error(SBBF_EINVAL, "filter is NULL");
  if (n == 0) return SBBF_OK;
  if (!d_hashes) return set_error(SBBF_EINVAL, "d_hashes is NULL");
  if (!aligned(d_hashes, 8)) return set_error(SBBF_EINVAL, "d_hashes must be 8-byte aligned");
  if (out_name) {
    if (!d_out) return set_error(SBBF_EINVAL, std::string(out_name) + " is NULL");
    if (!aligned(d_out, out_align))
      return set_error(SBBF_EINVAL, std::string(out_name) + " is not aligned to " + std::to_string(out_align));
  }
  return SBBF_OK;
}

// Slice size of the partitioned kernels: about four slices per compute unit
// so the slice phase fills the device, at least 64 blocks and at most the
// largest power of two of blocks (up to 128 KiB) whose words fit one
// workgroup's LDS (4096 blocks of eight words; 8192 of four, 2048 of sixteen).
static uint32_t partition_slice_shift(const sbbf_device_info &info, uint32_t num_blocks, uint32_t lanes) {
  const uint64_t block_bytes = 4u * (uint64_t)lanes;
  uint32_t max_shift = 6;
  while (max_shift < 13 && (block_bytes << (max_shift + 1)) <= (128u << 10) &&
         (block_bytes << (max_shift + 1)) <= info.lds_per_block)
    ++max_shift;
  const uint64_t target = (uint64_t)num_blocks / (4u * (uint64_t)info.compute_units);
  uint32_t shift = 6;
  while (shift < max_shift && ((uint64_t)1u << (shift + 1)) <= target) ++shift;
  return shift;
}

static uint32_t partition_slices(uint32_t num_blocks, uint32_t shift) {
  return (uint32_t)(((uint64_t)num_blocks + (1u << shift) - 1u) >> shift);
}

static bool partition_fits(const sbbf_device_info &info, const sbbf_filter *f) {
  return partition_slices(f->num_blocks, partition_slice_shift(info, f->num_blocks, f->lanes)) <=
         partition_max_slices();
}

// Library choice of insert strategy (SBBF_INSERT_AUTO): the partitioned insert
// when the batch has at least two keys per block (so the one-time read and
// write of the whole filter costs less than per-key atomics, which the device
// caps at about 27 G keys/s whatever the filter size), at least 4M keys (below
// that its fixed costs lose to the atomics: measured on MI355X for filters of
// 1 to 64 MiB) and the filter splits into few enough slices; otherwise global
// 32-bit atomics.
// Rate of the 32-bit atomic insert (G keys/s) on MI355X by filter size:
// one memory-side atomic request per key, slower once the filter is far
// beyond the 256 MB last-level cache.
static double atomic_rate_gkeys(uint64_t bytes) {
  const uint64_t MiB = 1ull << 20;
  if (bytes <= 256 * MiB) return 26.5;
  if (bytes <= 512 * MiB) return 22.5;
  if (bytes <= 2048 * MiB) return 19.0;
  return 18.0;
}

// Extra cost (us) of a partition in two levels: the level-1 count and
// scatter (about 6.2 us per million keys), one wait for the stream and the
// fixed cost of a one-level call per group of slices.
static double two_level_us(const sbbf_filter *f, size_t n, const sbbf_device_info &info) {
  const uint32_t slices = partition_slices(f->num_blocks, partition_slice_shift(info, f->num_blocks, f->lanes));
  if (slices <= partition_level_slices()) return 0.0;
  const double groups = (double)((slices + partition_group_slices() - 1u) / partition_group_slices());
  return 40.0 + 50.0 * groups + 6.2 * (double)n / 1e6;
}

// Library choice of insert strategy (SBBF_INSERT_AUTO) from a cost model
// fitted to MI355X measurements (filters of 1 MiB to 4 GiB, 1M to 200M
// keys): the partitioned insert takes about 100 us plus one read and one
// write of the filter at 5 TB/s plus 6.3 us per million keys (plus the
// second level's costs above 4,096 slices); the atomics take n / rate(filter
// size). The partitioned insert needs at least 4M keys (below, its
// workgroups are too few to be measured faster anywhere).
static uint32_t auto_insert_strategy(const sbbf_filter *f, size_t n, const sbbf_device_info &info) {
  if ((uint64_t)n < (4ull << 20) || !partition_fits(info, f)) return SBBF_INSERT_ATOMIC32;
  const double bytes = (double)filter_bytes(f);
  const double part_us = 100.0 + 2.0 * bytes / 5e6 + 6.3 * (double)n / 1e6 + two_level_us(f, n, info);
  const double atomic_us = (double)n / (atomic_rate_gkeys(filter_bytes(f)) * 1e3);
  return part_us < atomic_us ? SBBF_INSERT_PARTITIONED : SBBF_INSERT_ATOMIC32;
}

// Rate of the gather lookup (G keys/s) on MI355X by filter size, measured
// with about 24 keys per block: L2-resident up to 4 MiB, then falling as
// more of the random 32-byte reads miss (the 256 MB last-level cache, then
// HBM).
static double gather_rate_gkeys(uint64_t bytes) {
  const uint64_t MiB = 1ull << 20;
  if (bytes <= 4 * MiB) return 140.0;
  if (bytes <= 8 * MiB) return 98.0;
  if (bytes <= 16 * MiB) return 70.0;
  if (bytes <= 32 * MiB) return 57.0;
  if (bytes <= 64 * MiB) return 52.0;
  if (bytes <= 256 * MiB) return 50.0;
  return 43.0;
}

// Library choice of lookup strategy (SBBF_LOOKUP_AUTO) from a cost model
// fitted to MI355X measurements (filters of 1 MiB to 4 GiB, 1M to 200M
// keys): the partitioned lookup takes about 45 us plus one read of the
// filter at 5 TB/s plus 7.7 us per million keys (plus the second level's
// costs above 4,096 slices); the gather takes n / rate(filter size). The
// cheaper one is used (when the filter splits into few enough slices).
static uint32_t auto_lookup_strategy(const sbbf_filter *f, size_t n, const sbbf_device_info &info) {
  if (!partition_fits(info, f)) return SBBF_LOOKUP_GATHER;
  const double bytes = (double)filter_bytes(f);
  const double part_us = 45.0 + bytes / 5e6 + 7.7 * (double)n / 1e6 + two_level_us(f, n, info);
  const double gather_us = (double)n / (gather_rate_gkeys(filter_bytes(f)) * 1e3);
  return part_us < gather_us ? SBBF_LOOKUP_PARTITIONED : SBBF_LOOKUP_GATHER;
}

// Stream-ordered workspace: allocated from the device's default memory pool
// on the call's stream and released on it after the kernels, so concurrent
// calls on different streams never share it. The pool keeps freed memory for
// reuse instead of returning it at every synchronisation.
static hipError_t workspace_alloc(void **p, size_t bytes, hipStream_t stream, int device) {
  static std::mutex mu;
  static std::vector<bool> configured;
  {
    std::lock_guard<std::mutex> lock(mu);
    if ((int)configured.size() <= device) configured.resize(device + 1, false);
    if (!configured[device]) {
      hipMemPool_t pool;
      if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
      }
      (void)hipGetLastError();
      configured[device] = true;
    }
  }
  return dev_malloc_async(p, bytes, stream);
}

// Insert of n hashes, or of n keys hashed on load (key_hash) when keys is 1.
static sbbf_status insert_impl(sbbf_filter *f, const uint64_t *d_hashes, size_t n, const sbbf_launch *cfg,
                               sbbf_stream s, uint32_t keys) {
  sbbf_status st = check_batch(f, d_hashes, n, nullptr, nullptr, 1);
  if (st != SBBF_OK || n == 0) return st;
  uint32_t strategy = cfg ? cfg->strategy : SBBF_INSERT_AUTO;
  const sbbf_device_info *info = current_device_info(&st);
  if (!info) return st;
  if (strategy == SBBF_INSERT_AUTO) strategy = auto_insert_strategy(f, n, *info);
  Shape shape;
  hipStream_t stream = (hipStream_t)s;
  switch (strategy) {
    case SBBF_INSERT_ATOMIC32:
      if ((st = resolve_shape(cfg, n, 2, &shape)) != SBBF_OK) return st;
      shape.keys = keys;
      shape.lanes = f->lanes;
      return hip_error(launch_insert_atomic32(d_hashes, n, f->words, f->num_blocks, shape, stream), "insert");
    case SBBF_INSERT_ATOMIC64:
      if ((st = resolve_shape(cfg, n, 2, &shape)) != SBBF_OK) return st;
      shape.keys = keys;
      shape.lanes = f->lanes;
      return hip_error(launch_insert_atomic64(d_hashes, n, f->words, f->num_blocks, shape, stream), "insert");
    case SBBF_INSERT_PARTITIONED: {
      const uint32_t shift = partition_slice_shift(*info, f->num_blocks, f->lanes);
      const uint32_t slices = partition_slices(f->num_blocks, shift);
      if (slices > partition_max_slices())
        return set_error(SBBF_EUNSUPPORTED, "filter has more than " + std::to_string(partition_max_slices()) +
                                                " slices of " + std::to_string(1u << shift) + " blocks");
      const uint32_t groups = cfg && cfg->grid_blocks ? cfg->grid_blocks : (uint32_t)info->compute_units * 2u;
      const uint64_t step = partition_max_keys();
      void *ws = nullptr;
      hipError_t e = workspace_alloc(&ws, partition_workspace_bytes(n < step ? n : step, slices, groups, false),
                                     stream, info->device);
      if (e != hipSuccess) return hip_error(e, "hipMallocAsync(partition workspace)");
      for (uint64_t at = 0; at < n && e == hipSuccess; at += step) {
        const uint64_t m = n - at < step ? n - at : step;
        e = launch_insert_partitioned(d_hashes + at, m, f->words, f->num_blocks, shift, ws, groups, keys, stream,
                                      f->lanes);
      }
      hipError_t e2 = hipFreeAsync(ws, stream);
      if (e != hipSuccess) return hip_error(e, "partitioned insert");
      return hip_error(e2, "hipFreeAsync(partition workspace)");
    }
    case SBBF_INSERT_LDS: {
      if (filter_bytes(f) > info->lds_per_block)
        return set_error(SBBF_EUNSUPPORTED, "filter does not fit one workgroup's LDS (" +
                                                std::to_string(info->lds_per_block) + " bytes)");
      sbbf_launch c = cfg ? *cfg : sbbf_launch{0, 0, 0, 0, 0};
      if (c.block_threads == 0) c.block_threads = 1024;
      if (c.grid_blocks == 0) c.grid_blocks = 1;
      if ((st = resolve_shape(&c, n, 2, &shape)) != SBBF_OK) return st;
      shape.keys = keys;
      shape.lanes = f->lanes;
      return hip_error(launch_insert_lds(d_hashes, n, f->words, f->num_blocks, shape, stream), "insert");
    }
    default:
      return set_error(SBBF_EINVAL, "unknown insert strategy");
  }
}

sbbf_status sbbf_insert_batch_ex(sbbf_filter *f, const uint64_t *d_hashes, size_t n, const sbbf_launch *cfg,
                                 sbbf_stream s) {
  return insert_impl(f, d_hashes, n, cfg, s, 0u);
}

sbbf_status sbbf_insert_keys(sbbf_filter *f, const uint64_t *d_keys, size_t n, const sbbf_launch *cfg,
                             sbbf_stream s) {
  return insert_impl(f, d_keys, n, cfg, s, 1u);
}

uint64_t sbbf_key_hash(uint64_t key) { return key_hash(key); }

uint32_t sbbf_auto_insert_strategy(const sbbf_filter *f, size_t n) {
  sbbf_status st;
  const sbbf_device_info *info = f ? current_device_info(&st) : nullptr;
  return info ? auto_insert_strategy(f, n, *info) : 0u;
}

uint32_t sbbf_auto_lookup_strategy(const sbbf_filter *f, size_t n) {
  sbbf_status st;
  const sbbf_device_info *info = f ? current_device_info(&st) : nullptr;
  return info ? auto_lookup_strategy(f, n, *info) : 0u;
}

sbbf_status sbbf_insert_batch(sbbf_filter *f, const uint64_t *d_hashes, size_t n, sbbf_stream s) {
  return sbbf_insert_batch_ex(f, d_hashes, n, nullptr, s);
}

// Lookup of n hashes, or of n keys hashed on load (key_hash) when keys is 1.
static sbbf_status lookup_impl(const sbbf_filter *f, const uint64_t *d_hashes, size_t n, uint8_t *d_out,
                               uint32_t *d_bits, const sbbf_launch *cfg, sbbf_stream s, uint32_t keys) {
  if ((d_out == nullptr) == (d_bits == nullptr) && n > 0)
    return set_error(SBBF_EINVAL, "exactly one of d_out and d_bits must be non-NULL");
  sbbf_status st = d_bits ? check_batch(f, d_hashes, n, d_bits, "d_bits", 4)
                          : check_batch(f, d_hashes, n, d_out, "d_out", 1);
  if (st != SBBF_OK || n == 0) return st;
  const sbbf_device_info *info = current_device_info(&st);
  if (!info) return st;
  hipStream_t stream = (hipStream_t)s;
  uint32_t strategy = cfg ? cfg->strategy : SBBF_LOOKUP_AUTO;
  if (strategy == SBBF_LOOKUP_AUTO) strategy = auto_lookup_strategy(f, n, *info);
  if (strategy == SBBF_LOOKUP_PARTITIONED) {
    const uint32_t shift = partition_slice_shift(*info, f->num_blocks, f->lanes);
    const uint32_t slices = partition_slices(f->num_blocks, shift);
    if (slices > partition_max_slices())
      return set_error(SBBF_EUNSUPPORTED, "filter has more than " + std::to_string(partition_max_slices()) +
                                              " slices of " + std::to_string(1u << shift) + " blocks");
    const uint32_t groups = cfg && cfg->grid_blocks ? cfg->grid_blocks : (uint32_t)info->compute_units * 2u;
    const uint64_t step = partition_max_keys();  // a multiple of 32: packed outputs split on word boundaries
    void *ws = nullptr;
    hipError_t e = workspace_alloc(&ws, partition_workspace_bytes(n < step ? n : step, slices, groups, true), stream,
                                   info->device);
    if (e != hipSuccess) return hip_error(e, "hipMallocAsync(partition workspace)");
    for (uint64_t at = 0; at < n && e == hipSuccess; at += step) {
      const uint64_t m = n - at < step ? n - at : step;
      e = launch_lookup_partitioned(d_hashes + at, m, f->words, f->num_blocks, shift, ws, groups,
                                    d_out ? d_out + at : nullptr, d_bits ? d_bits + at / 32 : nullptr, keys, stream,
                                    f->lanes);
    }
    hipError_t e2 = hipFreeAsync(ws, stream);
    if (e != hipSuccess) return hip_error(e, "partitioned lookup");
    return hip_error(e2, "hipFreeAsync(partition workspace)");
  }
  if (strategy != SBBF_LOOKUP_GATHER) return set_error(SBBF_EINVAL, "unknown lookup strategy");
  Shape shape;
  if ((st = resolve_shape(cfg, n, 2, &shape, 4)) != SBBF_OK) return st;
  shape.keys = keys;
  shape.lanes = f->lanes;
  return hip_error(launch_lookup(d_hashes, n, f->words, f->num_blocks, d_out, d_bits, shape, stream), "lookup");
}

sbbf_status sbbf_lookup_batch_ex(const sbbf_filter *f, const uint64_t *d_hashes, size_t n, uint8_t *d_out,
                                 uint32_t *d_bits, const sbbf_launch *cfg, sbbf_stream s) {
  return lookup_impl(f, d_hashes, n, d_out, d_bits, cfg, s, 0u);
}

sbbf_status sbbf_lookup_keys(const sbbf_filter *f, const uint64_t *d_keys, size_t n, uint8_t *d_out,
                             const sbbf_launch *cfg, sbbf_stream s) {
  return lookup_impl(f, d_keys, n, d_out, nullptr, cfg, s, 1u);
}

sbbf_status sbbf_lookup_batch(const sbbf_filter *f, const uint64_t *d_hashes, size_t n, uint8_t *d_out,
                              sbbf_stream s) {
  return sbbf_lookup_batch_ex(f, d_hashes, n, d_out, nullptr, nullptr, s);
}

sbbf_status sbbf_lookup_select(const sbbf_filter *f, const uint64_t *d_hashes, size_t n, uint32_t *d_indices,
                               uint64_t *d_count, const sbbf_launch *cfg, sbbf_stream s) {
  sbbf_status st = check_batch(f, d_hashes, n, d_indices, "d_indices", 4);
  if (st != SBBF_OK) return st;
  if (!d_count) return set_error(SBBF_EINVAL, "d_count is NULL");
  if (!aligned(d_count, 8)) return set_error(SBBF_EINVAL, "d_count must be 8-byte aligned");
  if ((uint64_t)n > 0xFFFFFFFFull) return set_error(SBBF_EINVAL, "one call takes fewer than 2^32 keys");
  hipStream_t stream = (hipStream_t)s;
  if (n == 0) return hip_error(launch_fill(reinterpret_cast<uint32_t *>(d_count), 2, 0u, stream), "select count");
  const sbbf_device_info *info = current_device_info(&st);
  if (!info) return st;
  void *ws = nullptr;
  hipError_t e = workspace_alloc(&ws, select_workspace_bytes(n), stream, info->device);
  if (e != hipSuccess) return hip_error(e, "hipMallocAsync(select workspace)");
  st = sbbf_lookup_batch_ex(f, d_hashes, n, nullptr, select_bits(ws), cfg, s);
  if (st == SBBF_OK) st = hip_error(launch_select(n, ws, d_indices, reinterpret_cast<unsigned long long *>(d_count), stream),
                                    "select");
  const hipError_t e2 = hipFreeAsync(ws, stream);
  if (st != SBBF_OK) return st;
  return hip_error(e2, "hipFreeAsync(select workspace)");
}

sbbf_status sbbf_lookup_batch_bits(const sbbf_filter *f, const uint64_t *d_hashes, size_t n, uint32_t *d_bits,
                                   sbbf_stream s) {
  return sbbf_lookup_batch_ex(f, d_hashes, n, nullptr, d_bits, nullptr, s);
}

sbbf_status sbbf_bench_gather(const uint32_t *d_buf, uint32_t num_blocks, const uint64_t *d_hashes, size_t n,
                              uint8_t *d_out, const sbbf_launch *cfg, sbbf_stream s) {
  if (!d_buf || num_blocks == 0) return set_error(SBBF_EINVAL, "bad buffer");
  if (n == 0) return SBBF_OK;
  if (!d_hashes || !d_out || !aligned(d_hashes, 8)) return set_error(SBBF_EINVAL, "bad hashes or output");
  Shape shape;
  sbbf_status st = resolve_shape(cfg, n, 2, &shape, 4);
  if (st != SBBF_OK) return st;
  return hip_error(launch_bench_gather(d_buf, num_blocks, d_hashes, n, d_out, shape, (hipStream_t)s), "gather");
}

sbbf_status sbbf_bench_atomic(uint32_t *d_buf, uint32_t num_blocks, const uint64_t *d_hashes, size_t n,
                              const sbbf_launch *cfg, sbbf_stream s) {
  if (!d_buf || num_blocks == 0 || !aligned(d_buf, 32)) return set_error(SBBF_EINVAL, "bad buffer");
  if (n == 0) return SBBF_OK;
  if (!d_hashes || !aligned(d_hashes, 8)) return set_error(SBBF_EINVAL, "bad hashes");
  Shape shape;
  sbbf_status st = resolve_shape(cfg, n, 2, &shape);
  if (st != SBBF_OK) return st;
  const bool wide = cfg && cfg->strategy == SBBF_INSERT_ATOMIC64;
  return hip_error(launch_bench_atomic(d_buf, num_blocks, d_hashes, n, wide, shape, (hipStream_t)s), "atomic");
}

sbbf_status sbbf_bench_stream(const uint64_t *d_hashes, size_t n, uint8_t *d_out, const sbbf_launch *cfg,
                              sbbf_stream s) {
  if (n == 0) return SBBF_OK;
  if (!d_hashes || !d_out || !aligned(d_hashes, 8)) return set_error(SBBF_EINVAL, "bad hashes or output");
  Shape shape;
  sbbf_status st = resolve_shape(cfg, n, 2, &shape);
  if (st != SBBF_OK) return st;
  return hip_error(launch_bench_stream(d_hashes, n, d_out, shape, (hipStream_t)s), "stream");
}

}  // extern "C"
