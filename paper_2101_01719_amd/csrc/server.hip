// Serving runtime: resident filters in a budgeted device arena, requests of
// any size queued per filter, and continuous batching of the queued requests
// into steps (one insert kernel and one lookup kernel per step) while earlier
// steps are still running.
//
// Correctness rule of the batching: per filter, a step takes the longest prefix
// of the filter's FIFO that is some inserts followed by some lookups. Inside a
// step every insert runs before every lookup, and steps run in order on one
// stream, so a lookup sees exactly the inserts that arrived before it on its
// filter — the same result it gets when it is run alone. Filters are
// independent, so mixing filters in a step changes nothing.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"
#include "sbbf_device.h"

namespace sbbf {
namespace {

constexpr uint32_t kServeThreads = 256;
constexpr uint32_t kServeUnroll = 2;
constexpr uint32_t kArenaAlign = 256;
// Inserts into filters of at most this many blocks (32 KiB) are ORed into a
// zeroed LDS copy first and merged with one device atomic per non-zero 64-bit
// word pair: a tile's keys land on few blocks of such a filter, and per-key
// device atomics on the same words serialize.
constexpr uint32_t kServeLdsBlocks = 1024;
// Lookup tiles are laid out so that workgroup i runs on XCD i % 8 (workgroups
// are dealt to the eight XCDs in turn) and every tile of a filter on the same
// XCD, so a filter's blocks are cached in one L2 instead of eight.
constexpr uint32_t kServeXcds = 8;
constexpr uint64_t kServeSlack = 65536;
// Requests a replay without arrival times admits per round of its loop.
constexpr uint64_t kReplayAdmitBatch = 2048;
// A realtime replay that sleeps through an idle gap wakes this long (ns)
// before the next arrival.
constexpr uint64_t kReplaySleepMargin = 200000;

struct STile {
  const uint64_t *keys;
  uint8_t *out;
  uint32_t *words;
  uint32_t num_blocks;
  uint32_t count;
};

// One workgroup per tile; 8-lane layout. Small filters: 32-bit LDS atomics
// into a zeroed copy, then one 64-bit device atomic per non-zero word pair;
// larger filters: 32-bit device atomics.
__global__ void __launch_bounds__(kServeThreads) serve_insert_kernel(const STile *__restrict__ tiles) {
  __shared__ unsigned long long lds2[kServeLdsBlocks * 4u];
  const STile t = tiles[blockIdx.x];
  const uint32_t lane = lane_id();
  const uint32_t j = lane & 7u;
  const uint32_t group = lane & ~7u;
  const uint32_t seed = seed_of_word(j);
  constexpr uint32_t kChunk = 64u * kServeUnroll;
  const bool small = t.num_blocks <= kServeLdsBlocks;  // uniform over the workgroup
  if (small) {
    uint32_t *lds = reinterpret_cast<uint32_t *>(lds2);
    for (uint32_t i = threadIdx.x; i < t.num_blocks * 4u; i += blockDim.x) lds2[i] = 0ull;
    __syncthreads();
    for (uint32_t base = (threadIdx.x / kWave) * kChunk; base < t.count; base += (blockDim.x / kWave) * kChunk) {
      uint32_t blk[kServeUnroll], lo[kServeUnroll];
#pragma unroll
      for (uint32_t u = 0; u < kServeUnroll; ++u) {
        const uint32_t i = base + 64u * u + lane;
        const uint64_t h = load_hash<0>(t.keys + (i < t.count ? i : t.count - 1u));
        lo[u] = (uint32_t)h;
        blk[u] = block_of((uint32_t)(h >> 32), t.num_blocks);
      }
#pragma unroll
      for (uint32_t u = 0; u < kServeUnroll; ++u) {
#pragma unroll
        for (uint32_t p = 0; p < 8; ++p) {
          const uint32_t b = lane_read(blk[u], group + p);
          const uint32_t x = lane_read(lo[u], group + p);
          __hip_atomic_fetch_or(lds + b * 8u + j, 1u << bit_of(seed, x), __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
    }
    __syncthreads();
    unsigned long long *pairs = reinterpret_cast<unsigned long long *>(t.words);
    for (uint32_t i = threadIdx.x; i < t.num_blocks * 4u; i += blockDim.x) {
      const unsigned long long v = lds2[i];
      if (v) __hip_atomic_fetch_or(pairs + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  for (uint32_t base = (threadIdx.x / kWave) * kChunk; base < t.count; base += (blockDim.x / kWave) * kChunk) {
    uint32_t blk[kServeUnroll], lo[kServeUnroll];
#pragma unroll
    for (uint32_t u = 0; u < kServeUnroll; ++u) {
      const uint32_t i = base + 64u * u + lane;
      const uint64_t h = load_hash<0>(t.keys + (i < t.count ? i : t.count - 1u));
      lo[u] = (uint32_t)h;
      blk[u] = block_of((uint32_t)(h >> 32), t.num_blocks);
    }
#pragma unroll
    for (uint32_t u = 0; u < kServeUnroll; ++u) {
#pragma unroll
      for (uint32_t p = 0; p < 8; ++p) {
        const uint32_t b = lane_read(blk[u], group + p);
        const uint32_t x = lane_read(lo[u], group + p);
        // Lanes past the tile repeat its last key: OR-ing a mask again changes nothing.
        __hip_atomic_fetch_or(t.words + (uint64_t)b * 8u + j, 1u << bit_of(seed, x), __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// One workgroup per tile; 8-lane gather, one result byte per key.
__global__ void __launch_bounds__(kServeThreads) serve_lookup_kernel(const STile *__restrict__ tiles) {
  const STile t = tiles[blockIdx.x];
  const uint32_t lane = lane_id();
  const uint32_t j = lane & 7u;
  const uint32_t group = lane & ~7u;
  const uint32_t seed = seed_of_word(j);
  constexpr uint32_t kChunk = 64u * kServeUnroll;
  for (uint32_t base = (threadIdx.x / kWave) * kChunk; base < t.count; base += (blockDim.x / kWave) * kChunk) {
    uint32_t blk[kServeUnroll], lo[kServeUnroll];
#pragma unroll
    for (uint32_t u = 0; u < kServeUnroll; ++u) {
      const uint32_t i = base + 64u * u + lane;
      const uint64_t h = load_hash<0>(t.keys + (i < t.count ? i : t.count - 1u));
      lo[u] = (uint32_t)h;
      blk[u] = block_of((uint32_t)(h >> 32), t.num_blocks);
    }
    uint32_t word[kServeUnroll][8], bit[kServeUnroll][8];
#pragma unroll
    for (uint32_t u = 0; u < kServeUnroll; ++u) {
#pragma unroll
      for (uint32_t p = 0; p < 8; ++p) {
        const uint32_t b = lane_read(blk[u], group + p);
        bit[u][p] = bit_of(seed, lane_read(lo[u], group + p));
        word[u][p] = t.words[(uint64_t)b * 8u + j];
      }
    }
#pragma unroll
    for (uint32_t u = 0; u < kServeUnroll; ++u) {
      uint64_t r = 0;
#pragma unroll
      for (uint32_t p = 0; p < 8; ++p) r |= fold_pass(ballot((word[u][p] >> bit[u][p]) & 1u), p);
      const uint32_t i = base + 64u * u + lane;
      if (i < t.count) t.out[i] = (uint8_t)((r >> lane) & 1u);
    }
  }
}

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

uint64_t round_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

}  // namespace

// Device arena: chunks from hipMalloc, first-fit free lists, a byte budget.
struct Arena {
  struct Chunk {
    char *base;
    uint64_t size;
    std::map<uint64_t, uint64_t> free;  // offset -> length
  };
  uint64_t budget = 0, used = 0, reserved = 0;
  uint64_t chunk_bytes = 256ull << 20;
  std::vector<Chunk> chunks;

  sbbf_status alloc(uint64_t bytes, char **out, uint32_t *chunk_idx, uint64_t *off) {
    bytes = round_up(bytes, kArenaAlign);
    if (used + bytes > budget) return set_error(SBBF_EBUDGET, "filter does not fit the HBM budget");
    for (uint32_t c = 0; c < chunks.size(); ++c) {
      for (auto it = chunks[c].free.begin(); it != chunks[c].free.end(); ++it) {
        if (it->second >= bytes) {
          const uint64_t o = it->first, len = it->second;
          chunks[c].free.erase(it);
          if (len > bytes) chunks[c].free[o + bytes] = len - bytes;
          used += bytes;
          *out = chunks[c].base + o;
          *chunk_idx = c;
          *off = o;
          return SBBF_OK;
        }
      }
    }
    const uint64_t size = std::max(bytes, std::min(chunk_bytes, budget - reserved));
    if (reserved + size > budget) return set_error(SBBF_EBUDGET, "HBM budget exhausted");
    void *p = nullptr;
    hipError_t e = dev_malloc(&p, size);
    if (e != hipSuccess) return hip_error(e, "hipMalloc(arena chunk)");
    reserved += size;
    Chunk ch{static_cast<char *>(p), size, {}};
    if (size > bytes) ch.free[bytes] = size - bytes;
    chunks.push_back(std::move(ch));
    used += bytes;
    *out = static_cast<char *>(p);
    *chunk_idx = (uint32_t)chunks.size() - 1;
    *off = 0;
    return SBBF_OK;
  }

  void release(uint32_t c, uint64_t off, uint64_t bytes) {
    bytes = round_up(bytes, kArenaAlign);
    auto &fl = chunks[c].free;
    auto it = fl.emplace(off, bytes).first;
    // merge with the next and the previous free ranges
    auto nx = std::next(it);
    if (nx != fl.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      fl.erase(nx);
    }
    if (it != fl.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        fl.erase(it);
      }
    }
    used -= bytes;
  }

  ~Arena() {
    for (auto &c : chunks) (void)hipFree(c.base);
  }
};

struct ServeFilter {
  bool live = false;
  uint32_t *words = nullptr;
  uint32_t num_blocks = 0;
  uint32_t chunk = 0;
  uint64_t off = 0;
  std::deque<uint64_t> fifo;  // pending request ids
  bool queued = false;        // in the ready list
  uint64_t inflight = 0;      // requests of this filter in launched steps
};

struct Request {
  uint32_t filter;
  uint32_t op;  // 0 insert, 1 lookup
  const uint64_t *keys;
  uint8_t *out;
  uint64_t n;
  uint64_t arrival_ns;
  uint64_t done_ns;
};

struct Slot {
  bool busy = false;
  hipEvent_t done = nullptr;
  // The step's tile table, written by the host and read by the kernels in
  // place: pinned, mapped and coherent host memory (no copy to the device
  // ahead of the kernels: 12-35 % lower median latency at 25-90 % load).
  STile *host = nullptr;
  STile *dev = nullptr;   // the device's address of `host`
  uint32_t cap = 0;       // tiles
  std::vector<uint64_t> reqs;
  uint64_t keys = 0;
};

}  // namespace sbbf

struct sbbf_server {
  sbbf_server_config cfg;
  int device = 0;
  hipStream_t stream = nullptr;
  sbbf::Arena arena;
  std::vector<sbbf::ServeFilter> filters;
  std::vector<uint32_t> free_ids;
  std::vector<sbbf::Request> reqs;
  std::deque<uint32_t> ready;  // filters with pending requests, in order of first arrival
  std::vector<sbbf::Slot> slots;
  // completed request ids; those from completed_head on are not yet polled
  // (a head index, so that polling in small batches does not shift the rest)
  std::vector<uint64_t> completed;
  size_t completed_head = 0;
  uint64_t pending = 0, inflight = 0;
  // statistics
  uint64_t steps = 0, keys_done = 0, req_done = 0;
  uint64_t first_arrival = UINT64_MAX, last_done = 0;
  uint64_t step_tiles_max = 0;
  // step assembly scratch, reused from step to step
  std::vector<sbbf::STile> step_ins;
  std::vector<sbbf::STile> step_lq[sbbf::kServeXcds];
};

namespace sbbf {
namespace {

// A slot's tile table of `tiles` entries in mapped, coherent pinned memory.
sbbf_status slot_alloc(Slot &sl, size_t tiles) {
  hipError_t e = host_malloc_mapped((void **)&sl.host, tiles * sizeof(STile), hipHostMallocMapped | hipHostMallocCoherent);
  if (e != hipSuccess) {
    sl.host = nullptr;
    return hip_error(e, "hipHostMalloc(server slot)");
  }
  e = hipHostGetDevicePointer((void **)&sl.dev, sl.host, 0);
  if (e != hipSuccess) return hip_error(e, "hipHostGetDevicePointer(server slot)");
  sl.cap = (uint32_t)tiles;
  return SBBF_OK;
}

sbbf_status server_make_slots(sbbf_server *s) {
  // Real tiles of a full step, twice over for the padding of the per-XCD
  // lookup queues (a slot grows later if a step needs more).
  const uint32_t tiles = 2u * ((uint32_t)((s->cfg.max_step_keys + s->cfg.tile_keys - 1) / s->cfg.tile_keys) +
                               s->cfg.max_step_requests + 1) + 8u * 64u;
  s->slots.resize(s->cfg.max_inflight_steps);
  for (auto &sl : s->slots) {
    hipError_t e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e != hipSuccess) return hip_error(e, "hipEventCreate(server slot)");
    const sbbf_status st = slot_alloc(sl, tiles);
    if (st != SBBF_OK) return st;
  }
  return SBBF_OK;
}

// Record completions of finished steps (non-blocking unless `block`).
sbbf_status server_harvest(sbbf_server *s, bool block) {
  for (auto &sl : s->slots) {
    if (!sl.busy) continue;
    hipError_t e = block ? hipEventSynchronize(sl.done) : hipEventQuery(sl.done);
    if (e == hipErrorNotReady) continue;
    if (e != hipSuccess) return hip_error(e, "server step");
    const uint64_t t = now_ns();
    for (uint64_t id : sl.reqs) {
      Request &r = s->reqs[id];
      r.done_ns = t;
      s->completed.push_back(id);
      s->filters[r.filter].inflight -= 1;
      s->keys_done += r.n;
      s->req_done += 1;
    }
    s->inflight -= sl.reqs.size();
    s->last_done = std::max(s->last_done, t);
    sl.reqs.clear();
    sl.busy = false;
    block = false;  // one completed step is enough when blocking
  }
  return SBBF_OK;
}

// Build and launch one step into a free slot. Returns the number of requests taken.
sbbf_status server_launch_step(sbbf_server *s, Slot &sl, uint64_t *taken) {
  *taken = 0;
  const uint32_t T = s->cfg.tile_keys;
  std::vector<STile> &ins = s->step_ins;
  std::vector<STile> *lq = s->step_lq;  // lookup tiles per XCD queue
  ins.clear();
  for (uint32_t k = 0; k < kServeXcds; ++k) lq[k].clear();
  uint64_t lq_keys[kServeXcds] = {};
  uint64_t keys = 0;
  uint32_t nreq = 0;
  const size_t nready = s->ready.size();
  for (size_t k = 0; k < nready; ++k) {
    const uint32_t fid = s->ready.front();
    s->ready.pop_front();
    ServeFilter &f = s->filters[fid];
    // This filter's lookup tiles go to one XCD queue (the least loaded when
    // its first lookup is taken); a request moves the filter to the least
    // loaded queue when its own is more than kServeSlack keys ahead, so one
    // large filter still spreads over every XCD.
    uint32_t q = kServeXcds;
    bool seen_lookup = false;
    while (!f.fifo.empty() && nreq < s->cfg.max_step_requests) {
      Request &r = s->reqs[f.fifo.front()];
      if (r.op == 0 && seen_lookup) break;
      if (keys > 0 && keys + r.n > s->cfg.max_step_keys) break;
      seen_lookup |= r.op == 1;
      if (r.op) {
        uint32_t least = 0;
        for (uint32_t x = 1; x < kServeXcds; ++x)
          if (lq_keys[x] < lq_keys[least]) least = x;
        if (q == kServeXcds || lq_keys[q] > lq_keys[least] + kServeSlack) q = least;
      }
      for (uint64_t at = 0; at < r.n; at += T) {
        const uint32_t c = (uint32_t)std::min<uint64_t>(T, r.n - at);
        STile t{r.keys + at, r.op ? r.out + at : nullptr, f.words, f.num_blocks, c};
        (r.op ? lq[q] : ins).push_back(t);
      }
      if (r.op) lq_keys[q] += r.n;
      keys += r.n;
      sl.reqs.push_back(f.fifo.front());
      f.fifo.pop_front();
      f.inflight += 1;
      ++nreq;
    }
    if (!f.fifo.empty()) {
      s->ready.push_back(fid);  // more work left: back of the line
    } else {
      f.queued = false;
    }
    if (nreq >= s->cfg.max_step_requests || keys >= s->cfg.max_step_keys) break;
  }
  if (nreq == 0) return SBBF_OK;
  // Interleave the queues: tile i comes from queue i % 8; shorter queues are
  // padded with empty tiles (count 0: the workgroup does nothing).
  size_t qmax = 0;
  for (uint32_t k = 0; k < kServeXcds; ++k) qmax = std::max(qmax, lq[k].size());
  const size_t nlook = qmax * kServeXcds;
  const size_t nt = ins.size() + nlook;
  if (nt > sl.cap) {  // one request larger than the step budget: grow this slot's buffers (the slot is idle)
    (void)hipHostFree(sl.host);
    sl.host = nullptr;
    sl.dev = nullptr;
    sl.cap = 0;
    const sbbf_status sa = slot_alloc(sl, nt);
    if (sa != SBBF_OK) return sa;
  }
  // The slot is idle (its previous step has completed), so its table may be
  // rewritten; the kernels launched below read it in place.
  memcpy(sl.host, ins.data(), ins.size() * sizeof(STile));
  STile *dst = sl.host + ins.size();
  for (size_t i = 0; i < qmax; ++i)
    for (uint32_t k = 0; k < kServeXcds; ++k)
      *dst++ = i < lq[k].size() ? lq[k][i] : STile{nullptr, nullptr, nullptr, 1u, 0u};
  hipError_t e = hipSuccess;
  if (!ins.empty()) {
    hipLaunchKernelGGL(serve_insert_kernel, dim3((uint32_t)ins.size()), dim3(kServeThreads), 0, s->stream, sl.dev);
    if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "server insert");
  }
  if (nlook > 0) {
    hipLaunchKernelGGL(serve_lookup_kernel, dim3((uint32_t)nlook), dim3(kServeThreads), 0, s->stream,
                       sl.dev + ins.size());
    if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "server lookup");
  }
  if ((e = hipEventRecord(sl.done, s->stream)) != hipSuccess) return hip_error(e, "hipEventRecord(server)");
  sl.busy = true;
  sl.keys = keys;
  s->pending -= nreq;
  s->inflight += nreq;
  s->steps += 1;
  s->step_tiles_max = std::max<uint64_t>(s->step_tiles_max, nt);
  *taken = nreq;
  return SBBF_OK;
}

// One round of the loop: harvest, then fill free slots with steps.
sbbf_status server_pump(sbbf_server *s, bool wait) {
  sbbf_status st = server_harvest(s, false);
  if (st != SBBF_OK) return st;
  bool launched = false;
  for (auto &sl : s->slots) {
    if (sl.busy || s->pending == 0) continue;
    uint64_t taken = 0;
    if ((st = server_launch_step(s, sl, &taken)) != SBBF_OK) return st;
    launched |= taken > 0;
  }
  if (wait && !launched && s->inflight > 0) return server_harvest(s, true);
  return SBBF_OK;
}

sbbf_status server_enqueue(sbbf_server *s, uint32_t fid, uint32_t op, const uint64_t *keys, uint64_t n, uint8_t *out,
                           uint64_t arrival_ns, uint64_t *req_id) {
  if (fid >= s->filters.size() || !s->filters[fid].live) return set_error(SBBF_EINVAL, "unknown filter id");
  if (op > 1) return set_error(SBBF_EINVAL, "op must be 0 (insert) or 1 (lookup)");
  if (n > 0 && (!keys || ((uintptr_t)keys & 7))) return set_error(SBBF_EINVAL, "keys NULL or not 8-byte aligned");
  if (op == 1 && n > 0 && !out) return set_error(SBBF_EINVAL, "lookup output is NULL");
  const uint64_t id = s->reqs.size();
  s->reqs.push_back(Request{fid, op, keys, out, n, arrival_ns ? arrival_ns : now_ns(), 0});
  Request &r = s->reqs.back();
  s->first_arrival = std::min(s->first_arrival, r.arrival_ns);
  if (n == 0) {  // nothing to run: complete at once
    r.done_ns = r.arrival_ns;
    s->completed.push_back(id);
    s->req_done += 1;
  } else {
    ServeFilter &f = s->filters[fid];
    f.fifo.push_back(id);
    if (!f.queued) {
      f.queued = true;
      s->ready.push_back(fid);
    }
    s->pending += 1;
  }
  if (req_id) *req_id = id;
  return SBBF_OK;
}

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * (double)(v.size() - 1);
  const size_t i = (size_t)pos;
  const double frac = pos - (double)i;
  return i + 1 < v.size() ? v[i] * (1.0 - frac) + v[i + 1] * frac : v[i];
}

}  // namespace
}  // namespace sbbf

using namespace sbbf;

extern "C" {

sbbf_status sbbf_server_default_config(sbbf_server_config *out) {
  if (!out) return set_error(SBBF_EINVAL, "out is NULL");
  memset(out, 0, sizeof(*out));
  out->hbm_budget_bytes = 64ull << 30;
  out->max_inflight_steps = 2;
  out->max_step_keys = 4u << 20;
  out->max_step_requests = 4096;
  out->tile_keys = 2048;
  return SBBF_OK;
}

sbbf_status sbbf_server_create(const sbbf_server_config *cfg, sbbf_server **out) {
  if (!out) return set_error(SBBF_EINVAL, "out is NULL");
  *out = nullptr;
  sbbf_server_config c;
  sbbf_server_default_config(&c);
  if (cfg) c = *cfg;
  if (c.max_inflight_steps == 0 || c.max_inflight_steps > 64) return set_error(SBBF_EINVAL, "max_inflight_steps in 1..64");
  if (c.max_step_keys == 0 || c.max_step_requests == 0) return set_error(SBBF_EINVAL, "step limits must be positive");
  if (c.tile_keys < 64 || c.tile_keys % 64) return set_error(SBBF_EINVAL, "tile_keys must be a multiple of 64");
  if (c.hbm_budget_bytes == 0) return set_error(SBBF_EINVAL, "budget must be positive");
  sbbf_server *s = new (std::nothrow) sbbf_server();
  if (!s) return set_error(SBBF_ENOMEM, "server allocation failed");
  s->cfg = c;
  s->arena.budget = c.hbm_budget_bytes;
  hipError_t e = hipGetDevice(&s->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete s;
    return hip_error(e, "server stream");
  }
  sbbf_status st = server_make_slots(s);
  if (st != SBBF_OK) {
    sbbf_server_destroy(s);
    return st;
  }
  *out = s;
  return SBBF_OK;
}

sbbf_status sbbf_server_destroy(sbbf_server *s) {
  if (!s) return set_error(SBBF_EINVAL, "server is NULL");
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  for (auto &sl : s->slots) {
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.host) (void)hipHostFree(sl.host);
  }
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
  return SBBF_OK;
}

sbbf_status sbbf_server_add_filter(sbbf_server *s, uint32_t num_blocks, uint32_t *filter_id) {
  if (!s || !filter_id) return set_error(SBBF_EINVAL, "server or filter_id is NULL");
  if (num_blocks == 0) return set_error(SBBF_EINVAL, "num_blocks must be >= 1");
  char *p = nullptr;
  uint32_t chunk = 0;
  uint64_t off = 0;
  sbbf_status st = s->arena.alloc((uint64_t)num_blocks * 32u, &p, &chunk, &off);
  if (st != SBBF_OK) return st;
  hipError_t e = launch_fill(reinterpret_cast<uint32_t *>(p), (uint64_t)num_blocks * 8u, 0u, s->stream);
  if (e != hipSuccess) {
    s->arena.release(chunk, off, (uint64_t)num_blocks * 32u);
    return hip_error(e, "clear new filter");
  }
  uint32_t id;
  if (!s->free_ids.empty()) {
    id = s->free_ids.back();
    s->free_ids.pop_back();
  } else {
    id = (uint32_t)s->filters.size();
    s->filters.emplace_back();
  }
  ServeFilter &f = s->filters[id];
  f = ServeFilter();
  f.live = true;
  f.words = reinterpret_cast<uint32_t *>(p);
  f.num_blocks = num_blocks;
  f.chunk = chunk;
  f.off = off;
  *filter_id = id;
  return SBBF_OK;
}

sbbf_status sbbf_server_remove_filter(sbbf_server *s, uint32_t filter_id) {
  if (!s || filter_id >= s->filters.size() || !s->filters[filter_id].live)
    return set_error(SBBF_EINVAL, "unknown filter id");
  ServeFilter &f = s->filters[filter_id];
  while (!f.fifo.empty() || f.inflight > 0) {  // finish its work first
    sbbf_status st = server_pump(s, true);
    if (st != SBBF_OK) return st;
  }
  s->arena.release(f.chunk, f.off, (uint64_t)f.num_blocks * 32u);
  f.live = false;
  s->free_ids.push_back(filter_id);
  return SBBF_OK;
}

sbbf_status sbbf_server_arena_usage(const sbbf_server *s, uint64_t *used_bytes, uint64_t *reserved_bytes) {
  if (!s) return set_error(SBBF_EINVAL, "server is NULL");
  if (used_bytes) *used_bytes = s->arena.used;
  if (reserved_bytes) *reserved_bytes = s->arena.reserved;
  return SBBF_OK;
}

sbbf_status sbbf_server_submit(sbbf_server *s, uint32_t filter_id, int op, const uint64_t *d_hashes, uint64_t n,
                               uint8_t *d_out, uint64_t *req_id) {
  if (!s) return set_error(SBBF_EINVAL, "server is NULL");
  return server_enqueue(s, filter_id, (uint32_t)op, d_hashes, n, d_out, 0, req_id);
}

sbbf_status sbbf_server_pump(sbbf_server *s, int wait) {
  if (!s) return set_error(SBBF_EINVAL, "server is NULL");
  return server_pump(s, wait != 0);
}

sbbf_status sbbf_server_drain(sbbf_server *s) {
  if (!s) return set_error(SBBF_EINVAL, "server is NULL");
  while (s->pending > 0 || s->inflight > 0) {
    sbbf_status st = server_pump(s, true);
    if (st != SBBF_OK) return st;
  }
  return SBBF_OK;
}

sbbf_status sbbf_server_poll(sbbf_server *s, uint64_t *done_ids, uint32_t cap, uint32_t *n_done) {
  if (!s || !n_done || (cap && !done_ids)) return set_error(SBBF_EINVAL, "bad poll arguments");
  sbbf_status st = server_harvest(s, false);
  if (st != SBBF_OK) return st;
  const uint32_t n = (uint32_t)std::min<size_t>(cap, s->completed.size() - s->completed_head);
  for (uint32_t i = 0; i < n; ++i) done_ids[i] = s->completed[s->completed_head + i];
  s->completed_head += n;
  if (s->completed_head == s->completed.size()) {
    s->completed.clear();
    s->completed_head = 0;
  } else if (s->completed_head >= 4096 && 2 * s->completed_head >= s->completed.size()) {
    // drop the polled front once it is at least half of the list
    s->completed.erase(s->completed.begin(), s->completed.begin() + (ptrdiff_t)s->completed_head);
    s->completed_head = 0;
  }
  *n_done = n;
  return n ? SBBF_OK : SBBF_EAGAIN;
}

sbbf_status sbbf_server_request_times(const sbbf_server *s, uint64_t req_id, uint64_t *arrival_ns, uint64_t *done_ns) {
  if (!s || req_id >= s->reqs.size()) return set_error(SBBF_EINVAL, "unknown request id");
  if (arrival_ns) *arrival_ns = s->reqs[req_id].arrival_ns;
  if (done_ns) *done_ns = s->reqs[req_id].done_ns;
  return SBBF_OK;
}

sbbf_status sbbf_server_replay(sbbf_server *s, const sbbf_request *log, uint64_t count, int realtime,
                               uint64_t *first_id) {
  if (!s || (count && !log)) return set_error(SBBF_EINVAL, "server or log is NULL");
  for (uint64_t i = 1; i < count; ++i)
    if (log[i].arrival_ns < log[i - 1].arrival_ns) return set_error(SBBF_EINVAL, "log must be sorted by arrival");
  const uint64_t t0 = now_ns();
  if (first_id) *first_id = s->reqs.size();
  // room for the whole log up front (no reallocation while admitting)
  s->reqs.reserve(s->reqs.size() + count);
  s->completed.reserve(s->completed.size() + count);
  uint64_t next = 0;
  while (next < count || s->pending > 0 || s->inflight > 0) {
    const uint64_t t = now_ns();
    // Admit every request whose arrival time has passed; when not realtime
    // (all requests arrive at once), at most kReplayAdmitBatch per round, so
    // that the first steps run on the device while the rest are admitted.
    const uint64_t admit_end = realtime ? count : std::min<uint64_t>(count, next + kReplayAdmitBatch);
    while (next < admit_end && (!realtime || t0 + log[next].arrival_ns <= t)) {
      const sbbf_request &q = log[next];
      sbbf_status st = server_enqueue(s, q.filter_id, q.op, q.d_hashes, q.n, q.d_out,
                                      realtime ? t0 + q.arrival_ns : t, nullptr);
      if (st != SBBF_OK) return st;
      ++next;
    }
    sbbf_status st = server_pump(s, false);
    if (st != SBBF_OK) return st;
    if (next >= count && s->pending == 0 && s->inflight > 0) {
      if ((st = server_harvest(s, true)) != SBBF_OK) return st;
    } else if (s->pending == 0 && next < count) {
      // Idle until the next arrival. A sleep can overshoot its deadline by
      // tens of microseconds, and that delay lands on the request's latency,
      // so the loop sleeps only through long idle gaps, waking well before
      // the arrival, and polls through the rest.
      const uint64_t due = t0 + log[next].arrival_ns;
      const uint64_t now2 = now_ns();
      if (due > now2 + kReplaySleepMargin + 50000 && s->inflight == 0)
        std::this_thread::sleep_for(std::chrono::nanoseconds(due - now2 - kReplaySleepMargin));
    }
  }
  return SBBF_OK;
}

sbbf_status sbbf_server_replay_per_request(sbbf_server *s, const sbbf_request *log, uint64_t count,
                                           double *seconds) {
  if (!s || (count && !log)) return set_error(SBBF_EINVAL, "server or log is NULL");
  for (uint64_t i = 0; i < count; ++i) {
    const sbbf_request &q = log[i];
    if (q.filter_id >= s->filters.size() || !s->filters[q.filter_id].live)
      return set_error(SBBF_EINVAL, "unknown filter id in the log");
    if (q.op > 1) return set_error(SBBF_EINVAL, "op must be 0 (insert) or 1 (lookup)");
  }
  sbbf_status st = sbbf_server_drain(s);
  if (st != SBBF_OK) return st;
  // Borrowed handles on the resident filters' words (nothing is copied).
  std::vector<sbbf_filter *> h(s->filters.size(), nullptr);
  auto release = [&h]() {
    for (auto *f : h)
      if (f) (void)sbbf_destroy(f);
  };
  for (size_t f = 0; f < s->filters.size(); ++f) {
    if (!s->filters[f].live) continue;
    if ((st = sbbf_create_wrapped(s->filters[f].words, s->filters[f].num_blocks, &h[f])) != SBBF_OK) {
      release();
      return st;
    }
  }
  sbbf_launch ins_cfg{0, 0, 0, SBBF_INSERT_ATOMIC32, 0};
  sbbf_launch look_cfg{0, 0, 0, SBBF_LOOKUP_GATHER, 0};
  const uint64_t t0 = now_ns();
  for (uint64_t i = 0; i < count && st == SBBF_OK; ++i) {
    const sbbf_request &q = log[i];
    sbbf_filter *f = h[q.filter_id];
    st = q.op == 0 ? sbbf_insert_batch_ex(f, q.d_hashes, q.n, &ins_cfg, s->stream)
                   : sbbf_lookup_batch_ex(f, q.d_hashes, q.n, q.d_out, nullptr, &look_cfg, s->stream);
  }
  const hipError_t e = hipStreamSynchronize(s->stream);
  const uint64_t t1 = now_ns();
  release();
  if (st != SBBF_OK) return st;
  if (e != hipSuccess) return hip_error(e, "replay per request");
  if (seconds) *seconds = (double)(t1 - t0) / 1e9;
  return SBBF_OK;
}

sbbf_status sbbf_server_stats(const sbbf_server *s, sbbf_serving_stats *out) {
  if (!s || !out) return set_error(SBBF_EINVAL, "server or out is NULL");
  memset(out, 0, sizeof(*out));
  std::vector<double> lat;
  lat.reserve(s->reqs.size());
  for (const auto &r : s->reqs)
    if (r.done_ns) lat.push_back((double)(r.done_ns - r.arrival_ns) / 1e3);
  out->requests_done = s->req_done;
  out->keys_done = s->keys_done;
  out->steps = s->steps;
  out->p50_us = percentile(lat, 0.50);
  out->p99_us = percentile(lat, 0.99);
  out->max_us = lat.empty() ? 0.0 : *std::max_element(lat.begin(), lat.end());
  const double span = s->last_done > s->first_arrival && s->first_arrival != UINT64_MAX
                          ? (double)(s->last_done - s->first_arrival) / 1e9
                          : 0.0;
  out->span_s = span;
  out->gkeys_per_s = span > 0 ? (double)s->keys_done / span / 1e9 : 0.0;
  out->arena_used_bytes = s->arena.used;
  out->arena_reserved_bytes = s->arena.reserved;
  return SBBF_OK;
}

sbbf_status sbbf_server_snapshot(sbbf_server *s, uint32_t filter_id, void *host_dst) {
  if (!s || !host_dst || filter_id >= s->filters.size() || !s->filters[filter_id].live)
    return set_error(SBBF_EINVAL, "bad snapshot arguments");
  sbbf_status st = sbbf_server_drain(s);
  if (st != SBBF_OK) return st;
  const ServeFilter &f = s->filters[filter_id];
  hipError_t e = hipMemcpyAsync(host_dst, f.words, (size_t)f.num_blocks * 32u, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  return hip_error(e, "snapshot");
}

sbbf_status sbbf_server_restore(sbbf_server *s, uint32_t filter_id, const void *host_src) {
  if (!s || !host_src || filter_id >= s->filters.size() || !s->filters[filter_id].live)
    return set_error(SBBF_EINVAL, "bad restore arguments");
  sbbf_status st = sbbf_server_drain(s);
  if (st != SBBF_OK) return st;
  const ServeFilter &f = s->filters[filter_id];
  hipError_t e = hipMemcpyAsync(f.words, host_src, (size_t)f.num_blocks * 32u, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  return hip_error(e, "restore");
}

}  // extern "C"
