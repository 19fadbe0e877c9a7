"""Request logs for the serving workload.

Streams used (SplitMix64 seeds):
  5   per-filter capacities (as the grouped workload, with its own seed)
  6   inter-arrival times: exponential with rate `rate_per_s` (a Poisson stream)
  7   operation: insert with probability `insert_frac`, else lookup
  8   batch size: floor(max_size ** u), clamped to [1, max_size] (log-uniform)
  9   filter: uniform over the filters
  10  fresh hashes, consumed in request order
  11  per lookup key: drawn from the filter's earlier inserts with probability
      `member_frac` (when the filter has any), else a fresh hash
  12  which earlier insert a member draw takes (uniform over them)

Payloads of all requests are laid end to end in request order; lookup outputs
likewise (one byte per looked-up key).
"""

from __future__ import annotations

import dataclasses

import numpy as np

from .splitmix import GAMMA, splitmix64_stream, unit_double
from .workloads import grouped_sizes

SEED_SERVE_SIZES = 5


def _stream_at(seed: int, positions: np.ndarray) -> np.ndarray:
    """G(seed)[positions] for arbitrary positions, via the stream's closed form."""
    from .splitmix import _mix_numpy_inplace

    z = (positions.astype(np.uint64) + np.uint64(1)) * np.uint64(GAMMA) + np.uint64(seed)
    _mix_numpy_inplace(z)
    return z


def _stream_at_torch(seed: int, positions):
    """As _stream_at on an int64 tensor of positions (int64 bit views out)."""
    from .splitmix import _M1, _M2, _as_signed, _lsr_torch

    z = (positions + 1).mul_(_as_signed(GAMMA)).add_(_as_signed(seed))
    z.bitwise_xor_(_lsr_torch(z, 30)).mul_(_as_signed(_M1))
    z.bitwise_xor_(_lsr_torch(z, 27)).mul_(_as_signed(_M2))
    z.bitwise_xor_(_lsr_torch(z, 31))
    return z


def _unit_double_torch(z):
    import torch

    from .splitmix import _lsr_torch

    return _lsr_torch(z, 11).to(torch.float64) * (2.0 ** -53)


def _umod_torch(z, m):
    """(z as unsigned 64-bit) mod m, for int64 tensors z (bit views) and
    0 < m < 2**31, exact: z = hi * 2**32 + lo, so z mod m is
    ((hi mod m) * (2**32 mod m) + lo mod m) mod m with every term below 2**62."""
    from .splitmix import _lsr_torch

    hi = _lsr_torch(z, 32)
    lo = z & 0xFFFFFFFF
    return ((hi % m) * ((1 << 32) % m) + lo % m) % m


# Lookup keys per piece of the member draws (bounds the temporaries).
_DRAW_CHUNK = 1 << 25


@dataclasses.dataclass
class ServingLog:
    blocks: np.ndarray      # int64 [F] blocks per filter
    capacity: np.ndarray    # int64 [F] keys the filter was sized for
    arrival_ns: np.ndarray  # uint64 [R], non-decreasing
    filter: np.ndarray      # uint32 [R]
    op: np.ndarray          # uint32 [R] (0 insert, 1 lookup)
    n: np.ndarray           # int64 [R]
    key_off: np.ndarray     # int64 [R + 1] into payload
    out_off: np.ndarray     # int64 [R + 1] into the output bytes (lookups only advance it)
    payload: np.ndarray     # uint64 [sum n]

    @property
    def num_filters(self) -> int:
        return int(self.blocks.size)

    @property
    def num_requests(self) -> int:
        return int(self.n.size)


def serving_log(num_filters: int = 4096, num_requests: int = 200_000, rate_per_s: float = 1e6,
                insert_frac: float = 0.2, max_size: int = 65536, member_frac: float = 0.25,
                log10_min: float = 3.0, log10_max: float = 6.0, bits_per_key: float = 10.5,
                backend: str = "numpy", device=None) -> ServingLog:
    """The request log. Per-request fields are numpy arrays on the host with
    either backend; the payload is a uint64 ndarray (numpy) or an int64
    tensor of the same bits on ``device`` (torch)."""
    F, R = num_filters, num_requests
    cap, blocks = grouped_sizes(F, SEED_SERVE_SIZES, log10_min, log10_max, bits_per_key)
    u = unit_double(splitmix64_stream(6, R))
    dt = -np.log1p(-u) / rate_per_s * 1e9
    arrival = np.floor(np.cumsum(dt)).astype(np.uint64)
    op = (unit_double(splitmix64_stream(7, R)) >= insert_frac).astype(np.uint32)
    size = np.floor(np.power(float(max_size), unit_double(splitmix64_stream(8, R)))).astype(np.int64)
    size = np.clip(size, 1, max_size)
    filt = (splitmix64_stream(9, R) % np.uint64(F)).astype(np.uint32)

    key_off = np.zeros(R + 1, dtype=np.int64)
    key_off[1:] = np.cumsum(size)
    total = int(key_off[-1])
    payload = splitmix64_stream(10, total, backend=backend, device=device)
    out_off = np.zeros(R + 1, dtype=np.int64)
    out_off[1:] = np.cumsum(np.where(op == 1, size, 0))

    # Earlier inserts of each request's filter: order the requests by filter
    # (stable, so log order within a filter), count the keys inserted before
    # each request, and lay every filter's inserted keys (their payload
    # positions, in log order) end to end in one table.
    by_f = np.argsort(filt, kind="stable")
    ins_n = np.where(op[by_f] == 0, size[by_f], 0)
    f_sorted = filt[by_f].astype(np.int64)
    f_first = np.searchsorted(f_sorted, np.arange(F))           # first sorted request of each filter
    run = np.cumsum(ins_n) - ins_n                                # keys inserted before, over the sorted order
    base_of_f = run[np.minimum(f_first, R - 1)] if R else np.zeros(F, dtype=np.int64)
    before = np.empty(R, dtype=np.int64)
    before[by_f] = run - base_of_f[f_sorted]                      # per request: its filter's keys inserted earlier
    table_base = np.zeros(F, dtype=np.int64)                      # where each filter's inserted keys start in the table
    table_base[:] = base_of_f
    ins_req = by_f[ins_n > 0]                                     # insert requests, grouped by filter, log order
    lens = size[ins_req]
    starts = key_off[ins_req] - np.concatenate([[0], np.cumsum(lens)[:-1]])
    if backend == "numpy":
        table = np.repeat(starts, lens) + np.arange(int(lens.sum()))
    else:
        import torch

        table = torch.repeat_interleave(torch.from_numpy(starts).to(device), torch.from_numpy(lens).to(device)) + \
            torch.arange(int(lens.sum()), dtype=torch.int64, device=device)

    # Member draws for lookups with earlier inserts on their filter, a piece of
    # the lookup requests at a time. A draw reads the payload of an insert
    # request and writes into a lookup request, so the pieces are independent.
    look = np.nonzero((op == 1) & (before > 0))[0]
    if look.size and backend != "numpy" and int(before.max()) >= 1 << 31:
        raise ValueError("a filter has 2**31 or more earlier inserts")
    if backend != "numpy":
        import torch

        t_before = torch.from_numpy(before).to(device)
        t_filt = torch.from_numpy(filt.astype(np.int64)).to(device)
        t_base = torch.from_numpy(table_base).to(device)
    csum = np.cumsum(size[look])
    lo_r = 0
    while lo_r < look.size:
        done = int(csum[lo_r - 1]) if lo_r else 0
        hi_r = max(int(np.searchsorted(csum, done + _DRAW_CHUNK, side="right")), lo_r + 1)
        piece = look[lo_r:hi_r]
        lo_r = hi_r
        lens_p = size[piece]
        starts_p = key_off[piece] - np.concatenate([[0], np.cumsum(lens_p)[:-1]])
        if backend == "numpy":
            req_of_key = np.repeat(piece, lens_p)
            key_pos = np.repeat(starts_p, lens_p) + np.arange(int(lens_p.sum()))
            u = unit_double(_stream_at(11, key_pos))
            mem = u < member_frac
            key_pos, req_of_key = key_pos[mem], req_of_key[mem]
            idx = (_stream_at(12, key_pos) % before[req_of_key].astype(np.uint64)).astype(np.int64)
            payload[key_pos] = payload[table[table_base[filt[req_of_key]] + idx]]
        else:
            t_lens = torch.from_numpy(lens_p).to(device)
            req_of_key = torch.repeat_interleave(torch.from_numpy(piece.astype(np.int64)).to(device), t_lens)
            key_pos = torch.repeat_interleave(torch.from_numpy(starts_p).to(device), t_lens) + \
                torch.arange(int(lens_p.sum()), dtype=torch.int64, device=device)
            mem = _unit_double_torch(_stream_at_torch(11, key_pos)) < member_frac
            key_pos, req_of_key = key_pos[mem], req_of_key[mem]
            idx = _umod_torch(_stream_at_torch(12, key_pos), t_before[req_of_key])
            payload[key_pos] = payload[table[t_base[t_filt[req_of_key]] + idx]]
    return ServingLog(blocks=blocks, capacity=cap, arrival_ns=arrival, filter=filt, op=op, n=size,
                      key_off=key_off, out_off=out_off, payload=payload)
