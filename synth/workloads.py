"""Workload recipes: which hashes are inserted and which are looked up.

Streams used (SplitMix64 seeds):
  1  hashes inserted (the members)
  2  fresh hashes looked up as non-members
  3  shuffle keys (a stable sort by these keys, in unsigned order, is the shuffle)
  4  per-filter key counts of the grouped workload

The paper's own measurements use random keys from a third-party harness that is
not available; uniform 64-bit hashes at the paper's three filter geometries
(131 KB / 1 MB / 134 MB filters for 1e5 / 1e6 / 1e8 keys, the table in the
evaluation) stand in for them.

Members and non-members never collide: stream ``s`` at index ``i`` has state
``s + (i + 1) * GAMMA`` and the finaliser is a bijection, so G(1)[k] == G(2)[i]
only when (k - i) * GAMMA == 1 (mod 2**64), i.e. when k - i is the modular
inverse of GAMMA, a number far outside every index range used here.
``streams_disjoint`` checks that argument for given ranges, and the
de-duplication the recipes ask for is then the identity.
"""

from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from .splitmix import GAMMA, splitmix64_stream, unit_double

_MASK64 = (1 << 64) - 1
_GAMMA_INV = pow(GAMMA, -1, 1 << 64)

SEED_MEMBERS = 1
SEED_NONMEMBERS = 2
SEED_SHUFFLE = 3
SEED_GROUP_SIZES = 4


def streams_disjoint(seed_a: int, len_a: int, seed_b: int, len_b: int) -> bool:
    """True when G(seed_a)[0:len_a] and G(seed_b)[0:len_b] share no value.

    Values are equal exactly when the states are, i.e. when
    (k - i) * GAMMA == seed_b - seed_a (mod 2**64) for k < len_a, i < len_b.
    """
    d = ((seed_b - seed_a) * _GAMMA_INV) & _MASK64  # the only k - i that collides
    # k - i ranges over (-(len_b - 1)) .. (len_a - 1); map d into that signed window.
    if d <= len_a - 1:
        return False
    if (1 << 64) - d <= len_b - 1:
        return False
    return True


def _stable_unsigned_argsort(keys, backend: str):
    if backend == "numpy":
        return np.argsort(keys, kind="stable")
    import torch

    # Flip the sign bit so that signed order of the int64 view is unsigned order.
    flipped = torch.bitwise_xor(keys, -(1 << 63))
    return torch.sort(flipped, stable=True).indices


def _concat(parts, backend):
    if backend == "numpy":
        return np.concatenate(parts)
    import torch

    return torch.cat(parts)


def _take(arr, idx, backend):
    if backend == "numpy":
        return arr[idx]
    return arr.index_select(0, idx)


def _zeros_bool(n, backend, device):
    if backend == "numpy":
        return np.zeros(n, dtype=bool)
    import torch

    return torch.zeros(n, dtype=torch.bool, device=device)


def _ones_bool(n, backend, device):
    if backend == "numpy":
        return np.ones(n, dtype=bool)
    import torch

    return torch.ones(n, dtype=torch.bool, device=device)


@dataclasses.dataclass
class PlainWorkload:
    """One filter: hashes to insert, then hashes to look up."""

    name: str
    num_blocks: int
    inserts: object  # uint64 ndarray or int64 tensor
    lookups: object
    is_member: object  # bool per lookup: True when the looked-up hash was inserted
    n_member_lookups: int
    n_nonmember_lookups: int


# Plain single-filter workloads at the paper's three geometries (its table of
# insert/lookup rates; 131 KB, 1 MB and 134 MB filters).
PLAIN_CONFIGS = {
    # 4,096 blocks (128 KiB); 1e5 members looked up, then 1e6 non-members, unshuffled.
    "plain_100k": dict(num_blocks=4096, n_insert=100_000, n_member_lookups=100_000,
                       n_nonmember_lookups=1_000_000, member_source="prefix", shuffle=False),
    # 32,768 blocks (1 MiB); 1e7 lookups, half members (cycling over the 1e6), shuffled.
    "plain_1m": dict(num_blocks=32768, n_insert=1_000_000, n_member_lookups=5_000_000,
                     n_nonmember_lookups=5_000_000, member_source="cycle", shuffle=True),
    # 4,194,304 blocks (128 MiB, 10.74 bits/key); 2e8 lookups at a 10 % member rate, shuffled.
    "plain_100m": dict(num_blocks=4194304, n_insert=100_000_000, n_member_lookups=20_000_000,
                       n_nonmember_lookups=180_000_000, member_source="prefix", shuffle=True),
}


def plain_workload(name: str, backend: str = "numpy", device=None, scale: Optional[float] = None,
                   **overrides) -> PlainWorkload:
    """Build a plain workload by name.

    ``scale`` shrinks every count (and the block count, keeping bits per key)
    for quick tests; ``overrides`` replaces individual recipe fields.
    """
    cfg = dict(PLAIN_CONFIGS[name])
    cfg.update(overrides)
    if scale is not None:
        for k in ("n_insert", "n_member_lookups", "n_nonmember_lookups"):
            cfg[k] = max(1, int(round(cfg[k] * scale)))
        cfg["num_blocks"] = max(1, int(round(cfg["num_blocks"] * scale)))
    nb = int(cfg["num_blocks"])
    n_ins = int(cfg["n_insert"])
    n_mem = int(cfg["n_member_lookups"])
    n_non = int(cfg["n_nonmember_lookups"])

    members = splitmix64_stream(SEED_MEMBERS, n_ins, backend=backend, device=device)
    if cfg["member_source"] == "prefix":
        if n_mem > n_ins:
            raise ValueError("prefix member lookups cannot exceed the inserted count")
        mem_look = members[:n_mem]
    elif cfg["member_source"] == "cycle":
        if backend == "numpy":
            idx = np.arange(n_mem, dtype=np.int64) % n_ins
        else:
            import torch

            idx = torch.arange(n_mem, dtype=torch.int64, device=device) % n_ins
        mem_look = _take(members, idx, backend)
    else:
        raise ValueError(cfg["member_source"])

    if not streams_disjoint(SEED_MEMBERS, n_ins, SEED_NONMEMBERS, n_non):
        raise RuntimeError("member and non-member streams overlap; de-duplication needed")
    non = splitmix64_stream(SEED_NONMEMBERS, n_non, backend=backend, device=device)

    lookups = _concat([mem_look, non], backend)
    is_member = _concat([_ones_bool(n_mem, backend, device), _zeros_bool(n_non, backend, device)], backend)
    if cfg["shuffle"]:
        keys = splitmix64_stream(SEED_SHUFFLE, n_mem + n_non, backend=backend, device=device)
        perm = _stable_unsigned_argsort(keys, backend)
        del keys
        lookups = _take(lookups, perm, backend)
        is_member = _take(is_member, perm, backend)
    return PlainWorkload(name=name, num_blocks=nb, inserts=members, lookups=lookups,
                         is_member=is_member, n_member_lookups=n_mem, n_nonmember_lookups=n_non)


@dataclasses.dataclass
class GroupedWorkload:
    """Many independent filters of uneven sizes, in CSR form.

    Filter f inserts ``inserts[ins_off[f]:ins_off[f+1]]`` and then looks up
    ``lookups[look_off[f]:look_off[f+1]]``.
    """

    num_filters: int
    n: np.ndarray  # int64 keys inserted per filter
    blocks: np.ndarray  # int64 blocks per filter
    ins_off: np.ndarray  # int64 [F+1]
    look_off: np.ndarray  # int64 [F+1]
    inserts: object
    lookups: object
    is_member: object


def grouped_sizes(num_filters: int, seed: int = SEED_GROUP_SIZES, log10_min: float = 3.0,
                  log10_max: float = 6.0, bits_per_key: float = 10.5):
    """Per-filter key counts, log-uniform in [10**log10_min, 10**log10_max], and block counts.

    n_f = clamp(floor(10**(lo + (hi - lo) * u_f)), 10**lo, 10**hi) with u_f the
    top 53 bits of G(seed)[f]; blocks_f = ceil(n_f * bits_per_key / 256).
    """
    u = unit_double(splitmix64_stream(seed, num_filters))
    lo_n = int(round(10 ** log10_min))
    hi_n = int(round(10 ** log10_max))
    n = np.floor(np.power(10.0, log10_min + (log10_max - log10_min) * u)).astype(np.int64)
    n = np.clip(n, lo_n, hi_n)
    blocks = np.ceil(n.astype(np.float64) * bits_per_key / 256.0).astype(np.int64)
    blocks = np.maximum(blocks, 1)
    return n, blocks


def grouped_workload(num_filters: int = 2048, log10_min: float = 3.0, log10_max: float = 6.0,
                     bits_per_key: float = 10.5, nonmembers_per_member: int = 3,
                     backend: str = "numpy", device=None, size_seed: int = SEED_GROUP_SIZES) -> GroupedWorkload:
    """Grouped workload: every filter looks up its own members once each plus
    ``nonmembers_per_member`` fresh hashes per member, shuffled within the filter.

    Inserts come from one shared stream G(1), cut in filter order; non-members
    from one shared stream G(2). The within-filter shuffle is a stable sort by
    the composite key (f << 40) | (G(3)[i] >> 24).
    """
    n, blocks = grouped_sizes(num_filters, size_seed, log10_min, log10_max, bits_per_key)
    F = num_filters
    ins_off = np.zeros(F + 1, dtype=np.int64)
    ins_off[1:] = np.cumsum(n)
    look_n = n * (1 + nonmembers_per_member)
    look_off = np.zeros(F + 1, dtype=np.int64)
    look_off[1:] = np.cumsum(look_n)
    tot_ins = int(ins_off[-1])
    tot_look = int(look_off[-1])
    tot_non = tot_ins * nonmembers_per_member
    if not streams_disjoint(SEED_MEMBERS, tot_ins, SEED_NONMEMBERS, tot_non):
        raise RuntimeError("member and non-member streams overlap")

    inserts = splitmix64_stream(SEED_MEMBERS, tot_ins, backend=backend, device=device)
    non = splitmix64_stream(SEED_NONMEMBERS, tot_non, backend=backend, device=device)

    # Unshuffled layout per filter: [its n_f members, its 3 n_f non-members].
    # Build a gather index into concat(inserts, non) for every lookup slot,
    # then shuffle within each filter with a stable sort by a composite key.
    k = nonmembers_per_member
    if backend == "numpy":
        fid = np.repeat(np.arange(F, dtype=np.int64), look_n)
        pos = np.arange(tot_look, dtype=np.int64) - look_off[fid]
        nf = n[fid]
        is_mem = pos < nf
        src = np.where(is_mem, ins_off[fid] + pos, tot_ins + ins_off[fid] * k + (pos - nf))
        del pos, nf
        shuffle = splitmix64_stream(SEED_SHUFFLE, tot_look)
        comp = (fid.astype(np.uint64) << np.uint64(40)) | (shuffle >> np.uint64(24))
        del shuffle, fid
        perm = np.argsort(comp, kind="stable")
        del comp
        lookups = np.concatenate([inserts, non])[src[perm]]
        is_member = is_mem[perm]
    else:
        import torch

        t_look_n = torch.from_numpy(look_n).to(device)
        t_look_off = torch.from_numpy(look_off).to(device)
        t_ins_off = torch.from_numpy(ins_off).to(device)
        t_n = torch.from_numpy(n).to(device)
        fid = torch.repeat_interleave(torch.arange(F, dtype=torch.int64, device=device), t_look_n)
        pos = torch.arange(tot_look, dtype=torch.int64, device=device) - t_look_off[fid]
        nf = t_n[fid]
        is_mem = pos < nf
        src = torch.where(is_mem, t_ins_off[fid] + pos, tot_ins + t_ins_off[fid] * k + (pos - nf))
        del pos, nf
        shuffle = splitmix64_stream(SEED_SHUFFLE, tot_look, backend="torch", device=device)
        # (f << 40) | (G(3)[i] >>> 24): non-negative, so signed order is unsigned order.
        comp = (fid << 40) | torch.bitwise_and(shuffle >> 24, (1 << 40) - 1)
        del shuffle, fid
        perm = torch.sort(comp, stable=True).indices
        del comp
        src = src.index_select(0, perm)
        is_member = is_mem.index_select(0, perm)
        del perm, is_mem
        both = torch.cat([inserts, non])
        lookups = both.index_select(0, src)
        del both, src
    return GroupedWorkload(num_filters=F, n=n, blocks=blocks, ins_off=ins_off, look_off=look_off,
                           inserts=inserts, lookups=lookups, is_member=is_member)


def grouped_filter_inputs(n: np.ndarray, f: int, nonmembers_per_member: int = 3):
    """Filter ``f``'s inserts and lookups of the grouped workload (numpy),
    equal to ``grouped_workload``'s slices ``inserts[ins_off[f]:ins_off[f+1]]``
    and ``lookups[look_off[f]:look_off[f+1]]`` for the same per-filter counts
    ``n``, built from that filter's stream ranges alone.

    The workload's shuffle sorts by (filter << 40) | (G(3)[i] >> 24) over the
    whole lookup array; inside one filter's range the filter part is constant,
    so the filter's order is the stable sort of its own G(3)[i] >> 24.
    """
    k = nonmembers_per_member
    n = np.asarray(n, dtype=np.int64)
    ins0 = int(n[:f].sum())
    nf = int(n[f])
    look0 = ins0 * (1 + k)
    members = splitmix64_stream(SEED_MEMBERS, nf, start=ins0)
    non = splitmix64_stream(SEED_NONMEMBERS, k * nf, start=k * ins0)
    shuffle = splitmix64_stream(SEED_SHUFFLE, (1 + k) * nf, start=look0) >> np.uint64(24)
    perm = np.argsort(shuffle, kind="stable")
    lookups = np.concatenate([members, non])[perm]
    is_member = perm < nf
    return members, lookups, is_member
