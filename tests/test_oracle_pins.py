"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the
constants printed in the appendix figure, closed forms of the block selection,
the bijection property of odd multiply-shift, brute force with Python big
integers on tiny inputs, the algebra of OR (order independence, idempotence,
union), outputs of the paper's own C code, and the paper's false-positive
formula at the measured load.
"""

import hashlib
import math

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
from oracle import fpr
from synth import plain_workload, splitmix64_stream

M32 = 0xFFFFFFFF


# --- seeds (appendix figure, the mask routine) -------------------------------

def test_seeds_are_the_printed_constants_in_little_endian_lane_order(golden):
    rows = golden("appendix_seeds.txt")
    assert len(rows) == 4
    expect = []
    for hi, lo in rows:
        # constant k occupies lanes 2k (low half) and 2k+1 (high half)
        expect += [int(lo, 16), int(hi, 16)]
    assert [int(s) for s in oracle.seeds()] == expect


def test_seeds_are_odd():
    # multiply-shift hashing needs odd multipliers (construction paragraph)
    assert all(int(s) & 1 for s in oracle.seeds())


# --- block selection (appendix figure, block_index) --------------------------

@pytest.mark.parametrize("B", [1, 2, 3, 5, 7, 100, 4096, 32768, 4194304, 41016, (1 << 32) - 1])
def test_block_special_cases(B):
    assert oracle.block(0, B) == 0
    assert oracle.block(0xFFFFFFFF_FFFFFFFF, B) == B - 1
    # the low half never matters
    assert oracle.block(0x12345678_00000000, B) == oracle.block(0x12345678_FFFFFFFF, B)


@pytest.mark.parametrize("k", [0, 1, 5, 12, 22, 31])
def test_block_power_of_two_is_top_bits(k):
    B = 1 << k
    for h in splitmix64_stream(11, 200).tolist():
        assert oracle.block(h, B) == (h >> (64 - k) if k else 0)


@pytest.mark.parametrize("B", [1, 3, 7, 10, 97, 1000, 4095, 4097])
def test_block_boundaries_exact(B):
    """floor(x * B / 2**32) is a monotone step function; block b starts at
    x_b = ceil(b * 2**32 / B). Checking every boundary pins it exactly, and
    each block receives floor(2**32/B) or ceil(2**32/B) of the 2**32 values."""
    starts = [-(-b * (1 << 32) // B) for b in range(B + 1)]
    for b in range(B):
        x = starts[b]
        assert oracle.block(x << 32, B) == b
        if x > 0:
            assert oracle.block((x - 1) << 32, B) == b - 1
        width = starts[b + 1] - starts[b]
        assert width in ((1 << 32) // B, -(-(1 << 32) // B))


def test_block_is_uniform_on_random_hashes():
    B = 1000
    h = splitmix64_stream(12, 2_000_000)
    c = oracle.block_histogram(h, B).astype(float)
    expect = h.size / B
    chi2 = ((c - expect) ** 2 / expect).sum()
    # chi-square with 999 dof: mean 999, sd ~ 44.7
    assert abs(chi2 - 999) < 6 * 44.7


# --- mask (construction paragraph; appendix figure, make_mask) ---------------

def test_mask_has_one_bit_per_lane():
    for x in splitmix64_stream(13, 500).tolist():
        m = oracle.mask(x & M32)
        assert all(bin(int(w)).count("1") == 1 for w in m)


@pytest.mark.slow
def test_index_histogram_exhaustive():
    """Over all 2**32 low halves, an odd multiplier permutes the 32-bit values,
    so each lane picks every index 0..31 exactly 2**27 times. Fails for an
    even seed, a wrong shift, or keeping the high half of the product."""
    hist = oracle.index_histogram(0, 1 << 32)
    assert (hist == (1 << 27)).all()


def test_index_cosets_are_permutations():
    """For any fixed r, the 32 low halves x = r + t * 2**27 (t = 0..31) give
    idx_j = (c_r + s_j * t) mod 32, a permutation of 0..31 when s_j is odd.
    A cheap consequence of the exhaustive property, checked on many cosets."""
    for r in splitmix64_stream(14, 64).tolist():
        r &= (1 << 27) - 1
        rows = [oracle.bit_indices(r + (t << 27)) for t in range(32)]
        for j in range(8):
            assert sorted(int(row[j]) for row in rows) == list(range(32))


def test_worked_examples(golden):
    for row in golden("paper_code_examples.txt"):
        h, B, b = int(row[0], 16), int(row[1]), int(row[2])
        idx = [int(v) for v in row[3:11]]
        assert oracle.block(h, B) == b
        assert [int(v) for v in oracle.bit_indices(h & M32)] == idx
        assert [int(v) for v in oracle.mask(h & M32)] == [1 << i for i in idx]


# --- brute force with big integers on tiny inputs ----------------------------

def _bigint_filter(B, hashes):
    """Filter as one Python integer: bit 256*b + 32*j + k. Independent of the
    oracle's word array representation."""
    s = [int(v) for v in oracle.seeds()]
    bits = 0
    for h in hashes:
        b = ((h >> 32) * B) >> 32
        x = h & M32
        for j in range(8):
            bits |= 1 << (256 * b + 32 * j + (((s[j] * x) & M32) >> 27))
    return bits


def _bigint_contains(bits, B, h):
    s = [int(v) for v in oracle.seeds()]
    b = ((h >> 32) * B) >> 32
    x = h & M32
    return all((bits >> (256 * b + 32 * j + (((s[j] * x) & M32) >> 27))) & 1 for j in range(8))


@pytest.mark.parametrize("B", [1, 2, 3, 5, 8])
def test_brute_force_tiny(B):
    hs = splitmix64_stream(20 + B, 64).tolist()
    words = oracle.build_filter(B, np.array(hs, dtype=np.uint64))
    as_int = int.from_bytes(words.astype("<u4").tobytes(), "little")
    assert as_int == _bigint_filter(B, hs)
    probes = hs + splitmix64_stream(40 + B, 256).tolist()
    got = oracle.lookup(words, B, np.array(probes, dtype=np.uint64))
    assert [bool(v) for v in got] == [_bigint_contains(as_int, B, p) for p in probes]


# --- invariants ---------------------------------------------------------------

hash_lists = st.lists(st.integers(min_value=0, max_value=(1 << 64) - 1), min_size=0, max_size=200)


@settings(max_examples=60, deadline=None)
@given(hs=hash_lists, B=st.integers(min_value=1, max_value=64))
def test_no_false_negatives(hs, B):
    h = np.array(hs, dtype=np.uint64)
    words = oracle.build_filter(B, h)
    assert oracle.lookup(words, B, h).all()


@settings(max_examples=60, deadline=None)
@given(h=st.integers(min_value=0, max_value=(1 << 64) - 1), B=st.integers(min_value=1, max_value=1 << 20))
def test_single_insert_sets_one_bit_per_lane(h, B):
    words = oracle.build_filter(B, np.array([h], dtype=np.uint64))
    b = oracle.block(h, B)
    blk = words[8 * b: 8 * b + 8]
    assert all(bin(int(w)).count("1") == 1 for w in blk)
    assert oracle.popcount(words) == 8


@settings(max_examples=40, deadline=None)
@given(hs=hash_lists, B=st.integers(min_value=1, max_value=32), seed=st.integers(0, 1000))
def test_order_independence_idempotence_union(hs, B, seed):
    h = np.array(hs, dtype=np.uint64)
    base = oracle.build_filter(B, h)
    rng = np.random.default_rng(seed)
    perm = h[rng.permutation(h.size)] if h.size else h
    assert np.array_equal(oracle.build_filter(B, perm), base)
    twice = oracle.build_filter(B, np.concatenate([h, h]))
    assert np.array_equal(twice, base)
    cut = h.size // 2
    union = oracle.build_filter(B, h[:cut]) | oracle.build_filter(B, h[cut:])
    assert np.array_equal(union, base)


def test_all_ones_and_empty_filters():
    B = 17
    probes = splitmix64_stream(50, 1000)
    assert oracle.lookup(np.full(8 * B, M32, dtype=np.uint32), B, probes).all()
    assert not oracle.lookup(oracle.new_filter(B), B, probes).any()


def test_lookup_is_and_over_lanes():
    B = 4
    probes = splitmix64_stream(51, 2000).tolist()
    rng = np.random.default_rng(5)
    words = rng.integers(0, 1 << 32, size=8 * B, dtype=np.uint64).astype(np.uint32)
    words &= rng.integers(0, 1 << 32, size=8 * B, dtype=np.uint64).astype(np.uint32)  # ~25 % density
    got = oracle.lookup(words, B, np.array(probes, dtype=np.uint64))
    for p, g in zip(probes, got):
        b = oracle.block(p, B)
        idx = oracle.bit_indices(p & M32)
        want = all((int(words[8 * b + j]) >> int(idx[j])) & 1 for j in range(8))
        assert bool(g) == want


def test_lookup_bits_packing():
    B = 9
    h = splitmix64_stream(52, 1000)
    words = oracle.build_filter(B, h[:300])
    by = oracle.lookup(words, B, h)
    bits = oracle.lookup_bits(words, B, h)
    assert bits.size == (h.size + 31) // 32
    unpacked = np.unpackbits(bits.view(np.uint8), bitorder="little")[: h.size]
    assert np.array_equal(unpacked, by)
    assert (np.unpackbits(bits.view(np.uint8), bitorder="little")[h.size:] == 0).all()


def test_select_definition():
    """select = the ascending positions of the lookup's ones: every inserted
    hash is selected (no false negatives), nothing else but the lookup's
    false positives, and a brute-force tiny case written out by hand."""
    B = 13
    h = splitmix64_stream(53, 4000)
    words = oracle.build_filter(B, h[:500])
    sel = oracle.select(words, B, h)
    assert sel.dtype == np.uint32
    assert np.all(np.diff(sel.astype(np.int64)) > 0)          # ascending, unique
    assert np.isin(np.arange(500), sel).all()                  # members
    assert sel.size == int(oracle.lookup(words, B, h).sum())
    for i in range(h.size):                                    # one by one
        assert (i in set(sel.tolist())) == oracle.contains(words, B, int(h[i]))
    # all-ones filter selects every index; the empty filter none
    ones = np.full(8 * B, 0xFFFFFFFF, dtype=np.uint32)
    assert np.array_equal(oracle.select(ones, B, h), np.arange(h.size, dtype=np.uint32))
    assert oracle.select(oracle.new_filter(B), B, h).size == 0


# --- whole workloads against the paper's code and the paper's formula ------------

def _run(name):
    w = plain_workload(name)
    words = oracle.build_filter(w.num_blocks, w.inserts)
    res = oracle.lookup(words, w.num_blocks, w.lookups)
    return w, words, res


def _config_row(golden, name):
    for row in golden("paper_code_configs.txt"):
        if row[0] == name:
            return row
    raise KeyError(name)


@pytest.mark.parametrize("name", ["plain_100k", "plain_1m"])
def test_config_matches_paper_code(golden, name):
    row = _config_row(golden, name)
    w, words, res = _run(name)
    assert w.num_blocks == int(row[1]) and w.inserts.size == int(row[2])
    assert oracle.popcount(words) == int(row[3])
    assert (~w.is_member).sum() == int(row[4])
    assert int(res[~w.is_member].sum()) == int(row[5])
    assert hashlib.sha256(words.astype("<u4").tobytes()).hexdigest()[:16] == row[6]
    assert res[w.is_member].all()


@pytest.mark.slow
def test_config_100m_matches_paper_code(golden):
    row = _config_row(golden, "plain_100m")
    B = int(row[1])
    ins = splitmix64_stream(1, int(row[2]))
    words = oracle.build_filter(B, ins)
    del ins
    assert oracle.popcount(words) == int(row[3])
    assert hashlib.sha256(words.astype("<u4").tobytes()).hexdigest()[:16] == row[6]
    fp = 0
    step = 30_000_000
    for s in range(0, int(row[4]), step):
        non = splitmix64_stream(2, min(step, int(row[4]) - s), start=s)
        fp += int(oracle.lookup(words, B, non).sum())
    assert fp == int(row[5])


@pytest.mark.parametrize("name", ["plain_100k", "plain_1m"])
def test_measured_fpr_matches_paper_formula(name):
    """The measured false-positive rate of the oracle's filter agrees with the
    paper's Poisson-sum formula at the measured load a = n / B, within
    max(4 sigma, 3 % relative), and with the filter's own conditional estimate
    within 4 sigma + 0.5 % relative."""
    w, words, res = _run(name)
    non = ~w.is_member
    N = int(non.sum())
    measured = res[non].sum() / N
    a = w.inserts.size / w.num_blocks
    F = fpr.sbbf_fpr(a)
    sigma = math.sqrt(F * (1 - F) / N)
    assert abs(measured - F) <= max(4 * sigma, 0.03 * F)
    cond = oracle.conditional_fpr(words, w.num_blocks)
    assert abs(measured - cond) <= 4 * sigma + 0.005 * cond
