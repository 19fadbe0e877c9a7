"""Pins of the oracle's block variants with four and sixteen lanes.

The paper defines the method with eight 32-bit lanes per block and notes that
four or sixteen would work too (footnote to the list of central ideas); it
prints seeds for eight lanes only. The oracle's readings: four lanes use seeds
0..3 of the appendix figure; sixteen lanes use the figure's eight seeds, then
the low 32 bits (lowest bit forced to one) of the first eight outputs of
SplitMix64 seeded with 16. These tests pin the variants to the eight-lane
method (whose pins are the paper's printed constants and the paper's own
code), to brute force with Python integers, to the algebra of OR, and to the
false-positive formula of the analysis section with K words per block.
"""

import math

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
from oracle import fpr
from synth import splitmix64, splitmix64_stream

M32 = 0xFFFFFFFF


def _printed_seeds(golden):
    out = []
    for hi, lo in golden("appendix_seeds.txt"):
        out += [int(lo, 16), int(hi, 16)]
    return out


def _reading_seeds(golden, lanes):
    paper = _printed_seeds(golden)
    extra = [(splitmix64(16, i) & M32) | 1 for i in range(8)]
    return (paper + extra)[:lanes] if lanes > 8 else paper[:lanes]


@pytest.mark.parametrize("lanes", [4, 8, 16])
def test_variant_seeds_follow_the_readings(golden, lanes):
    s = [int(v) for v in oracle.variant_seeds(lanes)]
    assert s == _reading_seeds(golden, lanes)
    assert all(v & 1 for v in s)
    assert len(set(s)) == lanes


def test_variant_lanes_rejected():
    for bad in (0, 1, 2, 3, 5, 7, 12, 32):
        with pytest.raises(ValueError):
            oracle.variant_seeds(bad)


def test_variant_masks_extend_the_method():
    # Four lanes: the first half of the method's mask; sixteen: the method's
    # mask followed by eight more words.
    for x in splitmix64_stream(60, 2000).tolist():
        x &= M32
        m8 = oracle.mask(x)
        assert np.array_equal(oracle.variant_mask(4, x), m8[:4])
        m16 = oracle.variant_mask(16, x)
        assert np.array_equal(m16[:8], m8)
        assert all(bin(int(w)).count("1") == 1 for w in m16)


def test_variant_eight_lanes_is_the_method():
    B = 1000
    h = splitmix64_stream(61, 20000)
    w8 = oracle.build_filter(B, h)
    wv = oracle.variant_build_filter(8, B, h)
    assert np.array_equal(w8, wv)
    probes = splitmix64_stream(62, 20000)
    assert np.array_equal(oracle.lookup(w8, B, probes), oracle.variant_lookup(wv, 8, B, probes))


def _bigint_filter(seeds, B, hashes):
    K = len(seeds)
    bits = 0
    for h in hashes:
        b = ((h >> 32) * B) >> 32
        x = h & M32
        for j in range(K):
            bits |= 1 << (K * 32 * b + 32 * j + (((seeds[j] * x) & M32) >> 27))
    return bits


def _bigint_contains(bits, seeds, B, h):
    K = len(seeds)
    b = ((h >> 32) * B) >> 32
    x = h & M32
    return all((bits >> (K * 32 * b + 32 * j + (((seeds[j] * x) & M32) >> 27))) & 1 for j in range(K))


@pytest.mark.parametrize("lanes", [4, 16])
@pytest.mark.parametrize("B", [1, 2, 3, 7])
def test_variant_brute_force_tiny(golden, lanes, B):
    seeds = _reading_seeds(golden, lanes)
    hs = splitmix64_stream(70 + B, 48).tolist()
    words = oracle.variant_build_filter(lanes, B, np.array(hs, dtype=np.uint64))
    as_int = int.from_bytes(words.astype("<u4").tobytes(), "little")
    assert as_int == _bigint_filter(seeds, B, hs)
    probes = hs + splitmix64_stream(80 + B, 200).tolist()
    got = oracle.variant_lookup(words, lanes, B, np.array(probes, dtype=np.uint64))
    assert [bool(v) for v in got] == [_bigint_contains(as_int, seeds, B, p) for p in probes]


hash_lists = st.lists(st.integers(min_value=0, max_value=(1 << 64) - 1), min_size=0, max_size=150)


@settings(max_examples=40, deadline=None)
@given(hs=hash_lists, B=st.integers(min_value=1, max_value=40), lanes=st.sampled_from([4, 16]),
       seed=st.integers(0, 1000))
def test_variant_or_algebra(hs, B, lanes, seed):
    h = np.array(hs, dtype=np.uint64)
    base = oracle.variant_build_filter(lanes, B, h)
    assert oracle.variant_lookup(base, lanes, B, h).all()  # no false negatives
    perm = h[np.random.default_rng(seed).permutation(h.size)] if h.size else h
    assert np.array_equal(oracle.variant_build_filter(lanes, B, perm), base)
    assert np.array_equal(oracle.variant_build_filter(lanes, B, np.concatenate([h, h])), base)
    cut = h.size // 2
    union = oracle.variant_build_filter(lanes, B, h[:cut]) | oracle.variant_build_filter(lanes, B, h[cut:])
    assert np.array_equal(union, base)


@settings(max_examples=40, deadline=None)
@given(h=st.integers(min_value=0, max_value=(1 << 64) - 1), B=st.integers(min_value=1, max_value=1 << 16),
       lanes=st.sampled_from([4, 16]))
def test_variant_single_insert_one_bit_per_word(h, B, lanes):
    words = oracle.variant_build_filter(lanes, B, np.array([h], dtype=np.uint64))
    b = oracle.block(h, B)
    blk = words[lanes * b: lanes * b + lanes]
    assert all(bin(int(w)).count("1") == 1 for w in blk)
    assert oracle.popcount(words) == lanes


def test_variant_all_ones_and_empty():
    B = 13
    probes = splitmix64_stream(90, 500)
    for lanes in (4, 16):
        assert oracle.variant_lookup(np.full(lanes * B, M32, dtype=np.uint32), lanes, B, probes).all()
        assert not oracle.variant_lookup(oracle.variant_new_filter(lanes, B), lanes, B, probes).any()


def test_variant_extra_seed_cosets_are_permutations():
    # For an odd seed s, x -> s x mod 2^32 is a bijection, and on the coset
    # x = c + 2^27 t (t = 0..31) the top five bits of s x step through all 32
    # values: each word's index is a permutation of [0, 32) there. A seed
    # made even, or a product not reduced mod 2^32, breaks it.
    for j in range(16):
        for c in (0, 1, 12345, (1 << 27) - 1):
            words = [oracle.variant_mask(16, (c + (t << 27)) & M32)[j] for t in range(32)]
            idx = sorted(int(w).bit_length() - 1 for w in words)
            assert idx == list(range(32))


def test_variant_fpr_formula_k8_is_the_method():
    for a in (1.0, 10.0, 24.38, 52.0):
        assert fpr.sbbf_fpr(a, 8) == fpr.sbbf_fpr(a)


def test_variant_fpr_formula_small_load_limit():
    # With a -> 0 a block holds one or two keys or none: a probe is a false
    # positive when its block holds one key and every word agrees (chance
    # (1/32)^K), or two keys and every word matches one of them (chance
    # (1 - (31/32)^2)^K); three keys weigh a^2 3^K / 6 relative, negligible.
    for lanes in (4, 8, 16):
        a = 1e-8
        two = a * math.exp(-a) * (1 / 32) ** lanes + a * a / 2 * math.exp(-a) * (63 / 1024) ** lanes
        assert math.isclose(fpr.sbbf_fpr(a, lanes), two, rel_tol=1e-6)


@pytest.mark.parametrize("lanes,B,n", [(4, 65536, 800_000), (16, 16384, 800_000)])
def test_variant_measured_fpr_matches_formula(lanes, B, n):
    # Filters at the paper's 10.5-bit-per-key geometry scaled to K words per
    # block (a = 32 K / 10.5 keys per block), probed with fresh hashes.
    h = splitmix64_stream(91, n)
    words = oracle.variant_build_filter(lanes, B, h)
    probes = splitmix64_stream(92, 2_000_000)
    rate = float(oracle.variant_lookup(words, lanes, B, probes).mean())
    model = fpr.sbbf_fpr(n / B, lanes)
    sigma = math.sqrt(model * (1 - model) / probes.size)
    assert abs(rate - model) <= max(4 * sigma, 0.03 * model), (rate, model)
    # The per-filter predictor: mean over blocks of the product of the
    # words' fill fractions.
    pc = np.unpackbits(words.view(np.uint8)).reshape(B, lanes, 32).sum(axis=2) / 32.0
    pred = float(np.prod(pc, axis=1).mean())
    assert abs(rate - pred) <= 4 * sigma + 0.005 * pred, (rate, pred)
