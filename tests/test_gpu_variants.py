"""Block variants with four and sixteen 32-bit words per block (the paper notes
that four or sixteen lanes would work as well as eight): every insert and
lookup strategy against the oracle's variant functions, at small ragged sizes,
edge cases and a 128 MiB filter, plus select, keys, union and serialization."""

import struct

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from synth import splitmix64_stream  # noqa: E402

pytestmark = pytest.mark.gpu

INSERTS = {"auto": None, "atomic32": dict(strategy=1), "atomic64": dict(strategy=2), "lds": dict(strategy=3),
           "partitioned": dict(strategy=4)}
LOOKUPS = {"auto": None, "gather": dict(strategy=1), "partitioned": dict(strategy=2)}


@pytest.fixture(scope="module")
def P():
    import paper_2101_01719_amd as P

    return P


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to("cuda")


def host_words(f):
    torch.cuda.synchronize()
    return f.words.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("lanes", [4, 16])
@pytest.mark.parametrize("ins", list(INSERTS))
@pytest.mark.parametrize("look", list(LOOKUPS))
def test_variant_matches_oracle(P, lanes, ins, look):
    # LDS inserts need the whole filter in one workgroup's LDS.
    B = (1000 if lanes == 16 else 2000) if ins == "lds" else 3001
    h = splitmix64_stream(1100 + lanes, 7_777)
    probes = np.concatenate([h[::5], splitmix64_stream(1200 + lanes, 20_001)])
    ref = oracle.variant_build_filter(lanes, B, h)
    want = oracle.variant_lookup(ref, lanes, B, probes)
    f = P.Filter(B, lanes=lanes)
    f.insert(dev(h), launch=INSERTS[ins])
    assert np.array_equal(host_words(f), ref)
    got = f.lookup(dev(probes), launch=LOOKUPS[look]).cpu().numpy()
    assert np.array_equal(got, want)
    bits = f.lookup_bits(dev(probes), launch=LOOKUPS[look]).cpu().numpy().view(np.uint32)
    assert np.array_equal(bits, _pack(want))
    f.close()


def _pack(r):
    out = np.zeros((r.size + 31) // 32, dtype=np.uint32)
    idx = np.flatnonzero(r)
    np.bitwise_or.at(out, idx // 32, (np.uint32(1) << (idx % 32).astype(np.uint32)))
    return out


@pytest.mark.parametrize("lanes", [4, 16])
@pytest.mark.parametrize("B,n", [(1, 1), (1, 1000), (2, 65), (63, 0), (65, 63), (4097, 129), (70_001, 300_001)])
def test_variant_edge_sizes(P, lanes, B, n):
    h = splitmix64_stream(1300 + B + lanes, n)
    probes = np.concatenate([h, splitmix64_stream(1400 + B, 517)])
    ref = oracle.variant_build_filter(lanes, B, h)
    want = oracle.variant_lookup(ref, lanes, B, probes)
    for ins in ("atomic32", "partitioned"):
        f = P.Filter(B, lanes=lanes)
        if n:
            f.insert(dev(h), launch=INSERTS[ins])
        assert np.array_equal(host_words(f), ref), ins
        for look in ("gather", "partitioned"):
            assert np.array_equal(f.lookup(dev(probes), launch=LOOKUPS[look]).cpu().numpy(), want), (ins, look)
        f.close()


@pytest.mark.parametrize("lanes", [4, 16])
def test_variant_128mib_filter(P, lanes):
    """A 128 MiB filter (the size of the 100M-key workload's filter): the
    partitioned insert and lookup (what the library picks for large batches)
    against the oracle everywhere, and against the atomic insert and the
    gather lookup."""
    B = (128 << 20) // (4 * lanes)
    n = 8_000_000
    h = splitmix64_stream(1500, n)
    probes = np.concatenate([h[: n // 10], splitmix64_stream(1501, 3 * n)])
    rng = np.random.default_rng(lanes)
    probes = probes[rng.permutation(probes.size)]
    ref = oracle.variant_build_filter(lanes, B, h)
    want = oracle.variant_lookup(ref, lanes, B, probes)
    f = P.Filter(B, lanes=lanes)
    # batches of the 100M-key workload's size pick the partitioned paths
    assert P.sbbf_auto_insert_strategy(f.handle, 100_000_000) == 4
    assert P.sbbf_auto_lookup_strategy(f.handle, 200_000_000) == 2
    dh, dp = dev(h), dev(probes)
    f.insert(dh, launch=INSERTS["partitioned"])
    assert np.array_equal(host_words(f), ref)
    assert np.array_equal(f.lookup(dp, launch=LOOKUPS["partitioned"]).cpu().numpy(), want)
    assert np.array_equal(f.lookup(dp, launch=LOOKUPS["gather"]).cpu().numpy(), want)
    g = P.Filter(B, lanes=lanes)
    g.insert(dh, launch=INSERTS["atomic32"])
    torch.cuda.synchronize()
    assert torch.equal(f.words, g.words)
    f.close()
    g.close()


@pytest.mark.parametrize("lanes", [4, 16])
def test_variant_select_and_keys(P, lanes):
    B = 50_000
    h = splitmix64_stream(1600 + lanes, 400_000)
    probes = np.concatenate([h[::3], splitmix64_stream(1700, 900_001)])
    f = P.Filter(B, lanes=lanes)
    f.insert(dev(h))
    ref = oracle.variant_build_filter(lanes, B, h)
    assert np.array_equal(host_words(f), ref)
    want = np.flatnonzero(oracle.variant_lookup(ref, lanes, B, probes)).astype(np.uint32)
    for look in ("gather", "partitioned"):
        got = f.select(dev(probes), launch=LOOKUPS[look]).cpu().numpy().view(np.uint32)
        assert np.array_equal(got, want), look
    keys = np.arange(123_457, dtype=np.uint64) * np.uint64(7)
    k = P.Filter(B, lanes=lanes)
    k.insert_keys(dev(keys))
    kref = oracle.variant_build_filter(lanes, B, oracle.key_hash(keys))
    assert np.array_equal(host_words(k), kref)
    kp = np.arange(0, 2_000_000, 3, dtype=np.uint64)
    assert np.array_equal(k.lookup_keys(dev(kp)).cpu().numpy(), oracle.variant_lookup(kref, lanes, B, oracle.key_hash(kp)))
    f.close()
    k.close()


@pytest.mark.parametrize("lanes", [4, 16])
def test_variant_union_and_serialization(P, lanes):
    B = 20_011
    a_h, b_h = splitmix64_stream(1800, 100_000), splitmix64_stream(1801, 70_000)
    a, b = P.Filter(B, lanes=lanes), P.Filter(B, lanes=lanes)
    a.insert(dev(a_h))
    b.insert(dev(b_h))
    a.union(b)
    ref = oracle.variant_build_filter(lanes, B, np.concatenate([a_h, b_h]))
    assert np.array_equal(host_words(a), ref)
    blob = a.serialize()
    assert len(blob) == 32 + 4 * lanes * B == P.sbbf_serialized_bytes_variant(B, lanes)
    magic, version, seed_order, nb, word_bytes, hdr_lanes, reserved = struct.unpack("<8sIIIIII", blob[:32])
    assert (magic, version, seed_order, nb, word_bytes, hdr_lanes, reserved) == (b"SBBF256\0", 1, 1, B, 4, lanes, 0)
    assert np.array_equal(np.frombuffer(blob[32:], dtype="<u4"), ref)
    h = P.sbbf_deserialize(blob)
    assert P.sbbf_lanes(h) == lanes and P.sbbf_num_blocks(h) == B
    assert P.sbbf_serialize(h) == blob
    P.sbbf_destroy(h)
    # a size that does not match the header's lanes is refused
    with pytest.raises(P.SbbfError):
        P.sbbf_deserialize(blob[:-4])
    # another lane count does not union
    c = P.Filter(B, lanes=8 if lanes != 8 else 4)
    with pytest.raises(P.SbbfError):
        a.union(c)
    a.close()
    b.close()
    c.close()


def test_variant_eight_is_the_method(P):
    B = 30_000
    h = splitmix64_stream(1900, 500_000)
    v = P.Filter(B, lanes=8)
    m = P.Filter(B)
    v.insert(dev(h), launch=INSERTS["partitioned"])
    m.insert(dev(h), launch=INSERTS["partitioned"])
    torch.cuda.synchronize()
    assert torch.equal(v.words, m.words)
    assert np.array_equal(v.words.cpu().numpy().view(np.uint32), oracle.build_filter(B, h))
    handle = P.sbbf_create_variant(B, 8)
    assert P.sbbf_lanes(handle) == 8
    P.sbbf_destroy(handle)
    v.close()
    m.close()


def test_variant_errors(P):
    for bad in (0, 1, 2, 3, 5, 12, 32):
        with pytest.raises(P.SbbfError):
            P.sbbf_create_variant(100, bad)
    f4 = P.Filter(100, lanes=4)
    f8 = P.Filter(100)
    with pytest.raises(P.SbbfError):
        P.sbbf_grouped_create([f8.handle, f4.handle])
    # the LDS insert of a filter too large for one workgroup's LDS
    big = P.Filter(4096, lanes=16)  # 256 KiB
    with pytest.raises(P.SbbfError):
        big.insert(dev(splitmix64_stream(1, 10)), launch=INSERTS["lds"])
    f4.close()
    f8.close()
    big.close()


@pytest.mark.parametrize("lanes", [4, 16])
def test_variant_partitioned_lookup_overflow(P, lanes):
    """Four- and sixteen-word blocks through the count-free lookup when most
    probes are two repeated members and the rest crowd into one slice: runs
    past their room go to the overflow pass, whose gather tests K words.
    Bytes and bits (bits: the packing of the byte results, LSB first)."""
    B = 4096 * 300 + 1
    h = splitmix64_stream(1950 + lanes, 400_000)
    ref = oracle.variant_build_filter(lanes, B, h)
    f = P.Filter(B, lanes=lanes)
    f.insert(dev(h), launch=INSERTS["partitioned"])
    probes = splitmix64_stream(1960 + lanes, 1_200_001)
    probes[0::3] = h[99]
    span = (4096 << 32) // B  # high halves mapping into the first slice
    probes[1::3] = ((probes[1::3] >> np.uint64(32)) % np.uint64(span) << np.uint64(32)) | \
        (probes[1::3] & np.uint64(0xFFFFFFFF))
    want = oracle.variant_lookup(ref, lanes, B, probes)
    assert want.any() and not want.all()
    dp = dev(probes)
    assert np.array_equal(f.lookup(dp, launch=LOOKUPS["partitioned"]).cpu().numpy(), want)
    bits = f.lookup_bits(dp, launch=LOOKUPS["partitioned"]).cpu().numpy().view(np.uint32)
    packed = np.packbits(want.astype(np.uint8), bitorder="little")
    packed = np.concatenate([packed, np.zeros(-packed.size % 4, np.uint8)]).view(np.uint32)
    assert np.array_equal(bits, packed[: bits.size])
    f.close()
