"""Parity of the HIP path with the CPU oracle for single filters.

Every comparison is exact: filter words byte-for-byte, lookup bytes and packed
lookup bits element-for-element. All calls go through the C ABI (via the
Python binding of the same names).
"""

import hashlib
import re

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from conftest import read_golden  # noqa: E402
from synth import plain_workload, splitmix64_stream  # noqa: E402

pytestmark = pytest.mark.gpu

STRATEGIES = {
    "atomic32": dict(strategy=1),
    "atomic64": dict(strategy=2),
    "lds_owner": dict(strategy=3, grid_blocks=1),
    "lds_merge8": dict(strategy=3, grid_blocks=8),
    "partitioned": dict(strategy=4),
    "auto": dict(strategy=0),
}

LOOKUPS = {
    "gather": dict(strategy=1),
    "partitioned": dict(strategy=2),
    "auto": dict(strategy=0),
}


@pytest.fixture(scope="module")
def P():
    import paper_2101_01719_amd as P

    return P


def dev(a: np.ndarray) -> "torch.Tensor":
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to("cuda")


def words_of(f) -> np.ndarray:
    torch.cuda.synchronize()
    return f.words.cpu().numpy().view(np.uint32)


def sha16(words: np.ndarray) -> str:
    return hashlib.sha256(words.astype("<u4").tobytes()).hexdigest()[:16]


def test_device_and_runtime(P):
    info = P.sbbf_device_query()
    print("device:", info)
    assert info["arch"].startswith("gfx950")
    assert info["compute_units"] > 0 and info["warp_size"] == 64
    assert info["lds_per_block"] >= 65536
    maps = open("/proc/self/maps").read()
    assert len(set(re.findall(r"\S*libamdhip64\S*", maps))) == 1


@pytest.mark.parametrize("B", [1, 2, 3, 5, 8, 13])
@pytest.mark.parametrize("strategy", sorted(STRATEGIES))
def test_tiny_filters(P, B, strategy):
    h = splitmix64_stream(100 + B, 64)
    probes = np.concatenate([h, splitmix64_stream(200 + B, 300)])
    f = P.Filter(B)
    f.insert(dev(h), launch=STRATEGIES[strategy])
    got = f.lookup(dev(probes)).cpu().numpy()
    ref = oracle.build_filter(B, h)
    assert np.array_equal(words_of(f), ref)
    assert np.array_equal(got, oracle.lookup(ref, B, probes))


RAGGED = [1, 2, 7, 8, 9, 63, 64, 65, 127, 128, 129, 255, 257, 511, 513, 1000, 4095, 4097, 65537]


@pytest.mark.parametrize("n", RAGGED)
def test_ragged_counts(P, n):
    B = 37
    h = splitmix64_stream(300, n)
    probes = splitmix64_stream(301, n + 77)
    probes[: n // 2] = h[: n // 2]
    ref = oracle.build_filter(B, h)
    ref_look = oracle.lookup(ref, B, probes)
    ref_bits = oracle.lookup_bits(ref, B, probes)
    for name, launch in STRATEGIES.items():
        f = P.Filter(B)
        f.insert(dev(h), launch=launch)
        assert np.array_equal(words_of(f), ref), name
        for unroll in (1, 2, 4):
            got = f.lookup(dev(probes), launch=dict(unroll=unroll)).cpu().numpy()
            assert np.array_equal(got, ref_look), (name, unroll)
            bits = f.lookup_bits(dev(probes), launch=dict(unroll=unroll)).cpu().numpy().view(np.uint32)
            assert np.array_equal(bits, ref_bits), (name, unroll)
        got = f.lookup(dev(probes), launch=LOOKUPS["partitioned"]).cpu().numpy()
        assert np.array_equal(got, ref_look), (name, "partitioned lookup")
        bits = f.lookup_bits(dev(probes), launch=LOOKUPS["partitioned"]).cpu().numpy().view(np.uint32)
        assert np.array_equal(bits, ref_bits), (name, "partitioned lookup bits")
        f.close()


@pytest.mark.parametrize("threads", [64, 128, 256, 512, 1024])
@pytest.mark.parametrize("unroll", [1, 2, 4, 8])
def test_launch_shapes_insert(P, threads, unroll):
    B = 1000
    h = splitmix64_stream(400, 50_001)
    ref = oracle.build_filter(B, h)
    for strat in (1, 2):
        for grid in (0, 1, 3):
            f = P.Filter(B)
            f.insert(dev(h), launch=dict(block_threads=threads, unroll=unroll, strategy=strat, grid_blocks=grid))
            assert np.array_equal(words_of(f), ref), (strat, grid)
            f.close()


@pytest.mark.parametrize("threads", [64, 256, 1024])
@pytest.mark.parametrize("unroll", [1, 2, 4])
def test_launch_shapes_lookup(P, threads, unroll):
    B = 1000
    h = splitmix64_stream(401, 30_000)
    probes = np.concatenate([h[:10_000], splitmix64_stream(402, 40_003)])
    ref = oracle.build_filter(B, h)
    ref_look = oracle.lookup(ref, B, probes)
    f = P.Filter(B)
    f.insert(dev(h))
    for grid in (0, 1, 5):
        got = f.lookup(dev(probes), launch=dict(block_threads=threads, unroll=unroll, grid_blocks=grid)).cpu().numpy()
        assert np.array_equal(got, ref_look), grid


def _paper_row(name):
    return [r for r in read_golden("paper_code_configs.txt") if r[0] == name][0]


@pytest.mark.parametrize("name", ["plain_100k", "plain_1m"])
@pytest.mark.parametrize("strategy", sorted(STRATEGIES))
def test_plain_workloads(P, name, strategy):
    w = plain_workload(name)
    launch = STRATEGIES[strategy]
    if strategy.startswith("lds") and w.num_blocks * 32 > P.sbbf_device_query()["lds_per_block"]:
        pytest.skip("filter larger than one workgroup's LDS")
    f = P.Filter(w.num_blocks)
    f.insert(dev(w.inserts), launch=launch)
    look = dev(w.lookups)
    got = f.lookup(look).cpu().numpy()
    bits = f.lookup_bits(look).cpu().numpy().view(np.uint32)
    for lname, llaunch in LOOKUPS.items():
        assert np.array_equal(f.lookup(look, launch=llaunch).cpu().numpy(), got), lname
        assert np.array_equal(f.lookup_bits(look, launch=llaunch).cpu().numpy().view(np.uint32), bits), lname
    words = words_of(f)
    ref = oracle.build_filter(w.num_blocks, w.inserts)
    assert np.array_equal(words, ref)
    assert sha16(words) == _paper_row(name)[6]
    ref_look = oracle.lookup(ref, w.num_blocks, w.lookups)
    assert np.array_equal(got, ref_look)
    assert np.array_equal(bits, oracle.lookup_bits(ref, w.num_blocks, w.lookups))
    assert int(got[~w.is_member].sum()) == int(_paper_row(name)[5])


def test_insert_accumulates_into_existing_filter(P):
    B = 2000
    a = splitmix64_stream(500, 20_000)
    b = splitmix64_stream(501, 30_000)
    ref = oracle.build_filter(B, np.concatenate([a, b]))
    for name, launch in STRATEGIES.items():
        f = P.Filter(B)
        f.insert(dev(a), launch=STRATEGIES["atomic32"])
        f.insert(dev(b), launch=launch)
        assert np.array_equal(words_of(f), ref), name
        f.clear()
        assert not words_of(f).any()


def test_library_owned_filter_roundtrip(P):
    B = 777
    h = splitmix64_stream(510, 9000)
    ref = oracle.build_filter(B, h)
    fh = P.sbbf_create(B)
    try:
        P.sbbf_insert_batch(fh, dev(h))
        host = torch.empty(8 * B, dtype=torch.int32)
        P.sbbf_copy_words_to_host(fh, host)
        torch.cuda.synchronize()
        assert np.array_equal(host.numpy().view(np.uint32), ref)
        # restore a checkpoint into a fresh filter and keep using it
        g = P.sbbf_create(B)
        P.sbbf_copy_words_from_host(g, host)
        more = splitmix64_stream(511, 5000)
        P.sbbf_insert_batch(g, dev(more))
        out = torch.empty(8 * B, dtype=torch.int32)
        P.sbbf_copy_words_to_host(g, out)
        torch.cuda.synchronize()
        assert np.array_equal(out.numpy().view(np.uint32), oracle.insert(ref.copy(), B, more))
        P.sbbf_destroy(g)
    finally:
        P.sbbf_destroy(fh)


def test_empty_batches_and_errors(P):
    f = P.Filter(64)
    empty = torch.empty(0, dtype=torch.int64, device="cuda")
    f.insert(empty)
    assert f.lookup(empty).numel() == 0
    assert not words_of(f).any()
    # LDS strategy on a filter larger than one workgroup's LDS is refused
    lds = P.sbbf_device_query()["lds_per_block"]
    big = P.Filter(lds // 32 + 1)
    with pytest.raises(P.SbbfError) as e:
        big.insert(dev(splitmix64_stream(1, 10)), launch=dict(strategy=3))
    assert e.value.status == P.SBBF_EUNSUPPORTED
    with pytest.raises(P.SbbfError) as e:
        f.insert(dev(splitmix64_stream(1, 10)), launch=dict(block_threads=96))
    assert e.value.status == P.SBBF_EINVAL
    with pytest.raises(P.SbbfError):
        f.lookup(dev(splitmix64_stream(1, 10)), launch=dict(unroll=8))
    # misaligned hash pointer
    import ctypes

    h = dev(splitmix64_stream(1, 16))
    st = P._L().sbbf_insert_batch(f.handle, ctypes.c_void_p(h.data_ptr() + 4), 4, None)
    assert st == P.SBBF_EINVAL
    assert not words_of(f).any()


@pytest.mark.parametrize("B", [1, 63, 4096, 4097, 8191, 12288 + 5, 1 << 20, (1 << 20) + 3])
def test_partitioned_slice_edges(P, B):
    """Filters of one slice, exactly one slice, one block over, several slices
    with a short last slice, and many slices."""
    h = splitmix64_stream(540 + B % 97, max(3 * B, 10_000) if B < (1 << 20) else 2_500_000)
    ref = oracle.build_filter(B, h)
    f = P.Filter(B)
    f.insert(dev(h[: h.size // 3]), launch=dict(strategy=1))  # start from a non-empty filter
    f.insert(dev(h[h.size // 3:]), launch=dict(strategy=4))
    assert np.array_equal(words_of(f), ref)
    probes = np.concatenate([h[::7], splitmix64_stream(600 + B % 89, 3 * B + 1001)])
    want = oracle.lookup(ref, B, probes)
    got = f.lookup(dev(probes), launch=LOOKUPS["partitioned"]).cpu().numpy()
    assert np.array_equal(got, want)
    bits = f.lookup_bits(dev(probes), launch=LOOKUPS["partitioned"]).cpu().numpy().view(np.uint32)
    assert np.array_equal(bits, oracle.lookup_bits(ref, B, probes))


def test_partitioned_two_levels_minimal(P):
    """One block over 4,096 slices of 4,096 blocks: the two-level partition
    with a second group of one slice holding one block."""
    B = 4096 * 4096 + 1
    h = splitmix64_stream(570, 3_000_000)
    h[:5] = np.array([(1 << 64) - 1, 0xFFFFFFFF00000000, 0xFFFFFFFF12345678, 0, 1 << 63], dtype=np.uint64)
    ref = oracle.build_filter(B, h)
    f = P.Filter(B)
    f.insert(dev(h), launch=dict(strategy=4))
    assert np.array_equal(words_of(f), ref)
    probes = np.concatenate([h[::3], splitmix64_stream(571, 2_000_003)])
    want = oracle.lookup(ref, B, probes)
    assert np.array_equal(f.lookup(dev(probes), launch=LOOKUPS["partitioned"]).cpu().numpy(), want)
    bits = f.lookup_bits(dev(probes), launch=LOOKUPS["partitioned"]).cpu().numpy().view(np.uint32)
    assert np.array_equal(bits, oracle.lookup_bits(ref, B, probes))
    f.close()


def test_partitioned_two_levels_large(P):
    """A 1.5 GiB filter (12,289 slices: four groups, a short last one): the
    two-level insert and lookup, from hashes and from keys, against the
    oracle; the library picks the partitioned paths for batches this size."""
    B = 3 * (1 << 24) + 12_345
    free, _ = torch.cuda.mem_get_info()
    if free < 8 * 32 * B:
        pytest.skip("not enough device memory")
    h = splitmix64_stream(572, 20_000_000)
    ref = oracle.build_filter(B, h)
    f = P.Filter(B)
    f.insert(dev(h[:1_000_000]), launch=dict(strategy=1))  # start from a non-empty filter
    f.insert(dev(h[1_000_000:]), launch=dict(strategy=4))
    assert np.array_equal(words_of(f), ref)
    probes = np.concatenate([h[::9], splitmix64_stream(573, 18_000_000)])
    probes = probes[np.random.default_rng(5).permutation(probes.size)]
    want = oracle.lookup(ref, B, probes)
    assert np.array_equal(f.lookup(dev(probes), launch=LOOKUPS["partitioned"]).cpu().numpy(), want)
    assert np.array_equal(f.lookup(dev(probes), launch=LOOKUPS["gather"]).cpu().numpy(), want)
    keys = np.arange(5_000_000, dtype=np.uint64) * np.uint64(3)
    g = P.Filter(B)
    g.insert_keys(dev(keys), launch=dict(strategy=4))
    kref = oracle.build_filter(B, oracle.key_hash(keys))
    assert np.array_equal(words_of(g), kref)
    kp = np.arange(0, 6_000_000, dtype=np.uint64)
    got = g.lookup_keys(dev(kp), launch=LOOKUPS["partitioned"]).cpu().numpy()
    assert np.array_equal(got, oracle.lookup(kref, B, oracle.key_hash(kp)))
    f.close()
    g.close()


def test_all_ones_filter_reports_every_probe(P):
    B = 321
    f = P.Filter(B)
    f.words.fill_(-1)
    probes = dev(splitmix64_stream(520, 10_000))
    assert bool(f.lookup(probes).all())
    f.clear()
    assert not bool(f.lookup(probes).any())


def test_largest_block_count(P):
    """num_blocks = 2**32 - 1 (128 GiB of words): block offsets need 64-bit
    addressing. Checked sparsely: every block a key selects holds exactly the
    oracle's bits, and the total set-bit count matches."""
    B = (1 << 32) - 1
    free, _ = torch.cuda.mem_get_info()
    if free < 32 * B + (8 << 30):
        pytest.skip("not enough device memory for a 128 GiB filter")
    h = np.concatenate([splitmix64_stream(530, 4000), np.array([0, (1 << 64) - 1, 0xFFFFFFFF00000000], np.uint64)])
    f = P.Filter(B)
    f.insert(dev(h))
    torch.cuda.synchronize()
    blocks = np.array([oracle.block(int(x), B) for x in h.tolist()], dtype=np.int64)
    got = f.words.view(-1, 8).index_select(0, torch.from_numpy(blocks).to("cuda")).cpu().numpy().view(np.uint32)
    # oracle on a compacted filter holding only the touched blocks
    uniq, inv = np.unique(blocks, return_inverse=True)
    want = np.zeros((uniq.size, 8), dtype=np.uint32)
    for k, x in enumerate(h.tolist()):
        want[inv[k]] |= oracle.mask(x & 0xFFFFFFFF)
    assert np.array_equal(got, want[inv])
    look = f.lookup(dev(h)).cpu().numpy()
    assert look.all()
    f.close()
    del f
    torch.cuda.empty_cache()


@pytest.mark.parametrize("strategy", ["atomic32", "atomic64", "partitioned"])
def test_plain_100m_full(P, strategy):
    """The 100M-key workload at full size in the launch shape the benchmark
    times (library defaults): the whole filter and all 2e8 lookups are
    compared with the oracle."""
    w = plain_workload("plain_100m", backend="torch", device="cuda")
    f = P.Filter(w.num_blocks)
    f.insert(w.inserts, launch=STRATEGIES[strategy])
    got = {name: f.lookup(w.lookups, launch=launch).cpu().numpy() for name, launch in LOOKUPS.items()}
    torch.cuda.synchronize()
    words = words_of(f)
    assert sha16(words) == _paper_row("plain_100m")[6]
    ins = w.inserts.cpu().numpy().view(np.uint64)
    ref = oracle.build_filter(w.num_blocks, ins)
    assert np.array_equal(words, ref)
    look = w.lookups.cpu().numpy().view(np.uint64)
    ref_look = oracle.lookup(ref, w.num_blocks, look)
    for name, g in got.items():
        assert np.array_equal(g, ref_look), name


@pytest.mark.parametrize("B", [4096 * 2048 + 5, 4096 * 4096])
def test_partitioned_many_slices(P, B):
    """Filters above 128 MiB: 2,049 slices of 4,096 blocks (two slices per
    scatter thread, a five-block last slice) and the limit of 4,096 slices
    (512 MiB, four per thread). Whole filter and every lookup against the
    oracle, for the partitioned insert and lookup."""
    h = splitmix64_stream(560 + B % 7, 6_000_000)
    ref = oracle.build_filter(B, h)
    f = P.Filter(B)
    f.insert(dev(h), launch=dict(strategy=4))
    assert np.array_equal(words_of(f), ref)
    probes = np.concatenate([h[::5], splitmix64_stream(561, 5_000_001)])
    want = oracle.lookup(ref, B, probes)
    got = f.lookup(dev(probes), launch=LOOKUPS["partitioned"]).cpu().numpy()
    assert np.array_equal(got, want)
    f.close()


def test_partitioned_two_slices_per_thread(P):
    """1,537 slices (a 192 MiB filter with a seven-block last slice): two
    slices per scatter thread with carried four-key groups."""
    B = 4096 * 1536 + 7
    h = splitmix64_stream(575, 9_000_000)
    ref = oracle.build_filter(B, h)
    f = P.Filter(B)
    f.insert(dev(h[:2_000_000]), launch=dict(strategy=4))
    f.insert(dev(h[2_000_000:]), launch=dict(strategy=4))
    assert np.array_equal(words_of(f), ref)
    probes = np.concatenate([h[::4], splitmix64_stream(576, 7_000_001)])
    want = oracle.lookup(ref, B, probes)
    assert np.array_equal(f.lookup(dev(probes), launch=LOOKUPS["partitioned"]).cpu().numpy(), want)
    bits = f.lookup_bits(dev(probes), launch=LOOKUPS["partitioned"]).cpu().numpy().view(np.uint32)
    assert np.array_equal(bits, oracle.lookup_bits(ref, B, probes))
    f.close()


def _skewed(seed, n, B, slices_hot, frac_hot):
    """n hashes: a fraction frac_hot with high halves inside the first
    slices_hot slices of 4,096 blocks (so their per-slice runs far exceed an
    even share), the rest uniform."""
    h = splitmix64_stream(seed, n)
    hot = int(n * frac_hot)
    span = (slices_hot * 4096 << 32) // B  # high halves mapping below block slices_hot * 4096
    hi = (h[:hot] >> np.uint64(32)) % np.uint64(max(span, 1))
    h[:hot] = (hi << np.uint64(32)) | (h[:hot] & np.uint64(0xFFFFFFFF))
    return h


@pytest.mark.parametrize("B,slices_hot,frac_hot", [(4096 * 64, 1, 1.0), (4096 * 256 + 9, 3, 0.5),
                                                   (4096 * 1536 + 7, 1, 0.3)])
def test_partitioned_insert_skewed(P, B, slices_hot, frac_hot):
    """Batches whose keys crowd into a few slices: runs longer than a
    partition bucket holds go through the overflow path; the filter must
    still equal the oracle's, inserted into a non-empty filter."""
    h = _skewed(580 + slices_hot, 3_000_000, B, slices_hot, frac_hot)
    pre = splitmix64_stream(581, 50_000)
    ref = oracle.build_filter(B, np.concatenate([pre, h]))
    f = P.Filter(B)
    f.insert(dev(pre), launch=dict(strategy=1))
    f.insert(dev(h), launch=dict(strategy=4))
    assert np.array_equal(words_of(f), ref)
    f.close()


def test_partitioned_insert_repeated_hash(P):
    """Half the batch is one hash repeated: one bucket per partition
    workgroup overflows, everything else is spread evenly."""
    B = 4096 * 128
    h = splitmix64_stream(582, 4_000_000)
    h[::2] = np.uint64(0x9E3779B97F4A7C15)
    ref = oracle.build_filter(B, h)
    f = P.Filter(B)
    f.insert(dev(h), launch=dict(strategy=4))
    assert np.array_equal(words_of(f), ref)
    f.close()


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 8, 9, 15, 17, 63, 7167, 7168, 7169])
def test_partitioned_insert_tiny_batches(P, n):
    """Batches of a few keys over 40 slices: buckets of one to a few keys
    (padded to four with copies of their last key)."""
    B = 4096 * 40 + 3
    h = splitmix64_stream(583 + n, n)
    ref = oracle.build_filter(B, h)
    f = P.Filter(B)
    f.insert(dev(h), launch=dict(strategy=4))
    assert np.array_equal(words_of(f), ref)
    f.close()


@pytest.mark.parametrize("grid", [1, 3, 700, 1500])
def test_partitioned_insert_grid_sizes(P, grid):
    """Partition workgroup counts from one (one bucket per slice holding the
    whole batch's share) to more than a bucketed partition takes (the
    counted partition then)."""
    B = 4096 * 300 + 11
    h = splitmix64_stream(584 + grid, 6_000_000)
    ref = oracle.build_filter(B, h)
    f = P.Filter(B)
    f.insert(dev(h), launch=dict(strategy=4, grid_blocks=grid))
    assert np.array_equal(words_of(f), ref)
    f.close()


@pytest.mark.parametrize("B,slices_hot,frac_hot", [(4096 * 64, 1, 1.0), (4096 * 1024, 2, 0.4),
                                                   (4096 * 1536 + 7, 1, 0.2)])
def test_partitioned_lookup_skewed(P, B, slices_hot, frac_hot):
    """Lookups crowding into a few slices (members among them): a few slice
    runs hold most of the batch, the rest are short or empty; bytes and
    bits both match the oracle."""
    h = _skewed(590 + slices_hot, 400_000, B, slices_hot, frac_hot)
    ref = oracle.build_filter(B, h)
    f = P.Filter(B)
    f.insert(dev(h), launch=dict(strategy=1))
    probes = np.concatenate([_skewed(592 + slices_hot, 2_500_000, B, slices_hot, frac_hot), h[::2]])
    probes = probes[np.random.default_rng(slices_hot).permutation(probes.size)]
    want = oracle.lookup(ref, B, probes)
    assert want.any() and not want.all()
    got = f.lookup(dev(probes), launch=LOOKUPS["partitioned"]).cpu().numpy()
    assert np.array_equal(got, want)
    bits = f.lookup_bits(dev(probes), launch=LOOKUPS["partitioned"]).cpu().numpy().view(np.uint32)
    assert np.array_equal(bits, oracle.lookup_bits(ref, B, probes))
    f.close()


def test_partitioned_lookup_repeated_hash(P):
    """Every third probe is one member hash: one slice run per chunk holds a
    third of the chunk's keys; the rest are spread evenly."""
    B = 4096 * 512
    h = splitmix64_stream(594, 1_000_000)
    ref = oracle.build_filter(B, h)
    f = P.Filter(B)
    f.insert(dev(h), launch=dict(strategy=1))
    probes = splitmix64_stream(595, 3_000_001)
    probes[::3] = h[12345]
    want = oracle.lookup(ref, B, probes)
    got = f.lookup(dev(probes), launch=LOOKUPS["partitioned"]).cpu().numpy()
    assert np.array_equal(got, want)
    bits = f.lookup_bits(dev(probes), launch=LOOKUPS["partitioned"]).cpu().numpy().view(np.uint32)
    assert np.array_equal(bits, oracle.lookup_bits(ref, B, probes))
    f.close()


@pytest.mark.parametrize("n", [1, 3, 4, 5, 255, 256, 257, 43_007, 43_008, 43_009, 1_000_003])
def test_partitioned_lookup_batch_sizes(P, n):
    """Lookup batches from one key to several partition chunks (ragged last
    chunk; bit output words across chunk ends)."""
    B = 4096 * 1000 + 17
    h = splitmix64_stream(596, 500_000)
    ref = oracle.build_filter(B, h)
    f = P.Filter(B)
    f.insert(dev(h), launch=dict(strategy=1))
    probes = np.concatenate([h[: n // 2], splitmix64_stream(597 + n, n - n // 2)])
    want = oracle.lookup(ref, B, probes)
    assert np.array_equal(f.lookup(dev(probes), launch=LOOKUPS["partitioned"]).cpu().numpy(), want)
    bits = f.lookup_bits(dev(probes), launch=LOOKUPS["partitioned"]).cpu().numpy().view(np.uint32)
    assert np.array_equal(bits, oracle.lookup_bits(ref, B, probes))
    f.close()


@pytest.mark.parametrize("grid", [1, 2, 3, 7, 100, 1024])
def test_partitioned_lookup_grid_sizes(P, grid):
    """Lookup partitions over one to 1,024 scatter workgroups: buckets holding
    many chunks, unpermute workgroups splitting a scatter workgroup's chunks
    unevenly, and a last scatter workgroup with fewer chunks than the others;
    bytes and bits."""
    B = 4096 * 300 + 5
    h = splitmix64_stream(598, 300_000)
    ref = oracle.build_filter(B, h)
    f = P.Filter(B)
    f.insert(dev(h), launch=dict(strategy=1))
    probes = np.concatenate([h[::3], splitmix64_stream(599, 500_003)])
    want = oracle.lookup(ref, B, probes)
    launch = dict(strategy=2, grid_blocks=grid)
    assert np.array_equal(f.lookup(dev(probes), launch=launch).cpu().numpy(), want)
    bits = f.lookup_bits(dev(probes), launch=launch).cpu().numpy().view(np.uint32)
    assert np.array_equal(bits, oracle.lookup_bits(ref, B, probes))
    f.close()


def test_partitioned_lookup_past_the_per_call_limit(P):
    """2^31 + 1,000,003 lookups (a call takes at most 2^31 keys: the batch
    runs as one full-size count-free partition, the largest its 32-bit
    positions serve, then a 1M-key one; packed bits split at a word
    boundary). Every sixteenth probe is a member; results are compared with
    the oracle at 2M sampled positions plus both ends and the split, members
    must all be found, and the bit output must pack the byte output."""
    B = 4_194_304
    n_ins = 10_000_000
    n = (1 << 31) + 1_000_003
    ins = splitmix64_stream(601, n_ins)
    ref = oracle.build_filter(B, ins)
    f = P.Filter(B)
    f.insert(dev(ins), launch=dict(strategy=4))
    probes = splitmix64_stream(602, n, backend="torch", device="cuda")
    d_ins = dev(ins)
    members = torch.arange(0, n, 16, device="cuda")
    probes[members] = d_ins[members % n_ins]
    del d_ins
    out = f.lookup(probes, launch=dict(strategy=2))
    assert bool(out[members].all().item())
    rng = np.random.default_rng(603)
    edges = np.concatenate([np.arange(0, 100_000), np.arange((1 << 31) - 100_000, (1 << 31) + 100_000),
                            np.arange(n - 100_000, n)])
    idx = np.unique(np.concatenate([rng.integers(0, n, 2_000_000), edges]))
    d_idx = torch.from_numpy(idx.astype(np.int64)).to("cuda")
    sample = probes[d_idx].cpu().numpy().view(np.uint64)
    want = oracle.lookup(ref, B, sample)
    assert np.array_equal(out[d_idx].cpu().numpy(), want)
    bits = f.lookup_bits(probes, launch=dict(strategy=2))
    del probes
    got_bits = ((bits[d_idx // 32] >> (d_idx % 32).to(torch.int32)) & 1).to(torch.uint8).cpu().numpy()
    assert np.array_equal(got_bits, want)
    f.close()


def test_partitioned_insert_past_the_per_call_limit(P):
    """2^31 + 1,000,003 inserts (the partitioned insert takes at most 2^31
    keys a call: one full-size bucketed partition, then a 1M-key one) give the
    same filter as the 32-bit atomic insert of the same keys, and every
    sixty-fourth key (a sample the oracle also inserts into an empty filter)
    is then found. The atomic insert is compared with the oracle at smaller
    sizes throughout this file."""
    B = 4_194_304
    n = (1 << 31) + 1_000_003
    keys = splitmix64_stream(604, n, backend="torch", device="cuda")
    f, g = P.Filter(B), P.Filter(B)
    f.insert(keys, launch=dict(strategy=4))
    g.insert(keys, launch=dict(strategy=1))
    torch.cuda.synchronize()
    assert torch.equal(f.words, g.words)
    sample = keys[::64].contiguous()
    del keys
    assert bool(f.lookup(sample, launch=dict(strategy=2)).all().item())
    # the oracle's filter of the sample alone is contained in the library's
    ref = oracle.build_filter(B, sample[:2_000_000].cpu().numpy().view(np.uint64))
    words = words_of(f)
    assert np.array_equal(words & ref, ref)
    f.close()
    g.close()
