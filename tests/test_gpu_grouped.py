"""Parity of the grouped launch (many filters, one graph launch) with the CPU
oracle applied filter by filter, and with one plain launch per filter."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from synth import grouped_workload, splitmix64_stream  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2101_01719_amd as P

    return P


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to("cuda")


def make_group(P, w, cfg=None):
    filters = [P.Filter(int(b)) for b in w.blocks]
    return filters, P.Group(filters, w.ins_off, w.look_off, cfg)


def check_against_oracle(w, filters, out, which):
    out = out.cpu().numpy() if hasattr(out, "cpu") else out
    ins = w.inserts if isinstance(w.inserts, np.ndarray) else None
    for f in which:
        B = int(w.blocks[f])
        i0, i1 = int(w.ins_off[f]), int(w.ins_off[f + 1])
        l0, l1 = int(w.look_off[f]), int(w.look_off[f + 1])
        h = ins[i0:i1] if ins is not None else w.inserts[i0:i1].cpu().numpy().view(np.uint64)
        look = (w.lookups[l0:l1] if isinstance(w.lookups, np.ndarray)
                else w.lookups[l0:l1].cpu().numpy().view(np.uint64))
        ref = oracle.build_filter(B, h)
        got_words = filters[f].words.cpu().numpy().view(np.uint32)
        assert np.array_equal(got_words, ref), f"filter {f} words"
        assert np.array_equal(out[l0:l1], oracle.lookup(ref, B, look)), f"filter {f} lookups"


@pytest.fixture(scope="module")
def small():
    return grouped_workload(num_filters=64, log10_min=2.0, log10_max=5.2)


def test_grouped_small_matches_oracle(P, small):
    w = small
    filters, g = make_group(P, w)
    ins, look = dev(w.inserts), dev(w.lookups)
    out = torch.empty(look.numel(), dtype=torch.uint8, device="cuda")
    g.run(ins, look, out)
    torch.cuda.synchronize()
    check_against_oracle(w, filters, out, range(w.num_filters))
    # plain per-filter launches give the same filters and results
    d1 = g.digest(out)
    g.clear()
    out2 = torch.zeros_like(out)
    g.run_per_filter(ins, look, out2)
    torch.cuda.synchronize()
    assert torch.equal(out, out2)
    assert g.digest(out2) == d1
    g.close()


CONFIGS = [
    dict(xcd_queues=0),
    dict(lookup_tile_keys=64, lookup_threads=64, lookup_unroll=1, lookup_blocks_per_cu=1),
    dict(lookup_tile_keys=4096, lookup_unroll=4, lookup_threads=128),
    dict(insert_lds_bytes=2048, insert_slice_shift=6),   # every filter above 2 KiB cut into 64-block slices
    dict(insert_lds_bytes=1 << 16, insert_slice_shift=11),
    dict(lookup_lds_slices=1),                             # filters of one 128 KiB slice from LDS
    dict(lookup_lds_slices=1024),                          # every filter from LDS, slice by slice
    dict(lookup_lds_slices=2, lookup_tile_keys=4096, xcd_queues=0),
    dict(lookup_lds_slices=4, lookup_lds_threads=256),     # slices of 32 KiB
    dict(lookup_lds_slices=1024, lookup_lds_threads=512),  # slices of 64 KiB
]


@pytest.mark.parametrize("cfg", CONFIGS, ids=[str(i) for i in range(len(CONFIGS))])
def test_grouped_configs_identical(P, small, cfg):
    w = small
    filters, g = make_group(P, w, cfg)
    ins, look = dev(w.inserts), dev(w.lookups)
    out = torch.empty(look.numel(), dtype=torch.uint8, device="cuda")
    g.run(ins, look, out)
    torch.cuda.synchronize()
    check_against_oracle(w, filters, out, range(0, w.num_filters, 3))
    g.close()


def test_grouped_phases_and_graph_replays(P, small):
    """The graph is replayed several times with eager work (clears, copies,
    synchronisations) between replays; every replay matches the eager phases."""
    w = small
    filters, g = make_group(P, w)
    ins, look = dev(w.inserts), dev(w.lookups)
    ref_out = torch.empty(look.numel(), dtype=torch.uint8, device="cuda")
    P.sbbf_grouped_insert(g.handle, ins)
    P.sbbf_grouped_lookup(g.handle, look, ref_out)
    ref_digest = g.digest(ref_out)
    check_against_oracle(w, filters, ref_out, range(0, w.num_filters, 5))
    for k in range(4):
        g.clear()
        out = torch.full_like(ref_out, 7)
        junk = torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        g.run(ins, look, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref_out), k
        assert g.digest(out) == ref_digest, k
        del junk
    # new buffers: the graph's kernel arguments are updated
    ins2, look2 = ins.clone(), look.clone()
    out2 = torch.empty_like(ref_out)
    g.clear()
    g.run(ins2, look2, out2)
    torch.cuda.synchronize()
    assert torch.equal(out2, ref_out)
    g.close()


def test_grouped_autotune(P, small, tmp_path):
    w = small
    filters, g = make_group(P, w)
    ins, look = dev(w.inserts), dev(w.lookups)
    out = torch.empty(look.numel(), dtype=torch.uint8, device="cuda")
    before = g.digest()
    cache = str(tmp_path / "tune.txt")
    best = g.autotune(ins, look, out, reps=2, cache_path=cache)
    assert g.digest() == before  # tuning leaves the filters as they were
    assert g.config() == best
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and lines[0].startswith("gfx950")
    again = g.autotune(ins, look, out, reps=2, cache_path=cache)  # served from the cache
    assert again == best
    assert len(open(cache).read().strip().splitlines()) == 1
    g.run(ins, look, out)
    torch.cuda.synchronize()
    check_against_oracle(w, filters, out, range(0, w.num_filters, 4))
    g.close()


EDGE_CONFIGS = [
    None,
    # 64-block slices: the 9,000-block filter is partitioned into 141 slices,
    # the 70,000-block one has 1,094 slices (more than one partition chunk can
    # sort) and is inserted by stream tiles
    dict(insert_lds_bytes=2048, insert_slice_shift=6),
]


@pytest.mark.parametrize("cfg", EDGE_CONFIGS, ids=["default", "small-slices"])
def test_grouped_edge_cases(P, cfg):
    # empty filters (no inserts, no lookups), a single huge-but-sparse filter,
    # and filters whose counts are not multiples of anything
    blocks = np.array([1, 5000, 9000, 3, 70000], dtype=np.int64)
    n_ins = np.array([0, 7, 100_001, 0, 5], dtype=np.int64)
    n_look = np.array([0, 0, 33, 9, 65_537], dtype=np.int64)
    ins_off = np.concatenate([[0], np.cumsum(n_ins)])
    look_off = np.concatenate([[0], np.cumsum(n_look)])
    ins = splitmix64_stream(700, int(ins_off[-1]))
    look = splitmix64_stream(701, int(look_off[-1]))
    look[:3] = ins[:3]
    filters = [P.Filter(int(b)) for b in blocks]
    g = P.Group(filters, ins_off, look_off, cfg)
    out = torch.empty(int(look_off[-1]), dtype=torch.uint8, device="cuda")
    g.run(dev(ins), dev(look), out)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    for f, B in enumerate(blocks.tolist()):
        ref = oracle.build_filter(B, ins[ins_off[f]:ins_off[f + 1]])
        assert np.array_equal(filters[f].words.cpu().numpy().view(np.uint32), ref)
        assert np.array_equal(res[look_off[f]:look_off[f + 1]], oracle.lookup(ref, B, look[look_off[f]:look_off[f + 1]]))
    with pytest.raises(P.SbbfError):
        P.sbbf_grouped_plan(g.handle, ins_off[::-1].copy(), look_off)  # decreasing offsets
    g.close()


def _golden_digest(name):
    from conftest import read_golden

    rows = {r[0]: r for r in read_golden("full_digests.txt")}
    return rows[name][1], int(rows[name][2]), int(rows[name][3])


def _sha256_filters(filters):
    import hashlib

    h = hashlib.sha256()
    for f in filters:
        h.update(f.words.cpu().numpy().tobytes())
    return h.hexdigest()


def _sha256_bytes(t):
    import hashlib

    return hashlib.sha256(t.cpu().numpy().tobytes()).hexdigest()


def test_grouped_full_workload(P):
    """The 2,048-filter workload (key counts log-uniform in [1e3, 1e6], 10.5
    bits per key, four lookups per inserted key) in the launch shape the
    benchmark times: every filter's bytes and every lookup byte equal the
    oracle's (SHA-256 of both against digests the oracle wrote,
    tests/golden/full_digests.txt), a sample of filters equals the oracle
    directly, and the per-filter plain launches give the same outputs."""
    w = grouped_workload(num_filters=2048, backend="torch", device="cuda")
    filters, g = make_group(P, w)
    out = torch.empty(w.lookups.numel(), dtype=torch.uint8, device="cuda")
    g.run(w.inserts, w.lookups, out)
    torch.cuda.synchronize()
    sha_f, nbytes_f, _ = _golden_digest("grouped_2048_filters")
    sha_l, nbytes_l, positives = _golden_digest("grouped_2048_lookups")
    assert sum(f.words.numel() * 4 for f in filters) == nbytes_f and out.numel() == nbytes_l
    assert int(out.sum(dtype=torch.int64).item()) == positives
    assert _sha256_filters(filters) == sha_f
    assert _sha256_bytes(out) == sha_l
    digest = g.digest(out)
    order = np.argsort(w.n)
    rng = np.random.default_rng(7)
    sample = sorted(set(order[:2].tolist() + order[-2:].tolist() + rng.choice(2048, 16, replace=False).tolist()))
    check_against_oracle(w, filters, out, sample)
    g.clear()
    out2 = torch.empty_like(out)
    g.run_per_filter(w.inserts, w.lookups, out2)
    torch.cuda.synchronize()
    assert torch.equal(out, out2)
    assert g.digest(out2) == digest
    g.close()


def test_grouped_many_runs_per_slice(P):
    """A partitioned filter with more insert chunks than one batch of runs a
    slice tile stages at a time (7,400,000 keys: 1,033 chunks of 7,168, so
    every slice has more than 1,024 runs), next to a small filter."""
    blocks = np.array([300_000, 40], dtype=np.int64)
    n_ins = np.array([7_400_000, 1_000], dtype=np.int64)
    n_look = np.array([50_000, 3_000], dtype=np.int64)
    ins_off = np.concatenate([[0], np.cumsum(n_ins)])
    look_off = np.concatenate([[0], np.cumsum(n_look)])
    ins = splitmix64_stream(710, int(ins_off[-1]))
    look = splitmix64_stream(711, int(look_off[-1]))
    look[:1000] = ins[:1000]
    filters = [P.Filter(int(b)) for b in blocks]
    g = P.Group(filters, ins_off, look_off)
    out = torch.empty(int(look_off[-1]), dtype=torch.uint8, device="cuda")
    g.run(dev(ins), dev(look), out)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    for f, B in enumerate(blocks.tolist()):
        ref = oracle.build_filter(B, ins[ins_off[f]:ins_off[f + 1]])
        assert np.array_equal(filters[f].words.cpu().numpy().view(np.uint32), ref), f
        assert np.array_equal(res[look_off[f]:look_off[f + 1]], oracle.lookup(ref, B, look[look_off[f]:look_off[f + 1]]))
    g.close()


def _multi_slice_workload():
    """Filters around the LDS slice sizes (1,024, 2,048, 4,096 blocks) and
    well above them, with ragged lookup counts around the LDS tiles (4,096,
    8,192, 16,384 keys) and none."""
    from types import SimpleNamespace

    blocks = [1, 7, 4095, 4096, 4097, 8195, 5 * 4096 + 17, 40_000, 300, 1024, 2049, 70_000]
    n_look = [5, 16_385, 16_383, 16_384, 0, 40_000, 70_001, 100_000, 1, 4097, 8191, 5_000]
    ins, look = [], []
    for f, (b, nl) in enumerate(zip(blocks, n_look)):
        h = splitmix64_stream(700 + f, 24 * b)
        ins.append(h)
        m = min(nl // 3, h.size)
        probes = np.concatenate([h[:m], splitmix64_stream(800 + f, nl - m)])
        look.append(probes[np.random.default_rng(f).permutation(nl)])
    off = lambda parts: np.concatenate([[0], np.cumsum([len(a) for a in parts])]).astype(np.uint64)
    return SimpleNamespace(blocks=np.array(blocks, dtype=np.uint64), num_filters=len(blocks), ins_off=off(ins),
                           look_off=off(look), inserts=np.concatenate(ins), lookups=np.concatenate(look))


@pytest.mark.parametrize("slices,threads", [(0, 1024), (1, 1024), (3, 1024), (1024, 1024), (2, 256), (1024, 256),
                                            (5, 512)])
def test_grouped_lds_lookup_multi_slice(P, slices, threads):
    """LDS lookups of filters of one to ten slices (last slice partial),
    mixed with gather lookups of the filters above the threshold; bytes
    identical to the oracle's for every filter, also on graph replays."""
    w = _multi_slice_workload()
    filters, g = make_group(P, w, dict(lookup_lds_slices=slices, lookup_lds_threads=threads))
    ins, look = dev(w.inserts), dev(w.lookups)
    out = torch.full((look.numel(),), 9, dtype=torch.uint8, device="cuda")
    g.run(ins, look, out)
    torch.cuda.synchronize()
    check_against_oracle(w, filters, out, range(w.num_filters))
    first = out.clone()
    for _ in range(2):
        g.clear()
        out.fill_(9)
        torch.cuda.synchronize()
        g.run(ins, look, out)
        torch.cuda.synchronize()
        assert torch.equal(out, first)
    g.close()


def test_two_groups_planned_in_turn(P):
    """Two groups with different LDS needs (large filters: 128 KiB slices;
    small filters: a few KiB), planned one after the other, then run, the
    first after the second was planned: planning it must not break the first."""
    from types import SimpleNamespace

    def workload(blocks, seed):
        ins = [splitmix64_stream(seed + f, 20 * b) for f, b in enumerate(blocks)]
        look = [np.concatenate([h[::3], splitmix64_stream(seed + 100 + f, h.size)]) for f, h in enumerate(ins)]
        off = lambda parts: np.concatenate([[0], np.cumsum([len(a) for a in parts])]).astype(np.uint64)
        return SimpleNamespace(blocks=np.array(blocks, dtype=np.uint64), num_filters=len(blocks), ins_off=off(ins),
                               look_off=off(look), inserts=np.concatenate(ins), lookups=np.concatenate(look))

    wa = workload([20_000, 9_000, 4_096], 900)
    wb = workload([50, 300, 7], 950)
    fa, ga = make_group(P, wa, dict(lookup_lds_slices=8))
    fb, gb = make_group(P, wb, dict(lookup_lds_slices=8))
    for w, filters, g in ((wa, fa, ga), (wb, fb, gb)):
        ins, look = dev(w.inserts), dev(w.lookups)
        out = torch.empty(look.numel(), dtype=torch.uint8, device="cuda")
        g.run(ins, look, out)
        torch.cuda.synchronize()
        check_against_oracle(w, filters, out, range(w.num_filters))
    ga.close()
    gb.close()


def test_group_rejects_shared_memory(P):
    """A filter may appear once in a group, and two handles over overlapping
    words are refused: a slice is stored back whole by one workgroup."""
    a, b = P.Filter(300), P.Filter(20)
    off = np.zeros(3, dtype=np.uint64)
    with pytest.raises(P.SbbfError) as e:
        P.Group([a, b, a], np.zeros(4, dtype=np.uint64), np.zeros(4, dtype=np.uint64))
    assert e.value.status == P.SBBF_EINVAL
    words = torch.zeros(8 * 100, dtype=torch.int32, device="cuda")
    h1 = P.sbbf_create_wrapped(words, 60)
    h2 = P.sbbf_create_wrapped(words[8 * 50:], 50)  # blocks 50..99 overlap blocks 50..59 of h1
    with pytest.raises(P.SbbfError):
        P.sbbf_grouped_create([h1, h2])
    g = P.Group([a, b], off, off)  # distinct filters are fine
    g.close()
    P.sbbf_destroy(h1)
    P.sbbf_destroy(h2)
    a.close()
    b.close()


# ---- capacity plans: per-run key ranges from device offsets -------------------------

# Filters covering every tile kind: stream-inserted (whole filter in LDS),
# partitioned by slice, LDS lookups (at most four 128 KiB slices) and gathers.
CAP_BLOCKS = [50, 700, 4096, 9000, 16_384, 40_000, 3, 2_500, 70_000]
CAP_INS = [2_000, 30_000, 90_000, 200_000, 400_000, 900_000, 10, 50_000, 1_500_000]
CAP_LOOK = [9_000, 1_000, 300_000, 50_000, 500_000, 800_000, 40, 70_001, 1_000_000]


def _count_vectors():
    rng = np.random.default_rng(11)
    full = (np.array(CAP_INS), np.array(CAP_LOOK))
    part = (rng.integers(0, np.array(CAP_INS) + 1), rng.integers(0, np.array(CAP_LOOK) + 1))
    part[0][1] = 0
    part[1][4] = 0
    tiny = (np.where(np.arange(len(CAP_INS)) == 5, CAP_INS[5], np.arange(len(CAP_INS)) % 3),
            np.where(np.arange(len(CAP_LOOK)) == 8, CAP_LOOK[8], np.arange(len(CAP_LOOK)) % 4))
    return [full, part, tiny]


def _csr(n):
    off = np.zeros(len(n) + 1, dtype=np.int64)
    off[1:] = np.cumsum(n)
    return off


def _cap_inputs(step, n_ins, n_look):
    """Inserts and lookups of one run: fresh hashes per filter, lookups mixing
    the filter's members of this run with fresh hashes."""
    ins_off, look_off = _csr(n_ins), _csr(n_look)
    ins = splitmix64_stream(820 + step, int(ins_off[-1]))
    look = splitmix64_stream(830 + step, int(look_off[-1]))
    for f in range(len(n_ins)):
        m = min(int(n_ins[f]), int(n_look[f]) // 2)
        look[look_off[f]:look_off[f] + m] = ins[ins_off[f]:ins_off[f] + m]
    return ins, look, ins_off, look_off


def test_capacity_plan_three_count_vectors(P):
    """One capacity plan and one graph, replayed with three different
    per-filter count vectors written into the same device offset buffers:
    every run equals the oracle, and no run does host planning or touches the
    graph (one plan, one graph instantiation, no updates)."""
    filters = [P.Filter(b) for b in CAP_BLOCKS]
    g = P.Group.with_capacity(filters, CAP_INS, CAP_LOOK)
    d_ins = torch.empty(sum(CAP_INS), dtype=torch.int64, device="cuda")
    d_look = torch.empty(sum(CAP_LOOK), dtype=torch.int64, device="cuda")
    d_out = torch.empty(sum(CAP_LOOK), dtype=torch.uint8, device="cuda")
    d_ioff = torch.empty(len(CAP_BLOCKS) + 1, dtype=torch.int64, device="cuda")
    d_loff = torch.empty(len(CAP_BLOCKS) + 1, dtype=torch.int64, device="cuda")
    for step, (n_ins, n_look) in enumerate(_count_vectors()):
        ins, look, ins_off, look_off = _cap_inputs(step, n_ins, n_look)
        print(f"capacity run {step}: inserts {n_ins.tolist()} lookups {n_look.tolist()}", flush=True)
        g.clear()
        d_out.fill_(7)
        d_ins[:ins.size].copy_(dev(ins))
        d_look[:look.size].copy_(dev(look))
        d_ioff.copy_(torch.from_numpy(ins_off))
        d_loff.copy_(torch.from_numpy(look_off))
        g.run_offsets(d_ins, d_ioff, d_look, d_loff, d_out)
        assert g.check() is None
        out = d_out[:look.size].cpu().numpy()
        for f, B in enumerate(CAP_BLOCKS):
            ref = oracle.build_filter(B, ins[ins_off[f]:ins_off[f + 1]])
            assert np.array_equal(filters[f].words.cpu().numpy().view(np.uint32), ref), (step, f)
            assert np.array_equal(out[look_off[f]:look_off[f + 1]],
                                  oracle.lookup(ref, B, look[look_off[f]:look_off[f + 1]])), (step, f)
        assert bool((d_out[look.size:] == 7).all()), step  # nothing written past the run's lookups
    c = g.counters()
    assert c == dict(plans=1, graph_builds=1, graph_updates=0), c
    g.close()


def test_capacity_plan_over_capacity_is_clamped_and_reported(P):
    """A run whose offsets give one filter more keys than planned (and another
    a decreasing range) processes only the planned keys of those filters, the
    rest exactly, and sbbf_grouped_check names the lowest offending filter."""
    blocks, cap_ins, cap_look = [900, 9000, 300], [5_000, 80_000, 2_000], [6_000, 50_000, 3_000]
    filters = [P.Filter(b) for b in blocks]
    g = P.Group.with_capacity(filters, cap_ins, cap_look)
    n_ins = np.array([5_000, 80_100, 1_000])       # filter 1: 100 keys over its capacity
    n_look = np.array([6_000, 50_000, 3_000])
    ins, look, ins_off, look_off = _cap_inputs(9, n_ins, n_look)
    look_bad = look_off.copy()
    look_bad[2] = look_off[2] + 10_000             # filter 1's lookups reach past filter 2's start: decreasing for 2
    d_ioff, d_loff = torch.from_numpy(ins_off).cuda(), torch.from_numpy(look_bad).cuda()
    d_look = torch.cat([dev(look), torch.zeros(10_000, dtype=torch.int64, device="cuda")])
    d_out = torch.full((d_look.numel(),), 7, dtype=torch.uint8, device="cuda")
    g.run_offsets(dev(ins), d_ioff, d_look, d_loff, d_out)
    assert g.check() == 1
    assert g.check() is None  # the record was cleared
    ref1 = oracle.build_filter(9000, ins[ins_off[1]:ins_off[1] + cap_ins[1]])
    assert np.array_equal(filters[1].words.cpu().numpy().view(np.uint32), ref1)
    ref0 = oracle.build_filter(900, ins[:ins_off[1]])
    assert np.array_equal(filters[0].words.cpu().numpy().view(np.uint32), ref0)
    out = d_out.cpu().numpy()
    assert np.array_equal(out[:look_off[1]], oracle.lookup(ref0, 900, look[:look_off[1]]))
    # filter 1 looks up its first 50,000 keys of the (longer) range; filter 2 none
    assert np.array_equal(out[look_off[1]:look_off[1] + 50_000],
                          oracle.lookup(ref1, 9000, d_look[look_off[1]:look_off[1] + 50_000].cpu().numpy().view(np.uint64)))
    assert bool((torch.from_numpy(out[look_off[1] + 50_000:]) == 7).all())
    ref2 = oracle.build_filter(300, ins[ins_off[2]:ins_off[3]])
    assert np.array_equal(filters[2].words.cpu().numpy().view(np.uint32), ref2)
    g.close()


def test_capacity_plan_entry_point_rules(P):
    filters = [P.Filter(64), P.Filter(128)]
    g = P.Group.with_capacity(filters, [10, 10], [10, 10])
    x = torch.zeros(20, dtype=torch.int64, device="cuda")
    out = torch.zeros(20, dtype=torch.uint8, device="cuda")
    for call in (lambda: g.run(x, x, out), lambda: g.run_per_filter(x, x, out), lambda: g.digest(out),
                 lambda: P.sbbf_grouped_insert(g.handle, x)):
        with pytest.raises(P.SbbfError):
            call()
    g.close()
    fixed = P.Group(filters, np.array([0, 5, 10]), np.array([0, 5, 10]))
    offs = torch.tensor([0, 5, 10], dtype=torch.int64, device="cuda")
    with pytest.raises(P.SbbfError):
        fixed.run_offsets(x, offs, x, offs, out)
    fixed.close()
