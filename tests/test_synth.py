"""The seeded input generators: SplitMix64 against its published values, the
numpy and torch backends against each other, and the workload recipes."""

import numpy as np
import pytest

from synth import grouped_sizes, grouped_workload, plain_workload, splitmix64, splitmix64_stream, unit_double
from synth.splitmix import GAMMA
from synth.workloads import streams_disjoint


def test_splitmix64_published_vector():
    # Vigna's reference SplitMix64 seeded with 0: first two outputs.
    assert splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert splitmix64(0, 1) == 0x6E789E6AA1B965F4
    s = splitmix64_stream(0, 2)
    assert [int(v) for v in s] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4]


def test_stream_slices_and_scalar_reference():
    full = splitmix64_stream(7, 1000)
    for i in (0, 1, 499, 999):
        assert int(full[i]) == splitmix64(7, i)
    part = splitmix64_stream(7, 100, start=450)
    assert np.array_equal(part, full[450:550])


def test_torch_backend_matches_numpy():
    torch = pytest.importorskip("torch")
    for seed in (0, 1, 2, 3, (1 << 64) - 1):
        a = splitmix64_stream(seed, 5000, start=123)
        b = splitmix64_stream(seed, 5000, start=123, backend="torch", device="cpu")
        assert b.dtype == torch.int64
        assert np.array_equal(a, b.numpy().view(np.uint64))


def test_streams_disjoint_argument():
    # The only colliding index difference between seeds 1 and 2 is GAMMA^-1.
    d = pow(GAMMA, -1, 1 << 64)
    assert (d * GAMMA) % (1 << 64) == 1
    assert streams_disjoint(1, 10**9, 2, 10**10)
    # A window that contains that difference is reported as overlapping and
    # the values there really are equal.
    assert not streams_disjoint(2, 1, 1, d + 1)
    assert splitmix64(1, d) == splitmix64(2, 0)


def test_unit_double_range():
    u = unit_double(splitmix64_stream(9, 10000))
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.02


@pytest.mark.parametrize("name", ["plain_100k", "plain_1m"])
def test_plain_workload_recipe(name):
    w = plain_workload(name)
    assert w.lookups.dtype == np.uint64
    assert w.is_member.sum() == w.n_member_lookups
    assert w.lookups.size == w.n_member_lookups + w.n_nonmember_lookups
    members = set(w.inserts.tolist())
    look = w.lookups.tolist()
    flags = w.is_member.tolist()
    sample = range(0, len(look), max(1, len(look) // 20000))
    for i in sample:
        assert (look[i] in members) == flags[i]


def test_plain_workload_backends_agree():
    pytest.importorskip("torch")
    a = plain_workload("plain_1m", scale=0.05)
    b = plain_workload("plain_1m", scale=0.05, backend="torch", device="cpu")
    assert np.array_equal(a.inserts, b.inserts.numpy().view(np.uint64))
    assert np.array_equal(a.lookups, b.lookups.numpy().view(np.uint64))
    assert np.array_equal(a.is_member, b.is_member.numpy())


def test_grouped_sizes_statistics():
    n, blocks = grouped_sizes(2048)
    assert n.min() >= 1000 and n.max() <= 1_000_000
    assert np.array_equal(blocks, (21 * n + 511) // 512)  # ceil(n * 10.5 / 256)
    # log-uniform: about a third of the filters per decade
    dec = np.floor(np.log10(n)).astype(int)
    counts = np.bincount(dec, minlength=7)[3:6]
    assert all(abs(c - 2048 / 3) < 80 for c in counts)


def test_grouped_workload_layout_and_backends():
    pytest.importorskip("torch")
    g = grouped_workload(num_filters=32, log10_max=3.7)
    h = grouped_workload(num_filters=32, log10_max=3.7, backend="torch", device="cpu")
    assert np.array_equal(g.lookups, h.lookups.numpy().view(np.uint64))
    assert np.array_equal(g.is_member, h.is_member.numpy())
    for f in range(g.num_filters):
        ins = g.inserts[g.ins_off[f]:g.ins_off[f + 1]]
        look = g.lookups[g.look_off[f]:g.look_off[f + 1]]
        mem = g.is_member[g.look_off[f]:g.look_off[f + 1]]
        assert look.size == 4 * ins.size
        # every member looked up exactly once, the rest are not members
        assert np.array_equal(np.sort(look[mem]), np.sort(ins))
        assert not np.isin(look[~mem], ins).any()


def test_serving_log_recipe():
    from synth.serving import serving_log

    L = serving_log(num_filters=64, num_requests=3000, rate_per_s=1e6, max_size=1024, log10_min=2.0, log10_max=3.5)
    assert np.all(np.diff(L.arrival_ns.astype(np.int64)) >= 0)
    # Poisson arrivals: mean gap 1 us
    assert abs(float(L.arrival_ns[-1]) / L.num_requests - 1000.0) < 100.0
    assert abs((L.op == 0).mean() - 0.2) < 0.03
    assert L.n.min() >= 1 and L.n.max() <= 1024
    assert np.array_equal(np.diff(L.key_off), L.n)
    assert L.out_off[-1] == L.n[L.op == 1].sum()
    assert np.bincount(L.filter, minlength=64).min() > 0
    # lookups draw about a quarter of their keys from earlier inserts of their filter
    seen = {}
    hits = total = 0
    for r in range(L.num_requests):
        f = int(L.filter[r])
        keys = L.payload[L.key_off[r]:L.key_off[r + 1]]
        if L.op[r] == 0:
            seen.setdefault(f, set()).update(keys.tolist())
        elif f in seen:
            s = seen[f]
            hits += sum(k in s for k in keys.tolist())
            total += keys.size
    assert abs(hits / total - 0.25) < 0.02


def test_serving_log_stream_positions():
    from synth.serving import _stream_at

    pos = np.array([0, 1, 17, 999, 123456], dtype=np.int64)
    assert np.array_equal(_stream_at(11, pos), splitmix64_stream(11, 123457)[pos])


def test_grouped_filter_inputs_equal_the_workload_slices():
    from synth.workloads import grouped_filter_inputs

    w = grouped_workload(num_filters=12, log10_min=2.0, log10_max=4.0)
    for f in range(12):
        m, look, mem = grouped_filter_inputs(w.n, f)
        assert np.array_equal(m, w.inserts[w.ins_off[f]:w.ins_off[f + 1]])
        assert np.array_equal(look, w.lookups[w.look_off[f]:w.look_off[f + 1]])
        assert np.array_equal(mem, w.is_member[w.look_off[f]:w.look_off[f + 1]])


@pytest.mark.parametrize("chunk", [3, 5000, 1 << 25])
def test_serving_log_pieces_and_backends_agree(monkeypatch, chunk):
    """Member draws taken a piece at a time give the same log for any piece
    size, and the torch backend gives the numpy backend's payload bit for bit
    (its unsigned modulo and unit doubles are exact)."""
    torch = pytest.importorskip("torch")
    import synth.serving as S

    ref = S.serving_log(64, 3000, max_size=4096)
    monkeypatch.setattr(S, "_DRAW_CHUNK", chunk)
    a = S.serving_log(64, 3000, max_size=4096)
    b = S.serving_log(64, 3000, max_size=4096, backend="torch", device="cpu")
    for name in ("arrival_ns", "filter", "op", "n", "key_off", "out_off", "payload"):
        assert np.array_equal(getattr(a, name), getattr(ref, name)), name
    assert np.array_equal(b.payload.numpy().view(np.uint64), ref.payload)
    assert isinstance(b.payload, torch.Tensor)


def test_unsigned_modulo_of_bit_views():
    torch = pytest.importorskip("torch")
    from synth.serving import _umod_torch

    z = splitmix64_stream(77, 20_000)
    m = (splitmix64_stream(78, 20_000) % np.uint64((1 << 31) - 1)).astype(np.int64) + 1
    got = _umod_torch(torch.from_numpy(z.view(np.int64)), torch.from_numpy(m)).numpy()
    assert np.array_equal(got, (z % m.astype(np.uint64)).astype(np.int64))
