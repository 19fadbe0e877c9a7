"""The serving loop: results of continuous batching equal the oracle replaying
the same request log in arrival order, and equal each request run alone;
admission by budget; checkpoint and restore."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from synth.serving import serving_log  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2101_01719_amd as P

    return P


@pytest.fixture(scope="module")
def small_log():
    return serving_log(num_filters=256, num_requests=3000, rate_per_s=2e6, max_size=4096, log10_min=2.0,
                       log10_max=4.5)


@pytest.fixture(scope="module")
def small_ref(small_log):
    L = small_log
    return oracle.replay_requests(L.blocks, L.filter, L.op, L.key_off, L.payload, L.out_off)


def staged(L):
    d_payload = torch.from_numpy(L.payload.view(np.int64)).to("cuda")
    d_out = torch.full((int(L.out_off[-1]),), 7, dtype=torch.uint8, device="cuda")
    return d_payload, d_out


def make_server(P, L, **cfg):
    s = P.sbbf_server_create(cfg)
    ids = [P.sbbf_server_add_filter(s, int(b)) for b in L.blocks]
    assert ids == list(range(L.num_filters))
    return s


def snapshot_all(P, s, L):
    out = []
    for f, b in enumerate(L.blocks.tolist()):
        host = torch.empty(8 * b, dtype=torch.int32)
        P.sbbf_server_snapshot(s, f, host)
        out.append(host.numpy().view(np.uint32).copy())
    return out


def check(P, s, L, d_out, ref):
    filters, outputs = ref
    got = d_out.cpu().numpy()
    assert np.array_equal(got, outputs)
    for f, words in enumerate(snapshot_all(P, s, L)):
        assert np.array_equal(words, filters[f]), f


@pytest.mark.parametrize("realtime,inflight,step_keys", [(False, 2, 1 << 20), (True, 2, 1 << 20), (False, 1, 4096),
                                                         (True, 4, 65536), (False, 3, 1)])
def test_mix_matches_oracle(P, small_log, small_ref, realtime, inflight, step_keys):
    L = small_log
    s = make_server(P, L, max_inflight_steps=inflight, max_step_keys=step_keys, tile_keys=256)
    d_payload, d_out = staged(L)
    req = P.serving_requests(L, d_payload, d_out)
    first = P.sbbf_server_replay(s, req, realtime=realtime)
    assert first == 0
    st = P.sbbf_server_stats(s)
    assert st["requests_done"] == L.num_requests
    assert st["keys_done"] == int(L.key_off[-1])
    assert 0 < st["p50_us"] <= st["p99_us"] <= st["max_us"]
    if step_keys >= 65536:
        assert st["steps"] < L.num_requests  # requests were batched
    check(P, s, L, d_out, small_ref)
    P.sbbf_server_destroy(s)


def test_alone_equals_mix(P, small_log, small_ref):
    """Every request submitted alone (the loop drained after each one, in log
    order) gives the same bytes as the mixed replay and the oracle."""
    L = small_log
    s = make_server(P, L)
    d_payload, d_out = staged(L)
    ids = []
    for r in range(L.num_requests):
        h = d_payload[int(L.key_off[r]):int(L.key_off[r + 1])]
        out = d_out[int(L.out_off[r]):int(L.out_off[r + 1])] if L.op[r] == 1 else None
        ids.append(P.sbbf_server_submit(s, int(L.filter[r]), int(L.op[r]), h, out))
        P.sbbf_server_drain(s)
    assert ids == list(range(L.num_requests))
    done = []
    while True:
        got = P.sbbf_server_poll(s, 1024)
        if not got:
            break
        done += got
    assert sorted(done) == ids
    assert P.sbbf_server_stats(s)["steps"] == L.num_requests
    check(P, s, L, d_out, small_ref)
    P.sbbf_server_destroy(s)


def test_admission_by_budget(P):
    budget = 1 << 20  # 1 MiB of filters
    s = P.sbbf_server_create(dict(hbm_budget_bytes=budget))
    ids = []
    with pytest.raises(P.SbbfError) as e:
        while True:
            ids.append(P.sbbf_server_add_filter(s, 3000))  # 96,000 bytes each (rounded to 96,000)
    assert e.value.status == P.SBBF_EBUDGET
    used, reserved = P.sbbf_server_arena_usage(s)
    assert len(ids) == budget // 96000 and used <= budget and reserved <= budget
    # a filter is admitted again once memory is released
    P.sbbf_server_remove_filter(s, ids[3])
    fid = P.sbbf_server_add_filter(s, 3000)
    assert fid == ids[3]
    with pytest.raises(P.SbbfError):
        P.sbbf_server_add_filter(s, 3000)
    # the re-admitted filter starts empty and works
    h = torch.arange(1, 5001, dtype=torch.int64, device="cuda") * 0x9E3779B97F4A7C15 % (1 << 62)
    out = torch.empty(5000, dtype=torch.uint8, device="cuda")
    P.sbbf_server_submit(s, fid, 0, h)
    P.sbbf_server_submit(s, fid, 1, h, out)
    P.sbbf_server_drain(s)
    assert bool(out.all())
    P.sbbf_server_destroy(s)


def test_checkpoint_and_resume(P, small_log, small_ref):
    """Snapshot every filter half way through the log, tear the server down,
    restore the snapshots into a new server and replay the rest: the final
    filters and outputs equal an uninterrupted run."""
    L = small_log
    half = L.num_requests // 2
    d_payload, d_out = staged(L)
    req = P.serving_requests(L, d_payload, d_out)
    s = make_server(P, L)
    P.sbbf_server_replay(s, req[:half], realtime=False)
    snaps = snapshot_all(P, s, L)
    P.sbbf_server_destroy(s)
    s2 = make_server(P, L)
    for f, words in enumerate(snaps):
        P.sbbf_server_restore(s2, f, torch.from_numpy(words.view(np.int32)))
    tail = req[half:].copy()
    tail["arrival_ns"] -= tail["arrival_ns"][0]
    P.sbbf_server_replay(s2, tail, realtime=False)
    check(P, s2, L, d_out, small_ref)
    P.sbbf_server_destroy(s2)


def test_serving_workload_scale(P):
    """4,096 resident filters sized like the grouped workload and 20,000
    requests (sizes log-uniform in 1..65,536, 20 % inserts) replayed in real
    time: all outputs and all final filters equal the oracle's replay."""
    L = serving_log(num_filters=4096, num_requests=20_000, rate_per_s=2e5)
    ref = oracle.replay_requests(L.blocks, L.filter, L.op, L.key_off, L.payload, L.out_off)
    s = make_server(P, L)
    d_payload, d_out = staged(L)
    P.sbbf_server_replay(s, P.serving_requests(L, d_payload, d_out), realtime=True)
    st = P.sbbf_server_stats(s)
    print("serving stats:", st)
    assert st["requests_done"] == L.num_requests
    check(P, s, L, d_out, ref)
    P.sbbf_server_destroy(s)


def test_serving_full_log_against_oracle_digests(P):
    """The full serving workload: 4,096 resident filters and a log of 200,000
    requests (sizes log-uniform in 1..65,536, 20 % inserts, 1,185,987,198
    keys), generated on the device and replayed through the loop. Every final
    filter byte and every lookup byte equals the oracle's in-order replay of
    the same log (SHA-256 against tests/golden/full_digests.txt, written by
    tests/golden/make_full_digests.py from the oracle alone)."""
    import hashlib

    from conftest import read_golden

    rows = {r[0]: r for r in read_golden("full_digests.txt")}
    L = serving_log(num_filters=4096, num_requests=200_000, backend="torch", device="cuda")
    assert int(L.key_off[-1]) == L.payload.numel() == 1_185_987_198
    s = make_server(P, L)
    d_out = torch.full((int(L.out_off[-1]),), 7, dtype=torch.uint8, device="cuda")
    print(f"serving full log: {L.num_requests} requests, {L.payload.numel()} keys", flush=True)
    P.sbbf_server_replay(s, P.serving_requests(L, L.payload, d_out), realtime=False)
    st = P.sbbf_server_stats(s)
    print("serving stats:", st)
    assert st["requests_done"] == L.num_requests and st["keys_done"] == L.payload.numel()
    sha_l, nbytes_l, positives = rows["serving_4096x200000_lookups"][1:4]
    assert d_out.numel() == int(nbytes_l)
    assert int(d_out.sum(dtype=torch.int64).item()) == int(positives)
    assert hashlib.sha256(d_out.cpu().numpy().tobytes()).hexdigest() == sha_l
    hf = hashlib.sha256()
    total = 0
    for words in snapshot_all(P, s, L):
        hf.update(words.tobytes())
        total += words.nbytes
    assert total == int(rows["serving_4096x200000_filters"][2])
    assert hf.hexdigest() == rows["serving_4096x200000_filters"][1]
    P.sbbf_server_destroy(s)


def test_one_large_filter_spreads(P):
    """Steps whose lookups all hit one large filter (and a few small ones):
    the lookup tiles of that filter move between the per-XCD queues as they
    fill; inserts into the small filters take the LDS-merge path. Results
    equal the oracle's in-order replay."""
    from synth import splitmix64_stream
    from synth.serving import ServingLog

    blocks = np.array([41_016, 40, 1024, 1025], dtype=np.int64)
    ops, filt, sizes = [], [], []
    for f, n in ((0, 65_536), (0, 65_536), (1, 3_000), (2, 5_000), (3, 5_000)):
        ops.append(0); filt.append(f); sizes.append(n)
    for k in range(40):
        ops.append(1); filt.append(0 if k % 8 else 1 + (k // 8) % 3); sizes.append(65_536 if k % 8 else 777)
    ops, filt, sizes = (np.array(ops, dtype=np.uint32), np.array(filt, dtype=np.uint32),
                        np.array(sizes, dtype=np.int64))
    key_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    payload = splitmix64_stream(4242, int(key_off[-1]))
    ins = payload[: key_off[2]]
    payload[key_off[5]: key_off[5] + 1000] = ins[:1000]  # some members among the lookups
    out_off = np.concatenate([[0], np.cumsum(np.where(ops == 1, sizes, 0))]).astype(np.int64)
    L = ServingLog(blocks=blocks, capacity=blocks * 24, arrival_ns=np.arange(ops.size, dtype=np.uint64),
                   filter=filt, op=ops, n=sizes, key_off=key_off, out_off=out_off, payload=payload)
    ref = oracle.replay_requests(L.blocks, L.filter, L.op, L.key_off, L.payload, L.out_off)
    s = make_server(P, L, max_step_keys=4 << 20)
    d_payload, d_out = staged(L)
    P.sbbf_server_replay(s, P.serving_requests(L, d_payload, d_out), realtime=False)
    check(P, s, L, d_out, ref)
    P.sbbf_server_destroy(s)


def test_per_request_baseline_equals_oracle(P, small_log, small_ref):
    """The baseline that issues every request of the log as one plain call,
    in order, ends with the same filters and lookup bytes as the oracle's
    replay (and so as the serving loop's); an unknown filter id is refused
    before anything is issued."""
    L = small_log
    s = make_server(P, L)
    d_payload, d_out = staged(L)
    req = P.serving_requests(L, d_payload, d_out)
    sec = P.sbbf_server_replay_per_request(s, req)
    assert sec > 0
    check(P, s, L, d_out, small_ref)
    bad = req[:3].copy()
    bad["filter_id"][2] = L.num_filters + 5
    before = snapshot_all(P, s, L)
    with pytest.raises(P.SbbfError):
        P.sbbf_server_replay_per_request(s, bad)
    for f, words in enumerate(snapshot_all(P, s, L)):
        assert np.array_equal(words, before[f]), f
    P.sbbf_server_destroy(s)


def test_request_larger_than_a_step_grows_the_slot(P):
    """Steps of at most one request and 64 keys (tile tables of a few hundred
    64-key tiles): requests of 65,536 keys run alone in steps whose tile table
    has to grow, between small requests on the same filters; results equal
    the oracle's replay."""
    from types import SimpleNamespace

    from synth import splitmix64_stream

    blocks = np.array([3000, 41_000, 17], dtype=np.uint64)
    # (filter, op, n): big inserts and lookups around small ones
    spec = [(1, 0, 65_536), (0, 0, 100), (1, 1, 65_536), (0, 1, 3), (2, 0, 65_536), (1, 0, 5), (2, 1, 65_536),
            (1, 1, 70_000), (0, 1, 65_536)]
    filt = np.array([f for f, _, _ in spec], dtype=np.uint32)
    op = np.array([o for _, o, _ in spec], dtype=np.uint32)
    n = np.array([k for _, _, k in spec], dtype=np.uint64)
    key_off = np.concatenate([[0], np.cumsum(n)]).astype(np.uint64)
    payload = splitmix64_stream(31, int(key_off[-1]))
    # lookups ask for some earlier inserted hashes too
    payload[int(key_off[2]):int(key_off[2]) + 1000] = payload[:1000]
    out_n = np.where(op == 1, n, 0)
    out_off = np.concatenate([[0], np.cumsum(out_n)]).astype(np.uint64)
    L = SimpleNamespace(num_requests=len(spec), num_filters=len(blocks), blocks=blocks, filter=filt, op=op, n=n,
                        key_off=key_off, out_off=out_off, payload=payload,
                        arrival_ns=np.arange(len(spec), dtype=np.uint64) * 1000)
    ref = oracle.replay_requests(L.blocks, L.filter, L.op, L.key_off, L.payload, L.out_off)
    s = make_server(P, L, max_step_keys=64, max_step_requests=1, tile_keys=64)
    d_payload, d_out = staged(L)
    P.sbbf_server_replay(s, P.serving_requests(L, d_payload, d_out), realtime=False)
    st = P.sbbf_server_stats(s)
    assert st["requests_done"] == L.num_requests and st["steps"] == L.num_requests
    check(P, s, L, d_out, ref)
    P.sbbf_server_destroy(s)
