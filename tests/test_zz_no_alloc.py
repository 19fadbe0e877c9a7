"""The allocation-free select (sbbf_lookup_select_noalloc) against the
allocating one (sbbf_lookup_select) and the oracle, called through the C ABI.

The allocation-free entry point keeps its workspace in a static device array
that every call on the GPU shares and that keeps the last call's contents, so
the cases below run back to back in one process: a large call, then a smaller
one over the stale array, then the largest size the array admits.
"""

import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from synth import splitmix64_stream  # noqa: E402

pytestmark = pytest.mark.gpu

MAX_KEYS = 1 << 28


@pytest.fixture(scope="module")
def P():
    import paper_2101_01719_amd as P

    return P


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to("cuda")


def _both(P, f, probes_dev, n_room=None):
    """Indices and count from the allocation-free and the allocating select
    (gather lookups for both, as the allocation-free form always uses)."""
    n = probes_dev.numel()
    room = max(n if n_room is None else n_room, 1)
    idx_a = torch.full((room,), -1, dtype=torch.int32, device="cuda")
    cnt_a = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    P.sbbf_lookup_select_noalloc(f.handle, probes_dev, idx_a, cnt_a)
    idx_b, cnt_b = P.sbbf_lookup_select(f.handle, probes_dev, launch=dict(strategy=1))
    torch.cuda.synchronize()
    ca, cb = int(cnt_a.item()), int(cnt_b.item())
    return idx_a, ca, idx_b, cb


def test_two_calls_in_a_row_match_the_allocating_select_and_the_oracle(P):
    B = 3000
    ins = splitmix64_stream(910, 60_000)
    f = P.Filter(B)
    f.insert(dev(ins))
    ref_words = oracle.build_filter(B, ins)
    # First call: 1,000,003 probes (123 tiles of 8,192 keys and a ragged tail),
    # a third of them members. Second call, smaller, over the stale workspace.
    for step, (seed, n) in enumerate([(911, 1_000_003), (912, 40_001)]):
        probes = splitmix64_stream(seed, n)
        probes[: min(n, 60_000):3] = ins[: len(probes[: min(n, 60_000):3])]
        print(f"noalloc select call {step}: n={n} B={B}", flush=True)
        idx_a, ca, idx_b, cb = _both(P, f, dev(probes))
        ref = oracle.select(ref_words, B, probes)
        assert ca == cb == ref.size, (step, ca, cb, ref.size)
        got = idx_a[:ca].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, idx_b[:cb].cpu().numpy().view(np.uint32)), step
        assert np.array_equal(got, ref), step
        # Nothing is written past the count.
        assert bool((idx_a[ca:] == -1).all()), step
    f.close()


def test_largest_batch_matches_the_allocating_select(P):
    """n = 2^28, the most the static workspace admits: every output index
    against the allocating select, and 4,000 sampled probes against the
    oracle one by one."""
    B = 4_194_304
    f = P.Filter(B)
    ins = splitmix64_stream(1, 1_000_000, backend="torch", device="cuda")
    f.insert(ins)
    probes = splitmix64_stream(913, MAX_KEYS, backend="torch", device="cuda")
    probes[: 1_000_000] = ins
    print(f"noalloc select: n={MAX_KEYS} B={B}", flush=True)
    idx_a, ca, idx_b, cb = _both(P, f, probes)
    assert ca == cb
    assert torch.equal(idx_a[:ca], idx_b[:cb])
    assert ca >= 1_000_000
    assert bool((idx_a[:1_000_000] == torch.arange(1_000_000, device="cuda", dtype=torch.int32)).all())
    # Sampled against the oracle: a probe is selected iff the oracle's lookup says present.
    ref_words = oracle.build_filter(B, ins.cpu().numpy().view(np.uint64))
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(MAX_KEYS, 4000, replace=False))
    want = oracle.lookup(ref_words, B, probes[torch.from_numpy(sample).cuda()].cpu().numpy().view(np.uint64))
    got_idx = idx_a[:ca]
    pos = torch.searchsorted(got_idx.to(torch.int64), torch.from_numpy(sample).cuda())
    pos = pos.clamp(max=ca - 1)
    sel = (got_idx.to(torch.int64)[pos] == torch.from_numpy(sample).cuda()).cpu().numpy()
    assert np.array_equal(sel, want.astype(bool))
    del probes
    f.close()


def test_empty_and_errors(P):
    f = P.Filter(64)
    idx = torch.zeros(8, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), 7, dtype=torch.int64, device="cuda")
    P.sbbf_lookup_select_noalloc(f.handle, torch.empty(0, dtype=torch.int64, device="cuda"), idx, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0
    L = P._L()
    hashes = torch.zeros(8, dtype=torch.int64, device="cuda")
    # More keys than the static workspace admits: rejected before any device
    # work (the size check precedes every pointer use).
    st = L.sbbf_lookup_select_noalloc(f.handle, ctypes.c_void_p(hashes.data_ptr()), MAX_KEYS + 1,
                                      ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(cnt.data_ptr()), None, None)
    assert st == 1 and "2^28" in L.sbbf_last_error().decode()
    # The partitioned lookup would allocate: refused.
    with pytest.raises(P.SbbfError) as e:
        P.sbbf_lookup_select_noalloc(f.handle, hashes, idx, cnt, launch=dict(strategy=2))
    assert e.value.status == 5
    f.close()
