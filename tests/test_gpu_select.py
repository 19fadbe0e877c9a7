"""Lookup with stream compaction (sbbf_lookup_select) against the oracle's
select: the ascending indices of the hashes the lookup reports present."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from synth import plain_workload, splitmix64_stream  # noqa: E402

pytestmark = pytest.mark.gpu

LOOKUPS = {"auto": None, "gather": dict(strategy=1), "partitioned": dict(strategy=2)}


@pytest.fixture(scope="module")
def P():
    import paper_2101_01719_amd as P

    return P


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to("cuda")


@pytest.mark.parametrize("strategy", list(LOOKUPS))
@pytest.mark.parametrize("n", [1, 31, 32, 33, 8191, 8192, 8193, 100_003])
def test_select_matches_oracle(P, strategy, n):
    B = 1500
    ins = splitmix64_stream(900, 20_000)
    probes = splitmix64_stream(901, n)
    probes[: min(n, 5000):3] = ins[: len(probes[: min(n, 5000):3])]
    f = P.Filter(B)
    f.insert(dev(ins))
    ref = oracle.select(oracle.build_filter(B, ins), B, probes)
    idx, cnt = P.sbbf_lookup_select(f.handle, dev(probes), launch=LOOKUPS[strategy])
    torch.cuda.synchronize()
    c = int(cnt.item())
    assert c == ref.size, (strategy, n)
    assert np.array_equal(idx[:c].cpu().numpy().view(np.uint32), ref), (strategy, n)
    f.close()


def test_select_all_and_none(P):
    B = 64
    probes = splitmix64_stream(902, 50_001)
    f = P.Filter(B)
    got = f.select(dev(probes)).cpu().numpy()
    assert got.size == 0  # empty filter: nothing present
    f.words.fill_(-1)     # all-ones filter: everything present
    got = f.select(dev(probes)).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, np.arange(probes.size, dtype=np.uint32))
    f.close()


def test_select_empty_batch_writes_zero(P):
    f = P.Filter(8)
    cnt = torch.full((1,), 12345, dtype=torch.int64, device="cuda")
    idx = torch.empty(1, dtype=torch.int32, device="cuda")
    P.sbbf_lookup_select(f.handle, torch.empty(0, dtype=torch.int64, device="cuda"), idx, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0
    f.close()


def test_select_plain_100m(P):
    """The 100M-key workload's 2e8 lookups in the benchmark's launch (library
    defaults): the indices are exactly the positions of the byte lookup's ones
    (itself checked against the oracle at this size), every member is among
    them, and a sample of indices and of non-selected positions agrees with
    the oracle's single-key lookup."""
    w = plain_workload("plain_100m", backend="torch", device="cuda")
    f = P.Filter(w.num_blocks)
    f.insert(w.inserts)
    out = f.lookup(w.lookups)
    idx, cnt = P.sbbf_lookup_select(f.handle, w.lookups)
    torch.cuda.synchronize()
    c = int(cnt.item())
    ref = torch.nonzero(out).flatten().to(torch.int32)
    assert c == ref.numel()
    assert torch.equal(idx[:c], ref)
    assert bool(out[w.is_member].all().item())
    words = f.words.cpu().numpy().view(np.uint32)
    look = w.lookups.cpu().numpy().view(np.uint64)
    rng = np.random.default_rng(11)
    sel = idx[:c].cpu().numpy()
    for i in rng.choice(sel, 200, replace=False):
        assert oracle.contains(words, w.num_blocks, int(look[i]))
    mask = np.ones(look.size, dtype=bool)
    mask[sel] = False
    for i in rng.choice(np.flatnonzero(mask), 200, replace=False):
        assert not oracle.contains(words, w.num_blocks, int(look[i]))
    f.close()
