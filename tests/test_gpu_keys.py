"""Entry points that take keys: the filter and the lookups equal the oracle
applied to the keys' hashes, for every insert and lookup strategy."""

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


@pytest.mark.parametrize("ins", list(INSERTS))
@pytest.mark.parametrize("look", list(LOOKUPS))
def test_keys_match_oracle(P, ins, look):
    B = 1000 if ins == "lds" else 3001
    keys = np.arange(7_777, dtype=np.uint64) * np.uint64(3) + np.uint64(11)  # sequential-style keys
    probes = np.concatenate([keys[::5], np.arange(20_000, 30_001, dtype=np.uint64)])
    ref = oracle.build_filter(B, oracle.key_hash(keys))
    f = P.Filter(B)
    f.insert_keys(dev(keys), launch=INSERTS[ins])
    got = f.lookup_keys(dev(probes), launch=LOOKUPS[look]).cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(f.words.cpu().numpy().view(np.uint32), ref)
    assert np.array_equal(got, oracle.lookup(ref, B, oracle.key_hash(probes)))
    f.close()


def test_keys_equal_hashing_first(P):
    """insert_keys(k) gives the same filter as inserting sbbf_key_hash(k)."""
    B = 4_194_304
    keys = splitmix64_stream(950, 3_000_000)
    a, b = P.Filter(B), P.Filter(B)
    a.insert_keys(dev(keys))
    b.insert(dev(oracle.key_hash(keys)))
    torch.cuda.synchronize()
    assert torch.equal(a.words, b.words)
    probes = dev(np.arange(5_000_000, dtype=np.uint64))
    assert torch.equal(a.lookup_keys(probes), b.lookup(dev(oracle.key_hash(np.arange(5_000_000, dtype=np.uint64)))))
    a.close()
    b.close()


def test_partitioned_lookup_keys_overflow(P):
    """Keys hashed on load through the count-free lookup partition when most
    probes are one repeated key: its slice's runs overflow, and the overflow
    pass hashes those keys itself."""
    B = 4096 * 600 + 3
    keys = splitmix64_stream(952, 800_000)
    ref = oracle.build_filter(B, oracle.key_hash(keys))
    f = P.Filter(B)
    f.insert_keys(dev(keys), launch=dict(strategy=4))
    probes = splitmix64_stream(953, 1_500_001)
    probes[1::3] = keys[777]
    probes[2::3] = keys[4242]
    got = f.lookup_keys(dev(probes), launch=dict(strategy=2)).cpu().numpy()
    want = oracle.lookup(ref, B, oracle.key_hash(probes))
    assert want.any() and not want.all()
    assert np.array_equal(got, want)
    f.close()
