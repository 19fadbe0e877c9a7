"""Pins for the two oracle functions that sit above the method's arithmetic.

``oracle.replay_requests`` defines what the serving loop must compute: the
insert and lookup routines of the paper's appendix figure applied to a request
log one request at a time, in arrival order, so that each lookup sees exactly
the inserts that came before it on its own filter. It is pinned here by

  * a log worked out by hand, two filters interleaved, whose expected bits come
    from the worked examples of the paper's own code
    (``tests/golden/paper_code_examples.txt``), not from the oracle;
  * a brute-force model of the log with Python integers (the bits computed from
    the printed seed constants) on tiny random logs;
  * planted mistakes (inserts moved before lookups, lookups before inserts, one
    shared filter, keys shifted by one, outputs misplaced) that must each fail.

``oracle.fpr.blocks_for_fpr`` inverts the paper's false-positive model (the
analysis section's Poisson sum): the smallest block count B with
F(n / B) <= target. It is pinned exactly, with no slack, by the definition
itself checked at B and B - 1, by a linear search over the neighbourhood, by
the evaluation table's geometry (1e8 keys and the rate of 4,194,304 blocks give
back 4,194,304 blocks) and by the band endpoints the paper prints (20 and 52
hashes per block); and planted mistakes in the bisection must each fail.
"""

import inspect
import textwrap

import numpy as np
import pytest

import oracle
import oracle.fpr as fpr
from conftest import read_golden
from synth import splitmix64_stream

M32 = 0xFFFFFFFF


def _examples():
    """hash -> (block by num_blocks, the eight bit indices), from the paper's code."""
    ex = {}
    for row in read_golden("paper_code_examples.txt"):
        h, B, b = int(row[0], 16), int(row[1]), int(row[2])
        ex.setdefault(h, [{}, [int(v) for v in row[3:11]]])[0][B] = b
    return ex


def _words_from_examples(B, keys, ex):
    """Filter words holding ``keys``, set bit by bit from the worked examples."""
    w = np.zeros(8 * B, dtype=np.uint32)
    for h in keys:
        blocks, idx = ex[h]
        b = blocks[B] if B in blocks else (0 if h == 0 else None)  # high half 0: block 0 for every B
        for j in range(8):
            w[8 * b + j] |= np.uint32(1 << idx[j])
    return w


# Hashes whose block and bit indices the paper's code gives (golden file):
A = 0x0000000000000000          # block 0 for every B; all eight indices 0
BB = 0xFFFFFFFFFFFFFFFF         # block B - 1 (B = 3: block 2); indices 23 23 11 14 26 17 20 12
C = 0x910A2DEC89025CC1          # B = 4096: block 2320
D = 0x975835DE1C9756CE          # B = 4096: block 2421

# Two filters, interleaved requests: (filter, op, keys); op 0 insert, 1 lookup.
HAND_LOG = [
    (0, 0, [A]),
    (0, 1, [A, BB]),       # B's block (2) of filter 0 is still empty -> 1, 0
    (1, 1, [A]),           # filter 1 is still empty -> 0
    (1, 0, [C]),
    (0, 0, [BB]),
    (0, 1, [A, BB]),       # both inserted now -> 1, 1
    (1, 1, [A, C, D]),     # blocks 0 and 2421 of filter 1 are empty -> 0, 1, 0
    (1, 0, [D]),
    (1, 1, [D, C]),        # -> 1, 1
]
HAND_BLOCKS = [3, 4096]
HAND_OUT = [1, 0, 0, 1, 1, 0, 1, 0, 1, 1]


def _as_arrays(log, payload_extra=()):
    filt = np.array([f for f, _, _ in log], dtype=np.uint32)
    op = np.array([o for _, o, _ in log], dtype=np.uint32)
    n = np.array([len(k) for _, _, k in log], dtype=np.int64)
    key_off = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    payload = np.array([h for _, _, k in log for h in k] + list(payload_extra), dtype=np.uint64)
    out_off = np.concatenate([[0], np.cumsum(np.where(op == 1, n, 0))]).astype(np.int64)
    return filt, op, key_off, payload, out_off


def _bigint_replay(blocks, log, seeds):
    """The log applied request by request to filters held as Python integers
    (bit 256 b + 32 j + k): inserts set bits, lookups read them."""
    bits = [0] * len(blocks)
    out = []

    def pos(h, B, j):
        b = ((h >> 32) * B) >> 32
        return 256 * b + 32 * j + (((seeds[j] * (h & M32)) & M32) >> 27)

    for f, o, keys in log:
        B = blocks[f]
        for h in keys:
            if o == 0:
                for j in range(8):
                    bits[f] |= 1 << pos(h, B, j)
            else:
                out.append(int(all((bits[f] >> pos(h, B, j)) & 1 for j in range(8))))
    return bits, out


def _printed_seeds():
    s = []
    for hi, lo in read_golden("appendix_seeds.txt"):
        s += [int(lo, 16), int(hi, 16)]
    return s


def _random_log(seed, blocks, n_req):
    rng = np.random.default_rng(seed)
    keys = splitmix64_stream(300 + seed, 8 * n_req).tolist()
    log, used, at = [], [], 0
    for _ in range(n_req):
        f = int(rng.integers(len(blocks)))
        o = int(rng.random() < 0.6)
        k = int(rng.integers(1, 6))
        ks = []
        for _ in range(k):
            if o == 1 and used and rng.random() < 0.5:
                ks.append(used[int(rng.integers(len(used)))])  # some keys inserted before (maybe elsewhere)
            else:
                ks.append(keys[at])
                at += 1
        if o == 0:
            used += ks
        log.append((f, o, ks))
    return log


def _replay_pins_pass(replay):
    """True when ``replay`` (a replay_requests implementation) passes every pin."""
    try:
        ex = _examples()
        filt, op, key_off, payload, out_off = _as_arrays(HAND_LOG)
        filters, out = replay(np.array(HAND_BLOCKS), filt, op, key_off, payload, out_off)
        if [int(v) for v in out] != HAND_OUT:
            return False
        if not np.array_equal(filters[0], _words_from_examples(3, [A, BB], ex)):
            return False
        if not np.array_equal(filters[1], _words_from_examples(4096, [C, D], ex)):
            return False
        seeds = _printed_seeds()
        for seed, blocks in ((1, [1, 2, 7]), (2, [5]), (3, [1, 1, 3, 64])):
            log = _random_log(seed, blocks, 60)
            filt, op, key_off, payload, out_off = _as_arrays(log)
            filters, out = replay(np.array(blocks), filt, op, key_off, payload, out_off)
            want_bits, want_out = _bigint_replay(blocks, log, seeds)
            if [int(v) for v in out] != want_out:
                return False
            for f, B in enumerate(blocks):
                if int.from_bytes(filters[f].astype("<u4").tobytes(), "little") != want_bits[f]:
                    return False
        return True
    except (AssertionError, ValueError, IndexError, TypeError):
        return False


def test_replay_hand_worked_log():
    ex = _examples()
    filt, op, key_off, payload, out_off = _as_arrays(HAND_LOG)
    filters, out = oracle.replay_requests(np.array(HAND_BLOCKS), filt, op, key_off, payload, out_off)
    assert out.tolist() == HAND_OUT
    assert np.array_equal(filters[0], _words_from_examples(3, [A, BB], ex))
    assert np.array_equal(filters[1], _words_from_examples(4096, [C, D], ex))
    # The final filters are the filters of all their inserts (order-free), and
    # the second filter's requests do not touch the first.
    assert np.array_equal(filters[0], oracle.build_filter(3, np.array([A, BB], dtype=np.uint64)))
    alone = [r for r in HAND_LOG if r[0] == 0]
    f0, o0, k0, p0, q0 = _as_arrays(alone)
    only0, out0 = oracle.replay_requests(np.array([3]), f0, o0, k0, p0, q0)
    assert np.array_equal(only0[0], filters[0])
    assert out0.tolist() == [1, 0, 1, 1]


@pytest.mark.parametrize("seed,blocks", [(1, [1, 2, 7]), (2, [5]), (3, [1, 1, 3, 64])])
def test_replay_matches_bigint_model(seed, blocks):
    log = _random_log(seed, blocks, 60)
    filt, op, key_off, payload, out_off = _as_arrays(log)
    filters, out = oracle.replay_requests(np.array(blocks), filt, op, key_off, payload, out_off)
    want_bits, want_out = _bigint_replay(blocks, log, _printed_seeds())
    assert out.tolist() == want_out
    for f in range(len(blocks)):
        assert int.from_bytes(filters[f].astype("<u4").tobytes(), "little") == want_bits[f]


def test_replay_pins_pass_unmutated():
    assert _replay_pins_pass(oracle.replay_requests)


REPLAY_MUTANTS = {
    "inserts_before_lookups": ("for r in range(len(op)):",
                               "for r in sorted(range(len(op)), key=lambda r: int(op[r])):"),
    "lookups_before_inserts": ("for r in range(len(op)):",
                               "for r in sorted(range(len(op)), key=lambda r: -int(op[r])):"),
    "one_shared_filter": ("f = int(filt[r])", "f = 0"),
    "keys_shifted": ("h = payload[int(key_off[r]):int(key_off[r + 1])]",
                     "h = payload[int(key_off[r]) + 1:int(key_off[r + 1]) + 1]"),
    "outputs_not_advanced": ("at += h.size", "at += 0"),
    "lookup_after_insert_of_same_request": ("if op[r] == 0:", "if True:"),
}


def _mutated(func, old, new):
    src = textwrap.dedent(inspect.getsource(func))
    assert old in src, f"mutation site not found: {old!r}"
    ns = dict(func.__globals__)
    exec(compile(src.replace(old, new, 1), "<mutant>", "exec"), ns)
    return ns[func.__name__]


@pytest.mark.parametrize("name", sorted(REPLAY_MUTANTS))
def test_replay_mutant_is_caught(name):
    old, new = REPLAY_MUTANTS[name]
    assert not _replay_pins_pass(_mutated(oracle.replay_requests, old, new))


# --- sizing from a target rate --------------------------------------------------

SIZING_CASES = [(1, 0.5), (1000, 0.01), (100_000, 0.0103), (1_000_000, 0.0274), (123_457, 0.004),
                (50_000, 0.001), (7, 0.19), (2_000_000, 0.05)]


def _defined(n, target, B, lanes=8):
    """B is the smallest block count with F(n / B) <= target (F grows with the load)."""
    return fpr.sbbf_fpr(n / B, lanes) <= target and (B == 1 or fpr.sbbf_fpr(n / (B - 1), lanes) > target)


def _linear_search(n, target, lo, hi, lanes=8):
    for B in range(max(1, lo), hi + 1):
        if fpr.sbbf_fpr(n / B, lanes) <= target:
            return B
    return None


def _sizing_pins_pass(blocks_for_fpr):
    try:
        for n, t in SIZING_CASES:
            B = blocks_for_fpr(n, t)
            if not _defined(n, t, B):
                return False
            if _linear_search(n, t, B - 40, B + 40) != B:
                return False
        # The evaluation table's geometry, at exactly the model's rate for it.
        if blocks_for_fpr(100_000_000, fpr.sbbf_fpr(100_000_000 / 4_194_304)) != 4_194_304:
            return False
        # The band endpoints the analysis section prints: 20 and 52 hashes per block.
        if blocks_for_fpr(20 * 4096, fpr.sbbf_fpr(20.0)) != 4096:
            return False
        if blocks_for_fpr(52 * 1000, fpr.sbbf_fpr(52.0)) != 1000:
            return False
        # Four- and sixteen-word blocks at the same geometry (exponent K).
        for K in (4, 16):
            if blocks_for_fpr(100_000_000, fpr.sbbf_fpr(100_000_000 / 4_194_304, K), lanes=K) != 4_194_304:
                return False
        # No block count is enough: 0; a rate every count meets: 1.
        if blocks_for_fpr(2**62, 1e-6) != 0 or blocks_for_fpr(0, 0.01) != 1 or blocks_for_fpr(1, 0.99) != 1:
            return False
        return True
    except (AssertionError, ValueError, ZeroDivisionError):
        return False


@pytest.mark.parametrize("n,target", SIZING_CASES)
def test_blocks_for_fpr_is_the_defined_minimum(n, target):
    B = fpr.blocks_for_fpr(n, target)
    assert _defined(n, target, B)
    assert _linear_search(n, target, B - 40, B + 40) == B


def test_blocks_for_fpr_table_geometry_exact():
    assert fpr.blocks_for_fpr(100_000_000, fpr.sbbf_fpr(100_000_000 / 4_194_304)) == 4_194_304
    assert fpr.blocks_for_fpr(20 * 4096, fpr.sbbf_fpr(20.0)) == 4096
    assert fpr.blocks_for_fpr(52 * 1000, fpr.sbbf_fpr(52.0)) == 1000


def test_sizing_pins_pass_unmutated():
    assert _sizing_pins_pass(fpr.blocks_for_fpr)


SIZING_MUTANTS = {
    "returns_lower_bracket": ("    return hi\n", "    return lo\n"),
    "strict_comparison": ("if sbbf_fpr(n / mid, lanes) <= fpr:", "if sbbf_fpr(n / mid, lanes) < fpr:"),
    "lanes_dropped": ("if sbbf_fpr(n / mid, lanes) <= fpr:", "if sbbf_fpr(n / mid) <= fpr:"),
    "one_block_reported_as_two": ("if sbbf_fpr(float(n), lanes) <= fpr:\n        return 1",
                                  "if sbbf_fpr(float(n), lanes) <= fpr:\n        return 2"),
    "load_per_bit": ("if sbbf_fpr(n / mid, lanes) <= fpr:", "if sbbf_fpr(n / (256 * mid), lanes) <= fpr:"),
}


@pytest.mark.parametrize("name", sorted(SIZING_MUTANTS))
def test_sizing_mutant_is_caught(name):
    old, new = SIZING_MUTANTS[name]
    assert not _sizing_pins_pass(_mutated(fpr.blocks_for_fpr, old, new))
