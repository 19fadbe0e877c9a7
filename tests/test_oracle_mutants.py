"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a temporary copy of the oracle's C source
(on the CPU, never in the GPU library), builds it, and runs a short battery of
pins: the printed seeds, the worked examples of the paper's code, brute force
with big integers, and the 100k-key workload result of the paper's code. Every
mutant must fail at least one of them.
"""

import ctypes
import hashlib
import os
import subprocess

import numpy as np
import pytest

from conftest import ROOT, read_golden
from synth import plain_workload

SRC = os.path.join(ROOT, "oracle", "sbbf_oracle.c")

MUTANTS = {
    "shift_28": ("idx[j] = product >> 27;", "idx[j] = product >> 28;"),
    "lanes_swapped": ("seeds[2 * k] = (uint32_t)(kPrintedConstants[k] & UINT64_C(0xffffffff));\n"
                      "    seeds[2 * k + 1] = (uint32_t)(kPrintedConstants[k] >> 32);",
                      "seeds[2 * k + 1] = (uint32_t)(kPrintedConstants[k] & UINT64_C(0xffffffff));\n"
                      "    seeds[2 * k] = (uint32_t)(kPrintedConstants[k] >> 32);"),
    "block_low_half": ("uint64_t hi = hash >> 32;", "uint64_t hi = hash & UINT64_C(0xffffffff);"),
    "block_off_by_one": ("return (hi * (uint64_t)num_blocks) >> 32;",
                         "return (((hi * (uint64_t)num_blocks) >> 32) + 1) % num_blocks;"),
    "block_mod": ("return (hi * (uint64_t)num_blocks) >> 32;", "return hash % num_blocks;"),
    "mask_uses_high_half": ("sbbf_oracle_mask((uint32_t)(hashes[i] & UINT64_C(0xffffffff)), mask);",
                            "sbbf_oracle_mask((uint32_t)(hashes[i] >> 32), mask);"),
    "transposed_words": ("words[8 * b + (uint64_t)j] |= mask[j];", "words[b + (uint64_t)num_blocks * (uint64_t)j] |= mask[j];"),
    "xor_not_or": ("words[8 * b + (uint64_t)j] |= mask[j];", "words[8 * b + (uint64_t)j] ^= mask[j];"),
    "product_high_half": ("uint32_t product = (uint32_t)((uint64_t)seeds[j] * (uint64_t)x); /* mod 2^32 */",
                          "uint32_t product = (uint32_t)(((uint64_t)seeds[j] * (uint64_t)x) >> 32);"),
    "lookup_any_lane": ("if ((words[8 * b + (uint64_t)j] & mask[j]) == 0) return 0;\n  }\n  return 1;",
                        "if ((words[8 * b + (uint64_t)j] & mask[j]) != 0) return 1;\n  }\n  return 0;"),
    "seed_typo": ("UINT64_C(0x705495c72df1424b)", "UINT64_C(0x705495c72df1424d)"),
    "dropped_lane": ("for (int j = 0; j < 8; ++j) words[8 * b + (uint64_t)j] |= mask[j];",
                     "for (int j = 0; j < 7; ++j) words[8 * b + (uint64_t)j] |= mask[j];"),
}

M32 = 0xFFFFFFFF


def _build(src_text, path):
    c = path + ".c"
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", path, c], check=True,
                   stderr=subprocess.DEVNULL)
    lib = ctypes.CDLL(path)
    U64P, U32P, U8P = ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint8)
    lib.sbbf_oracle_seeds.argtypes = [U32P]
    lib.sbbf_oracle_block.argtypes = [ctypes.c_uint64, ctypes.c_uint32]
    lib.sbbf_oracle_block.restype = ctypes.c_uint64
    lib.sbbf_oracle_bit_indices.argtypes = [ctypes.c_uint32, U32P]
    lib.sbbf_oracle_insert.argtypes = [U32P, ctypes.c_uint32, U64P, ctypes.c_uint64]
    lib.sbbf_oracle_lookup.argtypes = [U32P, ctypes.c_uint32, U64P, ctypes.c_uint64, U8P]
    return lib


def _pins_pass(lib):
    """True when every pin in the battery passes."""
    U64P, U32P, U8P = ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint8)
    seeds = np.zeros(8, dtype=np.uint32)
    lib.sbbf_oracle_seeds(seeds.ctypes.data_as(U32P))
    expect = []
    for hi, lo in read_golden("appendix_seeds.txt"):
        expect += [int(lo, 16), int(hi, 16)]
    if [int(s) for s in seeds] != expect:
        return False
    for row in read_golden("paper_code_examples.txt"):
        h, B, b = int(row[0], 16), int(row[1]), int(row[2])
        if lib.sbbf_oracle_block(h, B) != b:
            return False
        idx = np.zeros(8, dtype=np.uint32)
        lib.sbbf_oracle_bit_indices(h & M32, idx.ctypes.data_as(U32P))
        if [int(v) for v in idx] != [int(v) for v in row[3:11]]:
            return False
    # the 100k-key workload as produced by the paper's code
    row = [r for r in read_golden("paper_code_configs.txt") if r[0] == "plain_100k"][0]
    w = plain_workload("plain_100k")
    words = np.zeros(8 * w.num_blocks, dtype=np.uint32)
    lib.sbbf_oracle_insert(words.ctypes.data_as(U32P), w.num_blocks, w.inserts.ctypes.data_as(U64P), w.inserts.size)
    if hashlib.sha256(words.astype("<u4").tobytes()).hexdigest()[:16] != row[6]:
        return False
    out = np.zeros(w.lookups.size, dtype=np.uint8)
    lib.sbbf_oracle_lookup(words.ctypes.data_as(U32P), w.num_blocks, w.lookups.ctypes.data_as(U64P),
                           w.lookups.size, out.ctypes.data_as(U8P))
    if int(out[~w.is_member].sum()) != int(row[5]) or not out[w.is_member].all():
        return False
    return True


def test_unmutated_copy_passes(tmp_path):
    with open(SRC) as f:
        text = f.read()
    assert _pins_pass(_build(text, str(tmp_path / "orig.so")))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    with open(SRC) as f:
        text = f.read()
    old, new = MUTANTS[name]
    assert old in text, f"mutation site for {name} not found in the oracle source"
    lib = _build(text.replace(old, new, 1), str(tmp_path / f"{name}.so"))
    assert not _pins_pass(lib)


# --- the four- and sixteen-lane variants ---------------------------------------

VARIANT_MUTANTS = {
    "extra_seed_typo": ("UINT32_C(0x7ea09599)", "UINT32_C(0x7ea0959b)"),
    "variant_transposed": ("words[(uint64_t)lanes * b + j] |= mask[j];",
                           "words[(uint64_t)num_blocks * j + b] |= mask[j];"),
    "variant_seed_shift": ("seeds[j] = j < 8 ? paper[j] : kExtraSeeds[j - 8];",
                           "seeds[j] = j < 8 ? paper[(j + 4) % 8] : kExtraSeeds[j - 8];"),
    "variant_lookup_skips_last": ("for (uint32_t j = 0; j < lanes; ++j) {\n    if ((words[(uint64_t)lanes * b + j] & mask[j]) == 0) return 0;",
                                  "for (uint32_t j = 0; j + 1 < lanes; ++j) {\n    if ((words[(uint64_t)lanes * b + j] & mask[j]) == 0) return 0;"),
}


def _variant_pins_pass(lib):
    """The variant battery: seeds against the readings (printed constants, then
    SplitMix64 seeded with 16), and brute force with Python integers."""
    from synth import splitmix64, splitmix64_stream

    U64P, U32P, U8P = ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint8)
    lib.sbbf_oracle_variant_seeds.argtypes = [ctypes.c_uint32, U32P]
    lib.sbbf_oracle_variant_insert.argtypes = [U32P, ctypes.c_uint32, ctypes.c_uint32, U64P, ctypes.c_uint64]
    lib.sbbf_oracle_variant_lookup.argtypes = [U32P, ctypes.c_uint32, ctypes.c_uint32, U64P, ctypes.c_uint64, U8P]
    paper = []
    for hi, lo in read_golden("appendix_seeds.txt"):
        paper += [int(lo, 16), int(hi, 16)]
    extra = [(splitmix64(16, i) & M32) | 1 for i in range(8)]
    for lanes in (4, 16):
        want = (paper + extra)[:lanes]
        got = np.zeros(16, dtype=np.uint32)
        lib.sbbf_oracle_variant_seeds(lanes, got.ctypes.data_as(U32P))
        if [int(v) for v in got[:lanes]] != want:
            return False
        B = 5
        hs = splitmix64_stream(95, 40)
        words = np.zeros(lanes * B, dtype=np.uint32)
        lib.sbbf_oracle_variant_insert(words.ctypes.data_as(U32P), lanes, B, hs.ctypes.data_as(U64P), hs.size)
        bits = 0
        for h in hs.tolist():
            b, x = ((h >> 32) * B) >> 32, h & M32
            for j in range(lanes):
                bits |= 1 << (lanes * 32 * b + 32 * j + (((want[j] * x) & M32) >> 27))
        if int.from_bytes(words.astype("<u4").tobytes(), "little") != bits:
            return False
        probes = np.concatenate([hs, splitmix64_stream(96, 300)])
        out = np.zeros(probes.size, dtype=np.uint8)
        lib.sbbf_oracle_variant_lookup(words.ctypes.data_as(U32P), lanes, B, probes.ctypes.data_as(U64P), probes.size,
                                       out.ctypes.data_as(U8P))
        for h, r in zip(probes.tolist(), out.tolist()):
            b, x = ((h >> 32) * B) >> 32, h & M32
            hit = all((bits >> (lanes * 32 * b + 32 * j + (((want[j] * x) & M32) >> 27))) & 1 for j in range(lanes))
            if bool(r) != hit:
                return False
    return True


def test_unmutated_copy_passes_variant_pins(tmp_path):
    with open(SRC) as f:
        text = f.read()
    assert _variant_pins_pass(_build(text, str(tmp_path / "orig_v.so")))


@pytest.mark.parametrize("name", sorted(VARIANT_MUTANTS))
def test_variant_mutant_is_caught(name, tmp_path):
    with open(SRC) as f:
        text = f.read()
    old, new = VARIANT_MUTANTS[name]
    assert old in text, f"mutation site for {name} not found in the oracle source"
    lib = _build(text.replace(old, new, 1), str(tmp_path / f"{name}.so"))
    assert not _variant_pins_pass(lib)
