"""CPU oracle for split block Bloom filters — TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never calls it and shares
no code with it. The arithmetic lives in ``sbbf_oracle.c`` (plain scalar C11,
one thread); this module compiles it with gcc, loads it with ctypes and wraps
it for numpy arrays. ``fpr`` holds the paper's false-positive formula.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sbbf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_sbbf.so")
_lib = None

_U64P = ctypes.POINTER(ctypes.c_uint64)
_U32P = ctypes.POINTER(ctypes.c_uint32)
_U8P = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = True) -> str:
    """Compile the oracle into a shared library next to its source."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-o", tmp, _SRC],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    lib.sbbf_oracle_seeds.argtypes = [_U32P]
    lib.sbbf_oracle_block.argtypes = [ctypes.c_uint64, ctypes.c_uint32]
    lib.sbbf_oracle_block.restype = ctypes.c_uint64
    lib.sbbf_oracle_bit_indices.argtypes = [ctypes.c_uint32, _U32P]
    lib.sbbf_oracle_mask.argtypes = [ctypes.c_uint32, _U32P]
    lib.sbbf_oracle_insert.argtypes = [_U32P, ctypes.c_uint32, _U64P, ctypes.c_uint64]
    lib.sbbf_oracle_contains.argtypes = [_U32P, ctypes.c_uint32, ctypes.c_uint64]
    lib.sbbf_oracle_contains.restype = ctypes.c_int
    lib.sbbf_oracle_lookup.argtypes = [_U32P, ctypes.c_uint32, _U64P, ctypes.c_uint64, _U8P]
    lib.sbbf_oracle_lookup_bits.argtypes = [_U32P, ctypes.c_uint32, _U64P, ctypes.c_uint64, _U32P]
    lib.sbbf_oracle_popcount.argtypes = [_U32P, ctypes.c_uint64]
    lib.sbbf_oracle_popcount.restype = ctypes.c_uint64
    lib.sbbf_oracle_conditional_fpr.argtypes = [_U32P, ctypes.c_uint32]
    lib.sbbf_oracle_conditional_fpr.restype = ctypes.c_double
    lib.sbbf_oracle_index_histogram.argtypes = [ctypes.c_uint64, ctypes.c_uint64, _U64P]
    lib.sbbf_oracle_block_histogram.argtypes = [_U64P, ctypes.c_uint64, ctypes.c_uint32, _U64P]
    lib.sbbf_oracle_key_hash.argtypes = [_U64P, ctypes.c_uint64, _U64P]
    lib.sbbf_oracle_variant_seeds.argtypes = [ctypes.c_uint32, _U32P]
    lib.sbbf_oracle_variant_seeds.restype = ctypes.c_int
    lib.sbbf_oracle_variant_mask.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _U32P]
    lib.sbbf_oracle_variant_insert.argtypes = [_U32P, ctypes.c_uint32, ctypes.c_uint32, _U64P, ctypes.c_uint64]
    lib.sbbf_oracle_variant_contains.argtypes = [_U32P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64]
    lib.sbbf_oracle_variant_contains.restype = ctypes.c_int
    lib.sbbf_oracle_variant_lookup.argtypes = [_U32P, ctypes.c_uint32, ctypes.c_uint32, _U64P, ctypes.c_uint64, _U8P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def _hashes(h) -> np.ndarray:
    a = np.ascontiguousarray(h)
    if a.dtype == np.int64:
        a = a.view(np.uint64)
    if a.dtype != np.uint64:
        raise TypeError("hashes must be uint64 (or an int64 bit view)")
    return a


def _check_filter(words: np.ndarray, num_blocks: int, lanes: int = 8):
    if words.dtype != np.uint32 or not words.flags.c_contiguous:
        raise TypeError("filter words must be a contiguous uint32 array")
    if words.size != lanes * num_blocks:
        raise ValueError(f"filter must hold {lanes} words per block")
    if not (1 <= num_blocks <= 0xFFFFFFFF):
        raise ValueError("num_blocks must be in [1, 2**32 - 1]")


def seeds() -> np.ndarray:
    out = np.zeros(8, dtype=np.uint32)
    _load().sbbf_oracle_seeds(_ptr(out, _U32P))
    return out


def block(h: int, num_blocks: int) -> int:
    return int(_load().sbbf_oracle_block(ctypes.c_uint64(h), ctypes.c_uint32(num_blocks)))


def bit_indices(x: int) -> np.ndarray:
    out = np.zeros(8, dtype=np.uint32)
    _load().sbbf_oracle_bit_indices(ctypes.c_uint32(x), _ptr(out, _U32P))
    return out


def mask(x: int) -> np.ndarray:
    out = np.zeros(8, dtype=np.uint32)
    _load().sbbf_oracle_mask(ctypes.c_uint32(x), _ptr(out, _U32P))
    return out


def new_filter(num_blocks: int) -> np.ndarray:
    return np.zeros(8 * int(num_blocks), dtype=np.uint32)


def insert(words: np.ndarray, num_blocks: int, hashes) -> np.ndarray:
    """OR the masks of ``hashes`` into ``words`` in place; returns ``words``."""
    _check_filter(words, num_blocks)
    h = _hashes(hashes)
    _load().sbbf_oracle_insert(_ptr(words, _U32P), num_blocks, _ptr(h, _U64P), h.size)
    return words


def contains(words: np.ndarray, num_blocks: int, h: int) -> bool:
    _check_filter(words, num_blocks)
    return bool(_load().sbbf_oracle_contains(_ptr(words, _U32P), num_blocks, ctypes.c_uint64(h)))


def lookup(words: np.ndarray, num_blocks: int, hashes) -> np.ndarray:
    """uint8 0/1 per hash."""
    _check_filter(words, num_blocks)
    h = _hashes(hashes)
    out = np.empty(h.size, dtype=np.uint8)
    _load().sbbf_oracle_lookup(_ptr(words, _U32P), num_blocks, _ptr(h, _U64P), h.size, _ptr(out, _U8P))
    return out


def lookup_bits(words: np.ndarray, num_blocks: int, hashes) -> np.ndarray:
    """Packed LSB-first bitmap: uint32[ceil(n/32)]."""
    _check_filter(words, num_blocks)
    h = _hashes(hashes)
    out = np.empty((h.size + 31) // 32, dtype=np.uint32)
    _load().sbbf_oracle_lookup_bits(_ptr(words, _U32P), num_blocks, _ptr(h, _U64P), h.size, _ptr(out, _U32P))
    return out


def select(words: np.ndarray, num_blocks: int, hashes) -> np.ndarray:
    """Ascending indices of the hashes the lookup reports present (the lookup
    routine of the appendix figure, then the positions of its ones)."""
    return np.flatnonzero(lookup(words, num_blocks, hashes)).astype(np.uint32)


def popcount(words: np.ndarray) -> int:
    w = np.ascontiguousarray(words, dtype=np.uint32)
    return int(_load().sbbf_oracle_popcount(_ptr(w, _U32P), w.size))


def conditional_fpr(words: np.ndarray, num_blocks: int) -> float:
    _check_filter(words, num_blocks)
    return float(_load().sbbf_oracle_conditional_fpr(_ptr(words, _U32P), num_blocks))


def index_histogram(x_begin: int, x_end: int) -> np.ndarray:
    """hist[j, k] = #{x in [x_begin, x_end): lane j picks bit k}."""
    hist = np.zeros(256, dtype=np.uint64)
    _load().sbbf_oracle_index_histogram(x_begin, x_end, _ptr(hist, _U64P))
    return hist.reshape(8, 32)


def block_histogram(hashes, num_blocks: int) -> np.ndarray:
    h = _hashes(hashes)
    count = np.zeros(int(num_blocks), dtype=np.uint64)
    _load().sbbf_oracle_block_histogram(_ptr(h, _U64P), h.size, num_blocks, _ptr(count, _U64P))
    return count


def key_hash(keys) -> np.ndarray:
    """The library's hash of 64-bit keys (the 64-bit finalizer of MurmurHash3)."""
    k = _hashes(np.asarray(keys, dtype=np.uint64))
    out = np.empty(k.size, dtype=np.uint64)
    _load().sbbf_oracle_key_hash(_ptr(k, _U64P), k.size, _ptr(out, _U64P))
    return out


def build_filter(num_blocks: int, hashes) -> np.ndarray:
    """A fresh filter holding ``hashes``."""
    return insert(new_filter(num_blocks), num_blocks, hashes)


# ---- block variants with K = 4, 8 or 16 lanes (K words per block) ----------

VARIANT_LANES = (4, 8, 16)


def _check_lanes(lanes: int):
    if lanes not in VARIANT_LANES:
        raise ValueError("lanes must be 4, 8 or 16")


def variant_seeds(lanes: int) -> np.ndarray:
    """Seeds of a K-lane block in word order."""
    _check_lanes(lanes)
    out = np.zeros(16, dtype=np.uint32)
    if _load().sbbf_oracle_variant_seeds(lanes, _ptr(out, _U32P)) != 0:
        raise ValueError("lanes must be 4, 8 or 16")
    return out[:lanes].copy()


def variant_mask(lanes: int, x: int) -> np.ndarray:
    _check_lanes(lanes)
    out = np.zeros(16, dtype=np.uint32)
    _load().sbbf_oracle_variant_mask(lanes, ctypes.c_uint32(x), _ptr(out, _U32P))
    return out[:lanes].copy()


def variant_new_filter(lanes: int, num_blocks: int) -> np.ndarray:
    _check_lanes(lanes)
    return np.zeros(lanes * int(num_blocks), dtype=np.uint32)


def variant_insert(words: np.ndarray, lanes: int, num_blocks: int, hashes) -> np.ndarray:
    """OR the K-word masks of ``hashes`` into a K-lane filter in place."""
    _check_lanes(lanes)
    _check_filter(words, num_blocks, lanes)
    h = _hashes(hashes)
    _load().sbbf_oracle_variant_insert(_ptr(words, _U32P), lanes, num_blocks, _ptr(h, _U64P), h.size)
    return words


def variant_contains(words: np.ndarray, lanes: int, num_blocks: int, h: int) -> bool:
    _check_lanes(lanes)
    _check_filter(words, num_blocks, lanes)
    return bool(_load().sbbf_oracle_variant_contains(_ptr(words, _U32P), lanes, num_blocks, ctypes.c_uint64(h)))


def variant_lookup(words: np.ndarray, lanes: int, num_blocks: int, hashes) -> np.ndarray:
    """uint8 0/1 per hash against a K-lane filter."""
    _check_lanes(lanes)
    _check_filter(words, num_blocks, lanes)
    h = _hashes(hashes)
    out = np.empty(h.size, dtype=np.uint8)
    _load().sbbf_oracle_variant_lookup(_ptr(words, _U32P), lanes, num_blocks, _ptr(h, _U64P), h.size,
                                       _ptr(out, _U8P))
    return out


def variant_build_filter(lanes: int, num_blocks: int, hashes) -> np.ndarray:
    return variant_insert(variant_new_filter(lanes, num_blocks), lanes, num_blocks, hashes)


def replay_requests(blocks, filt, op, key_off, payload, out_off=None):
    """Apply a request log in order, one request at a time: request r inserts
    payload[key_off[r]:key_off[r+1]] into filter filt[r] (op 0) or looks those
    hashes up (op 1). Returns (filters, outputs): the final word arrays and the
    lookup result bytes laid end to end in request order."""
    filters = [new_filter(int(b)) for b in blocks]
    n_out = int(sum(int(key_off[r + 1] - key_off[r]) for r in range(len(op)) if op[r] == 1))
    outputs = np.zeros(n_out, dtype=np.uint8)
    at = 0
    for r in range(len(op)):
        f = int(filt[r])
        h = payload[int(key_off[r]):int(key_off[r + 1])]
        if op[r] == 0:
            insert(filters[f], int(blocks[f]), h)
        else:
            if out_off is not None:
                assert int(out_off[r]) == at
            outputs[at:at + h.size] = lookup(filters[f], int(blocks[f]), h)
            at += h.size
    return filters, outputs
