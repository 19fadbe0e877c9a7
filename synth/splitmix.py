"""SplitMix64 streams, vectorised, with a numpy backend and a torch backend.

The generator is the published SplitMix64 (Steele, Lea and Flood, OOPSLA
2014; Vigna's public-domain reference code). Its state advances by the odd
constant GAMMA and each output is the state passed through a bijective
64-bit finaliser, so element ``i`` of stream ``seed`` depends only on
``seed + (i + 1) * GAMMA`` and any slice of a stream can be produced directly.

Published test vector: seed 0 gives 0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4.
"""

from __future__ import annotations

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_MASK64 = (1 << 64) - 1

# numpy chunk so that host generation of very long streams stays within a
# bounded amount of temporary memory.
_CHUNK = 1 << 24


def _as_signed(v: int) -> int:
    v &= _MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


def splitmix64(seed: int, i: int) -> int:
    """Element ``i`` of stream ``seed`` as a Python int (scalar reference)."""
    z = (seed + (i + 1) * GAMMA) & _MASK64
    z = ((z ^ (z >> 30)) * _M1) & _MASK64
    z = ((z ^ (z >> 27)) * _M2) & _MASK64
    return z ^ (z >> 31)


def _mix_numpy_inplace(z: np.ndarray) -> None:
    z ^= z >> np.uint64(30)
    z *= np.uint64(_M1)
    z ^= z >> np.uint64(27)
    z *= np.uint64(_M2)
    z ^= z >> np.uint64(31)


def _stream_numpy(seed: int, n: int, start: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    g = np.uint64(GAMMA)
    s = np.uint64(seed & _MASK64)
    for c0 in range(0, n, _CHUNK):
        c1 = min(n, c0 + _CHUNK)
        z = out[c0:c1]
        z[:] = np.arange(start + c0 + 1, start + c1 + 1, dtype=np.uint64)
        z *= g
        z += s
        _mix_numpy_inplace(z)
    return out


def _lsr_torch(z, k: int):
    # Logical right shift on an int64 bit view: torch's >> is arithmetic.
    import torch

    return torch.bitwise_and(z >> k, (1 << (64 - k)) - 1)


def _stream_torch(seed: int, n: int, start: int, device):
    import torch

    z = torch.arange(start + 1, start + n + 1, dtype=torch.int64, device=device)
    z.mul_(_as_signed(GAMMA)).add_(_as_signed(seed))
    z.bitwise_xor_(_lsr_torch(z, 30)).mul_(_as_signed(_M1))
    z.bitwise_xor_(_lsr_torch(z, 27)).mul_(_as_signed(_M2))
    z.bitwise_xor_(_lsr_torch(z, 31))
    return z


def splitmix64_stream(seed: int, n: int, start: int = 0, backend: str = "numpy", device=None):
    """Elements ``[start, start + n)`` of stream ``seed``.

    backend "numpy" returns a uint64 ndarray; backend "torch" returns an int64
    tensor (the same bits) on ``device``.
    """
    if n < 0 or start < 0:
        raise ValueError("n and start must be non-negative")
    if backend == "numpy":
        return _stream_numpy(seed, n, start)
    if backend == "torch":
        return _stream_torch(seed, n, start, device)
    raise ValueError(f"unknown backend {backend!r}")


def unit_double(x):
    """Map uint64 values to doubles in [0, 1) using their top 53 bits."""
    if isinstance(x, np.ndarray):
        return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return (int(x) >> 11) * (2.0 ** -53)
