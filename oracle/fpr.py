"""False-positive model of split block Bloom filters — TEST INFRASTRUCTURE ONLY.

The analysis section of the paper approximates the false-positive probability
of a filter with a mean of ``a`` distinct hashes per 256-bit block by a Poisson
mixture: a block holding ``i`` hashes has each of its eight 32-bit lanes set at
a given bit with probability 1 - (1 - 1/32)**i, and a non-member is reported
present when all eight of its lane bits are set:

    F(a) = sum_{i >= 0} Poisson_a(i) * (1 - (31/32)**i)**8,   a = 256 n / m

(n distinct hashes, m filter bits). All arithmetic is fp64. The Poisson sum is
taken over i within 40 sqrt(a) + 50 of a; the weight outside is far below fp64
resolution.

For comparison the standard Bloom filter with the same n and m and the best
integer number of hash functions k has false-positive probability
(1 - exp(-k n / m))**k.
"""

from __future__ import annotations

import math


def _poisson_terms(a: float):
    """Yield (i, Poisson_a(i)) for i within 40 sqrt(a) + 50 of a (the weight
    of the terms outside is far below fp64 resolution)."""
    if a < 0:
        raise ValueError("load must be non-negative")
    w = 40.0 * math.sqrt(a) + 50.0
    start = max(0, int(math.floor(a - w)))
    stop = int(math.ceil(a + w))
    for i in range(start, stop + 1):
        # log-space for stability at large a
        if a == 0.0:
            p = 1.0 if i == 0 else 0.0
        else:
            p = math.exp(-a + i * math.log(a) - math.lgamma(i + 1))
        yield i, p


def sbbf_fpr(a: float, lanes: int = 8) -> float:
    """The paper's Poisson-sum approximation F(a), a = mean hashes per block.
    With ``lanes`` = K other than 8 (blocks of K 32-bit words, one bit per
    word) the same argument gives the exponent K in place of 8."""
    total = 0.0
    for i, p in _poisson_terms(a):
        total += p * (1.0 - (31.0 / 32.0) ** i) ** lanes
    return total


def sbbf_fpr_binomial(n: int, num_blocks: int) -> float:
    """The same model with the exact Binomial(n, 1/B) block load in place of
    the Poisson approximation (uniform block choice)."""
    if num_blocks < 1:
        raise ValueError("num_blocks must be >= 1")
    q = 1.0 / num_blocks
    a = n * q
    stop = min(n, int(math.ceil(a + 40.0 * math.sqrt(a) + 50.0)))
    total = 0.0
    for i in range(stop + 1):
        if q == 1.0:
            p = 1.0 if i == n else 0.0
        else:
            logp = (math.lgamma(n + 1) - math.lgamma(i + 1) - math.lgamma(n - i + 1)
                    + i * math.log(q) + (n - i) * math.log1p(-q))
            p = math.exp(logp)
        total += p * (1.0 - (31.0 / 32.0) ** i) ** 8
    return total


def standard_bloom_fpr(bits_per_key: float, k: int) -> float:
    """Standard Bloom filter with k hash functions: (1 - exp(-k / bits_per_key))**k."""
    return (1.0 - math.exp(-k / bits_per_key)) ** k


def standard_bloom_best(bits_per_key: float):
    """(fpr, k) for the best integer k."""
    best = None
    for k in range(1, 64):
        f = standard_bloom_fpr(bits_per_key, k)
        if best is None or f < best[0]:
            best = (f, k)
    return best


def load_for_fpr(target: float, lo: float = 1e-3, hi: float = 256.0) -> float:
    """Invert F by bisection: the load a with F(a) = target (F increases with a)."""
    if not (sbbf_fpr(lo) < target < sbbf_fpr(hi)):
        raise ValueError("target outside the bracket")
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if sbbf_fpr(mid) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def blocks_for_fpr(n: int, fpr: float, max_blocks: int = 2**32 - 1, lanes: int = 8) -> int:
    """Smallest number of blocks B >= 1 with sbbf_fpr(n / B) <= fpr, by
    bisection (F grows with the load n / B). 0 when even max_blocks is not
    enough."""
    if not (0.0 < fpr < 1.0):
        raise ValueError("fpr must be in (0, 1)")
    if n == 0:
        return 1
    if sbbf_fpr(n / max_blocks, lanes) > fpr:
        return 0
    if sbbf_fpr(float(n), lanes) <= fpr:
        return 1
    lo, hi = 1, max_blocks
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if sbbf_fpr(n / mid, lanes) <= fpr:
            hi = mid
        else:
            lo = mid
    return hi

