"""Seeded synthetic inputs for the split block Bloom filter workloads.

This module is shared by the CPU oracle side and the GPU side. It holds only
the random-number streams and the workload recipes (how many keys, which
stream they come from, how members and non-members are mixed). It holds none
of the filter's arithmetic: no block selection, no masks, no bit tests.

Every array is a stream of uint64 values drawn from SplitMix64 (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014; the
public-domain reference by S. Vigna). Stream ``G(seed)`` is

    G(seed)[i] = mix(seed + (i + 1) * GAMMA  mod 2**64)

with GAMMA = 0x9e3779b97f4a7c15 and ``mix`` the published finaliser. The
paper's inputs are 64-bit hash values of keys (the filter consumes hashes, not
keys), and SplitMix64 output stands in for a good key hash.

Two backends produce bit-identical arrays: ``numpy`` (host, uint64) and
``torch`` (host or device, int64 bit views, since torch arithmetic on uint64 is
limited). Device generation keeps the large workloads quick to build.
"""

from .splitmix import GAMMA, splitmix64, splitmix64_stream, unit_double  # noqa: F401
from .workloads import (  # noqa: F401
    PlainWorkload,
    GroupedWorkload,
    plain_workload,
    grouped_sizes,
    grouped_workload,
    PLAIN_CONFIGS,
)
