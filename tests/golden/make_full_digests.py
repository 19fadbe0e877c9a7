"""Write tests/golden/full_digests.txt: SHA-256 digests of the oracle's
results on the two largest workloads, at full size.

    python tests/golden/make_full_digests.py [--jobs 6]

It imports only the oracle (oracle/) and the input generators (synth/), so
every stored value is the oracle's. Both workloads are systems patterns built
on the method (many filters in one launch; a serving loop over resident
filters): their results are defined as the oracle applied filter by filter,
and request by request in arrival order.

* grouped: 2,048 filters, key counts log-uniform in [1e3, 1e6] from G(4),
  ceil(10.5 n / 256) blocks each; filter f inserts its n_f keys and looks up
  its members once each plus 3 n_f fresh hashes, shuffled within the filter.
  Digests: all filters' byte images in filter order, laid end to end; and all
  lookup result bytes (one per lookup, 0 or 1) in workload order.
* serving: 4,096 filters sized from G(5); a log of 200,000 requests (20 %
  inserts, sizes log-uniform 1 .. 65,536, 25 % of a lookup's keys drawn from
  its filter's earlier inserts), replayed by the oracle one request at a time
  in log order. Digests: the final filters' byte images in id order; and the
  lookup result bytes of all lookup requests, laid end to end in log order.
"""

from __future__ import annotations

import argparse
import hashlib
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import grouped_sizes  # noqa: E402
from synth.serving import serving_log  # noqa: E402
from synth.workloads import grouped_filter_inputs  # noqa: E402

OUT = os.path.join(HERE, "full_digests.txt")
GROUPED_FILTERS = 2048
SERVING_FILTERS = 4096
SERVING_REQUESTS = 200_000


def _grouped_one(args):
    n, blocks, f = args
    members, lookups, _ = grouped_filter_inputs(n, f)
    words = oracle.build_filter(int(blocks[f]), members)
    res = oracle.lookup(words, int(blocks[f]), lookups)
    return f, words.tobytes(), res.tobytes(), int(res.sum())


def grouped_digests(jobs: int):
    n, blocks = grouped_sizes(GROUPED_FILTERS)
    hf, hl = hashlib.sha256(), hashlib.sha256()
    nf_bytes = nl_bytes = positives = 0
    with mp.get_context("fork").Pool(jobs) as pool:
        for f, fb, lb, pos in pool.imap(_grouped_one, [(n, blocks, f) for f in range(GROUPED_FILTERS)], chunksize=4):
            hf.update(fb)
            hl.update(lb)
            nf_bytes += len(fb)
            nl_bytes += len(lb)
            positives += pos
    return [("grouped_2048_filters", hf.hexdigest(), nf_bytes, int(n.sum())),
            ("grouped_2048_lookups", hl.hexdigest(), nl_bytes, positives)]


def serving_digests():
    L = serving_log(SERVING_FILTERS, SERVING_REQUESTS)
    filters, outputs = oracle.replay_requests(L.blocks, L.filter, L.op, L.key_off, L.payload, L.out_off)
    hf = hashlib.sha256()
    nf_bytes = 0
    for w in filters:
        b = w.tobytes()
        hf.update(b)
        nf_bytes += len(b)
    inserted = int(L.n[L.op == 0].sum())
    return [("serving_4096x200000_filters", hf.hexdigest(), nf_bytes, inserted),
            ("serving_4096x200000_lookups", hashlib.sha256(outputs.tobytes()).hexdigest(), outputs.size,
             int(outputs.sum()))]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=6)
    a = ap.parse_args()
    oracle.build(force=False)
    rows = []
    t = time.time()
    rows += grouped_digests(a.jobs)
    print(f"grouped done in {time.time() - t:.0f} s", flush=True)
    t = time.time()
    rows += serving_digests()
    print(f"serving done in {time.time() - t:.0f} s", flush=True)
    with open(OUT, "w") as f:
        f.write("# SHA-256 of the oracle's results on the full grouped and serving workloads, written by\n"
                "# tests/golden/make_full_digests.py (oracle/ and synth/ only; see its docstring).\n"
                "# name                          sha256                                                            "
                "bytes        count\n"
                "# count: keys inserted (filters rows), lookups reported present (lookups rows)\n")
        for name, dg, nbytes, count in rows:
            f.write(f"{name:32s}{dg}  {nbytes:<12d} {count}\n")
    print(open(OUT).read())


if __name__ == "__main__":
    main()
