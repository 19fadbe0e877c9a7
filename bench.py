#!/usr/bin/env python3
"""Benchmark of the split block Bloom filter hot path on one MI355X.

One step is one pass of the single-filter hot path over one batch: zero the
filter, insert every hash of the batch, look up every probe of the batch
(hash streaming, block selection, mask, insert, lookup). The default workload
is the 100M-key geometry of the paper's evaluation table: 4,194,304 blocks
(128 MiB), 1e8 inserted hashes, 2e8 lookups at a 10 % member rate, all
synthetic SplitMix64 hashes resident in device memory before timing starts.

Prints one JSON line. ``value`` is total keys (inserts + lookups) per second
over the timed steps; per-operation rates, the roofline of the dominant
operation (from HIP events recorded on the launch stream around every library
call in the timed region; an operation may be several kernels), the measured
gather / atomic / streaming ceilings and the CPU oracle's rate on a bounded
sample are reported beside it, then the grouped workload (2,048 filters, one
graph launch against one plain launch per filter) and the serving workload
(4,096 resident filters, Poisson request stream, p50/p99 latency).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "G lookups/s & G inserts/s at 100M keys vs roofline; serving p50/p99 latency"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# Algorithmic bytes per key: hash in (8 B) + the 32-byte block + result out.
LOOKUP_BYTES_PER_KEY = 8 + 32 + 1
INSERT_BYTES_PER_KEY = 8 + 32
PAPER_CONTEXT = {"insert_Mps": 32, "lookup_Mps": 43, "hardware": "not stated (CPU, AVX2 code)",
                 "source": "evaluation table, 100M elements"}


# Sources of the single-filter path's kernels and their launch choices: a
# change to any of them invalidates committed hardware-counter traffic.
PLAIN_SOURCES = ("sbbf_device.h", "internal.h", "plain_kernels.hip", "partition_kernels.hip", "api.cpp")
# The same for the grouped graph's kernels.
GROUPED_SOURCES = ("sbbf_device.h", "internal.h", "grouped.hip")


def _kernel_source_digest(sources=PLAIN_SOURCES) -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2101_01719_amd", "csrc")
    for name in sources:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def _traffic(kernel: str, workload: str, sources=PLAIN_SOURCES):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None when
    none exist or the kernels changed since they were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_digest") != _kernel_source_digest(sources):
        return None
    return t.get("hbm_bytes_per_launch")


def _short_kernel(name: str) -> str:
    import re

    name = name.replace("(anonymous namespace)::", "").replace("void ", "").replace("sbbf::", "")
    return re.sub(r"\(.*$", "", name)


def _counter_rows(path: str, counter: str):
    """(dispatch id, kernel, grid, value in KiB) of one counter, in dispatch order."""
    import csv

    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])))
    rows.sort()
    return rows


def _traffic_from_counters(fetch_csv: str, write_csv: str, workload: str, copy_mib: int, commands) -> int:
    """Turn two rocprofv3 --pmc runs of the same bench command (FETCH_SIZE, then
    WRITE_SIZE; KiB per dispatch) into HBM bytes per insert and per lookup
    call, each counter scaled by what it reads for the plain device copy of
    copy_mib MiB that the command ran first (a kernel of known traffic)."""
    fetch, write = _counter_rows(fetch_csv, "FETCH_SIZE"), _counter_rows(write_csv, "WRITE_SIZE")
    if [r[:3] for r in fetch] != [r[:3] for r in write]:
        raise SystemExit("the two counter runs did not dispatch the same kernels")
    others = sorted({_short_kernel(r[1]) for r in fetch if _short_kernel(r[1]).startswith(("select_", "union_"))})
    if others:
        raise SystemExit(f"the counter runs also dispatched {others}: collect them with --no-select so that "
                         "every call averaged is a step's insert or lookup")
    want_kib = copy_mib * 1024.0
    copies = [i for i, r in enumerate(write) if "copy" in r[1].lower() and abs(r[3] - want_kib) < 0.05 * want_kib]
    if not copies:
        raise SystemExit(f"no copy dispatch writing about {copy_mib} MiB found")
    ci = copies[0]
    f_fetch, f_write = want_kib / fetch[ci][3], want_kib / write[ci][3]
    if workload == "grouped_2048":
        return _grouped_traffic(fetch, write, ci, f_fetch, f_write, copy_mib, commands)
    # Library dispatches after the copy: fill (clear), then the insert
    # kernels (a bucketed insert starts with a fill of its overflow count and
    # ends with the overflow pass; a counted one ends with the slice insert),
    # then the lookup kernels (a count-free lookup starts with a fill of its
    # overflow count and ends with the unpermute and the overflow pass; a
    # counted one ends with the unpermute), step after step.
    ops = {"insert": [], "lookup": []}
    cur, cur_op = [], "insert"
    for i in range(ci + 1, len(fetch)):
        name = _short_kernel(fetch[i][1])
        if not name.startswith(("part_", "insert_", "lookup_kernel", "fill_kernel")):
            continue
        if name.startswith("fill_kernel"):
            cur, cur_op = [], "insert"
            continue
        if name.startswith("part_overflow_lookup") and ops["lookup"] and not cur:
            ops["lookup"][-1].append((name, fetch[i][3], write[i][3]))  # the count-free lookup's last pass
            continue
        cur.append((name, fetch[i][3], write[i][3]))
        if name.startswith(("part_slice_insert", "part_overflow_insert", "insert_")):
            ops["insert"].append(cur)
            cur, cur_op = [], "lookup"
        elif name.startswith(("part_unpermute", "lookup_kernel")):
            ops["lookup"].append(cur)
            cur = []
    out = {}
    for op, calls in ops.items():
        if not calls:
            continue
        per_kernel = {}
        for call in calls:
            for name, fk, wk in call:
                d = per_kernel.setdefault(name, [0.0, 0.0, 0])
                d[0] += fk
                d[1] += wk
                d[2] += 1
        kernels = {k: {"fetch_kib_per_call": v[0] / len(calls), "write_kib_per_call": v[1] / len(calls),
                       "dispatches_per_call": v[2] / len(calls)} for k, v in per_kernel.items()}
        hbm = sum(1024.0 * (k["fetch_kib_per_call"] * f_fetch + k["write_kib_per_call"] * f_write)
                  for k in kernels.values())
        out[op] = {
            "workload": workload,
            "operation": op,
            "calls_averaged": len(calls),
            "hbm_bytes_per_launch": int(round(hbm)),
            "kernels": kernels,
            "calibration": {"copy_mib": copy_mib, "copy_fetch_kib": fetch[ci][3], "copy_write_kib": write[ci][3],
                            "fetch_scale": f_fetch, "write_scale": f_write},
            "commands": list(commands),
            "kernel_source_digest": _kernel_source_digest(),
        }
        path = os.path.join(ROOT, "profiles", f"traffic_{op}_{workload}.json")
        with open(path, "w") as fh:
            json.dump(out[op], fh, indent=1)
            fh.write("\n")
    print(json.dumps({op: v["hbm_bytes_per_launch"] for op, v in out.items()}))
    return 0


def _grouped_traffic(fetch, write, ci, f_fetch, f_write, copy_mib, commands) -> int:
    """HBM bytes per grouped graph launch: the grouped_* kernels from each
    reset node to the gather lookup node that ends the graph, averaged over
    launches (the per-filter baseline's and the digest's kernels are not
    grouped_* and are left out)."""
    launches, cur = [], None
    for i in range(ci + 1, len(fetch)):
        name = _short_kernel(fetch[i][1])
        if not name.startswith("grouped_"):
            continue
        if name.startswith("grouped_reset"):
            cur = []
        if cur is None:
            continue
        cur.append((name, fetch[i][3], write[i][3]))
        if name.startswith("grouped_lookup_kernel"):
            launches.append(cur)
            cur = None
    if not launches:
        raise SystemExit("no grouped graph launch found after the copy")
    per_kernel = {}
    for call in launches:
        for name, fk, wk in call:
            d = per_kernel.setdefault(name, [0.0, 0.0, 0])
            d[0] += fk
            d[1] += wk
            d[2] += 1
    kernels = {k: {"fetch_kib_per_call": v[0] / len(launches), "write_kib_per_call": v[1] / len(launches),
                   "dispatches_per_call": v[2] / len(launches)} for k, v in per_kernel.items()}
    hbm = sum(1024.0 * (k["fetch_kib_per_call"] * f_fetch + k["write_kib_per_call"] * f_write)
              for k in kernels.values())
    out = {
        "workload": "grouped_2048",
        "operation": "graph",
        "calls_averaged": len(launches),
        "hbm_bytes_per_launch": int(round(hbm)),
        "kernels": kernels,
        "calibration": {"copy_mib": copy_mib, "copy_fetch_kib": fetch[ci][3], "copy_write_kib": write[ci][3],
                        "fetch_scale": f_fetch, "write_scale": f_write},
        "commands": list(commands),
        "kernel_source_digest": _kernel_source_digest(GROUPED_SOURCES),
    }
    with open(os.path.join(ROOT, "profiles", "traffic_graph_grouped_2048.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps({"graph": out["hbm_bytes_per_launch"]}))
    return 0


def _kernel_summary(stats_csv: str, out_md: str, title: str, command: str) -> int:
    """Short markdown table of the library's kernels from a rocprofv3
    kernel_stats.csv."""
    import csv

    lines = [f"# {title}", "", "Command (from the repository root, on one MI355X):", "", "```", command, "```", "",
             "Source: rocprofv3 `kernel_stats.csv` of that run; library kernels only (the rest are torch kernels "
             "of the input generator and the copy).", "",
             "| kernel | calls | average (us) | min (us) | max (us) | total (ms) |", "|---|---:|---:|---:|---:|---:|"]
    with open(stats_csv) as f:
        for r in csv.DictReader(f):
            if "sbbf" not in r["Name"]:
                continue
            lines.append(f"| `{_short_kernel(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                         f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                         f"{float(r['TotalDurationNs']) / 1e6:.2f} |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))
    return 0


def _counter_summary(out_md: str, csvs, title: str, commands) -> int:
    """Markdown table of hardware counters per library kernel from one or more
    rocprofv3 --pmc runs (counter_collection.csv): each counter's mean per
    dispatch, and the derived L2 hit rate (TCC_HIT / (TCC_HIT + TCC_MISS)),
    share of 32-byte memory read requests, and atomics per dispatch."""
    import collections
    import csv

    per = collections.OrderedDict()  # kernel -> counter -> [sum, dispatches]
    for path in csvs:
        with open(path) as f:
            for r in csv.DictReader(f):
                if "sbbf" not in r["Kernel_Name"]:
                    continue
                k = _short_kernel(r["Kernel_Name"])
                acc = per.setdefault(k, collections.OrderedDict()).setdefault(r["Counter_Name"], [0.0, 0])
                acc[0] += float(r["Counter_Value"])
                acc[1] += 1
    names = []
    for cs in per.values():
        for c in cs:
            if c not in names:
                names.append(c)

    def mean(cs, c):
        return cs[c][0] / cs[c][1] if c in cs and cs[c][1] else None

    lines = [f"# {title}", "", "Commands (from the repository root, on one MI355X; one counter set per run):", "",
             "```"] + list(commands) + ["```", "",
             "Source: rocprofv3 `counter_collection.csv` of those runs; library kernels only. Counters are means per "
             "dispatch over every dispatch of the kernel in the run. L2 hit = TCC_HIT / (TCC_HIT + TCC_MISS); "
             "32B rd = TCC_EA0_RDREQ_32B / TCC_EA0_RDREQ (share of the L2's memory read requests that are 32 "
             "bytes); a dash: not counted for that kernel.", "",
             "| kernel | " + " | ".join(names) + " | L2 hit | 32B rd |",
             "|---|" + "---:|" * (len(names) + 2)]
    for k, cs in per.items():
        cells = []
        for c in names:
            v = mean(cs, c)
            cells.append("-" if v is None else f"{v:.4g}")
        hit, miss = mean(cs, "TCC_HIT"), mean(cs, "TCC_MISS")
        rd, rd32 = mean(cs, "TCC_EA0_RDREQ"), mean(cs, "TCC_EA0_RDREQ_32B")
        hr = f"{hit / (hit + miss):.3f}" if hit is not None and miss is not None and hit + miss > 0 else "-"
        r32 = f"{rd32 / rd:.3f}" if rd and rd32 is not None else "-"
        lines.append(f"| `{k}` | " + " | ".join(cells) + f" | {hr} | {r32} |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))
    return 0


def _ensure_built():
    lib = os.path.join(ROOT, "paper_2101_01719_amd", "libsbbf.so")
    if not os.path.exists(lib):
        from paper_2101_01719_amd import build

        build.build()


def _select(P, torch, f, lookups, ref_out, launch, reps=5):
    """Lookup with stream compaction over the step's lookups (the filter as
    the last step left it): time per call, and the indices must equal the
    positions of the byte lookup's ones."""
    n = lookups.numel()
    idx = torch.empty(n, dtype=torch.int32, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    P.sbbf_lookup_select(f.handle, lookups, idx, cnt, launch=launch)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        P.sbbf_lookup_select(f.handle, lookups, idx, cnt, launch=launch)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    c = int(cnt.item())
    ref = torch.nonzero(ref_out).flatten()
    ok = c == ref.numel() and bool(torch.equal(idx[:c].to(torch.int64), ref))
    return {"keys": n, "selected": c, "ms": ms, "gkeys_per_s": n / (ms / 1e3) / 1e9, "matches_lookup": ok}


def _union(P, torch, f, reps=10):
    """Union of the step's filter into a second filter of the same size:
    time per call and HBM rate (two filters read, one written)."""
    g = P.Filter(P.sbbf_num_blocks(f.handle))
    g.union(f)
    torch.cuda.synchronize()
    ok = bool(torch.equal(g.words, f.words))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.union(f)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 3 * 32 * P.sbbf_num_blocks(f.handle)
    g.close()
    return {"filter_bytes": nbytes // 3, "ms": ms, "GBps": nbytes / (ms / 1e3) / 1e9, "correct": ok}


def _keys(P, torch, f, w, ins_launch, look_launch, reps=5):
    """The same step with the hashes taken as keys (hashed on the device as
    they are loaded): clear, insert_keys, lookup_keys; median of reps."""
    import numpy as np

    out = torch.empty(w.lookups.numel(), dtype=torch.uint8, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    def step(rec):
        f.clear()
        if rec:
            ev[0].record()
        P.sbbf_insert_keys(f.handle, w.inserts, launch=ins_launch)
        if rec:
            ev[1].record()
        P.sbbf_lookup_keys(f.handle, w.lookups, out, launch=look_launch)
        if rec:
            ev[2].record()

    step(False)
    torch.cuda.synchronize()
    t_ins, t_look = [], []
    for _ in range(reps):
        step(True)
        torch.cuda.synchronize()
        t_ins.append(ev[0].elapsed_time(ev[1]))
        t_look.append(ev[1].elapsed_time(ev[2]))
    ins_ms, look_ms = float(np.median(t_ins)), float(np.median(t_look))
    members_ok = bool(out[w.is_member].all().item())
    n = w.inserts.numel() + w.lookups.numel()
    return {"insert_ms": ins_ms, "lookup_ms": look_ms, "gkeys_per_s": n / ((ins_ms + look_ms) / 1e3) / 1e9,
            "members_all_found": members_ok}


def _variants(P, torch, w, reps=5):
    """The same step on the block variants with four and sixteen 32-bit words
    per block, each in a 128 MiB filter (the same bytes per key as the
    eight-word filter): clear, insert, lookup with the library's strategies
    (median of reps); measured false-positive rate against the model with K
    words per block."""
    import numpy as np

    out = torch.empty(w.lookups.numel(), dtype=torch.uint8, device="cuda")
    res = {}
    for lanes in (4, 16):
        B = (128 << 20) // (4 * lanes)
        f = P.Filter(B, lanes=lanes)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

        def step(rec):
            f.clear()
            if rec:
                ev[0].record()
            f.insert(w.inserts)
            if rec:
                ev[1].record()
            f.lookup(w.lookups, out=out)
            if rec:
                ev[2].record()

        step(False)
        torch.cuda.synchronize()
        t_ins, t_look = [], []
        for _ in range(reps):
            step(True)
            torch.cuda.synchronize()
            t_ins.append(ev[0].elapsed_time(ev[1]))
            t_look.append(ev[1].elapsed_time(ev[2]))
        ins_ms, look_ms = float(np.median(t_ins)), float(np.median(t_look))
        n_ins, n_look = w.inserts.numel(), w.lookups.numel()
        fpr = float(out[~w.is_member].float().mean().item())
        res[str(lanes)] = {
            "num_blocks": B, "block_bytes": 4 * lanes,
            "insert_ms": ins_ms, "lookup_ms": look_ms,
            "gkeys_per_s": (n_ins + n_look) / ((ins_ms + look_ms) / 1e3) / 1e9,
            "insert_strategy": P.sbbf_auto_insert_strategy(f.handle, n_ins),
            "lookup_strategy": P.sbbf_auto_lookup_strategy(f.handle, n_look),
            "lookup_GBps": n_look * (8 + 4 * lanes + 1) / (look_ms / 1e3) / 1e9,
            "insert_GBps": n_ins * (8 + 4 * lanes) / (ins_ms / 1e3) / 1e9,
            "false_positive_rate": fpr, "model_fpr": P.sbbf_fpr_model_variant(n_ins / B, lanes),
            "members_all_found": bool(out[w.is_member].all().item()),
        }
        f.close()
    return res


def _strategy_sweep(out_md: str) -> int:
    """Rates of both lookup and both insert strategies over filter sizes and
    batch sizes (about 24 keys per block inserted first, as in the 100M-key
    workload), with the strategy the library picks for each point."""
    _ensure_built()
    import torch

    import paper_2101_01719_amd as P
    from synth import splitmix64_stream

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    torch.cuda.set_device(0)
    h = splitmix64_stream(1, 64_000_000, backend="torch", device="cuda")
    o = torch.empty(h.numel(), dtype=torch.uint8, device="cuda")
    look_names, ins_names = {1: "gather", 2: "partitioned"}, {1: "atomic32", 4: "partitioned"}
    rows = []
    for mib in (1, 2, 4, 8, 16, 32, 64):
        B = (mib << 20) // 32
        f = P.Filter(B)
        f.insert(h[: B * 24])
        torch.cuda.synchronize()
        for n in (1 << 20, 4 << 20, 16 << 20, 64_000_000):
            x, y = h[:n], o[:n]
            lg = n / timed(lambda: f.lookup(x, out=y, launch=dict(strategy=1))) / 1e6
            lp = n / timed(lambda: f.lookup(x, out=y, launch=dict(strategy=2))) / 1e6
            ia = n / timed(lambda: f.insert(x, launch=dict(strategy=1))) / 1e6
            ip = n / timed(lambda: f.insert(x, launch=dict(strategy=4))) / 1e6
            al, ai = P.sbbf_auto_lookup_strategy(f.handle, n), P.sbbf_auto_insert_strategy(f.handle, n)
            rows.append((mib, n, lg, lp, look_names[al], ia, ip, ins_names[ai]))
            print(json.dumps({"mib": mib, "n": n, "lookup_gather": lg, "lookup_partitioned": lp, "auto_lookup": al,
                              "insert_atomic32": ia, "insert_partitioned": ip, "auto_insert": ai}), flush=True)
        f.close()
    # Filters above 128 MiB (one level up to 4,096 slices of 128 KiB, two levels above), with 64M keys inserted
    # and batches of 64M and 200M keys.
    del h, o
    h = splitmix64_stream(2, 200_000_000, backend="torch", device="cuda")
    o = torch.empty(h.numel(), dtype=torch.uint8, device="cuda")
    big = []
    for mib in (256, 512, 1536, 4096):
        B = (mib << 20) // 32
        f = P.Filter(B)
        f.insert(h[:64_000_000])
        torch.cuda.synchronize()
        for n in (64_000_000, 200_000_000):
            x, y = h[:n], o[:n]
            lg = n / timed(lambda: f.lookup(x, out=y, launch=dict(strategy=1)), reps=3) / 1e6
            lp = n / timed(lambda: f.lookup(x, out=y, launch=dict(strategy=2)), reps=3) / 1e6
            ia = n / timed(lambda: f.insert(x, launch=dict(strategy=1)), reps=3) / 1e6
            ip = n / timed(lambda: f.insert(x, launch=dict(strategy=4)), reps=3) / 1e6
            al, ai = P.sbbf_auto_lookup_strategy(f.handle, n), P.sbbf_auto_insert_strategy(f.handle, n)
            big.append((mib, n, lg, lp, look_names[al], ia, ip, ins_names[ai]))
            print(json.dumps({"mib": mib, "n": n, "lookup_gather": lg, "lookup_partitioned": lp, "auto_lookup": al,
                              "insert_atomic32": ia, "insert_partitioned": ip, "auto_insert": ai}), flush=True)
        f.close()
    with open(out_md, "w") as fh:
        fh.write("# Strategy sweep: gather vs partitioned lookup, atomic vs partitioned insert\n\n")
        fh.write("Command (from the repository root, on one MI355X):\n\n```\npython bench.py --strategy-sweep "
                 + out_md + "\n```\n\n")
        fh.write("G keys/s per strategy (HIP events around each call, mean of 5 after one warm-up), one filter of the "
                 "given size holding about 24 keys per block, SplitMix64 hashes (seed 1); `auto` is what the library "
                 "picks for that filter and batch (SBBF_*_AUTO). The faster strategy of each pair is in bold.\n\n")
        fh.write("| filter | keys | lookup gather | lookup partitioned | auto | insert atomic32 | insert partitioned "
                 "| auto |\n|---:|---:|---:|---:|---|---:|---:|---|\n")
        b = lambda v, w: f"**{v:.1f}**" if v >= w else f"{v:.1f}"
        for mib, n, lg, lp, al, ia, ip, ai in rows:
            fh.write(f"| {mib} MiB | {n:,} | {b(lg, lp)} | {b(lp, lg)} | {al} | {b(ia, ip)} | {b(ip, ia)} | {ai} |\n")
        fh.write("\nLarger filters (2,048 to 4,096 slices of 128 KiB take one level, more take two), 64M keys "
                 "inserted first (SplitMix64 seed 2), mean of 3 calls after one warm-up:\n\n")
        fh.write("| filter | keys | lookup gather | lookup partitioned | auto | insert atomic32 | insert partitioned "
                 "| auto |\n|---:|---:|---:|---:|---|---:|---:|---|\n")
        for mib, n, lg, lp, al, ia, ip, ai in big:
            fh.write(f"| {mib} MiB | {n:,} | {b(lg, lp)} | {b(lp, lg)} | {al} | {b(ia, ip)} | {b(ip, ia)} | {ai} |\n")
    return 0


def _cpu_baseline(w):
    """The oracle, untuned, on the host: all inserts into the full-size filter,
    then the first half of the lookups. One thread."""
    import numpy as np

    import oracle

    ins = w.inserts.cpu().numpy().view(np.uint64)
    n_look = w.lookups.numel() // 2
    look = w.lookups[:n_look].cpu().numpy().view(np.uint64)
    words = oracle.new_filter(w.num_blocks)
    t0 = time.perf_counter()
    oracle.insert(words, w.num_blocks, ins)
    t1 = time.perf_counter()
    oracle.lookup(words, w.num_blocks, look)
    t2 = time.perf_counter()
    keys = ins.size + look.size
    return {
        "value": keys / (t2 - t0) / 1e9,
        "unit": "G keys/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"all {ins.size:,} inserts into the {w.num_blocks:,}-block filter, then the first "
                  f"{look.size:,} of the {w.lookups.numel():,} lookups (insert {t1 - t0:.2f} s, "
                  f"lookup {t2 - t1:.2f} s)",
        "insert_gkeys_per_s": ins.size / (t1 - t0) / 1e9,
        "lookup_gkeys_per_s": look.size / (t2 - t1) / 1e9,
        "host_cpu": _host_cpu(),
    }


def _host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _ceilings(P, torch, w, look_launch, ins_launch, reps=5):
    """Measured ceilings with the same access pattern and launch shape:
    random 32-byte gather (lookup without the mask), random 8 x 32-bit atomic
    OR (insert without the mask), streaming (8 B in, 1 B out), and a plain
    device copy."""
    buf = torch.full((8 * w.num_blocks,), 1, dtype=torch.int32, device="cuda")
    out = torch.empty(w.lookups.numel(), dtype=torch.uint8, device="cuda")
    res = {}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps / 1e3

    t = timed(lambda: P.sbbf_bench_gather(buf, w.num_blocks, w.lookups, out, launch=look_launch))
    res["gather_gkeys_per_s"] = w.lookups.numel() / t / 1e9
    res["gather_GBps"] = LOOKUP_BYTES_PER_KEY * w.lookups.numel() / t / 1e9
    for name, strat in (("atomic32", 1), ("atomic64", 2)):
        launch = dict(ins_launch, strategy=strat)
        t = timed(lambda: P.sbbf_bench_atomic(buf, w.num_blocks, w.inserts, launch=launch))
        res[f"{name}_gkeys_per_s"] = w.inserts.numel() / t / 1e9
        res[f"{name}_GBps"] = INSERT_BYTES_PER_KEY * w.inserts.numel() / t / 1e9
    t = timed(lambda: P.sbbf_bench_stream(w.lookups, out, launch=look_launch))
    res["stream_gkeys_per_s"] = w.lookups.numel() / t / 1e9
    res["stream_GBps"] = 9 * w.lookups.numel() / t / 1e9
    # A plain device copy of the lookup hashes (equal read and write
    # traffic): the practical bandwidth of a read-and-write streaming pass.
    dst = torch.empty_like(w.lookups)
    t = timed(lambda: dst.copy_(w.lookups))
    res["copy_GBps"] = 2 * 8 * w.lookups.numel() / t / 1e9
    del buf, out, dst
    return res


def _plain_small(P, torch, name, reps=20):
    """One of the evaluation table's smaller geometries (4,096 blocks with 1e5
    inserts, 32,768 blocks with 1e6): median insert and lookup times over
    `reps` steps with the library's default strategies, and the filter bytes
    and lookup bytes of the last step compared with the oracle."""
    import numpy as np

    import oracle
    from synth import plain_workload

    w = plain_workload(name, backend="torch", device="cuda")
    f = P.Filter(w.num_blocks)
    out = torch.empty(w.lookups.numel(), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    t_ins, t_look = [], []
    for k in range(reps + 3):
        f.clear(stream)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(stream)
        f.insert(w.inserts, stream=stream)
        ev[1].record(stream)
        f.lookup(w.lookups, out=out, stream=stream)
        ev[2].record(stream)
        torch.cuda.synchronize()
        if k >= 3:
            t_ins.append(ev[0].elapsed_time(ev[1]))
            t_look.append(ev[1].elapsed_time(ev[2]))
    ins_ms, look_ms = float(np.median(t_ins)), float(np.median(t_look))
    ins_h = w.inserts.cpu().numpy().view(np.uint64)
    ref = oracle.build_filter(w.num_blocks, ins_h)
    ref_out = oracle.lookup(ref, w.num_blocks, w.lookups.cpu().numpy().view(np.uint64))
    same = bool(np.array_equal(f.words.cpu().numpy().view(np.uint32), ref) and
                np.array_equal(out.cpu().numpy(), ref_out))
    n_ins, n_look = w.inserts.numel(), w.lookups.numel()
    fp = int(out[~w.is_member].sum().item())
    res = {
        "workload": f"{name}: {w.num_blocks:,} blocks, {n_ins:,} inserts, {n_look:,} lookups",
        "insert_ms": ins_ms, "lookup_ms": look_ms,
        "insert_gkeys_per_s": n_ins / ins_ms / 1e6, "lookup_gkeys_per_s": n_look / look_ms / 1e6,
        "insert_strategy": int(P.sbbf_auto_insert_strategy(f.handle, n_ins)),
        "lookup_strategy": int(P.sbbf_auto_lookup_strategy(f.handle, n_look)),
        "false_positive_rate": fp / max(1, int((~w.is_member).sum().item())),
        "identical_to_oracle": same,
    }
    f.close()
    return res


def _grouped(P, torch, autotune=True, reps=5, cfg=None):
    """The grouped workload: 2,048 filters with key counts log-uniform in
    [1e3, 1e6], 10.5 bits per key, four lookups per inserted key at a 25 %
    member rate; one graph launch against one plain launch per filter per
    operation, same data, identical results (digest of every filter and every
    output byte)."""
    import numpy as np

    from synth import grouped_workload

    w = grouped_workload(num_filters=2048, backend="torch", device="cuda")
    filters = [P.Filter(int(b)) for b in w.blocks]
    g = P.Group(filters, w.ins_off, w.look_off, cfg)
    out = torch.empty(w.lookups.numel(), dtype=torch.uint8, device="cuda")
    tuned = g.autotune(w.inserts, w.lookups, out, reps=3) if autotune and cfg is None else g.config()

    def timed(fn, n):
        ts = []
        for k in range(n + 1):
            g.clear()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            if k:
                ts.append(e0.elapsed_time(e1))
        return sorted(ts)[len(ts) // 2]

    graph_ms = timed(lambda: g.run(w.inserts, w.lookups, out), reps)
    d_graph = g.digest(out)
    per_ms = timed(lambda: g.run_per_filter(w.inserts, w.lookups, out), max(2, reps // 2))
    d_per = g.digest(out)
    # The same batch through a capacity plan: key ranges from device offsets.
    cap = P.Group.with_capacity(filters, np.diff(w.ins_off), np.diff(w.look_off), tuned)
    d_ioff = torch.from_numpy(np.asarray(w.ins_off, dtype=np.int64)).cuda()
    d_loff = torch.from_numpy(np.asarray(w.look_off, dtype=np.int64)).cuda()
    t_host = []

    def cap_run():
        t = time.perf_counter()
        cap.run_offsets(w.inserts, d_ioff, w.lookups, d_loff, out)
        t_host.append(time.perf_counter() - t)

    cap_ms = timed(cap_run, reps)
    cap_identical = g.digest(out) == d_graph and cap.check() is None
    cap_counters = cap.counters()
    cap.close()
    n_ins, n_look = int(w.ins_off[-1]), int(w.look_off[-1])
    keys = n_ins + n_look
    alg_bytes = INSERT_BYTES_PER_KEY * n_ins + LOOKUP_BYTES_PER_KEY * n_look
    gbps = alg_bytes / (graph_ms / 1e3) / 1e9
    res = {
        "workload": "2,048 filters, key counts log-uniform in [1e3, 1e6] (SplitMix64 seed 4), 10.5 bits/key, "
                    f"{int(w.ins_off[-1]):,} inserts and {int(w.look_off[-1]):,} lookups (25 % members)",
        "graph_ms": graph_ms,
        "per_filter_ms": per_ms,
        "speedup_vs_per_filter": per_ms / graph_ms,
        "gkeys_per_s": keys / graph_ms / 1e6,
        "per_filter_gkeys_per_s": keys / per_ms / 1e6,
        "identical_results": d_graph == d_per,
        "per_filter_strategies": "library defaults per filter (sbbf_insert_batch / sbbf_lookup_batch)",
        "roofline": {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbps / HBM_PEAK_GBS, "traffic": _traffic("graph", "grouped_2048", GROUPED_SOURCES),
                     "bytes_per_key": {"insert": INSERT_BYTES_PER_KEY, "lookup": LOOKUP_BYTES_PER_KEY},
                     "algorithmic_bytes": alg_bytes, "avg_ms": graph_ms, "kernel": "grouped graph launch"},
        "capacity_plan": {"graph_ms": cap_ms, "identical_results": cap_identical,
                          "host_us_per_run": 1e6 * float(np.median(t_host)), "counters": cap_counters},
        "config": tuned,
    }
    g.close()
    del filters, out, w
    torch.cuda.empty_cache()
    return res


class _PinnedHost:
    """Mapped pinned host memory (hipHostMalloc from the HIP runtime torch
    loaded), holding a copy of a device tensor; ``device_ptr`` is the address
    kernels read it through (across PCIe)."""

    def __init__(self, torch, t):
        import ctypes
        import re

        import numpy as np

        path = next(p for p in re.findall(r"\S*libamdhip64\.so\S*", open("/proc/self/maps").read()))
        self.hip = ctypes.CDLL(path)
        self.nbytes = t.numel() * t.element_size()
        self.host = ctypes.c_void_p()
        mapped_portable = 0x2 | 0x1
        if self.hip.hipHostMalloc(ctypes.byref(self.host), ctypes.c_size_t(self.nbytes), mapped_portable) != 0:
            raise RuntimeError("hipHostMalloc failed")
        dev = ctypes.c_void_p()
        if self.hip.hipHostGetDevicePointer(ctypes.byref(dev), self.host, 0) != 0:
            raise RuntimeError("hipHostGetDevicePointer failed")
        self.device_ptr = dev.value
        buf = (ctypes.c_int64 * t.numel()).from_address(self.host.value)
        torch.from_numpy(np.frombuffer(buf, dtype=np.int64)).copy_(t)
        torch.cuda.synchronize()

    def close(self):
        if self.host:
            self.hip.hipHostFree(self.host)
            self.host = None


def _steady_latency(P, s, first, L, lo=0.1, hi=0.9):
    """p50 / p99 / max latency (us) of the requests whose arrival falls in the
    [lo, hi] part of the log's span: the first steps (empty queues, cold
    caches) and the drain at the end are left out."""
    import numpy as np

    n = L.num_requests
    arr = np.empty(n, dtype=np.float64)
    done = np.empty(n, dtype=np.float64)
    for r in range(n):
        a, d = P.sbbf_server_request_times(s, first + r)
        arr[r], done[r] = a, d
    t0 = arr.min()
    span = arr.max() - t0
    sel = (arr >= t0 + lo * span) & (arr <= t0 + hi * span)
    lat = (done[sel] - arr[sel]) / 1e3
    return {"p50_us": float(np.percentile(lat, 50)), "p99_us": float(np.percentile(lat, 99)),
            "max_us": float(lat.max()), "window_requests": int(sel.sum())}


def _serving(P, torch, num_requests=200_000, capacity_only=False):
    """The serving workload: 4,096 resident filters sized like the grouped
    workload (seed 5), Poisson arrivals, 20 % insert / 80 % lookup requests of
    log-uniform size 1..65,536, uniform filter choice, payloads generated on
    the device; capacity with every request queued at once (after one untimed
    warm-up replay), then latency at 25 / 50 / 90 % of that capacity over the
    steady-state window, and the same at 50 % with the payloads in pinned host
    memory read by the kernels across PCIe (the H2D variant)."""
    import numpy as np

    from synth.serving import serving_log

    base_rate = 1e6
    L = serving_log(num_filters=4096, num_requests=num_requests, rate_per_s=base_rate, backend="torch",
                    device="cuda")
    d_payload = L.payload
    d_out = torch.empty(int(L.out_off[-1]), dtype=torch.uint8, device="cuda")
    cfg = dict(max_step_keys=16 << 20, max_step_requests=16384)

    def run(rate, payload=d_payload, steady=False):
        s = P.sbbf_server_create(cfg)
        for b in L.blocks.tolist():
            P.sbbf_server_add_filter(s, b)
        req = P.serving_requests(L, payload, d_out)
        if rate:
            req["arrival_ns"] = (L.arrival_ns.astype(np.float64) * (base_rate / rate)).astype(np.uint64)
        torch.cuda.synchronize()
        first = P.sbbf_server_replay(s, req, realtime=bool(rate))
        st = P.sbbf_server_stats(s)
        if steady:
            st["steady"] = _steady_latency(P, s, first, L)
        P.sbbf_server_destroy(s)
        return st

    run(0)  # warm-up (first use of the arena, the pinned tile tables and the kernels), not reported
    cap = run(0)
    if capacity_only:
        return {"capacity_gkeys_per_s": cap["gkeys_per_s"], "steps": cap["steps"], "config": cfg}
    # Baseline with the same results: one plain call per request, in order.
    ref_out = d_out.clone()
    d_out.zero_()
    s = P.sbbf_server_create(cfg)
    for b in L.blocks.tolist():
        P.sbbf_server_add_filter(s, b)
    torch.cuda.synchronize()
    per_request_s = P.sbbf_server_replay_per_request(s, P.serving_requests(L, d_payload, d_out))
    P.sbbf_server_destroy(s)
    identical = bool(torch.equal(d_out, ref_out))
    keys = int(L.key_off[-1])
    mean_keys = float(L.n.mean())
    points = []
    for frac in (0.25, 0.5, 0.9):
        rate = frac * cap["gkeys_per_s"] * 1e9 / mean_keys
        st = run(rate, steady=True)
        points.append({"load": frac, "requests_per_s": rate, "offered_gkeys_per_s": rate * mean_keys / 1e9,
                       "p50_us": st["steady"]["p50_us"], "p99_us": st["steady"]["p99_us"],
                       "max_us": st["steady"]["max_us"], "window_requests": st["steady"]["window_requests"],
                       "p50_us_all": st["p50_us"], "p99_us_all": st["p99_us"],
                       "sustained_gkeys_per_s": st["gkeys_per_s"], "steps": st["steps"]})
    half = points[1]
    # H2D variant: the same log with its payloads in mapped pinned host memory.
    host = _PinnedHost(torch, d_payload)
    try:
        d_out.zero_()
        h2d_cap = run(0, payload=host.device_ptr)
        h2d_identical = bool(torch.equal(d_out, ref_out))
        rate = 0.5 * h2d_cap["gkeys_per_s"] * 1e9 / mean_keys
        h2d_half = run(rate, payload=host.device_ptr, steady=True)
    finally:
        host.close()
    del ref_out
    return {
        "workload": f"4,096 filters ({int(L.blocks.sum()) * 32 / 2**20:.1f} MiB resident), {num_requests:,} requests "
                    f"({keys:,} keys), 20 % inserts, sizes log-uniform 1..65,536",
        "capacity_gkeys_per_s": cap["gkeys_per_s"],
        "per_request_gkeys_per_s": keys / per_request_s / 1e9,
        "speedup_vs_per_request": cap["gkeys_per_s"] / (keys / per_request_s / 1e9),
        "identical_outputs_vs_per_request": identical,
        "p50_us": half["p50_us"],
        "p99_us": half["p99_us"],
        "latency_window": "requests arriving in the middle 80 % of the replay (first steps and final drain left out)",
        "at_load": points,
        "h2d_payload": {
            "what": "payloads in mapped pinned host memory, read by the step kernels across PCIe; outputs on the device",
            "capacity_gkeys_per_s": h2d_cap["gkeys_per_s"],
            "identical_outputs": h2d_identical,
            "at_half_load": {"offered_gkeys_per_s": rate * mean_keys / 1e9, **h2d_half["steady"],
                             "sustained_gkeys_per_s": h2d_half["gkeys_per_s"]},
        },
        "config": cfg,
    }


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plain_100m", choices=["plain_100k", "plain_1m", "plain_100m", "grouped_2048"],
                    help="the single-filter workload timed (grouped_2048 only names the counter files of "
                         "--traffic-from for the grouped graph)")
    ap.add_argument("--grouped-only", action="store_true",
                    help="run only the grouped leg (after --calibrate-copy-mib's copy), print its JSON")
    ap.add_argument("--insert-strategy", type=int, default=0,
                    help="0 = library choice, 1 atomic32, 2 atomic64, 3 LDS, 4 partitioned")
    ap.add_argument("--lookup-strategy", type=int, default=0, help="0 = library choice, 1 gather, 2 partitioned")
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--unroll", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ceilings", action="store_true")
    ap.add_argument("--no-grouped", action="store_true")
    ap.add_argument("--no-select", action="store_true", help="skip the select, union, key-hashing and block-variant measurements")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--grouped-config", metavar="JSON",
                    help="grouped plan settings over the defaults, e.g. '{\"xcd_queues\": 0}' (no autotuning)")
    ap.add_argument("--serving-requests", type=int, default=200_000)
    ap.add_argument("--serving-capacity-only", action="store_true",
                    help="serving leg: the capacity replays only (no baseline, no load levels), for profiling")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before the steps, copy this many MiB once with a plain device copy (a kernel of known "
                         "traffic for scaling hardware byte counters)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_*.json from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of "
                         "this script with --calibrate-copy-mib, then exit (no GPU use)")
    ap.add_argument("--traffic-commands", nargs="*", default=[], help="the commands of those runs, recorded")
    ap.add_argument("--kernel-summary", nargs=2, metavar=("STATS_CSV", "OUT_MD"),
                    help="write a markdown kernel-time summary of a rocprofv3 kernel_stats.csv, then exit")
    ap.add_argument("--counter-summary", nargs="+", metavar="PATH",
                    help="OUT_MD then one or more rocprofv3 --pmc counter_collection.csv files: write a markdown "
                         "table of counters per library kernel (with --summary-command once per run), then exit")
    ap.add_argument("--summary-title", default="Kernel time summary")
    ap.add_argument("--summary-command", action="append", default=[])
    ap.add_argument("--strategy-sweep", metavar="OUT_MD",
                    help="time the gather and partitioned lookups and the atomic and partitioned inserts over filter "
                         "sizes of 1 to 64 MiB and batches of 1M to 64M keys, write a markdown table, then exit")
    a = ap.parse_args(argv)

    if a.traffic_from:
        return _traffic_from_counters(a.traffic_from[0], a.traffic_from[1], a.workload,
                                      a.calibrate_copy_mib or 1024, a.traffic_commands)
    if a.strategy_sweep:
        return _strategy_sweep(a.strategy_sweep)
    if a.kernel_summary:
        return _kernel_summary(a.kernel_summary[0], a.kernel_summary[1], a.summary_title,
                               a.summary_command[0] if a.summary_command else "")
    if a.counter_summary:
        if len(a.counter_summary) < 2:
            ap.error("--counter-summary needs OUT_MD and at least one CSV")
        return _counter_summary(a.counter_summary[0], a.counter_summary[1:], a.summary_title, a.summary_command)

    if a.workload == "grouped_2048" and not a.grouped_only:
        ap.error("--workload grouped_2048 names counter files for --traffic-from; use --grouped-only to run the "
                 "grouped leg alone")
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only. Independent filters would shard across GPUs as whole "
              "filters, and one large filter by block range with an all-to-all exchange of hashes; "
              "neither is built here. Run with --gpus 1.", file=sys.stderr)
        return 2

    _ensure_built()
    import torch

    import paper_2101_01719_amd as P
    from synth import plain_workload

    torch.cuda.set_device(0)
    if a.grouped_only:
        if a.calibrate_copy_mib:
            src = torch.ones(a.calibrate_copy_mib << 18, dtype=torch.int32, device="cuda")
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
            del src, dst
        cfg = json.loads(a.grouped_config) if a.grouped_config else None
        print(json.dumps({"grouped": _grouped(P, torch, autotune=cfg is None, cfg=cfg)}), flush=True)
        return 0
    t_gen = time.perf_counter()
    w = plain_workload(a.workload, backend="torch", device="cuda")
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    n_ins, n_look = w.inserts.numel(), w.lookups.numel()

    ins_launch = dict(block_threads=a.threads, unroll=a.unroll, grid_blocks=a.grid, strategy=a.insert_strategy)
    look_launch = dict(block_threads=a.threads, unroll=min(a.unroll, 4), grid_blocks=a.grid,
                       strategy=a.lookup_strategy)
    f = P.Filter(w.num_blocks)
    names_ins = {1: "atomic32", 2: "atomic64", 3: "lds", 4: "partitioned"}
    names_look = {1: "gather", 2: "partitioned"}
    ins_used = names_ins[a.insert_strategy or P.sbbf_auto_insert_strategy(f.handle, n_ins)]
    look_used = names_look[a.lookup_strategy or P.sbbf_auto_lookup_strategy(f.handle, n_look)]
    out = torch.empty(n_look, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def step(ev=None):
        f.clear(stream)
        if ev:
            ev[0].record(stream)
        f.insert(w.inserts, launch=ins_launch, stream=stream)
        if ev:
            ev[1].record(stream)
        f.lookup(w.lookups, out=out, launch=look_launch, stream=stream)
        if ev:
            ev[2].record(stream)

    if a.calibrate_copy_mib:
        src = torch.ones(a.calibrate_copy_mib << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(a.steps)]
    t0 = time.perf_counter()
    for k in range(a.steps):
        step(events[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / a.steps
    insert_ms = sum(e[0].elapsed_time(e[1]) for e in events) / a.steps
    lookup_ms = sum(e[1].elapsed_time(e[2]) for e in events) / a.steps

    # correctness facts of the last step (cheap, device-side)
    fp = int(out[~w.is_member].sum().item())
    members_ok = bool(out[w.is_member].all().item())
    n_non = int((~w.is_member).sum().item())
    select = None if a.no_select else _select(P, torch, f, w.lookups, out, look_launch)
    union = None if a.no_select else _union(P, torch, f)
    keys = None if a.no_select else _keys(P, torch, f, w, ins_launch, look_launch)
    variants = None if a.no_select or a.workload != "plain_100m" else _variants(P, torch, w)

    ins_gbps = INSERT_BYTES_PER_KEY * n_ins / (insert_ms / 1e3) / 1e9
    look_gbps = LOOKUP_BYTES_PER_KEY * n_look / (lookup_ms / 1e3) / 1e9
    kernels = {
        "insert": dict(bound="hbm", achieved=ins_gbps, peak=HBM_PEAK_GBS, unit="GB/s", frac=ins_gbps / HBM_PEAK_GBS,
                       traffic=_traffic("insert", a.workload), avg_ms=insert_ms,
                       bytes_per_key=INSERT_BYTES_PER_KEY, keys_per_launch=n_ins),
        "lookup": dict(bound="hbm", achieved=look_gbps, peak=HBM_PEAK_GBS, unit="GB/s", frac=look_gbps / HBM_PEAK_GBS,
                       traffic=_traffic("lookup", a.workload), avg_ms=lookup_ms,
                       bytes_per_key=LOOKUP_BYTES_PER_KEY, keys_per_launch=n_look),
    }
    kernels["insert"]["kernel"] = f"insert ({ins_used})"
    kernels["lookup"]["kernel"] = f"lookup ({look_used})"
    dominant = "insert" if insert_ms >= lookup_ms else "lookup"
    roofline = kernels[dominant]

    result = {
        "metric": METRIC,
        "value": (n_ins + n_look) / (ms_per_step / 1e3) / 1e9,
        "unit": "G keys/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": f"{a.workload}: one filter of {w.num_blocks:,} blocks ({w.num_blocks * 32 / 2**20:.0f} MiB), "
                        f"{n_ins:,} inserts then {n_look:,} lookups ({w.n_member_lookups:,} members), "
                        "SplitMix64 hashes resident in HBM",
            "num_blocks": w.num_blocks,
            "inserts": n_ins,
            "lookups": n_look,
            "insert_launch": ins_launch,
            "lookup_launch": look_launch,
            "insert_strategy": ins_used,
            "lookup_strategy": look_used,
        },
        "insert_gkeys_per_s": n_ins / (insert_ms / 1e3) / 1e9,
        "lookup_gkeys_per_s": n_look / (lookup_ms / 1e3) / 1e9,
        "roofline": roofline,
        "roofline_other": kernels["lookup" if dominant == "insert" else "insert"],
        "false_positive_rate": fp / max(1, n_non),
        "members_all_found": members_ok,
        "input_generation_s": t_gen,
        "paper_context": PAPER_CONTEXT,
        "kernel_source_digest": _kernel_source_digest(),
    }
    if select is not None:
        result["select"] = select
    if union is not None:
        result["union"] = union
    if keys is not None:
        result["keys"] = keys
    if variants is not None:
        result["variants"] = variants
    if not a.no_ceilings:
        c = _ceilings(P, torch, w, look_launch, ins_launch)
        c["lookup_frac_of_gather"] = result["lookup_gkeys_per_s"] / c["gather_gkeys_per_s"]
        best_atomic = max(c["atomic32_gkeys_per_s"], c["atomic64_gkeys_per_s"])
        c["insert_frac_of_best_atomic"] = result["insert_gkeys_per_s"] / best_atomic
        result["ceilings"] = c
    if not a.no_cpu_baseline:
        result["cpu_baseline"] = _cpu_baseline(w)
        result["speedup_vs_cpu_baseline"] = result["value"] / result["cpu_baseline"]["value"]
    f.close()
    del w, out, f
    torch.cuda.empty_cache()
    if not a.no_select:
        result["plain_small"] = {name: _plain_small(P, torch, name) for name in ("plain_100k", "plain_1m")}
    if not a.no_grouped:
        result["grouped"] = _grouped(P, torch, cfg=json.loads(a.grouped_config) if a.grouped_config else None)
    if not a.no_serving:
        result["serving"] = _serving(P, torch, a.serving_requests, capacity_only=a.serving_capacity_only)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
