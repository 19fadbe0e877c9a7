"""Allocation failure forced from the host: with SBBF_FAULT_INJECT=alloc in a
child process's environment, every allocation the library would make fails
before it is attempted. Entry points that allocate return SBBF_ENOMEM and
enqueue nothing (the filter is unchanged); entry points that allocate
nothing (atomic inserts, gather lookups, the allocation-free select) still
give the oracle's results."""

import os
import subprocess
import sys

import pytest

from conftest import ROOT

pytestmark = pytest.mark.gpu

CHILD = r"""
import numpy as np
import torch

import oracle
import paper_2101_01719_amd as P
from synth import splitmix64_stream

ENOMEM = 2


def refused(what, fn):
    try:
        fn()
    except P.SbbfError as e:
        assert e.status == ENOMEM, (what, e.status, str(e))
        print("refused:", what, flush=True)
        return
    raise AssertionError(f"{what}: allocation was not refused")


torch.cuda.set_device(0)
B = 40_000  # 1.25 MiB: partitioned strategies apply
ins = splitmix64_stream(950, 200_000)
probes = splitmix64_stream(951, 300_000)
probes[:50_000] = ins[:50_000]
d_ins = torch.from_numpy(ins.view(np.int64)).cuda()
d_probes = torch.from_numpy(probes.view(np.int64)).cuda()
ref_words = oracle.build_filter(B, ins)
ref = oracle.lookup(ref_words, B, probes)

refused("sbbf_create", lambda: P.sbbf_create(64))
f = P.Filter(B)  # words in torch memory: nothing allocated by the library
before = f.words.clone()
refused("partitioned insert", lambda: f.insert(d_ins, launch=dict(strategy=4)))
torch.cuda.synchronize()
assert torch.equal(f.words, before), "a refused insert changed the filter"
f.insert(d_ins, launch=dict(strategy=1))  # 32-bit atomics: no workspace
torch.cuda.synchronize()
assert np.array_equal(f.words.cpu().numpy().view(np.uint32), ref_words)
refused("partitioned lookup", lambda: f.lookup(d_probes, launch=dict(strategy=2)))
out = f.lookup(d_probes, launch=dict(strategy=1))  # gather: no workspace
torch.cuda.synchronize()
assert np.array_equal(out.cpu().numpy(), ref)
refused("select", lambda: P.sbbf_lookup_select(f.handle, d_probes))
idx = torch.empty(probes.size, dtype=torch.int32, device="cuda")
cnt = torch.empty(1, dtype=torch.int64, device="cuda")
P.sbbf_lookup_select_noalloc(f.handle, d_probes, idx, cnt)
torch.cuda.synchronize()
c = int(cnt.item())
assert np.array_equal(idx[:c].cpu().numpy().view(np.uint32), np.flatnonzero(ref).astype(np.uint32))
g_filters = [P.Filter(100), P.Filter(9_000)]
refused("grouped plan", lambda: P.Group(g_filters, np.array([0, 10, 20]), np.array([0, 10, 20])))
refused("grouped capacity plan", lambda: P.Group.with_capacity(g_filters, [10, 10], [10, 10]))
refused("server", lambda: P.sbbf_server_create({}))
print("FAULT_INJECTION_OK", flush=True)
"""


def test_allocation_failures_are_reported_and_change_nothing():
    env = dict(os.environ, SBBF_FAULT_INJECT="alloc", PYTHONPATH=ROOT)
    print("fault injection child: SBBF_FAULT_INJECT=alloc", flush=True)
    r = subprocess.run([sys.executable, "-u", "-c", CHILD], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=240)
    print(r.stdout[-3000:], r.stderr[-3000:])
    assert r.returncode == 0 and "FAULT_INJECTION_OK" in r.stdout


def test_without_the_variable_nothing_is_refused():
    env = {k: v for k, v in os.environ.items() if k != "SBBF_FAULT_INJECT"}
    env["PYTHONPATH"] = ROOT
    code = ("import paper_2101_01719_amd as P, torch; torch.cuda.set_device(0); h = P.sbbf_create(64); "
            "P.sbbf_destroy(h); print('CREATE_OK')")
    r = subprocess.run([sys.executable, "-u", "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0 and "CREATE_OK" in r.stdout, r.stderr[-2000:]
