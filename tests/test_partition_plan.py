"""The partition planner's invariants, on the CPU.

tests/partition_plan_check.hip is compiled together with the planner's
source (paper_2101_01719_amd/csrc/partition_kernels.hip) and sweeps batch
sizes from 1 key to 2^31, filters of 1 to 4,096 slices and 1 to 2,048
partition workgroups. For every count-free lookup plan it checks what the
kernels' indexing relies on: result positions below 2^16 (slices * room),
room a power of two from 32 to 4,096, chunks of whole tiles, no scatter
workgroup without a chunk, bucket room in whole 32-key words, bucket
positions below 2^32, workspace sections 256-byte aligned, in order and large
enough, the unpermute's chunks from one scatter workgroup with 16-bit run
offsets, and every kernel's LDS within a compute unit's 160 KiB (two
unpermute workgroups per unit); for the counted lookup, chunks of at most
65,536 keys and a large enough layout. No device is used.
"""

import os
import shutil
import subprocess

import pytest

from conftest import ROOT


def _hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_partition_plans_keep_kernel_invariants(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not found")
    exe = tmp_path / "plan_check"
    src = os.path.join(ROOT, "tests", "partition_plan_check.hip")
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", f"-I{os.path.join(ROOT, 'include')}",
           f"-I{os.path.join(ROOT, 'paper_2101_01719_amd', 'csrc')}", "-x", "hip", src, "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "plan check ok" in r.stdout
