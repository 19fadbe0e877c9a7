"""Third implementation: the paper's own appendix code, compiled at test time.

When the environment variable SBBF_PAPER_SOURCE names a copy of the paper's
LaTeX source (never available on GPU machines) and the host has AVX2, this test extracts the C code of the appendix figure from the
source at run time, compiles it unchanged together with a small driver written
here, and compares its filter bytes, lookups and worked examples with the
oracle. Nothing of the listing is stored in this repository. Skipped otherwise.
"""

import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from conftest import read_golden
from synth import plain_workload, splitmix64_stream

# Path of the paper's LaTeX source, e.g. SBBF_PAPER_SOURCE=/path/to/paper.tex.
PAPER = os.environ.get("SBBF_PAPER_SOURCE", "")

DRIVER = r"""
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
int main(int argc, char **argv) {
  if (argc == 2 && strcmp(argv[1], "examples") == 0) {
    unsigned long long h; unsigned long B;
    while (scanf("%llx %lu", &h, &B) == 2) {
      uint32_t lanes[8];
      __m256i m = make_mask((uint32_t)h);
      _mm256_storeu_si256((__m256i *)lanes, m);
      printf("%llu", (unsigned long long)block_index(h, (uint32_t)B));
      for (int j = 0; j < 8; ++j) printf(" %u", lanes[j]);
      printf("\n");
    }
    return 0;
  }
  uint32_t B = (uint32_t)strtoul(argv[1], 0, 10);
  size_t ni = strtoull(argv[2], 0, 10), nl = strtoull(argv[3], 0, 10);
  uint64_t *h = malloc((ni + nl) * 8 + 8);
  FILE *f = fopen(argv[4], "rb");
  if (fread(h, 8, ni + nl, f) != ni + nl) return 2;
  fclose(f);
  __m256i *flt = aligned_alloc(32, (size_t)B * 32);
  memset(flt, 0, (size_t)B * 32);
  for (size_t i = 0; i < ni; ++i) add_hash(h[i], B, flt);
  unsigned char *r = malloc(nl + 1);
  for (size_t i = 0; i < nl; ++i) r[i] = find_hash(h[ni + i], B, flt);
  f = fopen(argv[5], "wb"); fwrite(flt, 32, B, f); fclose(f);
  f = fopen(argv[6], "wb"); fwrite(r, 1, nl, f); fclose(f);
  return 0;
}
"""


def _has_avx2():
    try:
        with open("/proc/cpuinfo") as f:
            return " avx2" in f.read()
    except OSError:
        return False


@pytest.fixture(scope="module")
def paper_binary(tmp_path_factory):
    if not PAPER or not os.path.exists(PAPER):
        pytest.skip("SBBF_PAPER_SOURCE does not name the paper's source on this machine")
    if not _has_avx2():
        pytest.skip("host has no AVX2")
    with open(PAPER) as f:
        text = f.read()
    m = re.search(r"\\begin\{verbatim\}\n(.*?)\\end\{verbatim\}", text, re.S)
    if not m:
        pytest.skip("appendix listing not found")
    d = tmp_path_factory.mktemp("paper")
    src = d / "paper_sbbf.c"
    src.write_text(m.group(1) + DRIVER)
    exe = d / "paper_sbbf"
    subprocess.run(["gcc", "-O2", "-mavx2", "-w", "-std=gnu11", "-o", str(exe), str(src)], check=True)
    return str(exe), d


def test_examples_match(paper_binary):
    exe, _ = paper_binary
    rows = read_golden("paper_code_examples.txt")
    extra = [(int(v), B) for v in splitmix64_stream(60, 200).tolist() for B in (1, 7, 4096, (1 << 32) - 1)]
    cases = [(int(r[0], 16), int(r[1])) for r in rows] + extra
    inp = "".join(f"{h:x} {B}\n" for h, B in cases)
    out = subprocess.run([exe, "examples"], input=inp, capture_output=True, text=True, check=True).stdout
    lines = out.strip().split("\n")
    assert len(lines) == len(cases)
    for (h, B), line in zip(cases, lines):
        vals = [int(v) for v in line.split()]
        assert vals[0] == oracle.block(h, B)
        assert vals[1:] == [int(v) for v in oracle.mask(h & 0xFFFFFFFF)]
    for r, line in zip(rows, lines):
        vals = [int(v) for v in line.split()]
        assert vals[0] == int(r[2])
        assert vals[1:] == [1 << int(i) for i in r[3:11]]


@pytest.mark.parametrize("name,B", [("plain_100k", None), ("plain_1m", None), ("plain_100k", 3), ("plain_100k", 1)])
def test_filters_and_lookups_match(paper_binary, name, B):
    exe, d = paper_binary
    w = plain_workload(name)
    nb = B or w.num_blocks
    ins = w.inserts if B is None else w.inserts[:500]
    look = w.lookups
    path = d / "in.bin"
    np.concatenate([ins, look]).astype("<u8").tofile(path)
    subprocess.run([exe, str(nb), str(ins.size), str(look.size), str(path), str(d / "f.bin"), str(d / "r.bin")],
                   check=True)
    got_f = np.fromfile(d / "f.bin", dtype="<u4")
    got_r = np.fromfile(d / "r.bin", dtype=np.uint8)
    words = oracle.build_filter(nb, ins)
    assert np.array_equal(got_f, words)
    assert np.array_equal(got_r, oracle.lookup(words, nb, look))
