"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer.

A small driver written here calls every function the oracle exports on edge
cases: one block, the largest block count for block selection, ragged packed
outputs (n not a multiple of 32), empty batches, all three block variants and a
bad lane count. Any out-of-bounds access, signed overflow, oversized shift or
other undefined behaviour aborts the run (no recovery), so the test passes only
on a clean run. Host code only; nothing here touches a GPU.
"""

import os
import shutil
import subprocess

import pytest

from conftest import ROOT

SRC = os.path.join(ROOT, "oracle", "sbbf_oracle.c")

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void sbbf_oracle_seeds(uint32_t seeds[8]);
uint64_t sbbf_oracle_block(uint64_t hash, uint32_t num_blocks);
void sbbf_oracle_bit_indices(uint32_t x, uint32_t idx[8]);
void sbbf_oracle_mask(uint32_t x, uint32_t mask[8]);
void sbbf_oracle_insert(uint32_t *words, uint32_t num_blocks, const uint64_t *hashes, uint64_t n);
int sbbf_oracle_contains(const uint32_t *words, uint32_t num_blocks, uint64_t hash);
void sbbf_oracle_lookup(const uint32_t *words, uint32_t num_blocks, const uint64_t *hashes, uint64_t n, uint8_t *out);
void sbbf_oracle_lookup_bits(const uint32_t *words, uint32_t num_blocks, const uint64_t *hashes, uint64_t n,
                             uint32_t *bits);
uint64_t sbbf_oracle_popcount(const uint32_t *words, uint64_t num_words);
double sbbf_oracle_conditional_fpr(const uint32_t *words, uint32_t num_blocks);
void sbbf_oracle_index_histogram(uint64_t x_begin, uint64_t x_end, uint64_t hist[256]);
void sbbf_oracle_block_histogram(const uint64_t *hashes, uint64_t n, uint32_t num_blocks, uint64_t *count);
void sbbf_oracle_key_hash(const uint64_t *keys, uint64_t n, uint64_t *out);
int sbbf_oracle_variant_seeds(uint32_t lanes, uint32_t seeds[16]);
void sbbf_oracle_variant_mask(uint32_t lanes, uint32_t x, uint32_t mask[16]);
void sbbf_oracle_variant_insert(uint32_t *words, uint32_t lanes, uint32_t num_blocks, const uint64_t *hashes,
                                uint64_t n);
int sbbf_oracle_variant_contains(const uint32_t *words, uint32_t lanes, uint32_t num_blocks, uint64_t hash);
void sbbf_oracle_variant_lookup(const uint32_t *words, uint32_t lanes, uint32_t num_blocks, const uint64_t *hashes,
                                uint64_t n, uint8_t *out);

static uint64_t sm(uint64_t *s) {  /* SplitMix64 */
  uint64_t z = (*s += UINT64_C(0x9e3779b97f4a7c15));
  z = (z ^ (z >> 30)) * UINT64_C(0xbf58476d1ce4e5b9);
  z = (z ^ (z >> 27)) * UINT64_C(0x94d049bb133111eb);
  return z ^ (z >> 31);
}

#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); return 1; } } while (0)

int main(void) {
  uint32_t s8[8], idx[8], m8[8], s16[16], m16[16];
  sbbf_oracle_seeds(s8);
  for (int j = 0; j < 8; ++j) CHECK(s8[j] & 1u);
  const uint64_t edge[] = {0, 1, UINT64_C(0xffffffff), UINT64_C(0x100000000), UINT64_MAX, UINT64_C(0x8000000000000000)};
  const uint32_t Bs[] = {1, 2, 3, 4096, 0x7fffffffu, 0xffffffffu};
  for (unsigned a = 0; a < sizeof edge / sizeof *edge; ++a)
    for (unsigned b = 0; b < sizeof Bs / sizeof *Bs; ++b) CHECK(sbbf_oracle_block(edge[a], Bs[b]) < Bs[b]);
  for (unsigned a = 0; a < sizeof edge / sizeof *edge; ++a) {
    sbbf_oracle_bit_indices((uint32_t)edge[a], idx);
    sbbf_oracle_mask((uint32_t)edge[a], m8);
    for (int j = 0; j < 8; ++j) CHECK(idx[j] < 32 && m8[j] == (1u << idx[j]));
  }
  uint64_t st = 7;
  enum { N = 1000, NL = 1037 };
  uint64_t *h = malloc(sizeof(uint64_t) * (N + NL));
  for (int i = 0; i < N + NL; ++i) h[i] = sm(&st);
  h[0] = 0; h[1] = UINT64_MAX;
  const uint32_t fb[] = {1, 2, 37, 4096};
  for (unsigned k = 0; k < sizeof fb / sizeof *fb; ++k) {
    const uint32_t B = fb[k];
    uint32_t *w = calloc((size_t)8 * B, 4);
    sbbf_oracle_insert(w, B, h, 0);                 /* empty batch */
    CHECK(sbbf_oracle_popcount(w, (uint64_t)8 * B) == 0);
    sbbf_oracle_insert(w, B, h, N);
    uint8_t *out = malloc(NL);
    uint32_t *bits = malloc(sizeof(uint32_t) * ((NL + 31) / 32));
    sbbf_oracle_lookup(w, B, h, N, out);            /* members */
    for (int i = 0; i < N; ++i) CHECK(out[i] == 1 && sbbf_oracle_contains(w, B, h[i]));
    sbbf_oracle_lookup(w, B, h + N, NL, out);
    sbbf_oracle_lookup_bits(w, B, h + N, NL, bits);  /* ragged: 1,037 = 32 * 32 + 13 */
    for (int i = 0; i < NL; ++i) CHECK(((bits[i / 32] >> (i % 32)) & 1u) == out[i]);
    CHECK(bits[NL / 32] >> (NL % 32) == 0);
    double c = sbbf_oracle_conditional_fpr(w, B);
    CHECK(c >= 0.0 && c <= 1.0);
    uint64_t *cnt = calloc(B, 8);
    sbbf_oracle_block_histogram(h, N + NL, B, cnt);
    uint64_t tot = 0;
    for (uint32_t b = 0; b < B; ++b) tot += cnt[b];
    CHECK(tot == N + NL);
    free(cnt); free(bits); free(out); free(w);
  }
  uint64_t hist[256];
  memset(hist, 0, sizeof hist);
  sbbf_oracle_index_histogram(UINT64_C(0xffffff00), UINT64_C(0x100000000), hist);  /* the top of the range */
  uint64_t tot = 0;
  for (int i = 0; i < 256; ++i) tot += hist[i];
  CHECK(tot == 8 * 256);
  uint64_t kh[4];
  const uint64_t keys[4] = {0, 1, UINT64_MAX, UINT64_C(0x8000000000000000)};
  sbbf_oracle_key_hash(keys, 4, kh);
  CHECK(kh[0] == 0);
  CHECK(sbbf_oracle_variant_seeds(3, s16) != 0);   /* bad lane count is refused */
  const uint32_t lanes[] = {4, 8, 16};
  for (unsigned k = 0; k < 3; ++k) {
    const uint32_t L = lanes[k], B = 29;
    CHECK(sbbf_oracle_variant_seeds(L, s16) == 0);
    sbbf_oracle_variant_mask(L, 0xffffffffu, m16);
    uint32_t *w = calloc((size_t)L * B, 4);
    uint8_t *out = malloc(NL);
    sbbf_oracle_variant_insert(w, L, B, h, N);
    sbbf_oracle_variant_lookup(w, L, B, h, N, out);
    for (int i = 0; i < N; ++i) CHECK(out[i] == 1 && sbbf_oracle_variant_contains(w, L, B, h[i]));
    sbbf_oracle_variant_lookup(w, L, B, h + N, NL, out);
    free(out); free(w);
  }
  free(h);
  printf("sanitized oracle ok\n");
  return 0;
}
"""


def test_oracle_clean_under_asan_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not available")
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "oracle_sanitized"
    cmd = [gcc, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-Wall", "-Wextra",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", str(exe), SRC, str(drv)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and ("cannot find" in r.stderr or "libasan" in r.stderr or "libubsan" in r.stderr):
        pytest.skip("sanitizer runtimes are not installed: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "sanitized oracle ok" in run.stdout
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr
