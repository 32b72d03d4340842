"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The library's host part (csrc/host.cpp: input handling, the F2/F4/isometry
constructions, logical pairs, qubit orders, mixed packages, the planner)
and the oracle (oracle/qdo.c) are compiled with the host compiler and the
sanitizers into small drivers that run them over seeded random codes; any
out-of-bounds access, use after free, leak or undefined operation aborts the
driver.  The drivers also check the constructions' own invariants and that
the oracle's brute force and BZ agree."""
import os
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.join(HERE, "..")
CSRC = os.path.join(ROOT, "paper_2408_10743_amd", "csrc")
ORACLE = os.path.join(ROOT, "oracle")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

HOST_DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "host.hpp"
#include "qdist.h"
using namespace qd;
static unsigned long long s = 88172645463325252ull;
static unsigned long long rnd() { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; }
int main() {
  int checked = 0;
  for (int it = 0; it < 160; ++it) {
    const int n = 1 + int(rnd() % 128);
    const int field = (it % 3 == 2) ? QD_FIELD_F4 : QD_FIELD_F2;
    const int m = 1 + int(rnd() % (field == QD_FIELD_F4 ? (n < 24 ? n : 24) : (2 * n < 40 ? 2 * n : 40)));
    std::vector<uint8_t> G(size_t(m) * (field == QD_FIELD_F4 ? n : 2 * n));
    for (auto &b : G) b = uint8_t(field == QD_FIELD_F4 ? rnd() % 4 : rnd() % 2);
    std::vector<BRow> basis;
    if (load_rows(G.data(), m, n, field, basis) != 0) return 2;
    const int rank = make_basis(basis, n);
    if (rank == 0) continue;
    std::vector<Gamma> f4 = build_f4(basis, n, kMaxGamma);
    Gamma f2 = build_f2(basis, n);
    std::vector<Gamma> iso = build_iso(basis, n, kMaxGamma);
    for (const Gamma &g : f4) if (!check_gamma(g, n)) return 3;
    if (!check_gamma(f2, n)) return 4;
    for (const Gamma &g : iso) if (!check_gamma_iso(g, n)) return 5;
    std::vector<BRow> logi;
    logical_pairs(basis, logi);
    for (const Gamma &g : f4) {
      QubitOrder o = qubit_order(g, n, false);
      for (const Package &p : g.pk) (void)permute_row(p.r, o);
    }
    std::vector<int> caps;
    if (field == QD_FIELD_F2 && rank < n && !try_mixed_f4(basis, n, rank, n / 4 + 1, kMaxGamma, f4, caps)) return 6;
    PlanChoice pc = choose_plan(f4, f2, iso, n, rank, QD_DIAG_AUTO, 0);
    if (pc.h_used < 1) return 7;
    ++checked;
  }
  std::printf("host checked %d\n", checked);
  return checked > 100 ? 0 : 8;
}
"""

ORACLE_DRIVER = r"""
#include <stdio.h>
#include <stdlib.h>
#include <stdint.h>
#include "qdo.h"
static unsigned long long s = 2463534242ull;
static unsigned long long rnd(void) { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; }
int main(void) {
  int checked = 0;
  for (int it = 0; it < 120; ++it) {
    const int n = 1 + (int)(rnd() % 24), m = 1 + (int)(rnd() % 16);
    uint8_t *B = malloc((size_t)m * 2 * n), *w = malloc((size_t)2 * n);
    for (int i = 0; i < m * 2 * n; ++i) B[i] = (uint8_t)(rnd() % 2);
    if (qdo_rank(B, m, n) == 0) { free(B); free(w); continue; }
    int d0 = -1, d2 = -1, d4 = -1, dh = -1, nlog = 0;
    long long log[5 * 512];
    if (qdo_brute(B, m, n, 1, &d0, w)) return 2;
    if (qdo_symplectic_weight(w, n) != d0 || !qdo_in_rowspace(B, m, n, w)) return 3;
    if (qdo_bz(B, m, n, QDO_DIAG_F2, 8, 1, &d2, w, log, 512, &nlog)) return 4;
    if (qdo_bz(B, m, n, QDO_DIAG_F4, 8, 1, &d4, w, log, 512, &nlog)) return 5;
    if (qdo_bz_iso(B, m, n, 8, 1, &dh, w, log, 512, &nlog)) return 6;
    if (d2 != d0 || d4 != d0 || dh != d0) return 7;
    free(B);
    free(w);
    ++checked;
  }
  printf("oracle checked %d\n", checked);
  return checked > 80 ? 0 : 8;
}
"""


def build_and_run(compiler, srcs, driver, name, extra):
    d = tempfile.mkdtemp(prefix="qd_san_")
    drv = os.path.join(d, name + (".cpp" if compiler == "g++" else ".c"))
    with open(drv, "w") as f:
        f.write(driver)
    exe = os.path.join(d, name)
    std = ["-std=c++17"] if compiler == "g++" else ["-std=c99"]
    subprocess.check_call([compiler] + std + SAN + extra + [drv] + srcs + ["-o", exe, "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    return r


def test_host_code_under_sanitizers():
    r = build_and_run("g++", [os.path.join(CSRC, "host.cpp")], HOST_DRIVER, "host_drv",
                      ["-I", CSRC, "-I", os.path.join(ROOT, "include")])
    print(r.stdout, r.stderr[-3000:])
    assert r.returncode == 0, r.stderr[-3000:]


def test_oracle_under_sanitizers():
    r = build_and_run("gcc", [os.path.join(ORACLE, "qdo.c")], ORACLE_DRIVER, "oracle_drv",
                      ["-I", ORACLE, "-mpopcnt", "-fopenmp"])
    print(r.stdout, r.stderr[-3000:])
    assert r.returncode == 0, r.stderr[-3000:]
