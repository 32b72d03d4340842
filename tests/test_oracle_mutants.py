"""The pins must catch plausible mistakes in the oracle.

Each mutant is a one-line change of oracle/qdo.c (a dropped term, a wrong
sign or bound, a missing clearing step), compiled on the CPU into a
temporary library; the pin checks below must fail for every one of them and
pass for the unmodified source.
"""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2408_10743_amd import workloads as W

from test_oracle_pins import GOLD, f4_to_bin, py_exhaustive, swt, esym
from test_oracle_rowspace_pins import all_vectors, py_span
from test_oracle_round_hist_pins import py_hist, _pauli_packages

SRC = os.path.join(os.path.dirname(O.__file__), "qdo.c")

MUTANTS = {
    "f2_no_full_clearing": ("      if (v != r && R[(size_t)v * len + col])\n        row_add(R + (size_t)v * len, R + (size_t)r * len, len);\n    rem[r] = 0;\n    second[q] = r;",
                            "      if (v != r && rem[v] && R[(size_t)v * len + col])\n        row_add(R + (size_t)v * len, R + (size_t)r * len, len);\n    rem[r] = 0;\n    second[q] = r;"),
    "bound_abs_not_max": ("int c = tdone[i] + 1 - delta[i];\n        L += c > 0 ? c : 0;",
                          "int c = tdone[i] + 1 - delta[i];\n        L += c > 0 ? c : -c;"),
    "bound_ignores_delta": ("int c = tdone[i] + 1 - delta[i];", "int c = tdone[i] + 1;"),
    "bound_off_by_one": ("int c = tdone[i] + 1 - delta[i];", "int c = tdone[i] + 2 - delta[i];"),
    "alpha_times_row_wrong": ("ag[n + q] = (uint8_t)(a ^ b);", "ag[n + q] = (uint8_t)a;"),
    "weight_xor_not_or": ("w += __builtin_popcountll(c[i] | c[W + i]);", "w += __builtin_popcountll(c[i] ^ c[W + i]);"),
    "one_row_clearing_skipped": ("if (sv == sr || sv == (sr ^ beta))", "if (0)"),
    "round_skips_last_package": ("  for (int i = start; i <= c->P - (c->t - depth); ++i)\n    for (int e = 0; e < c->ne[i]; ++e) {\n      const uint64_t *x = c->el + (size_t)(i * 3 + e) * W2;\n      for (int k = 0; k < W2; ++k) nxt[k] = cur[k] ^ x[k];\n      round_rec",
                                 "  for (int i = start; i < c->P - (c->t - depth); ++i)\n    for (int e = 0; e < c->ne[i]; ++e) {\n      const uint64_t *x = c->el + (size_t)(i * 3 + e) * W2;\n      for (int k = 0; k < W2; ++k) nxt[k] = cur[k] ^ x[k];\n      round_rec"),
    "hist_skips_last_package": ("  for (int i = start; i <= c->P - (c->t - depth); ++i)\n    for (int e = 0; e < c->ne[i]; ++e) {\n      const uint64_t *x = c->el + (size_t)(i * 3 + e) * W2;\n      for (int k = 0; k < W2; ++k) nxt[k] = cur[k] ^ x[k];\n      hist_rec",
                                "  for (int i = start; i < c->P - (c->t - depth); ++i)\n    for (int e = 0; e < c->ne[i]; ++e) {\n      const uint64_t *x = c->el + (size_t)(i * 3 + e) * W2;\n      for (int k = 0; k < W2; ++k) nxt[k] = cur[k] ^ x[k];\n      hist_rec"),
    "third_element_missing": ("      ne[i] = 3;", "      ne[i] = 2;"),
    "stop_one_early": ("if (L >= U || t == P[j]) finished = 1;", "if (L + 1 >= U || t == P[j]) finished = 1;"),
    "two_dim_clears_with_wrong_row": ("        } else if (sv == ss) {\n          row_add(R + (size_t)v * len, R + (size_t)s * len, len);",
                                      "        } else if (sv == ss) {\n          row_add(R + (size_t)v * len, R + (size_t)r * len, len);"),
    "iso_third_block_or": ("    out[2 * n + q] = row[q] ^ row[n + q];", "    out[2 * n + q] = row[q] | row[n + q];"),
    "iso_bound_ignores_delta": ("int c = tdone[i] + 1 - (r - k[i]);", "int c = tdone[i] + 1;"),
    "iso_echelon_not_reduced": ("        if (i != p && R[(size_t)i * len + c]) row_add(R + (size_t)i * len, R + (size_t)p * len, len);",
                                "        if (i > p && R[(size_t)i * len + c]) row_add(R + (size_t)i * len, R + (size_t)p * len, len);"),
    "iso_sets_not_disjoint": ("      if (piv[i] >= 0) used[piv[i]] = 1;", "      (void)used;"),
    "stab_test_inverted": ("    if (sym_product(c, chk + (size_t)r * 2 * W, W)) return 1;",
                           "    if (!sym_product(c, chk + (size_t)r * 2 * W, W)) return 1;"),
    "stab_product_missing_term": ("p ^= __builtin_parityll((a[i] & b[W + i]) ^ (a[W + i] & b[i]));",
                                  "p ^= __builtin_parityll(a[i] & b[W + i]);"),
    "stab_no_k0_rule": ("      if (sym_product(R + (size_t)i * 2 * W, R + (size_t)j * 2 * W, W)) return m;\n  return 0;",
                        "      if (sym_product(R + (size_t)i * 2 * W, R + (size_t)j * 2 * W, W)) return m;\n  return m;"),
    "stab_round_unfiltered": ("    if (w < c->best && admitted(cur, c->chk, c->nchk, c->W)) {", "    if (w < c->best) {"),
    "iso_round_skips_last_row": ("  for (int i = start; i <= c->m - (c->t - depth); ++i) {",
                                 "  for (int i = start; i < c->m - (c->t - depth); ++i) {"),
    "mixed_cap_ignored": ("    if (cnt >= 2 && allow2) { *dim = 2; return q; }", "    if (cnt >= 2) { *dim = 2; return q; }"),
    "mixed_one_row_clears_only_sr": ("        if (sv == sr || sv == (sr ^ beta))\n          row_add(R + (size_t)v * len, R + (size_t)r * len, len);\n      }\n      cand[r] = 0;",
                                     "        if (sv == sr)\n          row_add(R + (size_t)v * len, R + (size_t)r * len, len);\n      }\n      cand[r] = 0;"),
    "mixed_cap_counts_from_one": ("  int n2 = 0;\n  int *done", "  int n2 = 1;\n  int *done"),
    "in_rowspace_always_member": ("  return r0 == r1 ? 1 : 0;", "  return 1;"),
    "in_rowspace_compares_wrong_rank": ("  int r1 = reduce_basis(M, m + 1, n, NULL);", "  int r1 = reduce_basis(M, m, n, NULL);"),
    "symplectic_weight_and": ("    if (v[i] || v[n + i]) ++w;", "    if (v[i] && v[n + i]) ++w;"),
    "symplectic_weight_x_only": ("    if (v[i] || v[n + i]) ++w;", "    if (v[i]) ++w;"),
    "hist_repeats_a_package": ("      hist_rec(c, i + 1, depth + 1, nxt);", "      hist_rec(c, i, depth + 1, nxt);"),
    "hist_drops_weight_n": ("      for (int w = 0; w <= n; ++w) hist[w] += mine[w];",
                            "      for (int w = 0; w < n; ++w) hist[w] += mine[w];"),
    "hist_skips_third_element": ("    for (int e = 0; e < c->ne[i]; ++e) {\n      const uint64_t *x = c->el + (size_t)(i * 3 + e) * W2;\n      for (int k = 0; k < W2; ++k) nxt[k] = cur[k] ^ x[k];\n      hist_rec",
                                 "    for (int e = 0; e < c->ne[i] && e < 2; ++e) {\n      const uint64_t *x = c->el + (size_t)(i * 3 + e) * W2;\n      for (int k = 0; k < W2; ++k) nxt[k] = cur[k] ^ x[k];\n      hist_rec"),
}


def quick_pins():
    """A compact subset of the pins; True when all of them hold."""
    try:
        ex = GOLD["saved1_example"]
        A = np.array(ex["A"], dtype=np.uint8)
        if O.bz(A, O.DIAG_F2)[0] != ex["d_true"]:
            return False
        ex2 = GOLD["saved2_example"]
        A4 = f4_to_bin(ex2["A4"])
        d, _, log = O.bz(A4, O.DIAG_F4, 1)
        if d != ex2["d_true"] or [[t, L, U] for (t, j, L, U, _) in log] != ex2["trace_B4_after_rounds"]:
            return False
        for s in range(400):
            B = W.tiny_code(90000 + s)
            if not B.any():
                continue
            db = py_exhaustive(B[:10]) if B.shape[0] > 10 else None
            d0, wit = O.brute(B)
            if db is not None and O.brute(B[:10])[0] != db:
                return False
            if swt(wit) != d0:
                return False
            for diag in (O.DIAG_F2, O.DIAG_F4):
                if O.bz(B, diag, 8)[0] != d0:
                    return False
            if O.bz_iso(B, 8)[0] != d0:
                return False
        for s in range(10):
            G = W.f4_linear(5, 2, W.config_seed(14, s))
            B = O.expand(G, 4)
            ref = py_exhaustive(np.concatenate([f4_to_bin(G), f4_to_bin(np.array([[[0, 2, 3, 1][c] for c in r] for r in G]))]))
            if O.brute(B)[0] != ref:
                return False
        for s in range(40):
            B = W.tiny_code(91000 + s)
            if not B.any():
                continue
            r, gs = O.gamma_iso(B, 8, with_rows=True)
            for k, piv, rows in gs:
                for i, c in enumerate(piv):
                    if c >= 0 and (rows[i, c] != 1 or rows[:, c].sum() != 1):
                        return False
        for s in range(4):
            B = O.expand(*W.config1(s))
            _, _, log = O.bz_iso(B, 8)
            if max(t for t, *_ in log) < 2 or any(cnt != math.comb(20, t) for t, j, L, U, cnt in log):
                return False
        for name, dref in (("[[9,1,3]]", 3), ("[[5,1,3]]", 3), ("[[3,0,2]]", 2), ("[[4,2,2]]", 2)):
            A = W.textbook_code(name)
            if O.brute_stab(A)[0] != dref or O.bz_stab(A, O.DIAG_F4)[0] != dref:
                return False
        for s in range(40):
            rng = W.SplitMix64(W.config_seed(19, s))
            n = rng.uniform_int(2, 8)
            k = rng.uniform_int(0, n)
            A = W.random_stabilizer(n, k, rng.next())
            if O.bz_stab(A, O.DIAG_F4, 8)[0] != O.brute_stab(A)[0]:
                return False
        # mixed packages: brute force under caps, and the caps themselves
        for s in range(120):
            B = W.tiny_code(99000 + s, n_max=8)
            if not B.any():
                continue
            caps = [(s % 4) - 1, ((s // 4) % 4) - 1]
            if O.bz(B, O.DIAG_F4, 8, max2=caps)[0] != O.brute(B)[0]:
                return False
            for j, g in enumerate(O.gamma(B, O.DIAG_F4, 8, max2=caps)[:2]):
                two = sum(1 for d, p in zip(g["dims"], g["pivots"]) if d == 2 and p >= 0)
                if caps[j] >= 0 and two > caps[j]:
                    return False
        for s in range(10):
            B = W.additive(12, 8, W.config_seed(75, s))
            g = O.gamma(B, O.DIAG_F4, 1, max2=[2])[0]
            two = sum(1 for d, p in zip(g["dims"], g["pivots"]) if d == 2 and p >= 0)
            if two != 2:  # a random code has room for both two-row packages
                return False
        # membership: every vector of F2^6 against the span written out
        for s in range(6):
            B = W.additive(3, 1 + s % 4, W.config_seed(82, s))
            span = py_span(B)
            for v in all_vectors(3):
                if O.in_rowspace(B, v) != (v.tobytes() in span):
                    return False
        # symplectic weight: C(n, w) 3^w vectors of weight w
        hist = [0] * 4
        for v in all_vectors(3):
            hist[O.symplectic_weight(v, 3)] += 1
        if hist != [math.comb(3, w) * 3 ** w for w in range(4)]:
            return False
        rows, dims = W.random_packages(6, 20, W.config_seed(15, 0), 0.5)
        sizes = [3 if d == 2 else 1 for d in dims]
        for t in range(1, 7):
            if O.round_min(rows, dims, t)[2] != esym(sizes, t):
                return False
        # round weight distributions: Python enumeration and the full space
        for s in range(4):
            rows, dims = W.random_packages(5, 9 + 20 * s, W.config_seed(84, s), 0.6)
            for t in range(1, 6):
                if [int(x) for x in O.round_hist(rows, dims, t)] != [int(x) for x in py_hist(rows, dims, t)]:
                    return False
        rows, dims = _pauli_packages(4, 4, 2)
        tot = [0] * 5
        for t in range(1, 5):
            tot = [a + int(b) for a, b in zip(tot, O.round_hist(rows, dims, t))]
        if tot != [0] + [math.comb(4, w) * 3 ** w for w in range(1, 5)]:
            return False
        return True
    except O.OracleError:
        return False


def _load(path):
    O._lib = ctypes.CDLL(path)


@pytest.fixture
def restore_lib():
    saved = O._lib
    yield
    O._lib = saved


def test_unmodified_oracle_passes(restore_lib):
    O._lib = None
    assert quick_pins()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, restore_lib, tmp_path):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation site for {name} not unique/not found"
    mpath = tmp_path / "qdo_mut.c"
    mpath.write_text(src.replace(old, new))
    hdr = os.path.join(os.path.dirname(SRC), "qdo.h")
    (tmp_path / "qdo.h").write_text(open(hdr).read())
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-mpopcnt", "-fopenmp", "-std=c99", "-shared", "-fPIC",
                           str(mpath), "-o", str(so)])
    _load(str(so))
    assert not quick_pins(), f"mutant {name} survived the pins"
