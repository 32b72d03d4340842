"""Pins of the oracle's mixed-package F4 construction (not in the paper):
the F4 diagonalization of Sec. 2.3 with a cap on the two-row packages of
each matrix, after which every package has one row.

What fixes it independently of its own code: the exhaustive definition
(brute force) for every cap, the package invariants re-checked here symbol
by symbol, the caps themselves, the uncapped construction as the limit of a
large cap, and the round sizes e_t of the resulting package sizes.
"""
import itertools

import numpy as np

from oracle import oracle as O
from paper_2408_10743_amd import workloads as W

from test_oracle_pins import esym, py_exhaustive


def sym(row, q, n):
    return int(row[q]) | (int(row[n + q]) << 1)


def inside_two_row(g):
    return sum(1 for d, p in zip(g["dims"], g["pivots"]) if d == 2 and p >= 0)


def check_invariants(g, n):
    """Sec. 2.3 invariants, re-derived from the rows: a two-row package is
    the only one nonzero at its pivot; a one-row package's pivot symbol
    differs from the single other symbol any other row shows there."""
    rows, dims, piv = g["rows"], g["dims"], g["pivots"]
    els = []
    for i, d in enumerate(dims):
        r, s = rows[2 * i], rows[2 * i + 1]
        els.append([r, s, r ^ s] if d == 2 else [r])
    for i, q in enumerate(piv):
        if q < 0:
            continue
        own = {sym(e, q, n) for e in els[i]}
        assert 0 not in own
        if dims[i] == 2:
            assert len(own) == 3
        others = {sym(e, q, n) for j, es in enumerate(els) if j != i for e in es} - {0}
        if dims[i] == 2:
            assert not others, (i, q, others)
        else:
            assert len(others) <= 1 and not (others & own), (i, q, own, others)


def caps_for(seed, h):
    rng = W.SplitMix64(seed)
    return [rng.uniform_int(0, 4) - 1 for _ in range(h)]  # -1 (no cap) .. 3


def test_mixed_bz_matches_brute_tiny():
    checked = 0
    for s in range(600):
        B = W.tiny_code(95000 + s, n_max=8)
        if not B.any():
            continue
        d0 = O.brute(B)[0]
        caps = caps_for(96000 + s, 8)
        d, wit, _ = O.bz(B, O.DIAG_F4, 8, max2=caps)
        assert d == d0, (s, caps)
        assert int(np.count_nonzero(wit[:B.shape[1] // 2] | wit[B.shape[1] // 2:])) == d
        assert O.in_rowspace(B, wit)
        checked += 1
    assert checked > 500


def test_mixed_bz_matches_brute_rate_below_one():
    """Codes with fewer rows than qubits, where the planner uses caps."""
    for s in range(60):
        rng = W.SplitMix64(W.config_seed(70, s))
        n = rng.uniform_int(10, 16)
        m = rng.uniform_int(n // 2, n - 1)
        B = W.additive(n, m, rng.next())
        if O.rank(B) == 0:
            continue
        d0 = O.brute(B)[0]
        for a in range(0, m // 2 + 1, 2):
            assert O.bz(B, O.DIAG_F4, 8, max2=[a, a])[0] == d0, (s, a)


def test_mixed_invariants_and_caps():
    for s in range(80):
        rng = W.SplitMix64(W.config_seed(71, s))
        n = rng.uniform_int(8, 20)
        m = rng.uniform_int(4, n)
        B = W.additive(n, m, rng.next())
        if O.rank(B) == 0:
            continue
        caps = caps_for(97000 + s, 8)
        gs = O.gamma(B, O.DIAG_F4, 8, with_rows=True, max2=caps)
        used = set()
        for j, g in enumerate(gs):
            check_invariants(g, n)
            if caps[j] >= 0:
                assert inside_two_row(g) <= caps[j]
            piv = [q for q in g["pivots"] if q >= 0]
            assert not used & set(piv)  # disjoint qubit sets
            used |= set(piv)
            assert sum(g["dims"]) == O.rank(B)


def test_large_cap_is_the_uncapped_construction():
    for s in range(40):
        B = W.additive(12, 10 + s % 5, W.config_seed(72, s))
        if O.rank(B) == 0:
            continue
        a = O.gamma(B, O.DIAG_F4, 8)
        b = O.gamma(B, O.DIAG_F4, 8, max2=[64] * 8)
        c = O.gamma(B, O.DIAG_F4, 8, max2=[-1] * 8)
        assert a == b == c


def test_zero_cap_gives_one_row_packages():
    for s in range(40):
        B = W.additive(14, 9, W.config_seed(73, s))
        if O.rank(B) == 0:
            continue
        g = O.gamma(B, O.DIAG_F4, 1, max2=[0])[0]
        assert all(d == 1 for d, p in zip(g["dims"], g["pivots"]) if p >= 0)
        # one row per package and per pivot qubit: rank packages
        assert g["P"] == O.rank(B)


def test_mixed_round_sizes_are_esym():
    """Each logged round visits e_t(package sizes) combinations."""
    for s in range(20):
        B = W.additive(12, 9, W.config_seed(74, s))
        if O.rank(B) == 0:
            continue
        caps = [2, 3]
        gs = O.gamma(B, O.DIAG_F4, 8, max2=caps)
        d, _, log = O.bz(B, O.DIAG_F4, 8, max2=caps)
        for (t, j, L, U, combos) in log:
            sizes = [3 if x == 2 else 1 for x in gs[j]["dims"]]
            assert combos == esym(sizes, t), (s, t, j)


def test_mixed_exhaustive_python_small():
    """Independent of the C enumeration: tiny codes against a Python
    exhaustive search over the row space."""
    for s in range(60):
        B = W.tiny_code(98000 + s, n_max=6, m_max=8)
        if not B.any():
            continue
        assert O.bz(B, O.DIAG_F4, 8, max2=[1, 0, 2])[0] == py_exhaustive(B), s
