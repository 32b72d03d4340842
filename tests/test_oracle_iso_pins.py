"""Pins of the oracle's Saved_isometry (Sec. 2.4): Brouwer-Zimmermann for
the Hamming weight of the image (a, b, a+b), d = d_H / 2.

What fixes it independently of its own code: the exhaustive definition
(brute force), the textbook [[5,1,3]] code and closed forms, the structure
behind the bound (disjoint information sets in reduced form, checked row by
row) and the bound itself on every codeword, and the round sizes C(r, t).
"""
import itertools
import math

import numpy as np

from oracle import oracle as O
from paper_2408_10743_amd import workloads as W

from test_oracle_pins import _coords, pauli_rows, rand_code, swt


def iso(v):
    v = np.asarray(v, dtype=np.uint8)
    n = v.shape[-1] // 2
    return np.concatenate([v[..., :n], v[..., n:], v[..., :n] ^ v[..., n:]], axis=-1)


def test_bz_iso_matches_brute_random_tiny():
    for s in range(400):
        B = rand_code(50000 + s, 7)
        d0, _ = O.brute(B)
        d, wit, log = O.bz_iso(B)
        assert d == d0, s
        assert swt(wit) == d and O.in_rowspace(B, wit)
        # the log is in Hamming units: the final U is twice the distance
        assert log[-1][3] == 2 * d


def test_bz_iso_matches_brute_wider_codes():
    for s in range(40):
        rng = W.SplitMix64(W.config_seed(16, s))
        n = rng.uniform_int(8, 16)
        m = rng.uniform_int(4, 20)
        B = W.additive(n, m, rng.next())
        if O.rank(B) == 0:
            continue
        assert O.bz_iso(B)[0] == O.brute(B)[0], s
    for i in range(20):
        G, f = W.config1(i)
        B = O.expand(G, f)
        assert O.bz_iso(B)[0] == O.brute(B)[0], i


def test_bz_iso_textbook_and_closed_forms():
    five = pauli_rows(["XZZXI", "IXZZX", "XIXZZ", "ZXIXZ", "XXXXX", "ZZZZZ"])
    assert O.bz_iso(five)[0] == 3
    for n in (1, 4, 9):
        B = pauli_rows(["X" * n, "Z" * n])
        assert O.bz_iso(B)[0] == n
        I0 = np.concatenate([np.eye(n, dtype=np.uint8), np.zeros((n, n), np.uint8)], axis=1)
        assert O.bz_iso(I0)[0] == 1


def test_information_sets_structure():
    """Every Gamma_j: rows are images of codewords spanning the code, in
    reduced form on its own pivot columns; the pivot columns of different
    matrices are disjoint."""
    for s in range(200):
        B = rand_code(51000 + s, 7)
        r, gs = O.gamma_iso(B, 8, with_rows=True)
        n = B.shape[1] // 2
        assert r == O.rank(B)
        used = set()
        for k, piv, rows in gs:
            assert rows.shape == (r, 3 * n)
            # rows are isometric images of codewords and span the code
            assert np.array_equal(rows[:, 2 * n:], rows[:, :n] ^ rows[:, n:2 * n])
            ab = rows[:, :2 * n]
            assert O.rank(ab) == r and O.rank(np.concatenate([ab, B])) == r
            cols = [int(c) for c in piv if c >= 0]
            assert len(cols) == k and len(set(cols)) == k
            assert not (set(cols) & used)
            used |= set(cols)
            for i, c in enumerate(piv):
                if c < 0:
                    assert not rows[i, cols].any()  # delta rows vanish on the set
                    continue
                col = rows[:, c]
                assert col[i] == 1 and col.sum() == 1  # reduced on its pivot


def test_lower_bound_holds_for_every_codeword():
    """wt_H(iso c) >= sum_j max(0, g_j(c) - (r - k_j)), g_j = rows of Gamma_j
    that c uses, for every nonzero codeword c."""
    for s in range(150):
        B = rand_code(52000 + s, 6)
        r, gs = O.gamma_iso(B, 8, with_rows=True)
        if r > 10:
            continue
        n = B.shape[1] // 2
        rows0 = gs[0][2][:, :2 * n]
        for mask in range(1, 1 << r):
            c = np.zeros(2 * n, np.uint8)
            for i in range(r):
                if (mask >> i) & 1:
                    c ^= rows0[i]
            bound = 0
            for k, piv, rows in gs:
                x = _coords(rows[:, :2 * n], c)
                bound += max(0, int(x.sum()) - (r - k))
            assert int(iso(c).sum()) >= bound, (s, mask)
            assert int(iso(c).sum()) == 2 * swt(c)


def test_round_sizes_are_binomials():
    for s in range(20):
        B = rand_code(53000 + s, 7)
        r = O.rank(B)
        d, _, log = O.bz_iso(B, 8)
        for t, j, L, U, cnt in log:
            assert cnt == math.comb(r, t)
        # rounds run in order t = 1, 2, ... over the matrices
        ts = [t for t, *_ in log]
        assert ts == sorted(ts)


def test_config2_iso_equals_golden():
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_distances.json")))
    for i in range(2):
        G, f = W.config2(i)
        assert O.bz_iso(O.expand(G, f), 8)[0] == gold["config2"][i]


def test_brute_force_by_subsets_small():
    # the definition once more, with Python subsets of the image rows
    for s in range(30):
        B = rand_code(54000 + s, 4)
        if B.shape[0] > 8:
            B = B[:8]
            if not B.any():
                continue
        best = None
        I = iso(B)
        for k in range(1, B.shape[0] + 1):
            for sub in itertools.combinations(range(B.shape[0]), k):
                w = int(np.bitwise_xor.reduce(I[list(sub)], axis=0).sum())
                if w and (best is None or w < best):
                    best = w
        assert O.bz_iso(B)[0] * 2 == best
