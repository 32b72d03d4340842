"""The lower bound behind the kernel's partial weights, checked on the
oracle's generator matrices by enumeration.

Every package of a combination has a nonzero symbol at its own pivot qubit:
a 2-dim package is the only one nonzero there, and a 1-dim package's pivot
symbol differs from the one other symbol the rest of its matrix may carry
there (Sec. 2.2, Sec. 2.3).  So for any qubit set S, the weight of a
combination is at least its weight on S plus the number of its chosen
packages pivoted outside S.  For the isometry matrices (Sec. 2.4) each
chosen row has a 1 at its pivot image column; pivot columns are linearly
independent and a qubit's three image columns sum to zero, so at most two
pivot columns share a qubit and the credit is half of that count, rounded
up.  The library takes S = the first stored words, after moving every qubit
that carries no pivot to the front.
"""
import itertools

import numpy as np

from oracle import oracle as O
from paper_2408_10743_amd import workloads as W

from test_oracle_pins import rand_code


def elements(g, i):
    r, s = g["rows"][2 * i], g["rows"][2 * i + 1]
    return [r, s, r ^ s] if g["dims"][i] == 2 else [r]


def nonzero_qubits(c, n):
    return (c[:n] | c[n:]).astype(bool)


def stored_order(pivot_qubits, n):
    """Non-pivot qubits first (ascending), then pivot qubits."""
    piv = set(pivot_qubits)
    return [q for q in range(n) if q not in piv] + sorted(piv)


def combos(g, t):
    for pk in itertools.combinations(range(g["P"]), t):
        for choice in itertools.product(*[elements(g, i) for i in pk]):
            c = np.zeros_like(choice[0])
            for e in choice:
                c ^= e
            yield pk, c


def check_matrix(g, n, tmax, rng):
    pivots = g["pivots"]
    piv_q = [q for q in pivots if q >= 0]
    assert len(set(piv_q)) == len(piv_q)  # distinct pivot qubits
    order = stored_order(piv_q, n)
    subsets = [set(order[:k]) for k in (0, n // 4, n // 2, n - len(piv_q), n)]
    subsets += [set(np.flatnonzero(rng.random(n) < 0.5).tolist()) for _ in range(3)]
    seen = 0
    for t in range(1, min(tmax, g["P"]) + 1):
        for pk, c in combos(g, t):
            nz = nonzero_qubits(c, n)
            for i in pk:  # the lemma itself
                if pivots[i] >= 0:
                    assert nz[pivots[i]], (t, pk, i)
            w = int(nz.sum())
            for S in subsets:
                credit = sum(1 for i in pk if pivots[i] >= 0 and pivots[i] not in S)
                assert w >= int(sum(nz[q] for q in S)) + credit
            seen += 1
    return seen


def test_bound_f4_and_f2_matrices():
    rng = np.random.default_rng(7)
    total = 0
    codes = [O.expand(*W.config1(i)) for i in range(4)]
    codes += [rand_code(61000 + s, 9) for s in range(12)]
    for B in codes:
        if O.rank(B) == 0:
            continue
        n = B.shape[1] // 2
        for diag in (O.DIAG_F4, O.DIAG_F2):
            for g in O.gamma(B, diag, with_rows=True):
                total += check_matrix(g, n, 3, rng)
    assert total > 10000


def test_bound_wider_f4_code_low_rounds():
    # config 2's F4-linear shape (n = 48): rounds t <= 2 of both matrices
    rng = np.random.default_rng(8)
    B = O.expand(*W.config2(0))
    gs = O.gamma(B, O.DIAG_F4, with_rows=True)
    assert len(gs) >= 2
    for g in gs:
        assert check_matrix(g, B.shape[1] // 2, 2, rng) > 0


def test_bound_isometry_matrices():
    rng = np.random.default_rng(9)
    checked = 0
    for B in [O.expand(*W.config1(i)) for i in range(3)] + [rand_code(62000 + s, 8) for s in range(10)]:
        n = B.shape[1] // 2
        r, gs = O.gamma_iso(B, with_rows=True)
        for k, piv, rows in gs:
            cols = [int(c) for c in piv if c >= 0]
            per_qubit = np.bincount([c % n for c in cols], minlength=n)
            assert per_qubit.max(initial=0) <= 2
            for t in range(1, 4):
                for pk in itertools.combinations(range(len(piv)), t):
                    img = np.bitwise_xor.reduce(rows[list(pk)], axis=0)
                    assert all(img[piv[i]] == 1 for i in pk if piv[i] >= 0)
                    x, z = img[:n], img[n:2 * n]
                    nz = (x | z).astype(bool)
                    assert np.array_equal(img[2 * n:], x ^ z)
                    w = int(nz.sum())
                    for S in (set(range(n // 2)), set(np.flatnonzero(rng.random(n) < 0.5).tolist())):
                        outside = sum(1 for i in pk if piv[i] >= 0 and piv[i] % n not in S)
                        assert w >= int(sum(nz[q] for q in S)) + (outside + 1) // 2
                    checked += 1
    assert checked > 1000
