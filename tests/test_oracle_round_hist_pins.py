"""Pins of the oracle's round weight distribution (qdo_round_hist).

The distribution of one round (every choice of t distinct packages and one
nonzero element of each, Sec. 2.3; symplectic weight of the sum, Sec. 2) is
checked against an independent Python enumeration, against closed forms
whose every combination has a known weight, and against the oracle's own
round minimum and the e_t(sizes) count.  All run on the CPU.
"""
import itertools
import math

import numpy as np

from oracle import oracle as O
from paper_2408_10743_amd import workloads as W

from test_oracle_pins import elements, esym, swt


def py_hist(rows, dims, t):
    n = rows.shape[1] // 2
    els = elements(rows, dims)
    hist = np.zeros(n + 1, dtype=np.int64)
    for sub in itertools.combinations(range(len(dims)), t):
        for pick in itertools.product(*[els[i] for i in sub]):
            hist[swt(np.bitwise_xor.reduce(np.array(pick), axis=0))] += 1
    return hist


def test_hist_matches_python_enumeration():
    for s in range(30):
        rng = W.SplitMix64(W.config_seed(83, s))
        P = rng.uniform_int(1, 7)
        n = rng.uniform_int(1, 70)
        rows, dims = W.random_packages(P, n, rng.next(), two_dim_fraction=0.6)
        sizes = [3 if d == 2 else 1 for d in dims]
        for t in range(1, P + 1):
            h = O.round_hist(rows, dims, t)
            assert (h.astype(np.int64) == py_hist(rows, dims, t)).all()
            assert int(h.sum()) == esym(sizes, t)
            w, _, cnt = O.round_min(rows, dims, t)
            assert cnt == int(h.sum())
            assert w == int(np.flatnonzero(h)[0])


def _pauli_packages(P, n, dim):
    """Package i lives on qubit i alone: {X_i} (dim 1) or {X_i, Z_i, Y_i}."""
    rows = np.zeros((2 * P, 2 * n), dtype=np.uint8)
    for i in range(P):
        rows[2 * i, i] = 1
        rows[2 * i + 1, n + i] = 1
    return rows, [dim] * P


def test_closed_form_disjoint_qubits():
    # Every combination of t packages on t distinct qubits has weight t:
    # hist[t] = C(P, t) c^t for package size c, zero elsewhere.
    for dim, c in ((1, 1), (2, 3)):
        for P, n in ((5, 5), (9, 40), (12, 100)):
            rows, dims = _pauli_packages(P, n, dim)
            for t in range(1, min(P, 6) + 1):
                h = O.round_hist(rows, dims, t)
                ref = np.zeros(n + 1, dtype=np.uint64)
                ref[t] = math.comb(P, t) * c ** t
                assert (h == ref).all(), (dim, P, n, t)


def test_closed_form_repeated_row():
    # P one-row packages that are all X_1: a sum of t of them is X_1 for odd
    # t and zero for even t.
    for P in (3, 6, 9):
        n = 4
        rows = np.zeros((2 * P, 2 * n), dtype=np.uint8)
        rows[0::2, 0] = 1
        for t in range(1, P + 1):
            h = O.round_hist(rows, [1] * P, t)
            ref = np.zeros(n + 1, dtype=np.uint64)
            ref[t % 2] = math.comb(P, t)
            assert (h == ref).all()


def test_closed_form_weight_distribution_of_full_space():
    # The n two-row packages {X_i, Z_i, Y_i}, all rounds together, enumerate
    # every nonzero vector of F2^2n once: sum_t hist_t[w] = C(n, w) 3^w.
    for n in (3, 5, 8):
        rows, dims = _pauli_packages(n, n, 2)
        tot = np.zeros(n + 1, dtype=np.uint64)
        for t in range(1, n + 1):
            tot += O.round_hist(rows, dims, t)
        assert [int(x) for x in tot] == [0] + [math.comb(n, w) * 3 ** w for w in range(1, n + 1)]
