"""Pins of the oracle's membership test and symplectic weight.

Every GPU test checks that a witness lies in the row space with
O.in_rowspace, so that function must also say "no" to every vector outside
the span.  Here it is compared, for EVERY vector of F2^{2n} on small codes,
with the span written out in plain Python (all 2^m subset sums), on
full-rank, rank-deficient and all-zero generator sets.  The symplectic
weight (Sec. 2, #{i : a_i != 0 or b_i != 0}) is pinned by counting: over
all 4^n vectors of n qubits, exactly C(n, w) 3^w have weight w (each of the
w supporting qubits carries one of the three nonzero pairs (1,0), (0,1),
(1,1)).
"""
import itertools
import math

import numpy as np

from oracle import oracle as O
from paper_2408_10743_amd import workloads as W


def py_span(B):
    """Set of all F2 combinations of the rows of B (as byte strings)."""
    B = np.asarray(B, dtype=np.uint8)
    out = set()
    for mask in range(1 << B.shape[0]):
        c = np.zeros(B.shape[1], dtype=np.uint8)
        for i in range(B.shape[0]):
            if (mask >> i) & 1:
                c ^= B[i]
        out.add(c.tobytes())
    return out


def all_vectors(n):
    for bits in itertools.product((0, 1), repeat=2 * n):
        yield np.array(bits, dtype=np.uint8)


def check_membership(B):
    span = py_span(B)
    n = B.shape[1] // 2
    members = 0
    for v in all_vectors(n):
        inside = v.tobytes() in span
        assert O.in_rowspace(B, v) == inside, (B.tolist(), v.tolist())
        members += inside
    return members


def test_in_rowspace_every_vector_random_codes():
    seen_outside = 0
    for s in range(60):
        rng = W.SplitMix64(W.config_seed(80, s))
        n = rng.uniform_int(1, 4)
        m = rng.uniform_int(1, 2 * n + 2)  # m > 2n forces dependent rows
        B = W.additive(n, m, rng.next())
        members = check_membership(B)
        assert members == 2 ** O.rank(B) if B.any() else members == 1
        seen_outside += 4 ** n - members
    assert seen_outside > 1000  # most checked vectors are non-members


def test_in_rowspace_rank_deficient_and_zero():
    # duplicated and summed rows: rank 2 out of 4 rows
    r0 = np.array([1, 0, 1, 0, 0, 1], dtype=np.uint8)
    r1 = np.array([0, 1, 1, 1, 0, 0], dtype=np.uint8)
    B = np.stack([r0, r1, r0 ^ r1, r0])
    assert check_membership(B) == 4
    # a basis row plus a unit vector outside the span is not a member
    e = np.zeros(6, dtype=np.uint8)
    e[5] = 1
    assert O.in_rowspace(B, r0) and not O.in_rowspace(B, r0 ^ e)
    # the zero code holds only the zero vector
    Z = np.zeros((3, 6), dtype=np.uint8)
    assert check_membership(Z) == 1
    assert O.in_rowspace(Z, np.zeros(6, dtype=np.uint8))


def test_in_rowspace_wide_code_non_members():
    # n = 72 (the throughput workload's shape): a codeword is a member, and
    # flipping any single bit of it leaves the span unless that unit vector
    # is itself in the span (checked by rank)
    G, _ = W.config3(0)
    B = G[:40]
    rng = W.SplitMix64(W.config_seed(81, 0))
    c = np.zeros(144, dtype=np.uint8)
    for i in range(40):
        if rng.next() & 1:
            c ^= B[i]
    assert O.in_rowspace(B, c)
    r = O.rank(B)
    for bit in range(0, 144, 7):
        e = np.zeros(144, dtype=np.uint8)
        e[bit] = 1
        unit_inside = O.rank(np.vstack([B, e])) == r
        assert O.in_rowspace(B, c ^ e) == unit_inside
        assert not unit_inside  # 40 random rows of length 144 contain no unit vector


def test_symplectic_weight_counts():
    for n in range(1, 6):
        hist = [0] * (n + 1)
        for v in all_vectors(n):
            hist[O.symplectic_weight(v, n)] += 1
        assert hist == [math.comb(n, w) * 3 ** w for w in range(n + 1)]


def test_symplectic_weight_single_qubit_pairs():
    # (a_i, b_i) = (0,0) contributes 0; (1,0), (0,1), (1,1) contribute 1
    for a, b in itertools.product((0, 1), repeat=2):
        assert O.symplectic_weight(np.array([a, b], dtype=np.uint8), 1) == (1 if a or b else 0)
