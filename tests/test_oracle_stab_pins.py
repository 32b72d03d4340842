"""Pins of the oracle's Modified Brouwer-Zimmermann (Sec. 2.1) for quantum
stabilizer codes: the least weight over C^{perp_s} \\ C, with every codeword
counted when k = 0.

Independent facts: textbook codes ([[5,1,3]], Shor's degenerate [[9,1,3]],
Steane's [[7,1,3]], [[4,2,2]], a k = 0 state), a Python exhaustive search
with its own commutation test, and invariance under qubit permutations,
local symplectic maps and row operations.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2408_10743_amd import workloads as W

from test_oracle_pins import rand_code, swt

TEXTBOOK = {"[[5,1,3]]": 3, "[[9,1,3]]": 3, "[[7,1,3]]": 3, "[[4,2,2]]": 2, "[[3,0,2]]": 2}


def sym(a, b):
    n = a.shape[-1] // 2
    return int((a[:n].astype(int) @ b[n:].astype(int) + a[n:].astype(int) @ b[:n].astype(int)) % 2)


def py_stab(B):
    """Least weight over the nonzero span minus the codewords commuting with
    every row; every codeword counts when all rows commute (k = 0)."""
    B = np.asarray(B, dtype=np.uint8)
    m = B.shape[0]
    k0 = all(sym(B[i], B[j]) == 0 for i in range(m) for j in range(m))
    best = None
    for mask in range(1, 1 << m):
        c = np.zeros(B.shape[1], dtype=np.uint8)
        for i in range(m):
            if (mask >> i) & 1:
                c ^= B[i]
        w = swt(c)
        if not w:
            continue
        if not k0 and all(sym(c, B[i]) == 0 for i in range(m)):
            continue
        if best is None or w < best:
            best = w
    return best


def normalizer_ok(A, n, k):
    """Rank n + k and a radical (stabilizer) of dimension n - k."""
    m = A.shape[0]
    G = np.array([[sym(A[i], A[j]) for j in range(m)] for i in range(m)], dtype=np.uint8)
    return O.rank(A) == n + k and O.rank(np.concatenate([G, np.zeros_like(G)], axis=1)) == 2 * k


@pytest.mark.parametrize("name", sorted(TEXTBOOK))
def test_textbook_codes(name):
    A = W.textbook_code(name)
    d = TEXTBOOK[name]
    assert O.brute_stab(A)[0] == d
    for diag in (O.DIAG_F2, O.DIAG_F4):
        dd, wit, _ = O.bz_stab(A, diag)
        assert dd == d and swt(wit) == d and O.in_rowspace(A, wit)
    assert py_stab(A) == d


def test_filter_matters_for_shor_code():
    A = W.textbook_code("[[9,1,3]]")
    assert O.brute(A)[0] == 2  # weight-2 stabilizers: the whole span has d = 2
    d, wit, _ = O.bz_stab(A)
    assert d == 3
    assert any(sym(wit, A[i]) for i in range(A.shape[0]))  # the witness is no stabilizer


def test_random_stabilizer_generator_gives_normalizers():
    for s in range(30):
        rng = W.SplitMix64(W.config_seed(17, s))
        n = rng.uniform_int(2, 9)
        k = rng.uniform_int(0, n)
        A = W.random_stabilizer(n, k, rng.next())
        assert A.shape == (n + k, 2 * n)
        assert normalizer_ok(A, n, k), (s, n, k)
        # the first n - k rows commute with every row
        assert all(sym(A[i], A[j]) == 0 for i in range(n - k) for j in range(n + k))


def test_brute_matches_python_on_stabilizer_codes():
    for s in range(60):
        rng = W.SplitMix64(W.config_seed(18, s))
        n = rng.uniform_int(2, 6)
        k = rng.uniform_int(0, n)
        A = W.random_stabilizer(n, k, rng.next())
        if A.shape[0] > 11:
            continue
        d, wit = O.brute_stab(A)
        assert d == py_stab(A), (s, n, k)
        assert swt(wit) == d


def test_bz_matches_brute_on_stabilizer_codes():
    for s in range(200):
        rng = W.SplitMix64(W.config_seed(19, s))
        n = rng.uniform_int(2, 10)
        k = rng.uniform_int(0, n)
        A = W.random_stabilizer(n, k, rng.next())
        d0, _ = O.brute_stab(A)
        for diag in (O.DIAG_F2, O.DIAG_F4):
            d, wit, _ = O.bz_stab(A, diag, 8)
            assert d == d0, (s, n, k, diag)
            assert swt(wit) == d and O.in_rowspace(A, wit)
            if k > 0:
                assert any(sym(wit, A[i]) for i in range(A.shape[0]))


def test_bz_matches_brute_on_generic_spans():
    # any span: the filter removes its symplectic radical
    for s in range(300):
        B = rand_code(55000 + s, 6)
        if B.shape[0] > 11:
            B = B[:11]
        if not B.any():
            continue
        d0 = py_stab(B)
        assert O.brute_stab(B)[0] == d0, s
        assert O.bz_stab(B, O.DIAG_F4, 8)[0] == d0, s


def test_invariance():
    for s in range(40):
        rng = W.SplitMix64(W.config_seed(20, s))
        n = rng.uniform_int(3, 8)
        k = rng.uniform_int(1, n)
        A = W.random_stabilizer(n, k, rng.next())
        d = O.bz_stab(A)[0]
        # qubit permutation
        perm = np.array(sorted(range(n), key=lambda q: rng.next()))
        P = np.concatenate([A[:, perm], A[:, n + perm]], axis=1)
        assert O.bz_stab(P)[0] == d
        # local symplectic map on one qubit: (x, z) -> (z, x ^ z)
        q = rng.uniform_int(0, n - 1)
        L = A.copy()
        L[:, q], L[:, n + q] = A[:, n + q], A[:, q] ^ A[:, n + q]
        assert O.bz_stab(L)[0] == d
        # row operations
        R = A.copy()
        for i in range(1, R.shape[0]):
            R[i] ^= R[i - 1]
        assert O.bz_stab(R)[0] == d
