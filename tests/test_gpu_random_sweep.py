"""A seeded sweep of random codes through every path of the library
against the oracle's brute force (the definition of d).

Codes: additive with n = 3..60 and 2..20 rows (fewer, as many or more rows
than qubits, ragged word counts), F4-linear with k = 1..10.  Paths: the
automatic plan, each construction (F2, F4, isometry), partial weights
forced, mixed packages forced, and the plain walk; all codes also once as
a single batch.  Larger codes, beyond brute force, against the oracle's
BZ.  Every result is an integer and must match exactly, with a witness of
weight d in the row space."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import oracle as O
from paper_2408_10743_amd import workloads as W


@pytest.fixture(scope="module")
def Q():
    from paper_2408_10743_amd import qdist
    st, name = qdist.qd_device_check()
    assert st == 0, name
    return qdist


def swt(v):
    n = v.shape[-1] // 2
    return int(np.count_nonzero(v[:n] | v[n:]))


def codes(count=120):
    out = []
    for s in range(count):
        rng = W.SplitMix64(W.config_seed(90, s))
        if s % 3 == 2:
            n = rng.uniform_int(2, 40)
            k = rng.uniform_int(1, min(n, 10))
            out.append((W.f4_linear(n, k, rng.next()), 4))
        else:
            n = rng.uniform_int(3, 60)
            m = rng.uniform_int(2, 20)
            out.append((W.additive(n, m, rng.next()), 2))
    return out


def test_sweep_every_path(Q):
    cs = codes()
    Q_ = Q
    paths = [
        {},
        {"diag": Q_.QD_DIAG_F2},
        {"diag": Q_.QD_DIAG_F4},
        {"diag": Q_.QD_DIAG_ISO},
        {"partial_weight": 1},
        {"mixed_packages": 1, "partial_weight": 1},
        {"walk": 1},
        {"walk": 2, "diag": Q_.QD_DIAG_F4},
    ]
    checked = 0
    for i, (G, f) in enumerate(cs):
        B = O.expand(G, f)
        if O.rank(B) == 0:
            continue
        d_ref = O.brute(B)[0]
        for opts in paths:
            st, d, wit, s = Q.qd_distance_ex(G, f, **opts)
            if st == Q.QD_INCOMPLETE and opts.get("walk"):
                assert s.L <= d_ref <= s.U, (i, opts)  # the walk's depth limit
                continue
            assert st == 0, (i, opts, Q.qd_strerror(st))
            assert d == d_ref, (i, opts, d, d_ref)
            assert swt(wit) == d and O.in_rowspace(B, wit), (i, opts)
        checked += 1
    print(f"sweep: {checked} codes x {len(paths)} paths", flush=True)
    assert checked >= 100


def test_sweep_as_one_batch(Q):
    cs = [(G, f) for G, f in codes() if O.rank(O.expand(G, f)) > 0]
    st, ds, wits, sts, _ = Q.qd_distance_batch(cs)
    assert st == 0
    for (G, f), d, wit, s in zip(cs, ds, wits, sts):
        B = O.expand(G, f)
        assert s == 0 and d == O.brute(B)[0]
        assert swt(wit) == d and O.in_rowspace(B, wit)


def test_sweep_larger_codes_against_oracle_bz(Q):
    """Codes beyond brute force (additive, 22..30 rows and up to 120 qubits;
    F4-linear with k = 11..15), against the oracle's BZ, which the CPU tests
    pin to brute force: the automatic plan, F2, the isometry, the plain
    walk, 64-entry tiles, every word evaluated (partial_weight -1) and
    partial weights forced on every code with two or more words per half
    (partial_weight 1)."""
    paths = [{}, {"diag": Q.QD_DIAG_F2}, {"diag": Q.QD_DIAG_ISO}, {"walk": 1}, {"seg_len": 64},
             {"partial_weight": -1}, {"partial_weight": 1}]
    checked = 0
    for s in range(60):
        rng = W.SplitMix64(W.config_seed(92, s))
        if s % 4 == 3:
            n = rng.uniform_int(30, 64)
            G, f = W.f4_linear(n, rng.uniform_int(11, 15), rng.next()), 4
        else:
            n = rng.uniform_int(40, 120)
            m = rng.uniform_int(22, 30)
            G, f = W.additive(n, m, rng.next()), 2
        B = O.expand(G, f)
        d_ref = O.distance(G, f)[0]
        for opts in paths:
            st, d, wit, st_ = Q.qd_distance_ex(G, f, **opts)
            if st == Q.QD_INCOMPLETE and opts.get("walk"):
                assert st_.L <= d_ref <= st_.U, (s, opts)  # the walk's depth limit
                continue
            assert st == 0 and d == d_ref, (s, opts, st, d, d_ref)
            assert swt(wit) == d and O.in_rowspace(B, wit), (s, opts)
        checked += 1
    print(f"larger codes: {checked} x {len(paths)} paths", flush=True)
    assert checked == 60
