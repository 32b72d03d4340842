"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Distances and witness weights are integers and must match exactly; a
witness must lie in the row space.  Round-level checks compare one
enumeration round over seeded random package layouts with the oracle's
plain enumeration of the same round.
"""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import oracle as O
from paper_2408_10743_amd import workloads as W

GOLD_DIR = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def Q():
    from paper_2408_10743_amd import qdist
    st, name = qdist.qd_device_check()
    assert st == 0, f"no usable gfx950 device ({name}): {qdist.qd_strerror(st)}"
    return qdist


def swt(v):
    n = v.shape[-1] // 2
    return int(np.count_nonzero(v[:n] | v[n:]))


def check_distance(Q, G, field, d_ref, **opts):
    st, d, wit, stats = Q.qd_distance_ex(G, field, **opts)
    assert st == 0, Q.qd_strerror(st)
    assert d == d_ref
    assert swt(wit) == d
    assert O.in_rowspace(O.expand(G, field), wit)
    return stats


def test_device(Q):
    st, name = Q.qd_device_check()
    print("device", name, flush=True)
    assert st == 0 and "gfx950" in name


@pytest.mark.parametrize("n", [1, 5, 20, 31, 32, 33, 48, 64, 72, 96, 100, 128])
def test_round_min_random_packages(Q, n):
    for rep in range(3):
        rng = W.SplitMix64(W.config_seed(20, n * 10 + rep))
        P = rng.uniform_int(1, 14)
        frac = [1.0, 0.0, 0.5][rep]
        rows, dims = W.random_packages(P, n, rng.next(), frac)
        for t in range(1, min(P, 6) + 1):
            print(f"round n={n} rep={rep} P={P} t={t}", flush=True)
            st, w, wit, cnt = Q.qd_round_min(rows, dims, t)
            assert st == 0, Q.qd_strerror(st)
            wo, _, co = O.round_min(rows, dims, t)
            assert (w, cnt) == (wo, co)
            assert swt(wit) == w
            assert O.in_rowspace(rows, wit)


def test_round_min_large_round(Q):
    # several tiles per group, ragged item blocks and table tails
    rows, dims = W.random_packages(30, 72, W.config_seed(21, 0), 0.8)
    for t in (4, 5):
        print(f"large round t={t}", flush=True)
        st, w, wit, cnt = Q.qd_round_min(rows, dims, t)
        wo, _, co = O.round_min(rows, dims, t)
        assert st == 0 and (w, cnt) == (wo, co)
        assert swt(wit) == w


@pytest.mark.parametrize("D,w", [(2, 1), (3, 1), (3, 2), (4, 1), (4, 2), (4, 3)])
def test_round_min_partial_words(Q, D, w):
    """The partial-weight path of every (D, w): a round evaluated w words
    first gives the minimum and the count of the full evaluation and of the
    oracle's plain enumeration.  Dense random packages complete most blocks;
    packages confined to the first w words (so the full weight is the
    partial one) skip most of them.  t = 4 over 30 two-row packages is
    2.2e6 combinations, enough for saved tables and full blocks."""
    n = 32 * D - 3  # a ragged last word
    for concentrated in (False, True):
        rows, dims = W.random_packages(30, n, W.config_seed(26, 10 * D + w), 1.0)
        if concentrated:
            keep = np.zeros(2 * n, dtype=np.uint8)
            keep[:32 * w] = 1
            keep[n:n + 32 * w] = 1
            rows = rows * keep
        ref_w, _, ref_cnt = O.round_min(rows, dims, 4)
        st0, w0, wit0, c0 = Q.qd_round_min(rows, dims, 4)
        st1, w1, wit1, c1 = Q.qd_round_min(rows, dims, 4, partial_words=w)
        print(f"D={D} w={w} concentrated={concentrated} min={ref_w} count={ref_cnt}", flush=True)
        assert st0 == st1 == 0
        assert (w0, c0) == (w1, c1) == (ref_w, ref_cnt)
        assert swt(wit1) == w1
    # partial_words must be below D
    assert Q.qd_round_min(rows, dims, 4, partial_words=D)[0] == Q.QD_ERR_INVALID


def test_round_beyond_packages(Q):
    rows, dims = W.random_packages(3, 10, W.config_seed(21, 1))
    st, w, wit, cnt = Q.qd_round_min(rows, dims, 4)
    assert st == 0 and w == 11 and cnt == 0


def test_config1_against_brute_force(Q):
    for i in range(120):
        G, f = W.config1(i)
        d_ref, _ = O.brute(O.expand(G, f))
        print(f"config1 seed {i} d={d_ref}", flush=True)
        check_distance(Q, G, f, d_ref)


def test_config1_both_constructions(Q):
    for i in range(20):
        G, f = W.config1(i)
        d_ref, _ = O.brute(O.expand(G, f))
        for diag in (2, 4):
            s = check_distance(Q, G, f, d_ref, diag=diag)
            assert s.diag == diag


def test_config2_against_oracle(Q):
    gold = json.load(open(os.path.join(GOLD_DIR, "oracle_distances.json")))
    for i, d_ref in enumerate(gold["config2"][:10]):
        G, f = W.config2(i)
        print(f"config2 seed {i} d={d_ref}", flush=True)
        check_distance(Q, G, f, d_ref)


def test_config3_against_oracle(Q):
    gold = json.load(open(os.path.join(GOLD_DIR, "oracle_distances.json")))
    G, f = W.config3(0)
    print("config3 seed 0", flush=True)
    s = check_distance(Q, G, f, gold["config3"][0], timing=1)
    # every round enumerated the planned e_t(sizes) combinations except a
    # round cut short by the bound
    for r in s.rounds()[:-1]:
        assert r["combinations"] == r["planned"]


def test_structure_matches_oracle(Q):
    for i in range(10):
        G, f = W.config2(i) if i % 2 else W.config1(i)
        B = O.expand(G, f)
        st, d, wit, s = Q.qd_distance_ex(G, f)
        assert st == 0
        if s.diag == Q.QD_DIAG_ISO:  # the planner may pick the isometry for small codes
            r, gi = O.gamma_iso(B, 8)
            gs = [{"P": r, "delta": r - k} for k, _, _ in gi]
        else:
            gs = O.gamma(B, s.diag, 8)
        for j in range(s.h):
            assert (s.P[j], s.delta[j]) == (gs[j]["P"], gs[j]["delta"])


def test_edge_cases(Q):
    # one qubit, one row
    check_distance(Q, np.array([[1, 0]], np.uint8), 2, 1)
    # n = 128 (four words per half): span{X^n, Z^n} has d = n
    n = 128
    XZ = np.zeros((2, 2 * n), np.uint8); XZ[0, :n] = 1; XZ[1, n:] = 1
    check_distance(Q, XZ, 2, n)
    # full space: d = 1
    check_distance(Q, np.eye(2 * 9, dtype=np.uint8), 2, 1)
    # dependent rows
    G, f = W.config1(3)
    d_ref, _ = O.brute(O.expand(G, f))
    check_distance(Q, np.concatenate([G, G[:5] ^ G[5:10]]), 2, d_ref)
    # word boundaries
    for n in (31, 32, 33, 63, 64, 65, 95, 96, 97):
        G = W.additive(n, 14, W.config_seed(22, n))
        d_ref, _ = O.brute(O.expand(G, 2))
        check_distance(Q, G, 2, d_ref)
    # F4 input
    G = W.f4_linear(12, 5, W.config_seed(23, 0))
    d_ref, _ = O.brute(O.expand(G, 4))
    check_distance(Q, G, 4, d_ref)


def test_errors(Q):
    st, d, _ = Q.qd_distance(np.zeros((3, 8), np.uint8), 2)
    assert st == Q.QD_ERR_ZERO_CODE and d == -1
    st, d, _ = Q.qd_distance(np.full((2, 8), 2, np.uint8), 2)
    assert st == Q.QD_ERR_INVALID
    st, d, _ = Q.qd_distance(np.ones((2, 2 * 129), np.uint8), 2)
    assert st == Q.QD_ERR_TOO_LARGE


def test_tuning_overrides_do_not_change_results(Q):
    G, f = W.config2(1)
    gold = json.load(open(os.path.join(GOLD_DIR, "oracle_distances.json")))
    for seg, depth in ((8, 1), (64, 2), (4096, 4), (1024, 3)):
        check_distance(Q, G, f, gold["config2"][1], seg_len=seg, saved_depth=depth)


def test_tops_table_and_unranking_agree(Q):
    gold = json.load(open(os.path.join(GOLD_DIR, "oracle_distances.json")))
    for i in range(4):
        G, f = W.config2(i)
        for mode in (1, 2):
            for depth in (1, 3):
                check_distance(Q, G, f, gold["config2"][i], tops_mode=mode, saved_depth=depth)
    for i in range(10):
        G, f = W.config1(i)
        d_ref, _ = O.brute(O.expand(G, f))
        check_distance(Q, G, f, d_ref, tops_mode=2, diag=2)


def test_budget_gives_bounds(Q):
    G, f = W.config2(0)
    gold = json.load(open(os.path.join(GOLD_DIR, "oracle_distances.json")))
    st, d, wit, s = Q.qd_distance_ex(G, f, budget=100000)
    assert st == Q.QD_INCOMPLETE
    assert s.L <= gold["config2"][0] <= d
    assert swt(wit) == d


def test_invariance_on_gpu(Q):
    for i in range(10):
        G, f = W.config1(100 + i)
        n = G.shape[1] // 2
        st, d0, _ = Q.qd_distance(G, f)
        rng = W.SplitMix64(W.config_seed(24, i))
        perm = sorted(range(n), key=lambda _: rng.next())
        Gp = np.concatenate([G[:, perm], G[:, [n + q for q in perm]]], axis=1)
        Gs = np.concatenate([G[:, n:], G[:, :n]], axis=1)
        for V in (Gp, Gs):
            st2, d2, _ = Q.qd_distance(V, f)
            assert st == st2 == 0 and d2 == d0


def test_batch_equals_single(Q):
    codes = [W.config1(i) for i in range(6)] + [W.config2(i) for i in range(2)]
    st, ds, wits, sts, _ = Q.qd_distance_batch(codes)
    assert st == 0 and all(s == 0 for s in sts)
    for (G, f), d, w in zip(codes, ds, wits):
        st1, d1, _ = Q.qd_distance(G, f)
        assert st1 == 0 and d1 == d
        assert swt(w) == d


def test_valu_probes_run(Q):
    st, peak = Q.qd_valu_peak()
    assert st == 0 and peak > 1e12
    for name, mix in Q.QD_MIXES.items():
        st, v = Q.qd_valu_mix(mix)
        assert st == 0 and v > 1e12, name


def test_isometry_path_against_oracle(Q):
    """Saved_isometry on the GPU: the same distances as brute force and the
    oracle's Hamming BZ; every completed round visits C(r, t) rows subsets;
    the bound after each round is the oracle's Hamming bound, halved."""
    import math
    for i in range(30):
        G, f = W.config1(i)
        B = O.expand(G, f)
        d_ref, _ = O.brute(B)
        print(f"iso config1 seed {i} d={d_ref}", flush=True)
        s = check_distance(Q, G, f, d_ref, diag=Q.QD_DIAG_ISO)
        assert s.diag == Q.QD_DIAG_ISO
        d_o, _, olog = O.bz_iso(B, s.h)  # the matrices the planner kept
        assert d_o == d_ref
        rounds = s.rounds()
        for r, o in zip(rounds, olog):
            assert (r["t"], r["j"]) == (o[0], o[1])
            assert r["L"] == (o[2] + 1) // 2
            assert r["planned"] == math.comb(s.rank, r["t"])
        for r in rounds[:-1]:
            assert r["combinations"] == r["planned"]
    gold = json.load(open(os.path.join(GOLD_DIR, "oracle_distances.json")))
    for i in range(3):
        G, f = W.config2(i)
        print(f"iso config2 seed {i}", flush=True)
        check_distance(Q, G, f, gold["config2"][i], diag=Q.QD_DIAG_ISO)
    for n in (7, 33, 64, 65, 100, 128):
        G = W.additive(n, 14, W.config_seed(42, n))
        d_ref, _ = O.brute(O.expand(G, 2))
        print(f"iso additive n={n} d={d_ref}", flush=True)
        check_distance(Q, G, 2, d_ref, diag=Q.QD_DIAG_ISO)


def test_isometry_batch_and_mix(Q):
    codes = [W.config1(400 + i) for i in range(6)] + [W.config2(0)]
    st, ds, wits, sts, stats = Q.qd_distance_batch(codes, diag=Q.QD_DIAG_ISO)
    assert st == 0 and all(x == 0 for x in sts)
    for (G, f), d in zip(codes, ds):
        assert d == Q.qd_distance_ex(G, f, diag=Q.QD_DIAG_F4)[1]


def _stab_check(Q, A, d_ref, **opts):
    st, d, wit, s = Q.qd_distance_ex(A, 2, filter=Q.QD_FILTER_STABILIZER, **opts)
    assert st == 0, Q.qd_strerror(st)
    assert d == d_ref
    assert swt(wit) == d and O.in_rowspace(A, wit)
    n = A.shape[1] // 2
    if s.logical_pairs:
        prods = (A[:, :n].astype(int) @ wit[n:].astype(int) + A[:, n:].astype(int) @ wit[:n].astype(int)) % 2
        assert prods.any()  # the witness is no stabilizer
    return s


def test_stabilizer_filter_textbook(Q):
    ref = {"[[5,1,3]]": 3, "[[9,1,3]]": 3, "[[7,1,3]]": 3, "[[4,2,2]]": 2, "[[3,0,2]]": 2}
    for name, d in ref.items():
        A = W.textbook_code(name)
        for diag in (Q.QD_DIAG_F2, Q.QD_DIAG_F4):
            s = _stab_check(Q, A, d, diag=diag)
            assert s.logical_pairs == (A.shape[0] - A.shape[1] // 2 if name != "[[3,0,2]]" else 0)
    # the filter matters: without it Shor's code gives its weight-2 stabilizers
    assert Q.qd_distance(W.textbook_code("[[9,1,3]]"), 2)[1] == 2


def test_stabilizer_filter_random_codes(Q):
    for s in range(60):
        rng = W.SplitMix64(W.config_seed(21, s))
        n = rng.uniform_int(3, 14)
        k = rng.uniform_int(0, n)
        A = W.random_stabilizer(n, k, rng.next())
        d_ref = O.brute_stab(A)[0]
        print(f"stab n={n} k={k} d={d_ref}", flush=True)
        _stab_check(Q, A, d_ref)
    for s in range(12):
        rng = W.SplitMix64(W.config_seed(22, s))
        n = rng.uniform_int(16, 40)
        k = rng.uniform_int(1, n // 2)
        A = W.random_stabilizer(n, k, rng.next())
        d_ref = O.bz_stab(A, O.DIAG_F4, 8)[0]
        print(f"stab n={n} k={k} d={d_ref}", flush=True)
        _stab_check(Q, A, d_ref)
    # a generic span: the filter removes its radical
    for s in range(20):
        G = W.additive(12, 14, W.config_seed(23, s))
        _stab_check(Q, G, O.brute_stab(G)[0])


def test_stabilizer_filter_wide_code(Q):
    """D = 4: Shor's code on 9 of 100 qubits, single-qubit Z stabilizers on
    the others, qubits permuted.  d = 3; without the filter d = 1."""
    n = 100
    S = W.textbook_code("[[9,1,3]]")
    A = np.zeros((10 + 91, 2 * n), np.uint8)
    A[:10, :9] = S[:, :9]
    A[:10, n:n + 9] = S[:, 9:]
    for q in range(9, n):
        A[10 + q - 9, n + q] = 1
    rng = W.SplitMix64(W.config_seed(24, 0))
    perm = np.array(sorted(range(n), key=lambda q: rng.next()))
    A = np.concatenate([A[:, perm], A[:, n + perm]], axis=1)
    s = _stab_check(Q, A, 3)
    assert s.D == 4 and s.logical_pairs == 1
    assert Q.qd_distance(A, 2)[1] == 1


def test_stabilizer_filter_batch(Q):
    codes = [(W.random_stabilizer(10, 2, W.config_seed(25, i)), 2) for i in range(8)]
    codes.append((W.textbook_code("[[9,1,3]]"), 2))
    st, ds, wits, sts, stats = Q.qd_distance_batch(codes, filter=Q.QD_FILTER_STABILIZER)
    assert st == 0 and all(x == 0 for x in sts)
    for (A, f), d in zip(codes, ds):
        assert d == O.brute_stab(A)[0]


def test_f4_scalar_classes(Q):
    """F4-linear input: one codeword per class {c, alpha c, alpha^2 c} gives
    the same distance with a third of each round's combinations."""
    gold = json.load(open(os.path.join(GOLD_DIR, "oracle_distances.json")))
    for i in range(6):
        G, f = W.config2(i)
        print(f"scalar config2 seed {i}", flush=True)
        s1 = check_distance(Q, G, f, gold["config2"][i], diag=Q.QD_DIAG_F4)
        s0 = check_distance(Q, G, f, gold["config2"][i], diag=Q.QD_DIAG_F4, scalar_classes=-1)
        assert s1.scalar_classes == 1 and s0.scalar_classes == 0
        r1, r0 = s1.rounds(), s0.rounds()
        for a, b in zip(r1, r0):
            assert (a["t"], a["j"]) == (b["t"], b["j"])
            assert 3 * a["planned"] == b["planned"]
            assert a["L"] == b["L"]
        for a in r1[:-1]:
            assert a["combinations"] == a["planned"]
    for s in range(40):
        rng = W.SplitMix64(W.config_seed(26, s))
        n = rng.uniform_int(4, 40)
        k = rng.uniform_int(1, min(10, n))
        G = W.f4_linear(n, k, rng.next())
        d_ref = O.brute(O.expand(G, 4))[0]
        st, d, wit, s1 = Q.qd_distance_ex(G, 4)
        assert st == 0 and d == d_ref and swt(wit) == d, (s, n, k)
        assert O.in_rowspace(O.expand(G, 4), wit)
    # binary input never uses classes
    G, f = W.config1(0)
    assert Q.qd_distance_ex(G, f)[3].scalar_classes == 0


def test_stabilizer_filter_with_scalar_classes(Q):
    """F4-linear input with the filter: the radical of an F4-linear span is
    F4-linear, so one codeword per scalar class still finds the least
    admitted weight.  The five-qubit code in F4 form (two cyclic shifts of
    1 a a 1 0 and the logical 1 1 1 1 1), then random F4-linear spans."""
    base = [1, 2, 2, 1, 0]
    G4 = np.array([base[-i:] + base[:-i] for i in range(2)] + [[1, 1, 1, 1, 1]], dtype=np.uint8)
    for sc in (0, -1):
        st, d, wit, s = Q.qd_distance_ex(G4, 4, filter=Q.QD_FILTER_STABILIZER, scalar_classes=sc)
        assert st == 0 and d == 3 and s.logical_pairs == 1
        assert s.scalar_classes == (1 if sc == 0 and s.diag == Q.QD_DIAG_F4 else 0)
    for s_ in range(30):
        rng = W.SplitMix64(W.config_seed(27, s_))
        n = rng.uniform_int(3, 12)
        k = rng.uniform_int(1, min(6, n))
        G = W.f4_linear(n, k, rng.next())
        B = O.expand(G, 4)
        d_ref = O.brute_stab(B)[0]
        for sc in (0, -1):
            st, d, wit, s = Q.qd_distance_ex(G, 4, filter=Q.QD_FILTER_STABILIZER, scalar_classes=sc, diag=Q.QD_DIAG_F4)
            assert st == 0 and d == d_ref, (s_, n, k, sc)
            assert swt(wit) == d and O.in_rowspace(B, wit)


def test_scalar_classes_for_alpha_closed_binary_input(Q):
    gold = json.load(open(os.path.join(GOLD_DIR, "oracle_distances.json")))
    for i in range(3):
        G, f = W.config2(i)
        B = O.expand(G, f)
        st, d, wit, s = Q.qd_distance_ex(B, 2, diag=Q.QD_DIAG_F4)
        assert st == 0 and d == gold["config2"][i] and s.scalar_classes == 1
    A = W.textbook_code("[[5,1,3]]")
    st, d, wit, s = Q.qd_distance_ex(A, 2, filter=Q.QD_FILTER_STABILIZER, diag=Q.QD_DIAG_F4)
    assert st == 0 and d == 3 and s.scalar_classes == 1
