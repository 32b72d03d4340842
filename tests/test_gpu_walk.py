"""GPU parity of the plain walk kernel (qd_options.walk, qd_round_walk):
package sets in revolving-door order, element choices in reflected ternary
Gray order, one launch per round.

Round minima and combination counts equal the oracle's plain enumeration
of the same round.  The sum of the weights of every codeword walked equals
the sum over the round's combinations enumerated here with numpy, which a
skipped or repeated codeword would change.  Distances with the walk equal
the oracle's."""
import itertools
import json
import os

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


def round_weight_sum(rows, dims, t):
    """Sum of the symplectic weights of every combination of the round."""
    n = rows.shape[1] // 2
    els = []
    for i, d in enumerate(dims):
        r, s = rows[2 * i], rows[2 * i + 1]
        els.append(np.stack([r, s, r ^ s]) if d == 2 else r[None, :])
    total = 0
    for S in itertools.combinations(range(len(dims)), t):
        acc = np.zeros((1, 2 * n), dtype=np.uint8)
        for p in S:
            acc = (acc[:, None, :] ^ els[p][None, :, :]).reshape(-1, 2 * n)
        total += int(np.count_nonzero(acc[:, :n] | acc[:, n:], axis=1).sum())
    return total


def check_round(Q, rows, dims, t, per_lane, with_sum):
    st, w, wit, cnt, ws = Q.qd_round_walk(rows, dims, t, per_lane=per_lane, weight_sum=with_sum)
    assert st == 0, Q.qd_strerror(st)
    wo, _, co = O.round_min(rows, dims, t)
    assert (w, cnt) == (wo, co)
    assert swt(wit) == w and O.in_rowspace(rows, wit)
    if with_sum:
        assert ws == round_weight_sum(rows, dims, t)


@pytest.mark.parametrize("n", [5, 31, 33, 64, 72, 100, 128])
def test_walk_rounds_against_oracle(Q, n):
    """Two-row, one-row and mixed layouts, t up to 6, 1..5 sets per lane
    (ragged lane ranges and idle lanes in the last wave)."""
    for rep in range(3):
        rng = W.SplitMix64(W.config_seed(80, n * 10 + rep))
        P = rng.uniform_int(2, 11)
        frac = [1.0, 0.0, 0.5][rep]
        rows, dims = W.random_packages(P, n, rng.next(), frac)
        for t in range(1, min(P, 6) + 1):
            for per_lane in (1, 2, 5):
                small = len(list(itertools.combinations(range(P), t))) * 3 ** t <= 60000
                print(f"walk n={n} rep={rep} P={P} t={t} per_lane={per_lane}", flush=True)
                check_round(Q, rows, dims, t, per_lane, small)


def test_walk_deep_digits(Q):
    """t = 7 and 8: every slot's digit moves (digits 2..7 from the staged
    elements)."""
    for P, t, frac in [(8, 7, 1.0), (8, 8, 1.0), (9, 7, 0.7), (10, 8, 1.0)]:
        rows, dims = W.random_packages(P, 77, W.config_seed(81, P * 10 + t), frac)
        print(f"deep P={P} t={t}", flush=True)
        check_round(Q, rows, dims, t, 3, P <= 8)


def test_walk_many_packages(Q):
    """Up to 256 packages: the elements and binomials no longer fit the
    LDS staging (read from global memory instead), and package numbers above
    127 sit in the high digits' 8-bit fields.  The saved-sum engine runs the
    same rounds."""
    for P, t, frac, n in [(150, 3, 0.5, 100), (256, 4, 0.0, 128), (96, 4, 0.0, 64)]:
        rows, dims = W.random_packages(P, n, W.config_seed(86, P + t), frac)
        print(f"many packages P={P} t={t}", flush=True)
        check_round(Q, rows, dims, t, 2, False)
        # the saved-sum engine on the same round
        st0, w0, wit0, c0 = Q.qd_round_min(rows, dims, t)
        wo, _, co = O.round_min(rows, dims, t)
        assert st0 == 0 and (w0, c0) == (wo, co) and swt(wit0) == w0


def test_walk_many_waves(Q):
    """A round of 1.7e8 combinations over several thousand waves."""
    rows, dims = W.random_packages(30, 72, W.config_seed(82, 0), 1.0)
    for per_lane in (1, 4):
        st, w, wit, cnt, _ = Q.qd_round_walk(rows, dims, 5, per_lane=per_lane)
        st0, w0, wit0, c0 = Q.qd_round_min(rows, dims, 5)
        print(f"many waves per_lane={per_lane}: {w} {cnt}", flush=True)
        assert st == st0 == 0 and (w, cnt) == (w0, c0)
        assert swt(wit) == w and O.in_rowspace(rows, wit)


def test_walk_round_limits(Q):
    rows, dims = W.random_packages(10, 20, W.config_seed(83, 0))
    assert Q.qd_round_walk(rows, dims, 9)[0] == Q.QD_ERR_TOO_LARGE
    assert Q.qd_round_walk(rows, dims, 3, per_lane=0)[0] == Q.QD_ERR_INVALID
    st, w, _, cnt, ws = Q.qd_round_walk(rows[:6], dims[:3], 4, weight_sum=True)  # t > P
    assert st == 0 and w == 21 and cnt == 0 and ws == 0


def test_walk_distances(Q):
    """qd_distance with the walk: config 1 against brute force (F4, F2 and
    isometry constructions), config 2 and small additive codes against the oracle's
    BZ; every round but the last is walked whole."""
    for i in range(6):
        G, f = W.config1(i)
        d_ref = O.brute(O.expand(G, f))[0]
        for diag, walk in [(Q.QD_DIAG_F4, 1), (Q.QD_DIAG_F4, 3), (Q.QD_DIAG_F2, 2), (Q.QD_DIAG_ISO, 1)]:
            st, d, wit, s = Q.qd_distance_ex(G, f, diag=diag, walk=walk)
            print(f"config1 {i} diag={diag} walk={walk} d={d} ref={d_ref}", flush=True)
            assert st == 0 and d == d_ref and swt(wit) == d
            assert O.in_rowspace(O.expand(G, f), wit)
            rounds = s.rounds()  # every round walked whole; the last may stop once U meets L
            assert all(r["combinations"] == r["planned"] for r in rounds[:-1])
            assert rounds[-1]["combinations"] <= rounds[-1]["planned"]
    for i in range(3):
        G, f = W.config2(i)
        d_ref = O.distance(G, f)[0]
        st, d, wit, s = Q.qd_distance_ex(G, f, walk=1)
        st2, d2, _, s2 = Q.qd_distance_ex(G, f)
        print(f"config2 {i} d={d} ref={d_ref} walk combos {s.combinations} engine {s2.combinations}", flush=True)
        assert st == st2 == 0 and d == d2 == d_ref and swt(wit) == d
        assert s.scalar_classes == 0
    for s_ in range(8):
        rng = W.SplitMix64(W.config_seed(84, s_))
        n = rng.uniform_int(12, 40)
        B = W.additive(n, rng.uniform_int(n // 2, n), rng.next())
        if O.rank(B) == 0:
            continue
        d_ref = O.brute(B)[0] if O.rank(B) <= 22 else O.bz(B)[0]
        st, d, wit, s = Q.qd_distance_ex(B, 2, walk=1)
        print(f"additive n={n} d={d} ref={d_ref} status={st}", flush=True)
        assert st in (0, Q.QD_INCOMPLETE)
        if st == 0:
            assert d == d_ref and swt(wit) == d and O.in_rowspace(B, wit)
        else:  # a round deeper than 8 packages: certified bounds only
            assert s.L <= d_ref <= s.U


def test_walk_config3(Q):
    """Config 3 as bench.py's walk leg runs it: the golden distance, every
    round but the last walked whole, and the same per-round minima and
    bounds as the saved-sum engine with every word evaluated."""
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_distances.json")))
    G, f = W.config3(0)
    st, d, wit, s = Q.qd_distance_ex(G, f, walk=1, timing=1)
    st2, d2, _, s2 = Q.qd_distance_ex(G, f, partial_weight=-1, mixed_packages=-1)
    print(f"config3 walk d={d} in {s.wall_ms:.2f} ms, engine d={d2}", flush=True)
    assert st == st2 == 0 and d == d2 == gold["config3"][0]
    assert swt(wit) == d and O.in_rowspace(O.expand(G, f), wit)
    rw, re_ = s.rounds(), s2.rounds()
    assert [(r["t"], r["j"], r["L"]) for r in rw] == [(r["t"], r["j"], r["L"]) for r in re_]
    assert all(r["combinations"] == r["planned"] for r in rw[:-1])
    assert all(r["launches"] == 1 for r in rw)


def test_walk_depth_limit_gives_bounds(Q):
    """A round deeper than 8 packages ends the walk with QD_INCOMPLETE and
    certified bounds: 12 random rows on 128 qubits under the F2
    construction (one matrix of 12 packages, distance far above the L = 9
    that rounds t <= 8 certify)."""
    B = W.additive(128, 12, W.config_seed(85, 0))
    d_ref = O.brute(B)[0]
    st, d, wit, s = Q.qd_distance_ex(B, 2, diag=Q.QD_DIAG_F2, walk=1)
    print(f"depth limit: status={st} L={s.L} U={s.U} d={d_ref}", flush=True)
    assert st == Q.QD_INCOMPLETE
    assert s.L == 9 - s.delta[0] and s.L <= d_ref <= s.U == d
    assert swt(wit) == d and O.in_rowspace(B, wit)
    assert max(r["t"] for r in s.rounds()) == 8
    # the engine certifies the same code exactly
    st2, d2, _, _ = Q.qd_distance_ex(B, 2, diag=Q.QD_DIAG_F2)
    assert st2 == 0 and d2 == d_ref


def test_walk_and_engine_codes_share_steps(Q):
    """Requests on the walk and on the saved-sum engine in one serving
    engine: their pieces run in the same steps (one launch kind each), and
    every result equals the code alone on its own path."""
    import time
    codes = [W.config1(i) for i in range(6)] + [W.config2(i) for i in range(3)]
    alone = {}
    for i, (G, f) in enumerate(codes):
        walk = 1 if i % 2 else 0
        st, d, _, _ = Q.qd_distance_ex(G, f, walk=walk)
        assert st == 0
        alone[i] = d
    eng = Q.qd_engine_create()
    assert eng
    try:
        for i, (G, f) in enumerate(codes):
            assert Q.qd_engine_submit(eng, G, f, tag=i, walk=1 if i % 2 else 0) == 0
        got = {}
        t0 = time.time()
        while len(got) < len(codes) and time.time() - t0 < 60:
            for r, wit in Q.qd_engine_poll(eng, 64, 100):
                got[r.tag] = (r.status, r.d, swt(wit))
        print(f"mixed engine: {got}", flush=True)
        assert len(got) == len(codes)
        for i in range(len(codes)):
            assert got[i] == (0, alone[i], alone[i])
    finally:
        Q.qd_engine_destroy(eng)


def test_walk_options(Q):
    G, f = W.config1(0)
    assert Q.qd_distance_ex(G, f, walk=-1)[0] == Q.QD_ERR_INVALID
    assert Q.qd_distance_ex(G, f, walk=5000)[0] == Q.QD_ERR_INVALID
    assert Q.qd_distance_ex(G, f, walk=1, filter=Q.QD_FILTER_STABILIZER)[0] == Q.QD_ERR_INVALID
