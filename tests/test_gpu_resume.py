"""Resuming incomplete calls (qd_options.resume): a call stopped by its
budget, its cancel flag (also in the middle of a round) or the plain walk's
depth limit continues from its first unfinished round with the bounds it
had, and reaches the distance of an uninterrupted call (with the same
rounds in total when it stopped between rounds)."""
import ctypes
import json
import os
import threading

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


def test_resume_config3_in_pieces(Q):
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_distances.json")))
    G, f = W.config3(0)
    st0, d0, w0, s0 = Q.qd_distance_ex(G, f)
    assert st0 == 0 and d0 == gold["config3"][0]
    total, point, calls = 0, None, 0
    for budget in (10 ** 9, 2 * 10 ** 10, 0):
        opts = {"budget": budget}
        if point is not None:
            opts["resume"] = point
        st, d, w, s = Q.qd_distance_ex(G, f, **opts)
        rounds = s.rounds()
        print(f"budget {budget}: status {st} L={s.L} U={s.U} next=({s.next_t},{s.next_j}) "
              f"rounds {[(r['t'], r['j']) for r in rounds]}", flush=True)
        if point is not None and rounds:
            assert (rounds[0]["t"], rounds[0]["j"]) == point[:2]
        assert s.structure == s0.structure
        total += s.combinations
        calls += 1
        if st == 0:
            break
        assert st == Q.QD_INCOMPLETE and s.L <= d0 <= s.U
        point = Q.resume_point(s, w)
    assert st == 0 and d == d0 and swt(w) == d and O.in_rowspace(O.expand(G, f), w)
    assert calls >= 2
    assert total == s0.combinations


def test_resume_after_the_walks_depth_limit(Q):
    """The walk stops before round 9 with certified bounds; the saved-sum
    engine on the same matrices (F2 construction) finishes from there."""
    B = W.additive(128, 12, W.config_seed(85, 0))
    d_ref = O.brute(B)[0]
    st, d, w, s = Q.qd_distance_ex(B, 2, diag=Q.QD_DIAG_F2, walk=1)
    assert st == Q.QD_INCOMPLETE and (s.next_t, s.next_j) == (9, 0)
    st2, d2, w2, s2 = Q.qd_distance_ex(B, 2, diag=Q.QD_DIAG_F2, resume=Q.resume_point(s, w))
    print(f"walk then engine: L={s.L} U={s.U} -> d={d2} (brute {d_ref}), first round "
          f"{s2.rounds()[0]['t'] if s2.rounds() else None}", flush=True)
    assert st2 == 0 and d2 == d_ref and swt(w2) == d2 and O.in_rowspace(B, w2)
    assert all(r["t"] >= 9 for r in s2.rounds())


def test_resume_rejects_other_matrices_and_witnesses(Q):
    G, f = W.config2(0)
    st, d, w, s = Q.qd_distance_ex(G, f, budget=10 ** 5)
    assert st == Q.QD_INCOMPLETE
    point = Q.resume_point(s, w)
    # other matrices: the F2 construction of the same code
    assert Q.qd_distance_ex(G, f, diag=Q.QD_DIAG_F2, resume=point)[0] == Q.QD_ERR_INVALID
    # a witness that does not have weight U
    if point[3] is not None:
        bad = point[3].copy()
        bad[:] = 0
        assert Q.qd_distance_ex(G, f, resume=(point[0], point[1], point[2], bad, point[4]))[0] == Q.QD_ERR_INVALID
    # the right point still works
    st2, d2, w2, _ = Q.qd_distance_ex(G, f, resume=point)
    assert st2 == 0 and d2 == O.distance(G, f)[0]


def test_cancel_before_the_first_round_then_resume(Q):
    G, f = W.config1(3)
    d_ref = O.brute(O.expand(G, f))[0]
    flag = ctypes.c_int(1)
    st, d, w, s = Q.qd_distance_ex(G, f, cancel=flag)
    assert st == Q.QD_INCOMPLETE and (s.next_t, s.next_j) == (1, 0) and s.U == 21 and s.combinations == 0
    st2, d2, w2, _ = Q.qd_distance_ex(G, f, resume=Q.resume_point(s, w))
    assert st2 == 0 and d2 == d_ref and swt(w2) == d2


def test_cancel_mid_round_then_resume(Q):
    """With a cancel flag a long round spans several steps; a flag set while
    config 3 runs stops it at a step boundary with valid bounds and a resume
    point, and the resumed call reaches d."""
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_distances.json")))
    G, f = W.config3(0)
    d_ref = gold["config3"][0]
    for delay in (0.0005, 0.002):
        flag = ctypes.c_int(0)
        timer = threading.Timer(delay, lambda: setattr(flag, "value", 1))
        timer.start()
        st, d, w, s = Q.qd_distance_ex(G, f, cancel=flag)
        timer.join()
        print(f"cancel after {delay * 1e3:.1f} ms: status {st} L={s.L} U={s.U} next=({s.next_t},{s.next_j}) "
              f"{s.wall_ms:.2f} ms", flush=True)
        if st == 0:  # finished before the flag was seen
            assert d == d_ref
            continue
        assert st == Q.QD_INCOMPLETE and s.L <= d_ref <= s.U
        if s.U <= s.n:
            assert swt(w) == s.U and O.in_rowspace(O.expand(G, f), w)
        st2, d2, w2, s2 = Q.qd_distance_ex(G, f, resume=Q.resume_point(s, w))
        assert st2 == 0 and d2 == d_ref and swt(w2) == d2
