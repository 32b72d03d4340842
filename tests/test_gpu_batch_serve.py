"""GPU checks of the batched entry point and the serving engine: every
result equals the oracle's and the same code's qd_distance alone (exact,
tolerance 0), whatever else shares the device steps."""
import json
import os
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import oracle as O
from paper_2408_10743_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_distances.json")))


@pytest.fixture(scope="module")
def Q():
    from paper_2408_10743_amd import qdist
    st, name = qdist.qd_device_check()
    assert st == 0, name
    return qdist


def swt(v):
    n = v.shape[-1] // 2
    return int(np.count_nonzero(v[:n] | v[n:]))


def mixed_codes():
    codes, ref = [], []
    for i in range(16):
        G, f = W.config1(200 + i)
        codes.append((G, f)); ref.append(O.brute(O.expand(G, f))[0])
    for i in range(4):
        codes.append(W.config2(i)); ref.append(GOLD["config2"][i])
    for n in (12, 33, 64, 65, 97, 128):
        G = W.additive(n, 12, W.config_seed(40, n))
        codes.append((G, 2)); ref.append(O.brute(O.expand(G, 2))[0])
    G = W.f4_linear(30, 8, W.config_seed(41, 0))
    codes.append((G, 4)); ref.append(O.brute(O.expand(G, 4))[0])
    return codes, ref


def test_batch_matches_oracle_and_single(Q):
    codes, ref = mixed_codes()
    st, ds, wits, sts, stats = Q.qd_distance_batch(codes)
    assert st == 0 and all(s == 0 for s in sts), sts
    for (G, f), d, w, r in zip(codes, ds, wits, ref):
        assert d == r
        assert swt(w) == d and O.in_rowspace(O.expand(G, f), w)
        st1, d1, _ = Q.qd_distance(G, f)
        assert st1 == 0 and d1 == d


def test_batch_statuses_per_code(Q):
    G1, f1 = W.config1(7)
    codes = [(G1, f1), (np.zeros((3, 10), np.uint8), 2), (np.ones((2, 2 * 129), np.uint8), 2), (G1, f1)]
    st, ds, wits, sts, _ = Q.qd_distance_batch(codes)
    assert sts == [0, Q.QD_ERR_ZERO_CODE, Q.QD_ERR_TOO_LARGE, 0]
    assert st == Q.QD_ERR_ZERO_CODE
    d_ref = O.brute(O.expand(G1, f1))[0]
    assert ds[0] == ds[3] == d_ref and ds[1] == ds[2] == -1


def test_batch_budget(Q):
    codes = [W.config2(i) for i in range(3)] + [W.config1(0)]
    st, ds, wits, sts, stats = Q.qd_distance_batch(codes, budget=200000)
    for i in range(3):
        # either the bounds already meet inside the budget, or L <= d <= U
        if sts[i] == Q.QD_INCOMPLETE:
            assert stats[i].L <= GOLD["config2"][i] <= ds[i]
        else:
            assert sts[i] == 0 and ds[i] == GOLD["config2"][i]
    assert sts[0] == Q.QD_INCOMPLETE  # d = 11 needs round 4
    assert sts[3] == 0 and ds[3] == O.brute(O.expand(*W.config1(0)))[0]


def test_batch_empty(Q):
    st, ds, wits, sts, _ = Q.qd_distance_batch([])
    assert st == 0 and ds == []


def run_engine(Q, reqs, mem_budget=0, max_active=0, gap_s=0.0):
    e = Q.qd_engine_create(mem_budget, max_active)
    assert e
    got = {}
    try:
        for tag, (G, f) in enumerate(reqs):
            rc = Q.qd_engine_submit(e, G, f, tag)
            assert rc == 0
            if gap_s:
                time.sleep(gap_s)
            for r, w in Q.qd_engine_poll(e, 64, 0):
                got[r.tag] = (r.status, r.d, w, r.latency_ms, r.queue_ms)
        t_end = time.time() + 60
        while len(got) < len(reqs) and time.time() < t_end:
            for r, w in Q.qd_engine_poll(e, 64, 200):
                got[r.tag] = (r.status, r.d, w, r.latency_ms, r.queue_ms)
        assert Q.qd_engine_outstanding(e) == 0
    finally:
        Q.qd_engine_destroy(e)
    return got


def test_engine_alone_equals_in_mix(Q):
    reqs, ref = mixed_codes()
    got = run_engine(Q, reqs, gap_s=0.002)
    assert sorted(got) == list(range(len(reqs)))
    for tag, (G, f) in enumerate(reqs):
        status, d, w, lat, qms = got[tag]
        st1, d1, _ = Q.qd_distance(G, f)
        assert status == 0 and d == d1 == ref[tag]
        assert swt(w) == d and O.in_rowspace(O.expand(G, f), w)
        assert lat >= qms >= 0


def test_engine_small_budget_serializes(Q):
    reqs = [W.config1(300 + i) for i in range(6)]
    got = run_engine(Q, reqs, mem_budget=1, max_active=2)
    for tag, (G, f) in enumerate(reqs):
        assert got[tag][0] == 0 and got[tag][1] == O.brute(O.expand(G, f))[0]


def test_engine_rejects_bad_request(Q):
    e = Q.qd_engine_create()
    try:
        rc = Q.qd_engine_submit(e, np.zeros((2, 8), np.uint8), 2, 99)
        assert rc == Q.QD_ERR_ZERO_CODE
        res = Q.qd_engine_poll(e, 8, 2000)
        assert len(res) == 1 and res[0][0].tag == 99 and res[0][0].status == Q.QD_ERR_ZERO_CODE
    finally:
        Q.qd_engine_destroy(e)


def test_engine_destroy_with_work_outstanding(Q):
    e = Q.qd_engine_create()
    for i in range(8):
        Q.qd_engine_submit(e, *W.config2(i % 4), i)
    t0 = time.time()
    Q.qd_engine_destroy(e)
    assert time.time() - t0 < 30


def test_batch_of_every_word_count_in_one_launch(Q):
    """Codes of D = 1, 2, 3 and 4 words per half in one batch (each step
    launches the round kernel of every D).  Every code gives the oracle's
    distance and its result alone, on the default path, with every word
    evaluated, and with 64-entry tiles."""
    codes = []
    for i, n in enumerate((20, 30, 40, 60, 72, 90, 100, 120)):
        rng = W.SplitMix64(W.config_seed(93, i))
        codes.append((W.additive(n, rng.uniform_int(18, 24), rng.next()), 2))
    codes.append((W.f4_linear(70, 11, W.config_seed(93, 50)), 4))
    refs = [O.distance(G, f)[0] for G, f in codes]
    for opts in ({}, {"partial_weight": -1}, {"seg_len": 64}):
        st, ds, wits, sts, stats = Q.qd_distance_batch(codes, **opts)
        assert st == 0 and all(s == 0 for s in sts), (opts, sts)
        assert sorted({s.D for s in stats}) == [1, 2, 3, 4]
        for (G, f), d, w, r in zip(codes, ds, wits, refs):
            assert d == r, opts
            assert swt(w) == d and O.in_rowspace(O.expand(G, f), w)
            assert Q.qd_distance_ex(G, f, **opts)[1] == d
