"""GPU checks at the benchmark's full sizes, in the call patterns bench.py
times: every output is checked by its properties (witness weight equals d,
witness in the row space, the same d alone and in a batch), and samples
that the oracle finishes quickly are compared with it exactly."""
import json
import os
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import bench
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


def test_config1_every_seed(Q):
    """Config 1 at its stated size: all 1,000 seeds in one batch against the
    oracle's exhaustive search."""
    codes = [W.config1(i) for i in range(1000)]
    st, ds, wits, sts, _ = Q.qd_distance_batch(codes)
    assert st == 0 and all(x == 0 for x in sts)
    for i, ((G, f), d, w) in enumerate(zip(codes, ds, wits)):
        if i % 100 == 0:
            print(f"config1 seed {i}", flush=True)
        B = O.expand(G, f)
        assert d == O.brute(B)[0], i
        assert swt(w) == d and O.in_rowspace(B, w)


def test_config4_full_batch(Q):
    """The bench's config-4 batch (512 codes): each code's d equals its
    per-code result, witnesses check out, and the codes the oracle settles
    in well under a second agree with it."""
    codes, drawn = bench.config4_codes(Q, W, 512, 1e11)
    budget = int(4e11)
    print(f"config4 batch of {len(codes)} (of {drawn} drawn)", flush=True)
    st, ds, wits, sts, stats = Q.qd_distance_batch(codes, budget=budget)
    assert all(x in (0, Q.QD_INCOMPLETE) for x in sts)
    for (G, f), d, w, s, x in zip(codes, ds, wits, stats, sts):
        B = O.expand(G, f)
        assert swt(w) == d and O.in_rowspace(B, w)
        st1, d1, _, s1 = Q.qd_distance_ex(G, f, budget=budget)
        assert st1 == x and d1 == d
    # the same batch with every word evaluated and two-row packages first
    # (the paper's construction): the same statuses and distances
    st2, ds2, wits2, sts2, _ = Q.qd_distance_batch(codes, budget=budget, partial_weight=-1, mixed_packages=-1)
    assert sts2 == sts
    for i, (d, d2) in enumerate(zip(ds, ds2)):
        if sts[i] == 0:
            assert d == d2, i
    # exact oracle comparison on the cheapest codes of each field
    order = sorted(range(len(codes)), key=lambda i: stats[i].combinations)
    checked = {2: 0, 4: 0}
    for i in order:
        G, f = codes[i]
        if checked[f] >= 6 or sts[i] != 0:
            continue
        B = O.expand(G, f)
        t0 = time.perf_counter()
        d_ref = O.brute(B)[0] if O.rank(B) <= 22 else O.bz(B, O.DIAG_F4, 8)[0]
        print(f"config4 code {i} field {f} n {B.shape[1] // 2} d {d_ref} ({time.perf_counter() - t0:.2f} s)",
              flush=True)
        assert ds[i] == d_ref
        checked[f] += 1
    assert checked[2] == 6 and checked[4] == 6


def test_config5_engine_mix(Q):
    """The bench's config-5 request mix through the serving engine: every
    result equals the same code alone (tolerance 0)."""
    raw = W.config5(300 * 4, 1.0)
    reqs = []
    for _, G, f in raw:
        if bench.predicted_work(Q, G, f) <= 1e10:
            reqs.append((G, f))
            if len(reqs) == 300:
                break
    e = Q.qd_engine_create()
    got = {}
    try:
        for tag, (G, f) in enumerate(reqs):
            assert Q.qd_engine_submit(e, G, f, tag) == 0
        t_end = time.time() + 90
        while len(got) < len(reqs) and time.time() < t_end:
            for r, w in Q.qd_engine_poll(e, 64, 200):
                got[r.tag] = (r.status, r.d, w)
    finally:
        Q.qd_engine_destroy(e)
    assert len(got) == len(reqs)
    for tag, (G, f) in enumerate(reqs):
        status, d, w = got[tag]
        st1, d1, _ = Q.qd_distance(G, f)
        assert status == 0 and d == d1, tag
        assert swt(w) == d and O.in_rowspace(O.expand(G, f), w)


def test_config3_golden_seeds(Q):
    """Config 3 seeds 0-4 against the oracle's BZ distances, on the default
    path (partial weights, mixed packages allowed) and with every word
    evaluated and two-row packages first (the paper's construction), each
    on the matrix cores (the default) and on the vector ALU alone."""
    assert len(GOLD["config3"]) == 5
    for i, d_ref in enumerate(GOLD["config3"]):
        G, f = W.config3(i)
        B = O.expand(G, f)
        for base in ({}, {"partial_weight": -1, "mixed_packages": -1}):
            for mc in (0, -1):
                opts = dict(base, matrix_cores=mc)
                print(f"config3 seed {i} d={d_ref} {opts}", flush=True)
                st, d, w, s = Q.qd_distance_ex(G, f, **opts)
                assert st == 0 and d == d_ref, (i, opts, st, d)
                assert swt(w) == d and O.in_rowspace(B, w)
                assert (s.matrix_core_launches > 0) == (mc == 0), (i, opts)
                words_per_codeword = s.words / max(s.enumerated, 1)
                if base:
                    assert words_per_codeword == s.D
                else:
                    assert words_per_codeword < 1.1  # the partial-weight path decided the rounds


def test_config4_oracle_sample(Q):
    """A fixed sample of the bench's config-4 codes, spread over predicted
    work (1e4..1e11 combinations, both fields, n 28..80), against the
    oracle's BZ distances: the default path (partial weights on the codes
    planned at >= 1e8 combinations, capped two-row packages where the
    planner caps them), the same on the vector ALU alone, and every word
    evaluated with two-row packages first."""
    rows = GOLD["config4_sample"]
    pool = W.config4(800)  # draw i is the i-th code of the bench's draw sequence
    assert len(rows) >= 24
    big = capped = 0
    for r in rows:
        G, f = pool[r["index"]]
        assert bench.predicted_work(Q, G, f) <= 1e11  # a member of the bench's batch
        B = O.expand(G, f)
        for opts in ({}, {"matrix_cores": -1}, {"partial_weight": -1, "mixed_packages": -1}):
            print(f"config4 draw {r['index']} n={r['n']} field={f} d={r['d']} {opts}", flush=True)
            st, d, w, s = Q.qd_distance_ex(G, f, **opts)
            assert st == 0 and d == r["d"], (r, opts, st, d)
            assert swt(w) == d and O.in_rowspace(B, w)
            if not opts:
                if s.words < s.D * s.enumerated:
                    big += 1
                if any(c >= 0 for c in list(s.two_row_cap)[:s.h]):
                    capped += 1
    print(f"config4 sample: {len(rows)} codes, {big} on partial weights, {capped} with capped packages", flush=True)
    assert big >= 8 and capped >= 4


def test_config4_first_draws_bounds(Q):
    """Config 4 as drawn (the first 512 draws, n up to 96, no work filter)
    in one batch with the bench's per-code budget: every code ends exact or
    QD_INCOMPLETE; exact codes carry a valid witness, incomplete ones
    certified bounds L < U with a witness of weight U; the golden sample's
    codes among these draws give the oracle's distance."""
    codes = W.config4(512)
    st, ds, wits, sts, stats = Q.qd_distance_batch(codes, budget=int(4e11))
    assert st == 0
    gold = {r["index"]: r["d"] for r in GOLD["config4_sample"]}
    n_inc = 0
    for i, ((G, f), d, w, x, s) in enumerate(zip(codes, ds, wits, sts, stats)):
        assert x in (0, Q.QD_INCOMPLETE), (i, x)
        B = O.expand(G, f)
        assert swt(w) == d == s.U and O.in_rowspace(B, w), i
        if x == 0:
            assert s.L >= s.U
            if i in gold:
                assert d == gold[i], i
        else:
            n_inc += 1
            assert s.L < s.U, i
    ns = [G.shape[1] // 2 if f == 2 else G.shape[1] for G, f in codes]
    print(f"config4 first draws: {len(codes) - n_inc} exact, {n_inc} incomplete, n {min(ns)}..{max(ns)}", flush=True)
    assert max(ns) == 96


def test_config3_full_size_bench_call(Q):
    """Config 3 exactly as bench.py times it (stream, timing on): the oracle's
    golden distance, and every completed round visited its planned count."""
    import torch
    stream = torch.cuda.current_stream()
    G, f = W.config3(0)
    for _ in range(2):
        st, d, w, s = Q.qd_distance_ex(G, f, stream=stream.cuda_stream, timing=1)
        assert st == 0 and d == GOLD["config3"][0]
        assert swt(w) == d and O.in_rowspace(O.expand(G, f), w)
        assert s.combinations == sum(r["combinations"] for r in s.rounds())
        assert s.launches >= 1 and s.kernel_ms > 0
