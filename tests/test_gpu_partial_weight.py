"""GPU parity of the partial-weight path: every result with partial weights
(forced on for every code of two or more words per half, and automatic)
equals the oracle's and the result with every word evaluated
(partial_weight = -1), for each construction, the Modified BZ filter and
batches; the evaluated-word count shows which path ran."""
import json
import os

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


def both(Q, G, f, d_ref, **opts):
    """Runs with partial weights forced on (1), automatic (0) and off (-1);
    all must give d_ref and a valid witness.  Returns the stats of the
    forced and the off runs."""
    out = []
    B = O.expand(G, f)
    for pw in (1, 0, -1):
        st, d, wit, s = Q.qd_distance_ex(G, f, partial_weight=pw, **opts)
        assert st == 0, Q.qd_strerror(st)
        assert d == d_ref, (pw, d, d_ref)
        assert swt(wit) == d and O.in_rowspace(B, wit)
        assert s.enumerated >= s.combinations
        if pw == -1:
            assert s.words == s.D * s.enumerated
        else:
            assert s.words <= s.D * s.enumerated
        if pw != 0:
            out.append(s)
    return out


def test_config3_partial_weights_engage(Q):
    G, f = W.config3(0)
    print("config3 seed 0", flush=True)
    on, off = both(Q, G, f, GOLD["config3"][0], timing=1)
    assert on.D == 3
    # the large rounds evaluate one word of three for nearly every codeword
    assert on.words < 0.5 * on.D * on.enumerated
    print(f"words per codeword {on.words / on.enumerated:.3f}; kernel {on.kernel_ms:.2f} ms "
          f"vs {off.kernel_ms:.2f} ms", flush=True)


def test_config2_each_construction(Q):
    for i, d_ref in enumerate(GOLD["config2"][:6]):
        G, f = W.config2(i)
        for diag in (Q.QD_DIAG_AUTO, Q.QD_DIAG_F4, Q.QD_DIAG_F2, Q.QD_DIAG_ISO):
            print(f"config2 seed {i} diag {diag} d={d_ref}", flush=True)
            both(Q, G, f, d_ref, diag=diag)


def test_direct_sums_low_weight(Q):
    """Direct sums of small random codes spread over 40..100 qubits, qubits
    shuffled: pivots land everywhere, so the stored qubit order is far from
    the identity and every witness must be mapped back to qubit order.  (The
    rounds are small enough to run without saved tables, so the words
    evaluated stay D per codeword.)  d = the least component distance
    (brute force per component)."""
    for s in range(8):
        rng = W.SplitMix64(W.config_seed(60, s))
        parts, d_ref = [], 10 ** 9
        n = 0
        while n < 40 + 8 * s:
            nq = rng.uniform_int(6, 12)
            B = W.additive(nq, rng.uniform_int(nq - 2, nq + 2), rng.next())
            if O.rank(B) == 0:
                continue
            d_ref = min(d_ref, O.brute(B)[0])
            parts.append(B)
            n += nq
        m = sum(p.shape[0] for p in parts)
        A = np.zeros((m, 2 * n), np.uint8)
        r = c = 0
        for p in parts:
            k = p.shape[1] // 2
            A[r:r + p.shape[0], c:c + k] = p[:, :k]
            A[r:r + p.shape[0], n + c:n + c + k] = p[:, k:]
            r += p.shape[0]
            c += k
        perm = np.array(sorted(range(n), key=lambda q: rng.next()))
        A = np.concatenate([A[:, perm], A[:, n + perm]], axis=1)
        print(f"direct sum {s}: n={n} parts={len(parts)} d={d_ref}", flush=True)
        both(Q, A, 2, d_ref)


def test_filter_partial_weights(Q):
    for s in range(10):
        rng = W.SplitMix64(W.config_seed(61, s))
        n = rng.uniform_int(33, 50)
        k = rng.uniform_int(1, 4)
        A = W.random_stabilizer(n, k, rng.next())
        d_ref = O.bz_stab(A, O.DIAG_F4, 8)[0]
        print(f"stab n={n} k={k} d={d_ref}", flush=True)
        both(Q, A, 2, d_ref, filter=Q.QD_FILTER_STABILIZER)


def test_batch_partial_equals_full(Q):
    codes = []
    for i in range(48):
        rng = W.SplitMix64(W.config_seed(62, i))
        n = rng.uniform_int(33, 80)
        if i % 2:
            codes.append((W.f4_linear(n, n // 2, rng.next()), 4))
        else:
            codes.append((W.additive(n, n + rng.uniform_int(-6, 6), rng.next()), 2))
    budget = int(2e10)
    res = {}
    for pw in (1, -1):
        print(f"batch of {len(codes)}, partial_weight {pw}", flush=True)
        st, ds, wits, sts, stats = Q.qd_distance_batch(codes, budget=budget, partial_weight=pw)
        assert st == 0 and all(x in (0, Q.QD_INCOMPLETE) for x in sts)
        for (G, f), d, w in zip(codes, ds, wits):
            assert swt(w) == d and O.in_rowspace(O.expand(G, f), w)
        res[pw] = (ds, sts)
        words = sum(x.words for x in stats)
        full = sum(x.D * x.enumerated for x in stats)
        assert (words < full) if pw == 1 else (words == full)
    for i in range(len(codes)):
        if res[1][1][i] == 0 and res[-1][1][i] == 0:
            assert res[1][0][i] == res[-1][0][i], i
    assert sum(1 for x in res[1][1] if x == 0) >= len(codes) // 2
