"""GPU parity of the matrix-core path (fp4 MFMA over sign vectors) for every
word count and K-step layout: D = 1, 2, 3 and 4 words per half, the last
word packed into a spare group (n - 32 (D - 1) <= 10) or given its own
K-step.  Rounds are compared with the oracle's plain enumeration (minimum
and visited count, exact); whole calls with the vector-ALU path (same
status, bounds and distance) and the oracle's distance where it is cheap."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import oracle as O
from paper_2408_10743_amd import workloads as W

# n -> (D, packed last word); one word per half stays on the vector ALU (n = 20
# checks that the choice keeps it exact)
LAYOUTS = {20: (1, False), 50: (2, False), 70: (3, True), 90: (3, False), 100: (4, True), 120: (4, False)}


@pytest.fixture(scope="module")
def Q():
    from paper_2408_10743_amd import qdist
    st, name = qdist.qd_device_check()
    assert st == 0, name
    return qdist


def big_round(rd, D=2):
    """A round that takes the matrix cores: two or more words per half, a
    saved table and at least 2^20 combinations (smaller rounds and one-word
    codes stay on the vector ALU)."""
    return D >= 2 and rd["saved_depth"] > 0 and rd["planned"] >= 1 << 20


def swt(v):
    n = v.shape[-1] // 2
    return int(np.count_nonzero(v[:n] | v[n:]))


@pytest.mark.parametrize("n", sorted(LAYOUTS))
def test_round_min_vs_oracle(Q, n):
    """t = 4 over 30 packages (2.2e6 combinations with two-row packages:
    saved tables, several chunks per tile, ragged groups and tails) and t = 5
    over fewer packages; random and sparse rows (weights near the bottom of
    the range, where the minimum is decided)."""
    for rep, (P, t, frac, density) in enumerate([(30, 4, 0.8, 0.5), (24, 5, 1.0, 0.5), (30, 4, 1.0, 0.1)]):
        rows, dims = W.random_packages(P, n, W.config_seed(40, 100 * n + rep), frac)
        if density < 0.5:
            rng = np.random.default_rng(n * 7 + rep)
            rows = rows & (rng.random(rows.shape) < 2 * density).astype(np.uint8)
            for i in range(P):  # keep every package's rows independent and nonzero
                if not rows[2 * i].any():
                    rows[2 * i, i % (2 * n)] = 1
                if dims[i] == 2 and (not rows[2 * i + 1].any() or (rows[2 * i + 1] == rows[2 * i]).all()):
                    rows[2 * i + 1] = 0
                    rows[2 * i + 1, (i + n) % (2 * n)] = 1
        print(f"n={n} rep={rep} P={P} t={t}", flush=True)
        st, w, wit, cnt = Q.qd_round_min(rows, dims, t)
        assert st == 0, Q.qd_strerror(st)
        wo, _, co = O.round_min(rows, dims, t)
        assert (w, cnt) == (wo, co)
        assert swt(wit) == w and O.in_rowspace(rows, wit)


@pytest.mark.parametrize("n", sorted(LAYOUTS))
def test_distance_matches_vector_alu(Q, n):
    """A whole call with every word evaluated and the saved tables forced
    (saved_depth 2 and 3): the matrix cores and the vector ALU give the same
    status, bounds and distance, and only the first uses the matrix cores."""
    m = max(4, n // 2)
    for seed in range(2):
        G = W.additive(n, m, W.config_seed(41, 10 * n + seed))
        for depth in (2, 3):
            opts = dict(partial_weight=-1, saved_depth=depth, budget=int(2e9))
            print(f"n={n} m={m} seed={seed} depth={depth}", flush=True)
            r = [Q.qd_distance_ex(G, 2, matrix_cores=mc, **opts) for mc in (0, -1)]
            (st0, d0, w0, s0), (st1, d1, w1, s1) = r
            assert st0 == st1 and st0 in (0, Q.QD_INCOMPLETE)
            assert (d0, s0.L, s0.U) == (d1, s1.L, s1.U)
            assert s0.combinations == s1.combinations
            assert s1.matrix_core_launches == 0
            if any(big_round(rd, s0.D) for rd in s0.rounds()):
                assert s0.matrix_core_launches > 0
            B = O.expand(G, 2)
            assert swt(w0) == d0 and O.in_rowspace(B, w0)
            if st0 == 0 and O.rank(B) <= 18:
                assert d0 == O.brute(B)[0]


def test_batch_mixed_layouts(Q):
    """Codes of every layout in one batch (one launch per word count) give
    their results alone."""
    codes = [(W.additive(n, max(4, n // 3), W.config_seed(42, n)), 2) for n in sorted(LAYOUTS)]
    opts = dict(partial_weight=-1, saved_depth=2, budget=int(1e9))
    st, ds, wits, sts, stats = Q.qd_distance_batch(codes, **opts)
    assert st == 0
    for (G, f), d, w, x, s in zip(codes, ds, wits, sts, stats):
        st1, d1, _, s1 = Q.qd_distance_ex(G, f, **opts)
        assert (x, d) == (st1, d1)
        if any(big_round(rd, s.D) for rd in s.rounds()):
            assert s.matrix_core_launches > 0
        assert swt(w) == d and O.in_rowspace(O.expand(G, f), w)


@pytest.mark.parametrize("seg", [64, 128, 192])
def test_shared_chunks_ragged_ends(Q, seg):
    """Short tiles over a depth-2 saved table: the four waves of a workgroup
    share a segment's chunks up to the shortest wave's end, and each wave
    finishes its own remaining chunks (ends that are not a multiple of the
    shared group); with every word evaluated, tiles of odd chunk counts end
    the pipelined loop with a single chunk.  Config-4 draws of two and three
    words per half against the vector ALU."""
    pool = [c for c in W.config4(120) if 50 <= c[0].shape[1] // 2 <= 74 and c[1] == 2][:6]
    assert len(pool) >= 3
    for i, (G, f) in enumerate(pool):
        # Partial weights (shared chunks), then every word (the pipelined
        # loop over pairs of chunks, odd chunk counts in the short tiles).
        for pw in (0, -1):
            opts = dict(saved_depth=2, seg_len=seg, budget=int(2e10), partial_weight=pw)
            print(f"code {i} n={G.shape[1] // 2} seg={seg} partial_weight={pw}", flush=True)
            (st0, d0, w0, s0), (st1, d1, w1, s1) = [Q.qd_distance_ex(G, f, matrix_cores=mc, **opts)
                                                    for mc in (0, -1)]
            assert (st0, d0, s0.L, s0.U, s0.combinations) == (st1, d1, s1.L, s1.U, s1.combinations)
            assert swt(w0) == d0 and O.in_rowspace(O.expand(G, f), w0)
