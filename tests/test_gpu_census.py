"""GPU parity of the enumeration kernel's census (qd_round_census) against
the oracle's weight distribution of the same round (qdo_round_hist).

A minimum and a count can survive a kernel that skips or repeats table
entries inside a tile; the number of codewords below a threshold and the sum
of their weights do not.  The census is taken by the production enumeration
code (same tiles, blocks and partial-weight decisions) and must equal the
oracle's figures exactly, on every word path: every word evaluated, and w
words first with the blocks that may hold a codeword below the threshold
completed.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import oracle as O
from paper_2408_10743_amd import workloads as W


@pytest.fixture(scope="module")
def Q():
    from paper_2408_10743_amd import qdist
    st, name = qdist.qd_device_check()
    assert st == 0, f"no usable gfx950 device ({name}): {qdist.qd_strerror(st)}"
    return qdist


def swt(v):
    n = v.shape[-1] // 2
    return int(np.count_nonzero(v[:n] | v[n:]))


def below_figures(hist, below):
    w = np.arange(hist.shape[0], dtype=np.uint64)
    sel = w < below
    return int(hist[sel].sum()), int((hist[sel] * w[sel]).sum())


def check(Q, rows, dims, t, below, partial_words=0, hist=None):
    n = rows.shape[1] // 2
    if hist is None:
        hist = O.round_hist(rows, dims, t)
    st, w, wit, cnt, bc, bs = Q.qd_round_census(rows, dims, t, below, partial_words)
    assert st == 0, Q.qd_strerror(st)
    nz = np.flatnonzero(hist)
    assert w == (int(nz[0]) if nz.size else n + 1)
    assert cnt == int(hist.sum())
    assert (bc, bs) == below_figures(hist, below), (t, below, partial_words)
    if cnt:
        assert swt(wit) == w
    return hist


@pytest.mark.parametrize("n", [1, 7, 31, 32, 33, 64, 72, 96, 100, 128])
def test_census_random_packages(Q, n):
    for rep in range(3):
        rng = W.SplitMix64(W.config_seed(85, n * 10 + rep))
        P = rng.uniform_int(1, 14)
        rows, dims = W.random_packages(P, n, rng.next(), [1.0, 0.0, 0.5][rep])
        for t in range(1, min(P, 5) + 1):
            print(f"census n={n} rep={rep} P={P} t={t}", flush=True)
            hist = O.round_hist(rows, dims, t)
            nz = np.flatnonzero(hist)
            for below in (n + 2, int(nz[0]) + 2 if nz.size else 1, 1):
                check(Q, rows, dims, t, below, hist=hist)


@pytest.mark.parametrize("D,w", [(2, 1), (3, 1), (3, 2), (4, 1), (4, 2), (4, 3)])
def test_census_partial_words(Q, D, w):
    """t = 4 over 30 two-row packages (2.2e6 combinations: saved tables,
    full blocks, ragged tails) on every (D, w) path, with the threshold at
    the round minimum + 1, + 3 and above every weight."""
    n = 32 * D - 3
    for concentrated in (False, True):
        rows, dims = W.random_packages(30, n, W.config_seed(86, 10 * D + w), 1.0)
        if concentrated:
            keep = np.zeros(2 * n, dtype=np.uint8)
            keep[:32 * w] = 1
            keep[n:n + 32 * w] = 1
            rows = rows * keep
        hist = O.round_hist(rows, dims, 4)
        m = int(np.flatnonzero(hist)[0])
        for below in (m + 1, m + 3, n + 2):
            print(f"census D={D} w={w} concentrated={concentrated} below={below}", flush=True)
            check(Q, rows, dims, 4, below, 0, hist)
            check(Q, rows, dims, 4, below, w, hist)


def test_census_large_round(Q):
    rows, dims = W.random_packages(30, 72, W.config_seed(87, 0), 0.8)
    for t in (4, 5):
        hist = O.round_hist(rows, dims, t)
        m = int(np.flatnonzero(hist)[0])
        for below in (m + 2, 73):
            for pw in (0, 1, 2):
                print(f"census large t={t} below={below} pw={pw}", flush=True)
                check(Q, rows, dims, t, below, pw, hist)


def test_census_config3_matrices(Q):
    """Round t = 5 and t = 6 of both generator matrices of the n = 72
    benchmark code (config 3, seed 0): 1.4e9 combinations per matrix at
    t = 6, the kernel's production tiling at full size."""
    G, f = W.config3(0)
    gs = O.gamma(O.expand(G, f), O.DIAG_F4, 2, with_rows=True)
    for j, g in enumerate(gs):
        for t in (5, 6):
            hist = O.round_hist(g["rows"], g["dims"], t)
            m = int(np.flatnonzero(hist)[0])
            for below, pw in ((m + 4, 1), (m + 2, 2), (73, 0)):
                print(f"census config3 Gamma_{j + 1} t={t} below={below} pw={pw}", flush=True)
                check(Q, g["rows"], g["dims"], t, below, pw, hist)


def test_census_errors(Q):
    rows, dims = W.random_packages(4, 10, W.config_seed(87, 1))
    assert Q.qd_round_census(rows, dims, 2, 0)[0] == Q.QD_ERR_INVALID
    st, w, wit, cnt, bc, bs = Q.qd_round_census(rows, dims, 5, 3)
    assert st == 0 and w == 11 and cnt == bc == bs == 0
