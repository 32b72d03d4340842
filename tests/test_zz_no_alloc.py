"""The entry point that allocates nothing (qd_round_min_noalloc) against
qd_round_min and the oracle: two calls in a row, the second smaller; a
round too large for the fixed array; and, in a fresh process, that repeated
calls leave the device's free memory unchanged after the first (which loads
the library's code object with its array)."""
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import oracle as O
from paper_2408_10743_amd import workloads as W

ROOT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..")


@pytest.fixture(scope="module")
def Q():
    from paper_2408_10743_amd import qdist
    st, name = qdist.qd_device_check()
    assert st == 0, f"no usable gfx950 device ({name}): {qdist.qd_strerror(st)}"
    return qdist


def swt(v):
    n = v.shape[-1] // 2
    return int(np.count_nonzero(v[:n] | v[n:]))


CASES = [  # (packages, qubits, two-row fraction, t, partial words); each call smaller than the last
    (30, 72, 0.8, 5, 0),
    (12, 40, 0.5, 3, 0),
    (30, 93, 1.0, 4, 2),
    (9, 20, 0.0, 4, 0),
]


def test_noalloc_matches_round_min_two_calls(Q):
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    for i, (P, n, frac, t, pw) in enumerate(CASES):
        rows, dims = W.random_packages(P, n, W.config_seed(88, i), frac)
        print(f"noalloc call {i}: P={P} n={n} t={t} partial_words={pw}", flush=True)
        st, w, wit, cnt = Q.qd_round_min_noalloc(rows, dims, t, pw, stream)
        assert st == 0, Q.qd_strerror(st)
        st0, w0, wit0, cnt0 = Q.qd_round_min(rows, dims, t, pw)
        assert st0 == 0
        assert (w, cnt) == (w0, cnt0)
        wo, _, co = O.round_min(rows, dims, t)
        assert (w, cnt) == (wo, co)
        assert swt(wit) == w and O.in_rowspace(rows, wit)


def test_noalloc_null_stream_and_empty_round(Q):
    rows, dims = W.random_packages(14, 33, W.config_seed(88, 10), 0.5)
    st, w, wit, cnt = Q.qd_round_min_noalloc(rows, dims, 4)
    wo, _, co = O.round_min(rows, dims, 4)
    assert st == 0 and (w, cnt) == (wo, co)
    st, w, wit, cnt = Q.qd_round_min_noalloc(rows[:6], dims[:3], 4)  # t > P
    assert st == 0 and w == 34 and cnt == 0


def test_noalloc_rejects_a_round_beyond_its_array(Q):
    # 100 two-row packages at t = 6 (8.7e11 combinations): its tile plan
    # alone needs far more than the fixed array
    rows, dims = W.random_packages(100, 100, W.config_seed(88, 11), 1.0)
    st, w, wit, cnt = Q.qd_round_min_noalloc(rows, dims, 6)
    assert st == Q.QD_ERR_TOO_LARGE
    # the next call is unaffected
    rows, dims = W.random_packages(10, 50, W.config_seed(88, 12), 0.5)
    st, w, wit, cnt = Q.qd_round_min_noalloc(rows, dims, 3)
    wo, _, co = O.round_min(rows, dims, 3)
    assert st == 0 and (w, cnt) == (wo, co)


def test_noalloc_invalid_arguments(Q):
    rows, dims = W.random_packages(4, 10, W.config_seed(88, 13))
    assert Q.qd_round_min_noalloc(rows, dims, 0)[0] == Q.QD_ERR_INVALID
    assert Q.qd_round_min_noalloc(rows, dims, 2, partial_words=1)[0] == Q.QD_ERR_INVALID  # D = 1


PROBE = r"""
import sys
import torch
sys.path.insert(0, {root!r})
from paper_2408_10743_amd import qdist as Q
from paper_2408_10743_amd import workloads as W
torch.cuda.init()
cases = [(30, 72, 0.8, 5), (12, 40, 0.5, 3), (20, 60, 1.0, 4)]
def call(i):
    P, n, f, t = cases[i]
    rows, dims = W.random_packages(P, n, W.config_seed(89, i), f)
    st = Q.qd_round_min_noalloc(rows, dims, t)[0]
    assert st == 0, st
call(0)
torch.cuda.synchronize()
free0 = torch.cuda.mem_get_info()[0]
for i in (1, 2, 0, 1):
    call(i)
torch.cuda.synchronize()
free1 = torch.cuda.mem_get_info()[0]
print("free", free0, free1, flush=True)
assert free0 == free1, (free0, free1)
print("NOALLOC_OK", flush=True)
"""


def test_noalloc_leaves_free_memory_unchanged():
    r = subprocess.run([sys.executable, "-c", PROBE.format(root=ROOT)], capture_output=True, text=True,
                       timeout=240, cwd=ROOT)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0 and "NOALLOC_OK" in r.stdout
