"""ctypes wrapper of the CPU oracle (oracle/qdo.c).

Test infrastructure only: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The library under test never imports it.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

DIAG_F2 = 2
DIAG_F4 = 4


_NATIVE_PATH = os.path.join(_HERE, "liboracle_native.so")


def build(force=False, native=False):
    """Compile the oracle with gcc: plain -O2 with hardware popcount (the
    tests' checker), or native=True: -O3 -march=native, the CPU baseline of
    the benchmark, built on the machine that times it.  Same source, same
    OpenMP parallel outer loop."""
    src = os.path.join(_HERE, "qdo.c")
    path = _NATIVE_PATH if native else _LIB_PATH
    if not force and os.path.exists(path) and os.path.getmtime(path) >= os.path.getmtime(src):
        return path
    tmp = path + ".tmp"
    opt = ["-O3", "-march=native"] if native else ["-O2", "-mpopcnt"]
    subprocess.check_call(["gcc"] + opt + ["-fopenmp", "-std=c99", "-Wall", "-shared", "-fPIC", src, "-o", tmp])
    os.replace(tmp, path)
    return path


def use_native():
    """Route every later call of this module to the -O3 -march=native build
    (compiled here, for this CPU).  Used by the benchmark's CPU baseline."""
    global _lib
    _lib = ctypes.CDLL(build(force=True, native=True))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = ctypes.CDLL(_LIB_PATH)
    return _lib


_u8p = ctypes.POINTER(ctypes.c_uint8)
_ip = ctypes.POINTER(ctypes.c_int)


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(_u8p)


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_ip)


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc < 0:
        raise OracleError(f"{what} failed with status {rc}")
    return rc


def symplectic_weight(v, n):
    v, p = _u8(v)
    return lib().qdo_symplectic_weight(p, n)


def expand(G, field):
    """Binary rows of the code (F4 rows -> rows g and alpha*g)."""
    G = np.asarray(G, dtype=np.uint8)
    m = G.shape[0]
    n = G.shape[1] // 2 if field == 2 else G.shape[1]
    rows = m if field == 2 else 2 * m
    out = np.zeros((rows, 2 * n), dtype=np.uint8)
    G, gp = _u8(G)
    _check(lib().qdo_expand(gp, m, n, field, out.ctypes.data_as(_u8p)), "expand")
    return out


def rank(B):
    B, p = _u8(B)
    return _check(lib().qdo_rank(p, B.shape[0], B.shape[1] // 2), "rank")


def in_rowspace(B, v):
    B, p = _u8(B)
    v, vp = _u8(v)
    return bool(_check(lib().qdo_in_rowspace(p, B.shape[0], B.shape[1] // 2, vp), "in_rowspace"))


def brute(B, nthreads=0):
    """Exhaustive symplectic minimum distance: (d, witness)."""
    B, p = _u8(B)
    n = B.shape[1] // 2
    d = ctypes.c_int(-1)
    wit = np.zeros(2 * n, dtype=np.uint8)
    _check(lib().qdo_brute(p, B.shape[0], n, nthreads, ctypes.byref(d), wit.ctypes.data_as(_u8p)), "brute")
    return d.value, wit


def brute_iso_hamming(B):
    B, p = _u8(B)
    dH = ctypes.c_int(-1)
    _check(lib().qdo_brute_iso_hamming(p, B.shape[0], B.shape[1] // 2, ctypes.byref(dH)), "iso")
    return dH.value


def gamma(B, diag=DIAG_F4, max_gamma=8, with_rows=False, max2=None):
    """Generator matrices: list of dicts {P, delta, dims, pivots[, rows]}.
    max2 (F4 only): per-matrix caps on two-row packages (mixed packages;
    -1 or missing entries: no cap)."""
    B, p = _u8(B)
    m, n = B.shape[0], B.shape[1] // 2
    cap = 2 * n
    h = ctypes.c_int(0)
    P = np.zeros(max_gamma, dtype=np.int32)
    delta = np.zeros(max_gamma, dtype=np.int32)
    dims = np.zeros(max_gamma * cap, dtype=np.int32)
    piv = np.zeros(max_gamma * cap, dtype=np.int32)
    rows = np.zeros((max_gamma * cap * 2, 2 * n), dtype=np.uint8) if with_rows else None
    if max2 is None:
        rc = lib().qdo_gamma(p, m, n, diag, max_gamma, cap, ctypes.byref(h),
                             P.ctypes.data_as(_ip), delta.ctypes.data_as(_ip),
                             dims.ctypes.data_as(_ip), piv.ctypes.data_as(_ip),
                             rows.ctypes.data_as(_u8p) if with_rows else None)
    else:
        assert diag == DIAG_F4
        caps = _caps(max2, max_gamma)
        rc = lib().qdo_gamma_mixed(p, m, n, max_gamma, caps.ctypes.data_as(_ip), cap, ctypes.byref(h),
                                   P.ctypes.data_as(_ip), delta.ctypes.data_as(_ip),
                                   dims.ctypes.data_as(_ip), piv.ctypes.data_as(_ip),
                                   rows.ctypes.data_as(_u8p) if with_rows else None)
    _check(rc, "gamma")
    out = []
    for j in range(h.value):
        g = {"P": int(P[j]), "delta": int(delta[j]),
             "dims": dims[j * cap: j * cap + P[j]].tolist(),
             "pivots": piv[j * cap: j * cap + P[j]].tolist()}
        if with_rows:
            g["rows"] = rows[j * cap * 2: (j * cap + P[j]) * 2].copy()
        out.append(g)
    return out


def round_min(rows, dims, t, nthreads=0):
    """One round: (wmin, witness, count) over t packages (rows: P*2 x 2n)."""
    rows, rp = _u8(rows)
    dims, dp = _i32(dims)
    P = dims.shape[0]
    n = rows.shape[1] // 2
    w = ctypes.c_int(0)
    cnt = ctypes.c_ulonglong(0)
    wit = np.zeros(2 * n, dtype=np.uint8)
    _check(lib().qdo_round(rp, dp, P, n, t, nthreads, ctypes.byref(w), wit.ctypes.data_as(_u8p),
                           ctypes.byref(cnt)), "round")
    return w.value, wit, cnt.value


def round_hist(rows, dims, t, nthreads=0):
    """Weight distribution of one round: numpy array hist[w], w = 0..n."""
    rows, rp = _u8(rows)
    dims, dp = _i32(dims)
    P = dims.shape[0]
    n = rows.shape[1] // 2
    hist = np.zeros(n + 1, dtype=np.uint64)
    _check(lib().qdo_round_hist(rp, dp, P, n, t, nthreads,
                                hist.ctypes.data_as(ctypes.POINTER(ctypes.c_ulonglong))), "round_hist")
    return hist


def _log_records(log, nl):
    return [tuple(int(x) for x in log[i]) for i in range(min(nl, log.shape[0]))]


def bz_gamma(gammas, n, nthreads=0, log_cap=4096):
    """BZ over explicit generator matrices [{rows, dims, delta}, ...]."""
    h = len(gammas)
    P = np.array([len(g["dims"]) for g in gammas], dtype=np.int32)
    off = np.concatenate([[0], np.cumsum(P)[:-1]]).astype(np.int32)
    delta = np.array([g["delta"] for g in gammas], dtype=np.int32)
    rows = np.concatenate([np.asarray(g["rows"], dtype=np.uint8).reshape(-1, 2 * n) for g in gammas])
    dims = np.concatenate([np.asarray(g["dims"], dtype=np.int32) for g in gammas])
    d = ctypes.c_int(-1)
    wit = np.zeros(2 * n, dtype=np.uint8)
    log = np.zeros((log_cap, 5), dtype=np.int64)
    nl = ctypes.c_int(0)
    rows, rp = _u8(rows)
    dims, dp = _i32(dims)
    _check(lib().qdo_bz_gamma(h, P.ctypes.data_as(_ip), off.ctypes.data_as(_ip),
                              delta.ctypes.data_as(_ip), rp, dp, n, nthreads, ctypes.byref(d),
                              wit.ctypes.data_as(_u8p),
                              log.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)), log_cap,
                              ctypes.byref(nl)), "bz_gamma")
    return d.value, wit, _log_records(log, nl.value)


def _caps(max2, max_gamma):
    caps = np.full(max_gamma, -1, dtype=np.int32)
    for j, c in enumerate(list(max2)[:max_gamma]):
        caps[j] = c
    return caps


def bz(B, diag=DIAG_F4, max_gamma=8, nthreads=0, log_cap=4096, max2=None):
    """Full BZ pipeline: (d, witness, log[(t, j, L, U, combinations)]).
    max2: as for gamma (F4 with mixed packages)."""
    B, p = _u8(B)
    n = B.shape[1] // 2
    d = ctypes.c_int(-1)
    wit = np.zeros(2 * n, dtype=np.uint8)
    log = np.zeros((log_cap, 5), dtype=np.int64)
    nl = ctypes.c_int(0)
    logp = log.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong))
    if max2 is None:
        _check(lib().qdo_bz(p, B.shape[0], n, diag, max_gamma, nthreads, ctypes.byref(d),
                            wit.ctypes.data_as(_u8p), logp, log_cap, ctypes.byref(nl)), "bz")
    else:
        assert diag == DIAG_F4
        caps = _caps(max2, max_gamma)
        _check(lib().qdo_bz_mixed(p, B.shape[0], n, max_gamma, caps.ctypes.data_as(_ip), nthreads,
                                  ctypes.byref(d), wit.ctypes.data_as(_u8p), logp, log_cap,
                                  ctypes.byref(nl)), "bz_mixed")
    return d.value, wit, _log_records(log, nl.value)


def distance(G, field=2, nthreads=0):
    """Oracle distance of a product-ABI input: brute force when the rank is at
    most 24, Brouwer-Zimmermann otherwise.  Returns (d, witness)."""
    B = expand(G, field)
    if rank(B) <= 24:
        return brute(B, nthreads)
    d, w, _ = bz(B, DIAG_F4, 8, nthreads)
    return d, w


def gamma_iso(B, max_gamma=8, with_rows=False):
    """Information-set matrices of the isometric image (Sec. 2.4): returns
    (rank, [ (k_j, pivot columns per row (-1: none), rows or None) ])."""
    B, p = _u8(B)
    m, n = B.shape[0], B.shape[1] // 2
    h = ctypes.c_int(0)
    k = np.zeros(max_gamma, dtype=np.int32)
    piv = np.zeros(max_gamma * m, dtype=np.int32)
    rows = np.zeros((max_gamma * m, 3 * n), dtype=np.uint8) if with_rows else None
    r = lib().qdo_gamma_iso(p, m, n, max_gamma, ctypes.byref(h), k.ctypes.data_as(_ip),
                            piv.ctypes.data_as(_ip), rows.ctypes.data_as(_u8p) if with_rows else None)
    _check(r, "gamma_iso")
    out = []
    for j in range(h.value):
        out.append((int(k[j]), piv[j * r:(j + 1) * r].copy(),
                    rows[j * r:(j + 1) * r].copy() if with_rows else None))
    return r, out


def bz_iso(B, max_gamma=8, nthreads=0, log_cap=4096):
    """Saved_isometry: (d, witness (a|b), log[(t, j, L_H, U_H, combinations)])."""
    B, p = _u8(B)
    n = B.shape[1] // 2
    d = ctypes.c_int(-1)
    wit = np.zeros(2 * n, dtype=np.uint8)
    log = np.zeros((log_cap, 5), dtype=np.int64)
    nl = ctypes.c_int(0)
    _check(lib().qdo_bz_iso(p, B.shape[0], n, max_gamma, nthreads, ctypes.byref(d),
                            wit.ctypes.data_as(_u8p),
                            log.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)), log_cap,
                            ctypes.byref(nl)), "bz_iso")
    return d.value, wit, _log_records(log, nl.value)


def brute_stab(B, nthreads=0):
    """Exhaustive Modified-BZ minimum: least weight over span(B) minus its
    symplectic radical (the stabilizer when B generates a normalizer)."""
    B, p = _u8(B)
    n = B.shape[1] // 2
    d = ctypes.c_int(-1)
    wit = np.zeros(2 * n, dtype=np.uint8)
    _check(lib().qdo_brute_stab(p, B.shape[0], n, nthreads, ctypes.byref(d), wit.ctypes.data_as(_u8p)),
           "brute_stab")
    return d.value, wit


def bz_stab(B, diag=DIAG_F4, max_gamma=8, nthreads=0, log_cap=4096):
    """Modified BZ (Sec. 2.1) over the diag construction: (d, witness, log)."""
    B, p = _u8(B)
    n = B.shape[1] // 2
    d = ctypes.c_int(-1)
    wit = np.zeros(2 * n, dtype=np.uint8)
    log = np.zeros((log_cap, 5), dtype=np.int64)
    nl = ctypes.c_int(0)
    _check(lib().qdo_bz_stab(p, B.shape[0], n, diag, max_gamma, nthreads, ctypes.byref(d),
                             wit.ctypes.data_as(_u8p),
                             log.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)), log_cap,
                             ctypes.byref(nl)), "bz_stab")
    return d.value, wit, _log_records(log, nl.value)
