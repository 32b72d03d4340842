"""Python binding of libqdist (ctypes).  Argument marshalling only: every
step of the computation runs in the native library (host C++ and gfx950 HIP
kernels).  Importing this module fails loudly when libqdist.so has not been
built; there is no fallback implementation.

Names follow include/qdist.h.  Matrices are numpy uint8 arrays:
  field 2: (m, 2n), entries {0,1}, row = x_1..x_n | z_1..z_n
  field 4: (m, n),  entries {0..3}, code a + 2b for a + alpha*b
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqdist.so")

QD_FIELD_F2, QD_FIELD_F4 = 2, 4
QD_DIAG_AUTO, QD_DIAG_F2, QD_DIAG_F4, QD_DIAG_ISO = 0, 2, 4, 3
QD_FILTER_NONE, QD_FILTER_STABILIZER = 0, 1
QD_OK, QD_INCOMPLETE = 0, 1
QD_ERR_INVALID, QD_ERR_ZERO_CODE, QD_ERR_TOO_LARGE = -1, -2, -3
QD_ERR_NOMEM, QD_ERR_DEVICE, QD_ERR_INTERNAL = -4, -5, -6
QD_MAX_N, QD_MAX_GAMMA, QD_MAX_LOG = 128, 8, 96
QD_NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libqdist.so not found at {LIB_PATH}; build it with __graft_entry__.build()")
# PyTorch ships its own HIP runtime under the same soname as the system one
# the library links to, and whichever loads first serves the whole process.
# Load PyTorch's first when it is installed, so that both share one runtime:
# streams passed from PyTorch are then valid here, and PyTorch still finds
# the GPU after this library has used it.
try:
    import torch  # noqa: F401
except ImportError:
    pass
_lib = ctypes.CDLL(LIB_PATH)


class QdError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"{qd_strerror(status)} (status {status})")
        self.status = status


class qd_resume(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int), ("j", ctypes.c_int), ("U", ctypes.c_int),
                ("witness", ctypes.POINTER(ctypes.c_uint8)), ("structure", ctypes.c_ulonglong)]


class qd_options(ctypes.Structure):
    _fields_ = [("diag", ctypes.c_int), ("max_gamma", ctypes.c_int),
                ("budget", ctypes.c_ulonglong), ("cancel", ctypes.POINTER(ctypes.c_int)),
                ("stream", ctypes.c_void_p), ("seg_len", ctypes.c_int),
                ("saved_depth", ctypes.c_int), ("timing", ctypes.c_int), ("tops_mode", ctypes.c_int),
                ("filter", ctypes.c_int), ("scalar_classes", ctypes.c_int),
                ("partial_weight", ctypes.c_int), ("mixed_packages", ctypes.c_int), ("walk", ctypes.c_int),
                ("resume", ctypes.POINTER(qd_resume)), ("matrix_cores", ctypes.c_int)]


class qd_round_log(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int), ("j", ctypes.c_int), ("L", ctypes.c_int), ("U", ctypes.c_int),
                ("saved_depth", ctypes.c_int), ("launches", ctypes.c_int),
                ("combinations", ctypes.c_ulonglong), ("planned", ctypes.c_ulonglong),
                ("kernel_ms", ctypes.c_float)]


class qd_stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("rank", ctypes.c_int), ("D", ctypes.c_int), ("diag", ctypes.c_int),
                ("h", ctypes.c_int), ("P", ctypes.c_int * QD_MAX_GAMMA),
                ("delta", ctypes.c_int * QD_MAX_GAMMA), ("L", ctypes.c_int), ("U", ctypes.c_int),
                ("d_estimate", ctypes.c_int), ("predicted", ctypes.c_double),
                ("combinations", ctypes.c_ulonglong), ("enumerated", ctypes.c_ulonglong),
                ("words", ctypes.c_ulonglong), ("host_ms", ctypes.c_double),
                ("kernel_ms", ctypes.c_double), ("enumerated_kernel_ms", ctypes.c_double),
                ("wall_ms", ctypes.c_double),
                ("launches", ctypes.c_int), ("logical_pairs", ctypes.c_int),
                ("scalar_classes", ctypes.c_int), ("two_row_cap", ctypes.c_int * QD_MAX_GAMMA),
                ("next_t", ctypes.c_int), ("next_j", ctypes.c_int), ("structure", ctypes.c_ulonglong),
                ("nlog", ctypes.c_int),
                ("log", qd_round_log * QD_MAX_LOG), ("matrix_core_launches", ctypes.c_int)]

    def rounds(self):
        out = []
        for i in range(min(self.nlog, QD_MAX_LOG)):
            r = self.log[i]
            out.append({k: getattr(r, k) for k, _ in qd_round_log._fields_})
        return out

    def to_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("P", "delta", "log")}
        d["P"] = list(self.P)[: self.h]
        d["delta"] = list(self.delta)[: self.h]
        d["rounds"] = self.rounds()
        return d


class qd_result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_ulonglong), ("status", ctypes.c_int), ("d", ctypes.c_int), ("L", ctypes.c_int),
                ("n", ctypes.c_int), ("latency_ms", ctypes.c_double), ("queue_ms", ctypes.c_double),
                ("combinations", ctypes.c_ulonglong)]


class qd_plan_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("rank", ctypes.c_int), ("diag", ctypes.c_int), ("h", ctypes.c_int),
                ("h_used", ctypes.c_int), ("P", ctypes.c_int * QD_MAX_GAMMA),
                ("delta", ctypes.c_int * QD_MAX_GAMMA),
                ("dims", (ctypes.c_int * (2 * QD_MAX_N)) * QD_MAX_GAMMA),
                ("pivot", (ctypes.c_int * (2 * QD_MAX_N)) * QD_MAX_GAMMA),
                ("d_estimate", ctypes.c_int), ("predicted_f2", ctypes.c_double),
                ("predicted_f4", ctypes.c_double), ("predicted_iso", ctypes.c_double),
                ("f4_two_row_cap", ctypes.c_int * QD_MAX_GAMMA), ("f4_scalar_classes", ctypes.c_int)]


_u8p = ctypes.POINTER(ctypes.c_uint8)
_ip = ctypes.POINTER(ctypes.c_int)
_lib.qd_strerror.restype = ctypes.c_char_p
_lib.qd_distance.argtypes = [_u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _ip, _u8p]
_lib.qd_distance_ex.argtypes = [_u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(qd_options),
                                _ip, _u8p, ctypes.POINTER(qd_stats)]
_lib.qd_distance_batch_ex.argtypes = [ctypes.c_int, ctypes.POINTER(_u8p), _ip, _ip, _ip,
                                      ctypes.POINTER(qd_options), _ip, ctypes.POINTER(_u8p), _ip,
                                      ctypes.POINTER(qd_stats)]
_lib.qd_plan.argtypes = [_u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                         ctypes.POINTER(qd_plan_info)]
_lib.qd_round_min.argtypes = [_u8p, _ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, _ip, _u8p,
                              ctypes.POINTER(ctypes.c_ulonglong), ctypes.c_int]
_lib.qd_round_census.argtypes = [_u8p, _ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 _ip, _u8p, ctypes.POINTER(ctypes.c_ulonglong), ctypes.POINTER(ctypes.c_ulonglong),
                                 ctypes.POINTER(ctypes.c_ulonglong)]
_lib.qd_round_min_noalloc.argtypes = [_u8p, _ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, _ip, _u8p,
                                      ctypes.POINTER(ctypes.c_ulonglong), ctypes.c_int, ctypes.c_void_p]
_lib.qd_tune_run.argtypes = [ctypes.c_double, ctypes.c_char_p, ctypes.c_size_t]
_lib.qd_tune_load.argtypes = [ctypes.c_char_p]
_lib.qd_tune_get.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
_lib.qd_round_walk.argtypes = [_u8p, _ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _ip, _u8p,
                               ctypes.POINTER(ctypes.c_ulonglong), ctypes.POINTER(ctypes.c_ulonglong)]
_lib.qd_device_check.argtypes = [ctypes.c_char_p, ctypes.c_int]
_lib.qd_engine_create.restype = ctypes.c_void_p
_lib.qd_engine_create.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
_lib.qd_engine_submit.argtypes = [ctypes.c_void_p, _u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_ulonglong, ctypes.POINTER(qd_options)]
_lib.qd_engine_poll.argtypes = [ctypes.c_void_p, ctypes.POINTER(qd_result), _u8p, ctypes.c_int, ctypes.c_int]
_lib.qd_engine_outstanding.argtypes = [ctypes.c_void_p]
_lib.qd_engine_destroy.argtypes = [ctypes.c_void_p]
_lib.qd_valu_peak.argtypes = [ctypes.POINTER(ctypes.c_double)]
_lib.qd_valu_mix.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]


def qd_strerror(status):
    return _lib.qd_strerror(int(status)).decode()


def _matrix(G, field):
    G = np.ascontiguousarray(G, dtype=np.uint8)
    if G.ndim != 2:
        raise ValueError("G must be a 2-D uint8 array")
    m = G.shape[0]
    if field == QD_FIELD_F2:
        if G.shape[1] % 2:
            raise ValueError("a field-2 matrix has 2n columns")
        n = G.shape[1] // 2
    else:
        n = G.shape[1]
    return G, m, n


def resume_point(stats, witness):
    """The resume point (t, j, U, witness, structure) of a call that ended
    with QD_INCOMPLETE, from its qd_stats and returned witness."""
    return (stats.next_t, stats.next_j, stats.U, None if stats.U > stats.n else witness, stats.structure)


def _options(opts):
    o = qd_options()
    keep = []  # objects the options point into, alive until the call returns
    for k, v in (opts or {}).items():
        if k == "cancel":
            keep.append(v)  # a ctypes.c_int the caller keeps alive
            o.cancel = ctypes.pointer(v)
        elif k == "resume":  # (t, j, U, witness array or None, structure)
            t, j, U, wit, structure = v
            r = qd_resume(t, j, U, None, structure)
            if wit is not None:
                wbuf = np.ascontiguousarray(wit, dtype=np.uint8)
                r.witness = wbuf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
                keep.append(wbuf)
            keep.append(r)
            o.resume = ctypes.pointer(r)
        elif k == "stream":
            o.stream = ctypes.c_void_p(int(v))
        else:
            setattr(o, k, v)
    return o, keep


def qd_distance(G, field=QD_FIELD_F2):
    """Returns (status, d, witness)."""
    G, m, n = _matrix(G, field)
    d = ctypes.c_int(-1)
    wit = np.zeros(2 * n, dtype=np.uint8)
    st = _lib.qd_distance(G.ctypes.data_as(_u8p), m, n, field, ctypes.byref(d), wit.ctypes.data_as(_u8p))
    return st, d.value, wit


def qd_distance_ex(G, field=QD_FIELD_F2, **opts):
    """Returns (status, d, witness, qd_stats).  Options: diag, max_gamma,
    budget, cancel (ctypes.c_int), stream (hipStream_t as int), seg_len,
    saved_depth, timing, tops_mode, filter, scalar_classes, partial_weight,
    mixed_packages, walk, resume (a resume_point tuple), matrix_cores."""
    G, m, n = _matrix(G, field)
    o, _keep = _options(opts)
    d = ctypes.c_int(-1)
    wit = np.zeros(2 * n, dtype=np.uint8)
    s = qd_stats()
    st = _lib.qd_distance_ex(G.ctypes.data_as(_u8p), m, n, field, ctypes.byref(o), ctypes.byref(d),
                             wit.ctypes.data_as(_u8p), ctypes.byref(s))
    return st, d.value, wit, s


def qd_distance_batch(codes, **opts):
    """codes: list of (G, field).  Returns (status, d list, witness list,
    per-code status list, per-code qd_stats list)."""
    count = len(codes)
    mats, ms, ns, fs, wits = [], [], [], [], []
    for G, f in codes:
        G, m, n = _matrix(G, f)
        mats.append(G); ms.append(m); ns.append(n); fs.append(f)
        wits.append(np.zeros(2 * n, dtype=np.uint8))
    Gp = (_u8p * max(count, 1))(*[g.ctypes.data_as(_u8p) for g in mats])
    Wp = (_u8p * max(count, 1))(*[w.ctypes.data_as(_u8p) for w in wits])
    m_a = (ctypes.c_int * max(count, 1))(*ms)
    n_a = (ctypes.c_int * max(count, 1))(*ns)
    f_a = (ctypes.c_int * max(count, 1))(*fs)
    d_a = (ctypes.c_int * max(count, 1))()
    s_a = (ctypes.c_int * max(count, 1))()
    stats = (qd_stats * max(count, 1))()
    o, _keep = _options(opts)
    st = _lib.qd_distance_batch_ex(count, Gp, m_a, n_a, f_a, ctypes.byref(o), d_a, Wp, s_a, stats)
    return st, list(d_a)[:count], wits, list(s_a)[:count], list(stats)[:count]


def qd_plan(G, field=QD_FIELD_F2, diag=QD_DIAG_AUTO, max_gamma=0):
    """Host-only: generator-matrix structure and planner choice (dict)."""
    G, m, n = _matrix(G, field)
    info = qd_plan_info()
    st = _lib.qd_plan(G.ctypes.data_as(_u8p), m, n, field, diag, max_gamma, ctypes.byref(info))
    if st < 0:
        raise QdError(st)
    gs = []
    for j in range(info.h):
        P = info.P[j]
        gs.append({"P": P, "delta": info.delta[j], "dims": list(info.dims[j])[:P],
                   "pivots": list(info.pivot[j])[:P]})
    return {"n": info.n, "rank": info.rank, "diag": info.diag, "h": info.h, "h_used": info.h_used,
            "gammas": gs, "d_estimate": info.d_estimate, "predicted_f2": info.predicted_f2,
            "predicted_f4": info.predicted_f4, "predicted_iso": info.predicted_iso,
            "f4_two_row_cap": list(info.f4_two_row_cap), "f4_scalar_classes": info.f4_scalar_classes}


def qd_round_min(rows, dims, t, partial_words=0):
    """One GPU enumeration round: returns (status, wmin, witness, count).
    partial_words = w > 0: tiles evaluate w words first."""
    rows = np.ascontiguousarray(rows, dtype=np.uint8)
    dims = np.ascontiguousarray(dims, dtype=np.int32)
    P = dims.shape[0]
    n = rows.shape[1] // 2
    w = ctypes.c_int(0)
    cnt = ctypes.c_ulonglong(0)
    wit = np.zeros(2 * n, dtype=np.uint8)
    st = _lib.qd_round_min(rows.ctypes.data_as(_u8p), dims.ctypes.data_as(_ip), P, n, t, ctypes.byref(w),
                           wit.ctypes.data_as(_u8p), ctypes.byref(cnt), partial_words)
    return st, w.value, wit, cnt.value


def qd_tune_run(max_seconds=60.0):
    """Measures the launch shapes on the device and installs them: returns
    (status, table as JSON text)."""
    buf = ctypes.create_string_buffer(1 << 16)
    st = _lib.qd_tune_run(max_seconds, buf, len(buf))
    return st, buf.value.decode()


def qd_tune_load(text):
    return _lib.qd_tune_load(text.encode())


def qd_tune_get():
    buf = ctypes.create_string_buffer(1 << 16)
    st = _lib.qd_tune_get(buf, len(buf))
    return st, buf.value.decode()


def qd_tune_reset():
    return _lib.qd_tune_reset()


def qd_round_min_noalloc(rows, dims, t, partial_words=0, stream=None):
    """qd_round_min on the library's fixed device array (no device
    allocation): returns (status, wmin, witness, count)."""
    rows = np.ascontiguousarray(rows, dtype=np.uint8)
    dims = np.ascontiguousarray(dims, dtype=np.int32)
    P = dims.shape[0]
    n = rows.shape[1] // 2
    w = ctypes.c_int(0)
    cnt = ctypes.c_ulonglong(0)
    wit = np.zeros(2 * n, dtype=np.uint8)
    st = _lib.qd_round_min_noalloc(rows.ctypes.data_as(_u8p), dims.ctypes.data_as(_ip), P, n, t, ctypes.byref(w),
                                   wit.ctypes.data_as(_u8p), ctypes.byref(cnt), partial_words, stream)
    return st, w.value, wit, cnt.value


def qd_round_census(rows, dims, t, below, partial_words=0):
    """One GPU enumeration round with a census: returns (status, wmin,
    witness, count, below_count, below_weight_sum)."""
    rows = np.ascontiguousarray(rows, dtype=np.uint8)
    dims = np.ascontiguousarray(dims, dtype=np.int32)
    P = dims.shape[0]
    n = rows.shape[1] // 2
    w = ctypes.c_int(0)
    cnt, bc, bs = ctypes.c_ulonglong(0), ctypes.c_ulonglong(0), ctypes.c_ulonglong(0)
    wit = np.zeros(2 * n, dtype=np.uint8)
    st = _lib.qd_round_census(rows.ctypes.data_as(_u8p), dims.ctypes.data_as(_ip), P, n, t, partial_words, below,
                              ctypes.byref(w), wit.ctypes.data_as(_u8p), ctypes.byref(cnt), ctypes.byref(bc),
                              ctypes.byref(bs))
    return st, w.value, wit, cnt.value, bc.value, bs.value


def qd_round_walk(rows, dims, t, per_lane=1, weight_sum=False):
    """One round with the plain walk kernel: returns (status, wmin, witness,
    count, weight sum or None)."""
    rows = np.ascontiguousarray(rows, dtype=np.uint8)
    dims = np.ascontiguousarray(dims, dtype=np.int32)
    P = dims.shape[0]
    n = rows.shape[1] // 2
    w = ctypes.c_int(0)
    cnt = ctypes.c_ulonglong(0)
    ws = ctypes.c_ulonglong(0)
    wit = np.zeros(2 * n, dtype=np.uint8)
    st = _lib.qd_round_walk(rows.ctypes.data_as(_u8p), dims.ctypes.data_as(_ip), P, n, t, per_lane,
                            ctypes.byref(w), wit.ctypes.data_as(_u8p), ctypes.byref(cnt),
                            ctypes.byref(ws) if weight_sum else None)
    return st, w.value, wit, cnt.value, (ws.value if weight_sum else None)


def qd_device_check():
    buf = ctypes.create_string_buffer(64)
    st = _lib.qd_device_check(buf, 64)
    return st, buf.value.decode()


def qd_valu_peak():
    v = ctypes.c_double(0)
    st = _lib.qd_valu_peak(ctypes.byref(v))
    return st, v.value


QD_MIXES = {"hotloop_sgpr": 0, "hotloop_vgpr": 1, "bcnt": 2, "xor_vgpr": 3, "xor_sgpr": 4}


def qd_valu_mix(mix):
    """(status, lane-ops/s) of one QD_MIX_* instruction mix."""
    v = ctypes.c_double(0)
    st = _lib.qd_valu_mix(int(mix), ctypes.byref(v))
    return st, v.value


def qd_engine_create(mem_budget=0, max_active=0, stream=None):
    """Returns an engine handle (int) or None."""
    h = _lib.qd_engine_create(mem_budget, max_active, ctypes.c_void_p(int(stream)) if stream else None)
    return h


def qd_engine_submit(engine, G, field=QD_FIELD_F2, tag=0, **opts):
    G, m, n = _matrix(G, field)
    o, _keep = _options(opts)
    return _lib.qd_engine_submit(engine, G.ctypes.data_as(_u8p), m, n, field, tag, ctypes.byref(o))


def qd_engine_poll(engine, max_results=64, wait_ms=0):
    """Returns a list of (qd_result, witness array of 2n bytes)."""
    res = (qd_result * max_results)()
    wit = np.zeros((max_results, 2 * QD_MAX_N), dtype=np.uint8)
    k = _lib.qd_engine_poll(engine, res, wit.ctypes.data_as(_u8p), max_results, wait_ms)
    if k < 0:
        raise QdError(k)
    return [(res[i], wit[i, : 2 * res[i].n].copy()) for i in range(k)]


def qd_engine_outstanding(engine):
    return _lib.qd_engine_outstanding(engine)


def qd_engine_destroy(engine):
    _lib.qd_engine_destroy(engine)


def exported_symbols():
    """Names of the C ABI entry points declared in include/qdist.h."""
    return ["qd_distance", "qd_distance_ex", "qd_distance_batch", "qd_distance_batch_ex", "qd_plan",
            "qd_round_min", "qd_round_census", "qd_round_min_noalloc", "qd_round_walk",
            "qd_tune_run", "qd_tune_load", "qd_tune_get", "qd_tune_reset", "qd_strerror", "qd_device_check", "qd_valu_peak", "qd_valu_mix", "qd_engine_create",
            "qd_engine_submit", "qd_engine_poll", "qd_engine_outstanding", "qd_engine_destroy"]
