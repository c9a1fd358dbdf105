"""Python binding of the oracle (TEST INFRASTRUCTURE ONLY).

The oracle is a plain, exact CPU tracker written from the paper (Guo et al., FTK; Sec. 3.3, Sec. 4.1-4.3,
Eq. 2, Alg. 1).  Only tests/, the smoke check and the benchmark's CPU-baseline leg may import this module.  It
shares no code with the HIP library and never calls it.

All arrays are numpy; field layouts: scalar [nt][(nz)][ny][nx] float32, vector [nt][n][(nz)][ny][nx] float32.
"""
import ctypes
import os

import numpy as np

from . import build_oracle

STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_NONFINITE", 3: "ERR_RANGE", 5: "ERR_OOM", 7: "ERR_INVARIANT"}
TYPES = ["DEGENERATE", "MIN", "MAX", "SADDLE", "SADDLE1", "SADDLE2", "SOURCE", "SINK",
         "REPELLING_FOCUS", "ATTRACTING_FOCUS", "CENTER"]
FLAG_DEGENERATE_SUBLOC = 1
FLAG_WIDE = 4

_i64p = ctypes.POINTER(ctypes.c_int64)
_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i8p = ctypes.POINTER(ctypes.c_int8)


class _Result(ctypes.Structure):
    _fields_ = [("n_hits", ctypes.c_int64), ("n_traj", ctypes.c_int64),
                ("face_id", _i64p), ("pos", _f64p), ("mu", _f64p),
                ("type", _u8p), ("flags", _u8p), ("label", _i64p),
                ("simplices_tested", ctypes.c_int64), ("cells_with_hits", ctypes.c_int64),
                ("invariant_violations", ctypes.c_int64),
                ("t_quantise", ctypes.c_double), ("t_detect", ctypes.c_double),
                ("t_subloc", ctypes.c_double), ("t_stitch", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build_oracle.build(force=False)
        L = ctypes.CDLL(path)
        L.orc_kuhn_types.argtypes = [ctypes.c_int, ctypes.c_int, _i8p]
        L.orc_kuhn_types.restype = ctypes.c_int
        L.orc_sos_sign.argtypes = [ctypes.c_int, _i64p]
        L.orc_sos_sign.restype = ctypes.c_int
        L.orc_face_punctured.argtypes = [ctypes.c_int, _i64p]
        L.orc_face_punctured.restype = ctypes.c_int
        L.orc_track.argtypes = [ctypes.c_int, _f32p, ctypes.c_int, _i64p, ctypes.c_int, ctypes.c_int,
                                ctypes.POINTER(_Result)]
        L.orc_track.restype = ctypes.c_int
        L.orc_result_free.argtypes = [ctypes.POINTER(_Result)]
        L.orc_detect_count.argtypes = [ctypes.c_int, _f32p, ctypes.c_int, _i64p, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int64, ctypes.c_int64, _i64p]
        L.orc_detect_count.restype = ctypes.c_int64
        L.orc_eval_faces.argtypes = [ctypes.c_int, _f32p, ctypes.c_int, _i64p, ctypes.c_int, ctypes.c_int64,
                                     _i64p, _u8p, _f64p, _f64p, _u8p, _u8p]
        L.orc_eval_faces.restype = ctypes.c_int
        L.orc_cell_sides.argtypes = [ctypes.c_int, _i64p, ctypes.c_int64, _i64p, _i64p]
        L.orc_cell_sides.restype = ctypes.c_int
        L.orc_face_cofaces.argtypes = [ctypes.c_int, _i64p, ctypes.c_int64, _i64p]
        L.orc_face_cofaces.restype = ctypes.c_int
        L.orc_trace.argtypes = [ctypes.c_int, _f32p, ctypes.c_int, _i64p, ctypes.c_int, ctypes.c_int64,
                                ctypes.c_int64, _i64p, ctypes.POINTER(ctypes.c_int)]
        L.orc_trace.restype = ctypes.c_int64
        L.orc_quantise_all.argtypes = [ctypes.c_int, _f32p, ctypes.c_int, _i64p, ctypes.c_int, _i64p]
        L.orc_quantise_all.restype = ctypes.c_int
        L.orc_jacobian_all.argtypes = [ctypes.c_int, _f32p, ctypes.c_int, _i64p, _f32p]
        L.orc_jacobian_all.restype = ctypes.c_int
        L.orc_simplex_count.argtypes = [ctypes.c_int, _i64p]
        L.orc_simplex_count.restype = ctypes.c_int64
        L.orc_classify_matrix.argtypes = [ctypes.c_int, ctypes.c_int, _f64p]
        L.orc_classify_matrix.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _field(field, n, kind):
    f = np.ascontiguousarray(field, dtype=np.float32)
    if kind == 0:
        dims = f.shape[::-1]  # (nx, ny, [nz], nt)
    else:
        if f.shape[1] != n:
            raise ValueError("vector field must be [nt][n][...]")
        sp = f.shape[2:][::-1]
        dims = tuple(sp) + (f.shape[0],)
    if len(dims) != n + 1:
        raise ValueError("field rank does not match n")
    return f, np.asarray(dims, dtype=np.int64)


def kuhn_types(d, k):
    cnt = lib().orc_kuhn_types(d, k, None)
    out = np.zeros((cnt, 4), dtype=np.int8)
    lib().orc_kuhn_types(d, k, _p(out, _i8p))
    return out[:, :k].copy()


def sos_sign(m):
    """SoS sign of a square integer matrix m[j][k] (rows = components, columns = vertices in index order)."""
    m = np.asarray(m, dtype=np.int64)
    n = m.shape[0]
    cols = np.ascontiguousarray(m.T)
    return lib().orc_sos_sign(n, _p(cols, _i64p))


def face_punctured(vecs):
    """Puncture predicate on [n+1][n] integer vectors in chain order."""
    v = np.ascontiguousarray(vecs, dtype=np.int64)
    return lib().orc_face_punctured(v.shape[1], _p(v, _i64p))


def simplex_count(n, dims):
    d = np.asarray(dims, dtype=np.int64)
    return lib().orc_simplex_count(n, _p(d, _i64p))


def classify_matrix(J, kind):
    J = np.ascontiguousarray(J, dtype=np.float64)
    return lib().orc_classify_matrix(J.shape[0], kind, _p(J, _f64p))


class Track:
    """Result of a whole-field oracle run (host arrays)."""

    def __init__(self, status, r, n):
        self.status = status
        self.n_hits = int(r.n_hits)
        self.n_traj = int(r.n_traj)
        nh = self.n_hits
        self.face_id = np.ctypeslib.as_array(r.face_id, (nh,)).copy() if nh else np.zeros(0, np.int64)
        self.pos = np.ctypeslib.as_array(r.pos, (nh * (n + 1),)).reshape(nh, n + 1).copy() if nh else np.zeros((0, n + 1))
        self.mu = np.ctypeslib.as_array(r.mu, (nh * (n + 1),)).reshape(nh, n + 1).copy() if nh else np.zeros((0, n + 1))
        self.type = np.ctypeslib.as_array(r.type, (nh,)).copy() if nh else np.zeros(0, np.uint8)
        self.flags = np.ctypeslib.as_array(r.flags, (nh,)).copy() if nh else np.zeros(0, np.uint8)
        self.label = np.ctypeslib.as_array(r.label, (nh,)).copy() if nh else np.zeros(0, np.int64)
        self.simplices_tested = int(r.simplices_tested)
        self.cells_with_hits = int(r.cells_with_hits)
        self.invariant_violations = int(r.invariant_violations)
        self.times = dict(quantise=r.t_quantise, detect=r.t_detect, subloc=r.t_subloc, stitch=r.t_stitch)


def track(field, n=2, kind=0, qshift=20, nthreads=0):
    f, dims = _field(field, n, kind)
    r = _Result()
    st = lib().orc_track(n, _p(f, _f32p), kind, _p(dims, _i64p), qshift, nthreads, ctypes.byref(r))
    if st not in (0, 7):
        return Track(st, _Result(), n)
    out = Track(st, r, n)
    lib().orc_result_free(ctypes.byref(r))
    return out


def detect_count(field, n=2, kind=0, qshift=20, nthreads=0, t_begin=0, t_end=None):
    f, dims = _field(field, n, kind)
    nt = int(dims[-1])
    t_end = nt if t_end is None else t_end
    tested = np.zeros(1, np.int64)
    nh = lib().orc_detect_count(n, _p(f, _f32p), kind, _p(dims, _i64p), qshift, nthreads, t_begin, t_end,
                                _p(tested, _i64p))
    return int(nh), int(tested[0])


def eval_faces(field, face_ids, n=2, kind=0, qshift=20):
    f, dims = _field(field, n, kind)
    fids = np.ascontiguousarray(face_ids, dtype=np.int64)
    k = fids.shape[0]
    punct = np.zeros(k, np.uint8)
    mu = np.zeros((k, n + 1), np.float64)
    pos = np.zeros((k, n + 1), np.float64)
    typ = np.zeros(k, np.uint8)
    flg = np.zeros(k, np.uint8)
    st = lib().orc_eval_faces(n, _p(f, _f32p), kind, _p(dims, _i64p), qshift, k, _p(fids, _i64p),
                              _p(punct, _u8p), _p(mu, _f64p), _p(pos, _f64p), _p(typ, _u8p), _p(flg, _u8p))
    return dict(status=st, punctured=punct, mu=mu, pos=pos, type=typ, flags=flg)


def cell_sides(dims, cell_ids, n=2):
    dims = np.asarray(dims, dtype=np.int64)
    c = np.ascontiguousarray(cell_ids, dtype=np.int64)
    out = np.zeros((c.shape[0], n + 2), np.int64)
    lib().orc_cell_sides(n, _p(dims, _i64p), c.shape[0], _p(c, _i64p), _p(out, _i64p))
    return out


def face_cofaces(dims, face_id, n=2):
    dims = np.asarray(dims, dtype=np.int64)
    out = np.zeros(8, np.int64)
    k = lib().orc_face_cofaces(n, _p(dims, _i64p), int(face_id), _p(out, _i64p))
    return out[:k].copy()


def trace(field, face_id, n=2, kind=0, qshift=20, max_steps=1 << 20):
    f, dims = _field(field, n, kind)
    mn = np.zeros(1, np.int64)
    closed = ctypes.c_int(0)
    cnt = lib().orc_trace(n, _p(f, _f32p), kind, _p(dims, _i64p), qshift, int(face_id), max_steps,
                          _p(mn, _i64p), ctypes.byref(closed))
    return dict(length=int(cnt), min_face=int(mn[0]), closed=int(closed.value))


def quantise_all(field, n=2, kind=0, qshift=20):
    f, dims = _field(field, n, kind)
    V = int(np.prod(dims))
    q = np.zeros((V, n), np.int64)
    st = lib().orc_quantise_all(n, _p(f, _f32p), kind, _p(dims, _i64p), qshift, _p(q, _i64p))
    return st, q


def jacobian_all(field, n=2, kind=0):
    f, dims = _field(field, n, kind)
    V = int(np.prod(dims))
    J = np.zeros((V, n, n), np.float32)
    st = lib().orc_jacobian_all(n, _p(f, _f32p), kind, _p(dims, _i64p), _p(J, _f32p))
    return st, J
