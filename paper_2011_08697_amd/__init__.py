"""Python binding of libftk_mi355x.so (critical-point tracking on the simplicial spacetime mesh, gfx950).

Argument marshalling only: every step of the computation runs in the HIP library.  Device memory for outputs and
scratch comes from PyTorch's caching allocator through the library's allocator hooks, on PyTorch's current
stream.  If the library is missing the calls raise; there is no CPU fallback.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libftk_mi355x.so")

TYPES = ["DEGENERATE", "MIN", "MAX", "SADDLE", "SADDLE1", "SADDLE2", "SOURCE", "SINK",
         "REPELLING_FOCUS", "ATTRACTING_FOCUS", "CENTER"]
STATUS = ["OK", "ERR_ARG", "ERR_NONFINITE", "ERR_RANGE", "ERR_CAPACITY", "ERR_OOM", "ERR_HIP",
          "ERR_INVARIANT", "ERR_STATE"]
FLAG_DEGENERATE_SUBLOC, FLAG_FP64_FALLBACK, FLAG_WIDE = 1, 2, 4
OUT_POS, OUT_MU, OUT_TYPE, OUT_LABEL, OUT_FLAGS, OUT_ALL, OUT_DEFAULT = 1, 2, 4, 8, 16, 31, 29
SCALAR, VECTOR = 0, 1

EXPORTS = ["ftk_default_options", "ftk_track_cp2d", "ftk_track_cp3d", "ftk_cp_create", "ftk_cp_push",
           "ftk_cp_finish", "ftk_cp_destroy", "ftk_track_cp2d_batched", "ftk_result_free", "ftk_simplex_count",
           "ftk_last_error", "ftk_version", "ftk_traj_table_build", "ftk_traj_table_free", "ftk_cp_slice",
           "ftk_cp_filter_loops", "ftk_buffer_free", "ftk_autotune_cp2d", "ftk_traj_order",
           "ftk_traj_smooth_types", "ftk_traj_simplify_types", "ftk_track_iso3d", "ftk_iso_result_free",
           "ftk_edge_count", "ftk_track_vortex3d", "ftk_vortex_result_free", "ftk_triangle_count",
           "ftk_track_cp_mesh2d", "ftk_mesh_result_free", "ftk_mesh_create", "ftk_mesh_destroy",
           "ftk_track_cp_mesh", "ftk_track_cp2d_into"]

_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class FtkError(RuntimeError):
    def __init__(self, status, msg):
        self.status = status
        name = STATUS[status] if 0 <= status < len(STATUS) else str(status)
        super().__init__(f"{name}: {msg}")


class Options(ctypes.Structure):
    _fields_ = [("quant_log2", ctypes.c_int32), ("precision", ctypes.c_int32), ("outputs", ctypes.c_uint32),
                ("tile_y", ctypes.c_int32), ("slab_depth", ctypes.c_int32),
                ("alloc", _ALLOC_FN), ("free", _FREE_FN), ("alloc_ctx", ctypes.c_void_p),
                ("profile", ctypes.c_int32), ("debug", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("simplices_tested", ctypes.c_int64), ("cells_linked", ctypes.c_int64),
                ("fp64_fallbacks", ctypes.c_int64), ("degenerate_sublocations", ctypes.c_int64),
                ("wide_path", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("t_detect_ms", ctypes.c_float), ("t_scan_ms", ctypes.c_float), ("t_emit_ms", ctypes.c_float),
                ("t_link_ms", ctypes.c_float)]


class Result(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("reserved", ctypes.c_int32), ("n_hits", ctypes.c_int64),
                ("n_trajectories", ctypes.c_int64), ("face_id", ctypes.c_void_p), ("pos", ctypes.c_void_p),
                ("mu", ctypes.c_void_p), ("type", ctypes.c_void_p), ("flags", ctypes.c_void_p),
                ("label", ctypes.c_void_p), ("stats", Stats)]


class IsoResult(ctypes.Structure):
    _fields_ = [("n_hits", ctypes.c_int64), ("n_components", ctypes.c_int64), ("n_tets", ctypes.c_int64),
                ("edge_id", ctypes.c_void_p), ("pos", ctypes.c_void_p), ("label", ctypes.c_void_p),
                ("tets", ctypes.c_void_p)]


class VortexResult(ctypes.Structure):
    _fields_ = [("n_hits", ctypes.c_int64), ("n_components", ctypes.c_int64), ("tri_id", ctypes.c_void_p),
                ("pos", ctypes.c_void_p), ("label", ctypes.c_void_p)]


class MeshResult(ctypes.Structure):
    _fields_ = [("n_hits", ctypes.c_int64), ("n_trajectories", ctypes.c_int64), ("faces_per_step", ctypes.c_int64),
                ("n_edges", ctypes.c_int64), ("face_id", ctypes.c_void_p), ("pos", ctypes.c_void_p),
                ("label", ctypes.c_void_p)]


class TrajTable(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("label", ctypes.c_void_p), ("n_points", ctypes.c_void_p),
                ("t_min", ctypes.c_void_p), ("t_max", ctypes.c_void_p), ("n_ends", ctypes.c_void_p)]


_lib = None


def lib():
    """Load the HIP library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2011_08697_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        i64, vp = ctypes.c_int64, ctypes.c_void_p
        L.ftk_default_options.argtypes = [ctypes.POINTER(Options)]
        L.ftk_track_cp2d.argtypes = [vp, ctypes.c_int, i64, i64, i64, ctypes.POINTER(Options), vp,
                                     ctypes.POINTER(Result)]
        L.ftk_track_cp2d.restype = ctypes.c_int
        L.ftk_track_cp2d_into.argtypes = [vp, ctypes.c_int, i64, i64, i64, ctypes.POINTER(Options), vp, i64,
                                          ctypes.POINTER(Result)]
        L.ftk_track_cp2d_into.restype = ctypes.c_int
        L.ftk_track_cp3d.argtypes = [vp, ctypes.c_int, i64, i64, i64, i64, ctypes.POINTER(Options), vp,
                                     ctypes.POINTER(Result)]
        L.ftk_track_cp3d.restype = ctypes.c_int
        L.ftk_cp_create.argtypes = [ctypes.c_int32, ctypes.POINTER(i64), ctypes.c_int, ctypes.POINTER(Options), vp,
                                    ctypes.POINTER(vp)]
        L.ftk_cp_create.restype = ctypes.c_int
        L.ftk_cp_push.argtypes = [vp, vp]
        L.ftk_cp_push.restype = ctypes.c_int
        L.ftk_cp_finish.argtypes = [vp, ctypes.POINTER(Result)]
        L.ftk_cp_finish.restype = ctypes.c_int
        L.ftk_cp_destroy.argtypes = [vp]
        L.ftk_cp_destroy.restype = None
        L.ftk_track_cp2d_batched.argtypes = [ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(i64),
                                             ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.c_int,
                                             ctypes.POINTER(Options), vp, ctypes.POINTER(Result)]
        L.ftk_track_cp2d_batched.restype = ctypes.c_int
        L.ftk_result_free.argtypes = [ctypes.POINTER(Result), ctypes.POINTER(Options), vp]
        L.ftk_result_free.restype = None
        L.ftk_simplex_count.argtypes = [ctypes.c_int32, ctypes.POINTER(i64)]
        L.ftk_simplex_count.restype = i64
        L.ftk_traj_table_build.argtypes = [ctypes.POINTER(Result), ctypes.c_int32, ctypes.POINTER(i64),
                                           ctypes.POINTER(Options), vp, ctypes.POINTER(TrajTable)]
        L.ftk_traj_table_build.restype = ctypes.c_int
        L.ftk_traj_table_free.argtypes = [ctypes.POINTER(TrajTable), ctypes.POINTER(Options), vp]
        L.ftk_traj_table_free.restype = None
        L.ftk_cp_slice.argtypes = [ctypes.POINTER(Result), ctypes.c_int32, ctypes.POINTER(i64), i64,
                                   ctypes.POINTER(Options), vp, ctypes.POINTER(vp), ctypes.POINTER(i64)]
        L.ftk_cp_slice.restype = ctypes.c_int
        L.ftk_cp_filter_loops.argtypes = [ctypes.POINTER(Result), ctypes.POINTER(TrajTable), ctypes.c_float, vp, vp]
        L.ftk_cp_filter_loops.restype = ctypes.c_int
        L.ftk_buffer_free.argtypes = [vp, ctypes.POINTER(Options), vp]
        L.ftk_track_iso3d.argtypes = [vp, i64, i64, i64, i64, ctypes.c_float, ctypes.POINTER(Options), vp,
                                      ctypes.POINTER(IsoResult)]
        L.ftk_track_iso3d.restype = ctypes.c_int
        L.ftk_iso_result_free.argtypes = [ctypes.POINTER(IsoResult), ctypes.POINTER(Options), vp]
        L.ftk_iso_result_free.restype = None
        L.ftk_edge_count.argtypes = [ctypes.POINTER(i64)]
        L.ftk_edge_count.restype = i64
        L.ftk_track_vortex3d.argtypes = [vp, i64, i64, i64, i64, ctypes.POINTER(Options), vp,
                                         ctypes.POINTER(VortexResult)]
        L.ftk_track_vortex3d.restype = ctypes.c_int
        L.ftk_vortex_result_free.argtypes = [ctypes.POINTER(VortexResult), ctypes.POINTER(Options), vp]
        L.ftk_vortex_result_free.restype = None
        L.ftk_triangle_count.argtypes = [ctypes.POINTER(i64)]
        L.ftk_triangle_count.restype = i64
        L.ftk_track_cp_mesh2d.argtypes = [vp, i64, vp, i64, vp, i64, ctypes.POINTER(Options), vp,
                                          ctypes.POINTER(MeshResult)]
        L.ftk_track_cp_mesh2d.restype = ctypes.c_int
        L.ftk_mesh_result_free.argtypes = [ctypes.POINTER(MeshResult), ctypes.POINTER(Options), vp]
        L.ftk_mesh_result_free.restype = None
        L.ftk_mesh_create.argtypes = [vp, i64, vp, i64, vp, ctypes.POINTER(vp)]
        L.ftk_mesh_create.restype = ctypes.c_int
        L.ftk_mesh_destroy.argtypes = [vp]
        L.ftk_mesh_destroy.restype = None
        L.ftk_track_cp_mesh.argtypes = [vp, vp, i64, ctypes.POINTER(Options), vp, ctypes.POINTER(MeshResult)]
        L.ftk_track_cp_mesh.restype = ctypes.c_int
        L.ftk_traj_order.argtypes = [ctypes.POINTER(Result), ctypes.c_int32, ctypes.POINTER(i64),
                                     ctypes.POINTER(TrajTable), ctypes.POINTER(Options), vp, vp, vp]
        L.ftk_traj_order.restype = ctypes.c_int
        L.ftk_traj_smooth_types.argtypes = [ctypes.POINTER(Result), ctypes.POINTER(TrajTable), vp, vp, vp,
                                            ctypes.c_int32, ctypes.POINTER(Options), vp, vp]
        L.ftk_traj_smooth_types.restype = ctypes.c_int
        L.ftk_traj_simplify_types.argtypes = [ctypes.POINTER(Result), ctypes.POINTER(TrajTable), vp, vp, vp,
                                              ctypes.c_float, ctypes.POINTER(Options), vp, vp]
        L.ftk_traj_simplify_types.restype = ctypes.c_int
        L.ftk_buffer_free.restype = None
        L.ftk_autotune_cp2d.argtypes = [vp, ctypes.c_int, i64, i64, i64, ctypes.POINTER(Options), vp,
                                        ctypes.POINTER(Options)]
        L.ftk_autotune_cp2d.restype = ctypes.c_int
        L.ftk_last_error.restype = ctypes.c_char_p
        L.ftk_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def last_error():
    return lib().ftk_last_error().decode()


def simplex_count(n, dims_with_t):
    arr = (ctypes.c_int64 * len(dims_with_t))(*dims_with_t)
    return lib().ftk_simplex_count(n, arr)


class _TorchPool:
    """Allocator hooks backed by torch's caching allocator; keeps the tensors alive by pointer."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = device
        self.live = {}
        self._alloc = _ALLOC_FN(self.alloc)
        self._free = _FREE_FN(self.free)

    def alloc(self, nbytes, stream, ctx):
        try:
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=self.device)
        except Exception:
            return None
        p = t.data_ptr()
        self.live[p] = t
        return p

    def free(self, ptr, stream, ctx):
        self.live.pop(ptr, None)

    def take(self, ptr, dtype, shape):
        if not ptr:
            return None
        t = self.live.pop(ptr)
        n = 1
        for s in shape:
            n *= s
        return t.view(dtype)[:n].view(*shape) if n else t.view(dtype)[:0].view(*shape)


def _options(pool, quant_log2=20, precision=0, outputs=OUT_DEFAULT, tile_y=0, slab_depth=0, profile=0, debug=0):
    o = Options()
    lib().ftk_default_options(ctypes.byref(o))
    o.quant_log2, o.precision, o.outputs = quant_log2, precision, outputs
    o.tile_y, o.slab_depth, o.profile, o.debug = tile_y, slab_depth, profile, debug
    if pool is not None:
        o.alloc, o.free = pool._alloc, pool._free
    return o


def _stream_handle(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _wrap(pool, r):
    import torch
    n, nh = r.n, int(r.n_hits)
    out = dict(n=n, n_hits=nh, n_trajectories=int(r.n_trajectories),
               face_id=pool.take(r.face_id, torch.int64, (nh,)),
               pos=pool.take(r.pos, torch.float32, (nh, n + 1)),
               mu=pool.take(r.mu, torch.float32, (nh, n + 1)),
               type=pool.take(r.type, torch.uint8, (nh,)),
               flags=pool.take(r.flags, torch.uint8, (nh,)),
               label=pool.take(r.label, torch.int64, (nh,)),
               stats={f: getattr(r.stats, f) for f, _ in Stats._fields_ if f != "reserved"})
    return out


def _check(st):
    if st != 0:
        raise FtkError(st, last_error())


def track_cp2d(field, kind=SCALAR, **opts):
    """field: contiguous float32 CUDA tensor [nt][ny][nx] (scalar) or [nt][2][ny][nx] (vector)."""
    if not field.is_contiguous() or field.dtype.itemsize != 4 or not field.is_cuda:
        raise ValueError("field must be a contiguous float32 device tensor")
    if kind == SCALAR:
        nt, ny, nx = field.shape
    else:
        nt, c, ny, nx = field.shape
        if c != 2:
            raise ValueError("vector field must be [nt][2][ny][nx]")
    pool = _TorchPool(field.device)
    o = _options(pool, **opts)
    r = Result()
    st = lib().ftk_track_cp2d(ctypes.c_void_p(field.data_ptr()), kind, nx, ny, nt, ctypes.byref(o),
                              _stream_handle(field.device), ctypes.byref(r))
    _check(st)
    return _wrap(pool, r)


STATIC_SCRATCH_BYTES = 256 << 20


def track_cp2d_into(field, kind=SCALAR, capacity=None, out=None, **opts):
    """ftk_track_cp2d_into: the library allocates nothing; outputs go to `out` (a dict of device tensors face_id,
    pos, mu, type, flags, label with room for `capacity` hits, as many as opts' outputs ask for), allocated here with
    torch when not given.  Returns the same dict layout as track_cp2d (views of the first n_hits entries)."""
    import torch
    if not field.is_contiguous() or field.dtype.itemsize != 4 or not field.is_cuda:
        raise ValueError("field must be a contiguous float32 device tensor")
    if kind == SCALAR:
        nt, ny, nx = field.shape
    else:
        nt, c, ny, nx = field.shape
        if c != 2:
            raise ValueError("vector field must be [nt][2][ny][nx]")
    o = _options(None, **opts)
    outs = o.outputs
    dev = field.device
    if out is None:
        if capacity is None:
            raise ValueError("give capacity or out")
        out = dict(face_id=torch.empty(capacity, dtype=torch.int64, device=dev))
        if outs & OUT_POS:
            out["pos"] = torch.empty((capacity, 3), dtype=torch.float32, device=dev)
        if outs & OUT_MU:
            out["mu"] = torch.empty((capacity, 3), dtype=torch.float32, device=dev)
        if outs & OUT_TYPE:
            out["type"] = torch.empty(capacity, dtype=torch.uint8, device=dev)
        if outs & OUT_FLAGS:
            out["flags"] = torch.empty(capacity, dtype=torch.uint8, device=dev)
        if outs & OUT_LABEL:
            out["label"] = torch.empty(capacity, dtype=torch.int64, device=dev)
    capacity = out["face_id"].numel()
    r = Result()
    for k in ("face_id", "pos", "mu", "type", "flags", "label"):
        t = out.get(k)
        setattr(r, k, t.data_ptr() if t is not None else None)
    st = lib().ftk_track_cp2d_into(ctypes.c_void_p(field.data_ptr()), kind, nx, ny, nt, ctypes.byref(o),
                                   _stream_handle(dev), capacity, ctypes.byref(r))
    if st != 0:
        raise FtkError(st, last_error() + (f" (n_hits {r.n_hits})" if st == 4 else ""))
    nh = int(r.n_hits)

    def view(k, shape):
        t = out.get(k)
        return None if t is None or not getattr(r, k) else t.reshape(-1)[:nh * (shape[1] if len(shape) > 1 else 1)].view(*shape)
    return dict(n=2, n_hits=nh, n_trajectories=int(r.n_trajectories),
                face_id=view("face_id", (nh,)), pos=view("pos", (nh, 3)), mu=view("mu", (nh, 3)),
                type=view("type", (nh,)), flags=view("flags", (nh,)), label=view("label", (nh,)),
                stats={f: getattr(r.stats, f) for f, _ in Stats._fields_ if f != "reserved"})


def track_cp3d(field, **opts):
    """field: contiguous float32 CUDA tensor [nt][nz][ny][nx] (scalar; the gradient is tracked)."""
    if not field.is_contiguous() or field.dtype.itemsize != 4 or not field.is_cuda:
        raise ValueError("field must be a contiguous float32 device tensor")
    nt, nz, ny, nx = field.shape
    pool = _TorchPool(field.device)
    o = _options(pool, **opts)
    r = Result()
    st = lib().ftk_track_cp3d(ctypes.c_void_p(field.data_ptr()), SCALAR, nx, ny, nz, nt, ctypes.byref(o),
                              _stream_handle(field.device), ctypes.byref(r))
    _check(st)
    return _wrap(pool, r)


class Tracker:
    """Streaming form: push one time step at a time, then finish()."""

    def __init__(self, n, dims, kind=SCALAR, device=None, **opts):
        import torch
        self.device = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.pool = _TorchPool(self.device)
        self.opts = _options(self.pool, **opts)
        self.h = ctypes.c_void_p()
        arr = (ctypes.c_int64 * len(dims))(*dims)
        self.stream = _stream_handle(self.device)
        _check(lib().ftk_cp_create(n, arr, kind, ctypes.byref(self.opts), self.stream, ctypes.byref(self.h)))

    def push(self, step):
        if not step.is_contiguous() or not step.is_cuda:
            raise ValueError("step must be a contiguous device tensor")
        _check(lib().ftk_cp_push(self.h, ctypes.c_void_p(step.data_ptr())))

    def finish(self):
        r = Result()
        _check(lib().ftk_cp_finish(self.h, ctypes.byref(r)))
        return _wrap(self.pool, r)

    def close(self):
        if self.h:
            lib().ftk_cp_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def track_cp2d_batched(fields, kind=SCALAR, **opts):
    """fields: list of contiguous float32 device tensors (each as for track_cp2d)."""
    k = len(fields)
    if k == 0:
        return []
    pool = _TorchPool(fields[0].device)
    o = _options(pool, **opts)
    ptrs = (ctypes.c_void_p * k)(*[f.data_ptr() for f in fields])
    nx = (ctypes.c_int64 * k)(*[f.shape[-1] for f in fields])
    ny = (ctypes.c_int64 * k)(*[f.shape[-2] for f in fields])
    nt = (ctypes.c_int64 * k)(*[f.shape[0] for f in fields])
    res = (Result * k)()
    st = lib().ftk_track_cp2d_batched(k, ptrs, nx, ny, nt, kind, ctypes.byref(o), _stream_handle(fields[0].device),
                                      res)
    _check(st)
    return [_wrap(pool, res[i]) for i in range(k)]


# ---------------------------------------------------------------------------------------------------------------
# Trajectory post-processing (slicing at a time step, per-trajectory table, loop filter)
# ---------------------------------------------------------------------------------------------------------------
def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p()


def _device_of(res):
    import torch
    for k in ("face_id", "label", "pos", "type"):
        if res.get(k) is not None:
            return res[k].device
    return torch.device("cuda", torch.cuda.current_device())


def _dims_arg(res, dims_with_t):
    if len(dims_with_t) != res["n"] + 1:
        raise ValueError(f"dims_with_t must have {res['n'] + 1} entries for a {res['n']}D result")
    return (ctypes.c_int64 * len(dims_with_t))(*dims_with_t)


def _as_result(res):
    """Result struct view of a result dict from the tracking calls (device pointers only)."""
    r = Result()
    r.n = res["n"]
    r.n_hits = res["n_hits"]
    r.n_trajectories = res["n_trajectories"]
    for f in ("face_id", "pos", "mu", "type", "flags", "label"):
        setattr(r, f, _ptr(res[f]).value)
    return r


def trajectory_table(res, dims_with_t):
    """Per-trajectory attributes of a tracking result: label (ascending), n_points, t_min, t_max, n_ends."""
    import torch
    dev = _device_of(res)
    pool = _TorchPool(dev)
    o = _options(pool)
    r = _as_result(res)
    arr = _dims_arg(res, dims_with_t)
    t = TrajTable()
    _check(lib().ftk_traj_table_build(ctypes.byref(r), res["n"], arr, ctypes.byref(o), _stream_handle(dev),
                                      ctypes.byref(t)))
    n = int(t.n)
    return dict(n=n, label=pool.take(t.label, torch.int64, (n,)), n_points=pool.take(t.n_points, torch.int64, (n,)),
                t_min=pool.take(t.t_min, torch.float32, (n,)), t_max=pool.take(t.t_max, torch.float32, (n,)),
                n_ends=pool.take(t.n_ends, torch.int32, (n,)))


def slice_at(res, dims_with_t, t0):
    """Indices (ascending) of the critical points at time step t0: punctured ordinal faces anchored at t0."""
    import torch
    dev = _device_of(res)
    pool = _TorchPool(dev)
    o = _options(pool)
    r = _as_result(res)
    arr = _dims_arg(res, dims_with_t)
    p = ctypes.c_void_p()
    cnt = ctypes.c_int64()
    _check(lib().ftk_cp_slice(ctypes.byref(r), res["n"], arr, t0, ctypes.byref(o), _stream_handle(dev),
                              ctypes.byref(p), ctypes.byref(cnt)))
    k = int(cnt.value)
    t = pool.take(p.value, torch.int64, (max(k, 1),))
    return t[:k]


def filter_loops(res, table, min_duration):
    """uint8 keep mask: 0 for the points of closed loops shorter than min_duration (in step units)."""
    import torch
    dev = _device_of(res)
    keep = torch.empty(res["n_hits"], dtype=torch.uint8, device=dev)
    r = _as_result(res)
    t = _table_struct(table)
    _check(lib().ftk_cp_filter_loops(ctypes.byref(r), ctypes.byref(t), float(min_duration), _stream_handle(dev),
                                     _ptr(keep)))
    return keep


def track_iso3d(field, isovalue):
    """Isovolume of f = isovalue in a 3D series: field is a contiguous float32 CUDA tensor [nt][nz][ny][nx].
    Returns crossed edges (edge_id ascending, pos [n][4] as x, y, z, t), labels (smallest edge id of each
    isovolume), n_components and the tessellation tets [m][4] (indices into the hits)."""
    import torch
    if not field.is_contiguous() or field.dtype != torch.float32 or not field.is_cuda or field.dim() != 4:
        raise ValueError("field must be a contiguous 4D float32 device tensor")
    nt, nz, ny, nx = field.shape
    pool = _TorchPool(field.device)
    o = _options(pool)
    r = IsoResult()
    _check(lib().ftk_track_iso3d(ctypes.c_void_p(field.data_ptr()), nx, ny, nz, nt, float(isovalue), ctypes.byref(o),
                                 _stream_handle(field.device), ctypes.byref(r)))
    nh, nt4 = int(r.n_hits), int(r.n_tets)
    return dict(n_hits=nh, n_components=int(r.n_components), n_tets=nt4,
                edge_id=pool.take(r.edge_id, torch.int64, (max(nh, 1),))[:nh],
                pos=pool.take(r.pos, torch.float32, (max(nh, 1), 4))[:nh],
                label=pool.take(r.label, torch.int64, (max(nh, 1),))[:nh],
                tets=pool.take(r.tets, torch.int32, (max(nt4, 1), 4))[:nt4])


def track_vortex3d(psi, **opts):
    """Vortex surfaces of a 3D complex series: psi is a contiguous float32 CUDA tensor [nt][2][nz][ny][nx] (real and
    imaginary planes).  Returns positive triangles (tri_id ascending, pos [n][4] as x, y, z, t), labels (smallest
    triangle id of each surface) and n_components."""
    import torch
    if not psi.is_contiguous() or psi.dtype != torch.float32 or not psi.is_cuda or psi.dim() != 5 or psi.shape[1] != 2:
        raise ValueError("psi must be a contiguous float32 device tensor [nt][2][nz][ny][nx]")
    nt, _, nz, ny, nx = psi.shape
    pool = _TorchPool(psi.device)
    o = _options(pool, **opts)
    r = VortexResult()
    _check(lib().ftk_track_vortex3d(ctypes.c_void_p(psi.data_ptr()), nx, ny, nz, nt, ctypes.byref(o),
                                    _stream_handle(psi.device), ctypes.byref(r)))
    nh = int(r.n_hits)
    return dict(n_hits=nh, n_components=int(r.n_components),
                tri_id=pool.take(r.tri_id, torch.int64, (max(nh, 1),))[:nh],
                pos=pool.take(r.pos, torch.float32, (max(nh, 1), 4))[:nh],
                label=pool.take(r.label, torch.int64, (max(nh, 1),))[:nh])


def track_cp_mesh2d(xy, tri, field, **opts):
    """Critical points of a 2D vector field on a triangle mesh extruded in time: xy float32 [nv][2], tri int32
    [nf][3], field float32 [nt][2][nv], all contiguous CUDA tensors.  Returns punctured faces (face_id ascending, pos
    [n][3] as x, y, t), labels, n_trajectories, faces_per_step and n_edges."""
    import torch
    ok = (xy.is_cuda and tri.is_cuda and field.is_cuda and xy.dtype == torch.float32 and tri.dtype == torch.int32
          and field.dtype == torch.float32 and xy.is_contiguous() and tri.is_contiguous() and field.is_contiguous()
          and xy.dim() == 2 and xy.shape[1] == 2 and tri.dim() == 2 and tri.shape[1] == 3 and field.dim() == 3
          and field.shape[1] == 2 and field.shape[2] == xy.shape[0])
    if not ok:
        raise ValueError("need contiguous CUDA tensors xy float32 [nv][2], tri int32 [nf][3], field float32 [nt][2][nv]")
    pool = _TorchPool(xy.device)
    o = _options(pool, **opts)
    r = MeshResult()
    _check(lib().ftk_track_cp_mesh2d(ctypes.c_void_p(xy.data_ptr()), xy.shape[0], ctypes.c_void_p(tri.data_ptr()),
                                     tri.shape[0], ctypes.c_void_p(field.data_ptr()), field.shape[0], ctypes.byref(o),
                                     _stream_handle(xy.device), ctypes.byref(r)))
    nh = int(r.n_hits)
    return dict(n_hits=nh, n_trajectories=int(r.n_trajectories), faces_per_step=int(r.faces_per_step),
                n_edges=int(r.n_edges), face_id=pool.take(r.face_id, torch.int64, (max(nh, 1),))[:nh],
                pos=pool.take(r.pos, torch.float32, (max(nh, 1), 3))[:nh],
                label=pool.take(r.label, torch.int64, (max(nh, 1),))[:nh])


class Mesh:
    """Mesh handle: the topology of a triangle mesh (xy float32 [nv][2], tri int32 [nf][3], contiguous CUDA
    tensors) built once; track(field) then runs on the device only.  xy is referenced, not copied."""

    def __init__(self, xy, tri):
        import torch
        if not (xy.is_cuda and tri.is_cuda and xy.dtype == torch.float32 and tri.dtype == torch.int32
                and xy.is_contiguous() and tri.is_contiguous() and xy.dim() == 2 and xy.shape[1] == 2
                and tri.dim() == 2 and tri.shape[1] == 3):
            raise ValueError("need contiguous CUDA tensors xy float32 [nv][2] and tri int32 [nf][3]")
        self.xy, self.tri, self.device = xy, tri, xy.device
        self.h = ctypes.c_void_p()
        _check(lib().ftk_mesh_create(ctypes.c_void_p(xy.data_ptr()), xy.shape[0], ctypes.c_void_p(tri.data_ptr()),
                                     tri.shape[0], _stream_handle(xy.device), ctypes.byref(self.h)))

    def track(self, field, **opts):
        """field: contiguous float32 CUDA tensor [nt][2][nv]; returns the same dict as track_cp_mesh2d."""
        import torch
        if not (field.is_cuda and field.dtype == torch.float32 and field.is_contiguous() and field.dim() == 3
                and field.shape[1] == 2 and field.shape[2] == self.xy.shape[0]):
            raise ValueError("field must be a contiguous float32 CUDA tensor [nt][2][nv]")
        pool = _TorchPool(self.device)
        o = _options(pool, **opts)
        r = MeshResult()
        _check(lib().ftk_track_cp_mesh(self.h, ctypes.c_void_p(field.data_ptr()), field.shape[0], ctypes.byref(o),
                                       _stream_handle(self.device), ctypes.byref(r)))
        nh = int(r.n_hits)
        return dict(n_hits=nh, n_trajectories=int(r.n_trajectories), faces_per_step=int(r.faces_per_step),
                    n_edges=int(r.n_edges), face_id=pool.take(r.face_id, torch.int64, (max(nh, 1),))[:nh],
                    pos=pool.take(r.pos, torch.float32, (max(nh, 1), 3))[:nh],
                    label=pool.take(r.label, torch.int64, (max(nh, 1),))[:nh])

    def close(self):
        if self.h:
            lib().ftk_mesh_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def triangle_count(dims_with_t):
    """Spacetime triangles tested for a 3D grid (nx, ny, nz, nt)."""
    arr = (ctypes.c_int64 * 4)(*dims_with_t)
    return int(lib().ftk_triangle_count(arr))


def edge_count(dims_with_t):
    """Spacetime edges tested for a 3D grid (nx, ny, nz, nt)."""
    arr = (ctypes.c_int64 * 4)(*dims_with_t)
    return int(lib().ftk_edge_count(arr))


def _table_struct(table):
    t = TrajTable()
    t.n = table["n"]
    for f in ("label", "n_points", "t_min", "t_max", "n_ends"):
        setattr(t, f, _ptr(table[f]).value)
    return t


def trajectory_order(res, dims_with_t, table):
    """(order, offsets): hit indices grouped by trajectory (table order), each in curve order; offsets[j] is the
    start of trajectory j in order, offsets[-1] = n_hits."""
    import torch
    dev = _device_of(res)
    pool = _TorchPool(dev)
    o = _options(pool)
    r = _as_result(res)
    arr = _dims_arg(res, dims_with_t)
    t = _table_struct(table)
    order = torch.empty(max(res["n_hits"], 1), dtype=torch.int64, device=dev)
    offsets = torch.empty(table["n"] + 1, dtype=torch.int64, device=dev)
    _check(lib().ftk_traj_order(ctypes.byref(r), res["n"], arr, ctypes.byref(t), ctypes.byref(o),
                                _stream_handle(dev), _ptr(order), _ptr(offsets)))
    return order[:res["n_hits"]], offsets


def _walk_types(fn, res, table, order, offsets, arg, types):
    import torch
    dev = _device_of(res)
    pool = _TorchPool(dev)
    o = _options(pool)
    r = _as_result(res)
    t = _table_struct(table)
    tin = res["type"] if types is None else types
    if tin is None:
        raise ValueError("the result carries no types; pass types")
    if tin.dtype != torch.uint8 or tin.numel() != res["n_hits"] or not tin.is_contiguous():
        raise ValueError("types must be a contiguous uint8 tensor of n_hits entries")
    tout = torch.empty(max(res["n_hits"], 1), dtype=torch.uint8, device=dev)
    _check(fn(ctypes.byref(r), ctypes.byref(t), _ptr(order), _ptr(offsets), _ptr(tin), arg, ctypes.byref(o),
              _stream_handle(dev), _ptr(tout)))
    return tout[:res["n_hits"]]


def smooth_types(res, table, order, offsets, half_window=2, types=None):
    """Window-shifting type smoothing along the trajectories (types default to the result's)."""
    return _walk_types(lib().ftk_traj_smooth_types, res, table, order, offsets, int(half_window), types)


def simplify_types(res, table, order, offsets, min_persistence, types=None):
    """Run simplification: short runs of one type between two persistent runs of another take their type."""
    return _walk_types(lib().ftk_traj_simplify_types, res, table, order, offsets, float(min_persistence), types)


def autotune_cp2d(field, kind=SCALAR):
    """Time the detection tilings on this field; returns (tile_y, slab_depth), also remembered for the shape."""
    if not field.is_contiguous() or field.dtype.itemsize != 4 or not field.is_cuda:
        raise ValueError("field must be a contiguous float32 device tensor")
    nt, ny, nx = (field.shape[0], field.shape[-2], field.shape[-1])
    o = _options(None)
    t = Options()
    _check(lib().ftk_autotune_cp2d(ctypes.c_void_p(field.data_ptr()), kind, nx, ny, nt, ctypes.byref(o),
                                   _stream_handle(field.device), ctypes.byref(t)))
    return int(t.tile_y), int(t.slab_depth)
