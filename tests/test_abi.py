"""The C ABI library loads and exports every symbol include/ftk.h declares; host-side argument checks (no GPU
compute is launched by these tests)."""
import ctypes
import os
import re

import pytest

import paper_2011_08697_amd as F
from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "ftk.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(ftk_[a-z0-9_]+)\s*\(", text)
    return sorted(set(n for n in names if not n.endswith("_fn")))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 12
    L = F.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(F.EXPORTS)


def test_version_and_defaults():
    L = F.lib()
    assert b"gfx950" in L.ftk_version()
    o = F.Options()
    L.ftk_default_options(ctypes.byref(o))
    assert o.quant_log2 == 20 and o.precision == 0 and o.outputs == 29


@pytest.mark.parametrize("n,dims", [(2, (64, 64, 10)), (2, (1024, 1024, 100)), (2, (4096, 4096, 50)),
                                    (3, (256, 256, 256, 16)), (2, (5, 3, 2)), (3, (2, 3, 4, 5))])
def test_simplex_count_matches_oracle(n, dims):
    assert F.simplex_count(n, dims) == O.simplex_count(n, dims)


def test_simplex_count_rejects_bad_dims():
    assert F.simplex_count(2, (1, 5, 5)) == -1
    assert F.simplex_count(4, (5, 5, 5, 5, 5)) == -1


def _call2d(field_ptr, kind, nx, ny, nt, opt=None):
    L = F.lib()
    r = F.Result()
    st = L.ftk_track_cp2d(field_ptr, kind, nx, ny, nt, ctypes.byref(opt) if opt else None, None, ctypes.byref(r))
    return st, r


def test_argument_errors_are_reported_before_any_device_work():
    # null field, bad kind, too-small dims and bad options are rejected on the host
    st, _ = _call2d(None, 0, 8, 8, 4)
    assert st == 1 and "NULL" in F.last_error()
    st, _ = _call2d(ctypes.c_void_p(16), 5, 8, 8, 4)
    assert st == 1
    st, _ = _call2d(ctypes.c_void_p(16), 0, 1, 8, 4)
    assert st == 1 and ">= 2" in F.last_error()
    o = F.Options()
    F.lib().ftk_default_options(ctypes.byref(o))
    o.quant_log2 = 70
    st, _ = _call2d(ctypes.c_void_p(16), 0, 8, 8, 4, o)
    assert st == 1 and "quant_log2" in F.last_error()
    o.quant_log2 = 20
    o.tile_y = 7
    st, _ = _call2d(ctypes.c_void_p(16), 0, 8, 8, 4, o)
    assert st == 1


def test_result_free_of_empty_result_is_safe():
    r = F.Result()
    F.lib().ftk_result_free(ctypes.byref(r), None, None)


def _brute_count(dims, types):
    """Anchors whose whole simplex lies in the grid, summed over the types (direct enumeration)."""
    import itertools
    tot = 0
    for masks in types:
        used = 0
        for m in masks:
            used |= int(m)
        for c in itertools.product(*[range(d) for d in dims]):
            tot += all(c[a] + ((used >> a) & 1) < dims[a] for a in range(len(dims)))
    return tot


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (3, 4, 2, 5), (5, 3, 3, 2)])
def test_edge_and_triangle_counts(dims):
    arr = (ctypes.c_int64 * 4)(*dims)
    L = F.lib()
    assert L.ftk_edge_count(arr) == _brute_count(dims, [[m] for m in range(1, 16)])
    assert L.ftk_triangle_count(arr) == _brute_count(dims, O.kuhn_types(4, 2))
    bad = (ctypes.c_int64 * 4)(1, 3, 3, 3)
    assert L.ftk_edge_count(bad) == -1 and L.ftk_triangle_count(bad) == -1


def test_iso_and_vortex_argument_errors():
    """Host-side checks return before any device work: missing pointers, small or oversized grids."""
    L = F.lib()
    o = F.Options()
    L.ftk_default_options(ctypes.byref(o))
    ir = F.IsoResult()
    vr = F.VortexResult()
    dummy = ctypes.c_void_p(1)
    assert L.ftk_track_iso3d(None, 4, 4, 4, 4, 0.0, ctypes.byref(o), None, ctypes.byref(ir)) != 0
    assert L.ftk_track_iso3d(dummy, 1, 4, 4, 4, 0.0, ctypes.byref(o), None, ctypes.byref(ir)) != 0
    assert L.ftk_track_iso3d(dummy, 4, 70000, 4, 4, 0.0, ctypes.byref(o), None, ctypes.byref(ir)) != 0
    assert L.ftk_track_iso3d(dummy, 4, 4, 4, 4, float("nan"), ctypes.byref(o), None, ctypes.byref(ir)) != 0
    assert L.ftk_track_vortex3d(None, 4, 4, 4, 4, ctypes.byref(o), None, ctypes.byref(vr)) != 0
    assert L.ftk_track_vortex3d(dummy, 4, 4, 300, 300, ctypes.byref(o), None, ctypes.byref(vr)) != 0
    assert b"dimension" in L.ftk_last_error() or b"large" in L.ftk_last_error()


def test_refusing_allocator_reports_oom_before_device_work():
    """Scratch comes from the caller's allocator hooks when given: a refusal of the first request is FTK_ERR_OOM,
    returned before anything reaches the device (no GPU is needed for this)."""
    calls = []

    def alloc(nbytes, stream, ctx):
        calls.append(nbytes)
        return None

    def free(ptr, stream, ctx):
        calls.append(-1)

    a, f = F._ALLOC_FN(alloc), F._FREE_FN(free)
    o = F.Options()
    F.lib().ftk_default_options(ctypes.byref(o))
    o.alloc, o.free = a, f
    st, r = _call2d(ctypes.c_void_p(256), 0, 64, 64, 10, o)
    assert st == 5, F.last_error()
    assert len(calls) == 1 and calls[0] >= 64 * 64 * 10 * 2
    assert r.n_hits == 0 and not r.face_id


def test_no_alloc_entry_point_argument_errors():
    """ftk_track_cp2d_into rejects bad arguments on the host, before it looks up its scratch region."""
    L = F.lib()
    r = F.Result()
    st = L.ftk_track_cp2d_into(None, 0, 8, 8, 4, None, None, 10, ctypes.byref(r))
    assert st == 1 and "field" in F.last_error()
    st = L.ftk_track_cp2d_into(ctypes.c_void_p(256), 0, 8, 8, 4, None, None, 10, None)
    assert st == 1 and "io" in F.last_error()
    st = L.ftk_track_cp2d_into(ctypes.c_void_p(256), 0, 8, 8, 4, None, None, -1, ctypes.byref(r))
    assert st == 1 and "capacity" in F.last_error()
    st = L.ftk_track_cp2d_into(ctypes.c_void_p(256), 0, 8, 8, 4, None, None, 10, ctypes.byref(r))
    assert st == 1 and "output array" in F.last_error()  # default outputs need face_id, pos, type, flags, label
    assert r.n_hits == 0 and not r.face_id
