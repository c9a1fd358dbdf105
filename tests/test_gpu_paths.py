"""GPU tests of paths that realistic inputs rarely reach: the emission's workgroup-local capacity overflows (global
link list only for a crowded tile step, link stage overflow), invariant errors reaching the caller through every
form, the 128-bit path through the streaming and batched forms, and allocator refusals."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_08697_amd import synth
from tests.parity import assert_full_parity, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2011_08697_amd as F  # noqa: E402

DEV = torch.device("cuda", 0)
SMALL_LDS, INVARIANT = 1, 2
KEYS = ("face_id", "pos", "type", "flags", "label")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def stream(field, kind=0, **kw):
    f = dev(field)
    dims = [field.shape[-1], field.shape[-2]]
    tr = F.Tracker(2, dims, kind=kind, **kw)
    try:
        for t in range(field.shape[0]):
            tr.push(f[t].contiguous())
        return tr.finish()
    finally:
        tr.close()


def same(a, b):
    a, b = to_np(a), to_np(b)
    assert a["n_hits"] == b["n_hits"] and a["n_trajectories"] == b["n_trajectories"]
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k


FIELDS = {
    # dense: about 1.8 hits per vertex, every tile step beyond the small capacity (global-list-only steps)
    "noise": lambda: (synth.moving_gaussians_2d(200, 150, 12, 12, seed=1, noise_std=1e-3), 0),
    # sparse: chunks of many steps with time links attached at flush, stage overflowing to the list
    "blobs": lambda: (synth.moving_gaussians_2d(300, 200, 20, 24, seed=3), 0),
    # degenerate: ties everywhere
    "levels": lambda: (synth.quantise_levels(synth.moving_gaussians_2d(257, 131, 9, 16, seed=1, noise_std=1e-3)), 0),
    "vector": lambda: (synth.vortex_sources_2d(300, 220, 6, 24, seed=4), 1),
}


@pytest.mark.parametrize("name", sorted(FIELDS))
def test_small_local_capacities_keep_parity(name):
    f, kind = FIELDS[name]()
    ref = O.track(f, n=2, kind=kind)
    g = F.track_cp2d(dev(f), kind=kind, debug=SMALL_LDS)
    assert_full_parity(g, ref)
    same(g, F.track_cp2d(dev(f), kind=kind))


def test_small_local_capacities_streaming_and_batched():
    xs = [FIELDS["noise"]()[0], FIELDS["blobs"]()[0]]
    one = [F.track_cp2d(dev(x)) for x in xs]
    for x, r in zip(xs, one):
        same(stream(x, debug=SMALL_LDS), r)
    for r, ref in zip(F.track_cp2d_batched([dev(x) for x in xs], debug=SMALL_LDS), one):
        same(r, ref)


def test_invariant_error_reaches_the_caller_in_every_form():
    f = synth.moving_gaussians_2d(130, 70, 9, 10, seed=2, noise_std=1e-3)
    opt = INVARIANT | (4 << 8)  # report a bad cell at step 4
    with pytest.raises(F.FtkError) as e:
        F.track_cp2d(dev(f), debug=opt)
    assert e.value.status == 7
    with pytest.raises(F.FtkError) as e:
        stream(f, debug=opt)  # the error of step 4's emission (during the push of step 6) is reported at finish
    assert e.value.status == 7
    with pytest.raises(F.FtkError) as e:
        F.track_cp2d_batched([dev(f), dev(f[:6])], debug=opt)
    assert e.value.status == 7
    # a step beyond the series: no report
    assert_full_parity(F.track_cp2d(dev(f), debug=INVARIANT | (50 << 8)), O.track(f))


def wide_field(seed, shape=(4, 2, 20, 70)):
    rng = np.random.default_rng(seed)
    return (rng.integers(-3, 4, size=shape) * 2.0 ** 12).astype(np.float32)  # |q| up to 3 * 2^32


def test_wide_path_streaming_and_batched():
    u = wide_field(11)
    ref = O.track(u, n=2, kind=1)
    s = stream(u, kind=1)
    assert s["stats"]["wide_path"] == 1
    assert_full_parity(s, ref)
    narrow = synth.vortex_sources_2d(90, 70, 5, 6, seed=4)
    u2 = wide_field(12, (6, 2, 33, 41))
    res = F.track_cp2d_batched([dev(narrow), dev(u), dev(u2)], kind=1)
    assert_full_parity(res[0], O.track(narrow, n=2, kind=1))
    assert_full_parity(res[1], ref)
    assert_full_parity(res[2], O.track(u2, n=2, kind=1))


class RefusingPool(F._TorchPool):
    """torch-backed allocator hooks that refuse the k-th request and every later one."""

    def __init__(self, device, refuse_from):
        super().__init__(device)
        self.refuse_from = refuse_from
        self.calls = 0

    def alloc(self, nbytes, stream, ctx):
        self.calls += 1
        if self.calls >= self.refuse_from:
            return None
        return super().alloc(nbytes, stream, ctx)


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_refusing_allocator_gives_oom_and_releases_everything(k):
    """Scratch and outputs both come from the caller's hooks: a refusal anywhere gives FTK_ERR_OOM and every block
    taken so far is handed back."""
    f = dev(synth.make("blobs64"))
    pool = RefusingPool(DEV, k)
    o = F._options(pool)
    r = F.Result()
    nt, ny, nx = f.shape
    st = F.lib().ftk_track_cp2d(ctypes.c_void_p(f.data_ptr()), 0, nx, ny, nt, ctypes.byref(o),
                                F._stream_handle(DEV), ctypes.byref(r))
    torch.cuda.synchronize()
    assert st == 5, F.last_error()
    assert r.n_hits == 0 and not r.face_id
    assert pool.live == {}


TILED, SPARSE = 4, 8  # FTK_DEBUG_TILED_EMIT, FTK_DEBUG_SPARSE_EMIT


@pytest.mark.parametrize("name", sorted(FIELDS))
def test_emission_forms_are_identical(name):
    """The sparse emission (a wavefront per non-empty row segment, every link through the global list) and the tiled
    one give the same outputs bit for bit on dense, sparse, degenerate and vector fields, and both equal the
    oracle."""
    f, kind = FIELDS[name]()
    tiled = F.track_cp2d(dev(f), kind=kind, debug=TILED)
    sparse = F.track_cp2d(dev(f), kind=kind, debug=SPARSE)
    same(sparse, tiled)
    assert_full_parity(sparse, O.track(f, n=2, kind=kind))


def test_sparse_emission_wide_path_batched_and_invariant():
    u = wide_field(11)
    r = F.track_cp2d(dev(u), kind=1, debug=SPARSE)
    assert r["stats"]["wide_path"] == 1
    assert_full_parity(r, O.track(u, n=2, kind=1))
    # batched: every series in one form, or the per-series default (a dense and two sparse series)
    xs = [FIELDS["noise"]()[0], FIELDS["blobs"]()[0], synth.moving_gaussians_2d(70, 333, 7, 5, seed=9)]
    one = [F.track_cp2d(dev(x)) for x in xs]
    for dbg in (TILED, SPARSE, 0):
        for r, ref in zip(F.track_cp2d_batched([dev(x) for x in xs], debug=dbg), one):
            same(r, ref)
    f = synth.moving_gaussians_2d(130, 70, 9, 10, seed=2, noise_std=1e-3)
    opt = SPARSE | INVARIANT | (4 << 8)
    with pytest.raises(F.FtkError) as e:
        F.track_cp2d(dev(f), debug=opt)
    assert e.value.status == 7
    with pytest.raises(F.FtkError) as e:
        F.track_cp2d_batched([dev(f), dev(f[:6])], debug=opt)
    assert e.value.status == 7
