"""GPU parity of isovolume tracking (ftk_track_iso3d through the C ABI) against the oracle (oracle/iso.py): crossed
edge ids, labels, component counts and tetrahedra bit-exact, intersection points within 1e-5 relative; plus
errors, the empty case and sampled properties of the full 256^3 x 16 blob series."""
import ctypes

import numpy as np
import pytest

from oracle import iso as I
from paper_2011_08697_amd import synth
from parity import assert_pos_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2011_08697_amd as F  # noqa: E402

DEV = torch.device("cuda", 0)


def _linear(nx, ny, nz, nt, fn):
    X, Y, Z, T = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64),
                             np.arange(nz, dtype=np.float64), np.arange(nt, dtype=np.float64), indexing="ij")
    return np.transpose(fn(X, Y, Z, T), (3, 2, 1, 0)).astype(np.float32)


def _run(f, c):
    g = F.track_iso3d(torch.from_numpy(np.ascontiguousarray(f)).to(DEV), c)
    torch.cuda.synchronize()
    return g


def _check(g, o):
    assert g["n_hits"] == o.n_hits
    assert g["n_components"] == o.n_components
    assert np.array_equal(g["edge_id"].cpu().numpy(), o.edge_id)
    assert np.array_equal(g["label"].cpu().numpy(), o.label)
    assert_pos_close(g["pos"].cpu().numpy(), o.pos)
    assert g["n_tets"] == len(o.tets)
    assert np.array_equal(g["tets"].cpu().numpy(), o.tets)


CASES = {
    "moving_plane": lambda: (_linear(21, 21, 21, 12, lambda X, Y, Z, T: X - 0.9 * T), 0.0),
    "diagonal": lambda: (_linear(9, 9, 9, 4, lambda X, Y, Z, T: X + Y - 8.0), 0.0),
    "tied_0": lambda: (np.random.default_rng(0).integers(-1, 2, size=(4, 4, 5, 5)).astype(np.float32), 0.0),
    "tied_1": lambda: (np.random.default_rng(1).integers(-1, 2, size=(3, 5, 4, 6)).astype(np.float32), 0.0),
    "blobs": lambda: (synth.moving_gaussians_3d(24, 20, 18, 4, 6, seed=2), 0.3),
    "blobs_ragged": lambda: (synth.moving_gaussians_3d(131, 7, 5, 3, 4, seed=5), 0.2),
}


@pytest.mark.parametrize("case", list(CASES))
def test_matches_oracle(case):
    f, c = CASES[case]()
    _check(_run(f, c), I.track_iso(f, c))


def test_edge_count_and_empty():
    assert F.edge_count((5, 6, 7, 8)) == sum(
        np.prod([d - ((M >> a) & 1) for a, d in enumerate((5, 6, 7, 8))]) for M in range(1, 16))
    g = _run(np.ones((3, 4, 5, 6), np.float32), 0.5)
    assert g["n_hits"] == 0 and g["n_tets"] == 0 and g["n_components"] == 0


def test_errors():
    f = np.ones((3, 4, 5, 6), np.float32)
    f[1, 2, 3, 4] = np.nan
    with pytest.raises(F.FtkError):
        _run(f, 0.5)
    with pytest.raises(F.FtkError):
        _run(np.ones((1, 4, 5, 6), np.float32), 0.5)  # nt < 2
    with pytest.raises(F.FtkError):
        _run(np.ones((3, 4, 5, 6), np.float32), float("inf"))


def test_full_size_blobs3d256_sampled():
    """The 256^3 x 16 blob series at isovalue 0.5: sampled crossed edges checked against the field on the host
    (exact side tests, binary64 intersection points), ascending edge ids, and sampled tetrahedra whose four edges
    lie in one unit 4-cube."""
    t = torch.from_numpy(synth.make("blobs3d256", device=DEV)).to(DEV)
    g = F.track_iso3d(t, 0.5)
    torch.cuda.synchronize()
    f = t.cpu().numpy()
    del t
    nt, nz, ny, nx = f.shape
    nh = g["n_hits"]
    assert nh > 1000 and g["n_tets"] > nh
    eid = g["edge_id"]
    assert bool((eid[1:] > eid[:-1]).all())
    rng = np.random.default_rng(3)
    ks = rng.integers(0, nh, size=4000)
    e = eid[ks].cpu().numpy()
    pos = g["pos"][ks].cpu().numpy()
    c = np.float32(0.5)
    M = e % 15 + 1
    gv = e // 15
    x, y, z, tt = gv % nx, (gv // nx) % ny, (gv // (nx * ny)) % nz, gv // (nx * ny * nz)
    d = np.stack([(M >> a) & 1 for a in range(4)], 1)
    fa = f[tt, z, y, x]
    fb = f[tt + d[:, 3], z + d[:, 2], y + d[:, 1], x + d[:, 0]]
    assert np.all((fa >= c) != (fb >= c))
    mu = (np.float64(c) - fa.astype(np.float64)) / (fb.astype(np.float64) - fa.astype(np.float64))
    want = np.stack([x, y, z, tt], 1) + mu[:, None] * d
    assert_pos_close(pos, want)
    tk = rng.integers(0, g["n_tets"], size=2000)
    te = eid[g["tets"][tk].reshape(-1)].cpu().numpy().reshape(-1, 4)
    for row in te:
        gv = row // 15
        Mr = row % 15 + 1
        pts = []
        for gg, mm in zip(gv, Mr):
            a = np.array([gg % nx, (gg // nx) % ny, (gg // (nx * ny)) % nz, gg // (nx * ny * nz)])
            pts += [a, a + np.array([(mm >> b) & 1 for b in range(4)])]
        pts = np.array(pts)
        assert np.all(pts.max(0) - pts.min(0) <= 1)


class _ShiftPool(F._TorchPool):
    """torch-backed hooks that record the size of every request and hand out request number `shift` (if any) 4 bytes
    past a 16-byte boundary."""

    def __init__(self, device, shift=None):
        super().__init__(device)
        self.sizes = []
        self.shift = shift
        self.shifted = {}

    def alloc(self, nbytes, stream, ctx):
        self.sizes.append(int(nbytes))
        if len(self.sizes) - 1 != self.shift:
            return super().alloc(nbytes, stream, ctx)
        p = super().alloc(nbytes + 16, stream, ctx)
        if p is None:
            return None
        self.shifted[p + 4] = p
        return p + 4

    def free(self, ptr, stream, ctx):
        super().free(self.shifted.pop(ptr, ptr), stream, ctx)


def _iso_call(f, c, pool):
    nt, nz, ny, nx = f.shape
    o = F._options(pool)
    r = F.IsoResult()
    st = F.lib().ftk_track_iso3d(ctypes.c_void_p(f.data_ptr()), nx, ny, nz, nt, ctypes.c_float(c), ctypes.byref(o),
                                 F._stream_handle(DEV), ctypes.byref(r))
    torch.cuda.synchronize()
    return st, r, o


def test_misaligned_tetrahedron_array_is_refused():
    """Tetrahedra are written with 16-byte stores: an allocator that returns a misaligned tetrahedron array gets
    FTK_ERR_ARG before any kernel runs on it, and every block is handed back.  The tetrahedron request is found in
    a first call's request sequence as the last of the four consecutive output requests (edge ids, positions,
    labels, tetrahedra); only that request is shifted in the second call."""
    f = torch.from_numpy(np.ascontiguousarray(
        _linear(12, 11, 10, 3, lambda X, Y, Z, T: np.sin(0.7 * X) + np.cos(0.5 * Y) * np.sin(0.3 * Z + 0.4 * T)))
    ).to(DEV)
    rec = _ShiftPool(DEV)
    st, r, o = _iso_call(f, 0.1, rec)
    assert st == 0, F.last_error()
    nh, ntets = int(r.n_hits), int(r.n_tets)
    assert nh > 0 and ntets > 0
    F.lib().ftk_iso_result_free(ctypes.byref(r), ctypes.byref(o), F._stream_handle(DEV))
    torch.cuda.synchronize()
    up = lambda b: (b + 255) & ~255  # noqa: E731
    outs = [up(8 * nh), up(16 * nh), up(8 * nh), up(16 * ntets)]
    idx = [i for i in range(3, len(rec.sizes)) if rec.sizes[i - 3:i + 1] == outs]
    assert len(idx) == 1, rec.sizes
    pool = _ShiftPool(DEV, shift=idx[0])
    st, r, _ = _iso_call(f, 0.1, pool)
    assert st == 1, F.last_error()
    assert "16 bytes" in F.last_error()
    assert pool.sizes == rec.sizes[:len(pool.sizes)] and len(pool.sizes) > idx[0]
    assert pool.shifted == {} and pool.live == {}
