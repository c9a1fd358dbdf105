"""GPU parity of critical-point tracking on extruded triangle meshes (ftk_track_cp_mesh2d through the C ABI) against
the oracle (oracle/mesh.py): face ids, labels and trajectory counts bit-exact, points within 1e-5 relative; errors;
and a sampled check of a large Delaunay mesh against the oracle's per-face predicate."""
import numpy as np
import pytest

from oracle import mesh as M
from oracle import oracle as O
from paper_2011_08697_amd import synth
from parity import assert_pos_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2011_08697_amd as F  # noqa: E402

DEV = torch.device("cuda", 0)


def _run(xy, tri, field, **kw):
    g = F.track_cp_mesh2d(torch.from_numpy(np.ascontiguousarray(xy, np.float32)).to(DEV),
                          torch.from_numpy(np.ascontiguousarray(tri, np.int32)).to(DEV),
                          torch.from_numpy(np.ascontiguousarray(field, np.float32)).to(DEV), **kw)
    torch.cuda.synchronize()
    return g


def _swirl(xy, nt, seed):
    """Sum of a few moving source/vortex terms sampled at the vertices."""
    rng = np.random.default_rng(seed)
    f = np.zeros((nt, 2, len(xy)), np.float64)
    for _ in range(4):
        c = rng.uniform(2, 8, 2)
        v = rng.uniform(-0.5, 0.5, 2)
        rot = rng.uniform(0, np.pi)
        for t in range(nt):
            d = xy - (c + v * t)
            w = np.exp(-(d ** 2).sum(1) / 6.0)
            f[t, 0] += w * (np.cos(rot) * d[:, 0] - np.sin(rot) * d[:, 1])
            f[t, 1] += w * (np.sin(rot) * d[:, 0] + np.cos(rot) * d[:, 1])
    return f.astype(np.float32)


def _cases():
    xy_k, tri_k = synth.kuhn_grid_mesh(9, 7)
    xy_d, tri_d = synth.delaunay_mesh(60, seed=3)
    rng = np.random.default_rng(1)
    return {
        "kuhn_tied": (xy_k, tri_k, rng.integers(-2, 3, size=(5, 2, len(xy_k))).astype(np.float32) / 2 ** 20),
        "delaunay_tied": (xy_d, tri_d, rng.integers(-1, 2, size=(4, 2, len(xy_d))).astype(np.float32) / 2 ** 20),
        "delaunay_swirl": (xy_d, tri_d, _swirl(xy_d.astype(np.float64), 6, 2)),
        "delaunay_shuffled_rows": (xy_d, tri_d[:, ::-1].copy(), _swirl(xy_d.astype(np.float64), 4, 5)),
    }


@pytest.mark.parametrize("case", ["kuhn_tied", "delaunay_tied", "delaunay_swirl", "delaunay_shuffled_rows"])
def test_matches_oracle(case):
    xy, tri, field = _cases()[case]
    g = _run(xy, tri, field)
    o = M.track_cp_mesh(xy, tri, field)
    assert g["n_hits"] == o.n_hits and g["n_trajectories"] == o.n_traj
    assert g["faces_per_step"] == o.S and g["n_edges"] == o.ne
    assert np.array_equal(g["face_id"].cpu().numpy(), o.face_id)
    assert np.array_equal(g["label"].cpu().numpy(), o.label)
    assert_pos_close(g["pos"].cpu().numpy(), o.pos)


def test_edge_of_three_triangles_matches_oracle():
    """A mesh with an edge shared by three triangles (one more triangle on an interior edge of a grid mesh): the
    unions then visit every prism instead of starting from the hits; results equal the oracle's."""
    xy, tri = synth.kuhn_grid_mesh(9, 7)
    a, b = (int(v) for v in sorted(tri[len(tri) // 2][:2]))
    xy = np.concatenate([xy, (0.5 * (xy[a] + xy[b]) + np.array([0.13, 0.29], np.float32))[None]]).astype(np.float32)
    tri = np.concatenate([tri, np.array([[a, b, len(xy) - 1]], np.int32)])
    edges = np.sort(np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [0, 2]]]), axis=1)
    _, counts = np.unique(edges, axis=0, return_counts=True)
    assert counts.max() == 3
    rng = np.random.default_rng(4)
    for field in (rng.integers(-2, 3, size=(5, 2, len(xy))).astype(np.float32) / 2 ** 20,
                  _swirl(xy.astype(np.float64), 5, 7)):
        g = _run(xy, tri, field)
        o = M.track_cp_mesh(xy, tri, field)
        assert g["n_hits"] == o.n_hits and g["n_trajectories"] == o.n_traj
        assert np.array_equal(g["face_id"].cpu().numpy(), o.face_id)
        assert np.array_equal(g["label"].cpu().numpy(), o.label)
        assert_pos_close(g["pos"].cpu().numpy(), o.pos)


def test_errors():
    xy, tri = synth.delaunay_mesh(20, seed=1)
    field = np.zeros((3, 2, len(xy)), np.float32)
    bad = tri.copy()
    bad[0, 0] = len(xy)
    with pytest.raises(F.FtkError):
        _run(xy, bad, field)
    bad = tri.copy()
    bad[1, 1] = bad[1, 0]
    with pytest.raises(F.FtkError):
        _run(xy, bad, field)
    f2 = field.copy()
    f2[1, 0, 3] = np.inf
    with pytest.raises(F.FtkError):
        _run(xy, tri, f2)
    g = _run(xy, tri, np.ones((3, 2, len(xy)), np.float32))
    assert g["n_hits"] == 0 and g["n_trajectories"] == 0


def test_large_delaunay_mesh_sampled():
    """200,000-point Delaunay mesh over 12 steps: ids ascending; sampled punctured faces re-tested with the oracle's
    predicate on the host-quantised vectors and their points against the exact barycentric formula."""
    xy, tri = synth.delaunay_mesh(200000, extent=100.0, seed=9)
    nt = 12
    field = _swirl(xy.astype(np.float64) / 10.0, nt, 7)
    g = _run(xy, tri, field)
    nh = g["n_hits"]
    assert nh > 100
    fid = g["face_id"].cpu().numpy()
    assert np.all(fid[1:] > fid[:-1])
    trs = np.sort(tri.astype(np.int64), axis=1)
    edges = M.mesh_edges(tri)
    nf, ne, S = len(trs), len(edges), g["faces_per_step"]
    assert S == 3 * nf + 2 * ne
    q = np.rint(field * np.float32(2 ** 20)).astype(np.int64)
    rng = np.random.default_rng(0)
    pos = g["pos"].cpu().numpy()
    for k in rng.integers(0, nh, size=min(nh, 1500)):
        t, loc = divmod(int(fid[k]), S)
        if loc < nf:
            vs = [(trs[loc][0], t), (trs[loc][1], t), (trs[loc][2], t)]
        elif loc < nf + 2 * ne:
            E, up = divmod(loc - nf, 2)
            a, b = edges[E]
            vs = [(a, t), (a, t + 1), (b, t + 1)] if up else [(a, t), (b, t), (b, t + 1)]
        else:
            T, up = divmod(loc - nf - 2 * ne, 2)
            a = trs[T]
            vs = [(a[0], t), (a[1], t + 1), (a[2], t + 1)] if up else [(a[0], t), (a[1], t), (a[2], t + 1)]
        V = np.array([[q[tt, 0, v], q[tt, 1, v]] for v, tt in vs])
        assert O.face_punctured(V)
        d = lambda A, B: int(A[0]) * int(B[1]) - int(A[1]) * int(B[0])
        C = [d(V[1], V[2]), -d(V[0], V[2]), d(V[0], V[1])]
        D = sum(C)
        mu = [1 / 3] * 3 if D == 0 else [c / D for c in C]
        want = sum(m * np.array([xy[v, 0], xy[v, 1], tt], float) for m, (v, tt) in zip(mu, vs))
        assert_pos_close(pos[k:k + 1], want[None, :])


def test_mesh_handle_tracks_several_fields():
    """One mesh handle, two fields: each result equals the one-shot call."""
    import ctypes
    xy, tri = synth.delaunay_mesh(80, seed=4)
    dxy = torch.from_numpy(np.ascontiguousarray(xy)).to(DEV)
    dtri = torch.from_numpy(np.ascontiguousarray(tri, np.int32)).to(DEV)
    L = F.lib()
    sh = F._stream_handle(DEV)
    mesh = ctypes.c_void_p()
    assert L.ftk_mesh_create(ctypes.c_void_p(dxy.data_ptr()), len(xy), ctypes.c_void_p(dtri.data_ptr()), len(tri), sh,
                             ctypes.byref(mesh)) == 0
    try:
        for seed in (1, 2):
            field = _swirl(xy.astype(np.float64), 5, seed)
            df = torch.from_numpy(field).to(DEV)
            pool = F._TorchPool(DEV)
            o = F._options(pool)
            r = F.MeshResult()
            assert L.ftk_track_cp_mesh(mesh, ctypes.c_void_p(df.data_ptr()), 5, ctypes.byref(o), sh,
                                       ctypes.byref(r)) == 0
            nh = int(r.n_hits)
            fid = pool.take(r.face_id, torch.int64, (max(nh, 1),))[:nh].cpu().numpy()
            lab = pool.take(r.label, torch.int64, (max(nh, 1),))[:nh].cpu().numpy()
            g = _run(xy, tri, field)
            assert nh == g["n_hits"] and int(r.n_trajectories) == g["n_trajectories"]
            assert np.array_equal(fid, g["face_id"].cpu().numpy())
            assert np.array_equal(lab, g["label"].cpu().numpy())
    finally:
        L.ftk_mesh_destroy(mesh)


def test_mesh_class_binding():
    xy, tri = synth.delaunay_mesh(50, seed=6)
    m = F.Mesh(torch.from_numpy(xy).to(DEV), torch.from_numpy(np.ascontiguousarray(tri, np.int32)).to(DEV))
    field = _swirl(xy.astype(np.float64), 4, 3)
    g = m.track(torch.from_numpy(field).to(DEV))
    o = M.track_cp_mesh(xy, tri, field)
    assert np.array_equal(g["face_id"].cpu().numpy(), o.face_id)
    assert np.array_equal(g["label"].cpu().numpy(), o.label)
    m.close()
