"""Pins of the prismatic-mesh oracle (oracle/mesh.py): on a Kuhn-triangulated grid the staircase extrusion is the
regular spacetime mesh with the same vertex order, so the result must equal the regular-grid oracle (punctured
faces as vertex sets, points, trajectories); on random Delaunay meshes every tetrahedron has 0 or 2 punctured faces,
and a linear field with a moving zero gives one trajectory on the line with one punctured triangle per step."""
import numpy as np
import pytest

from oracle import mesh as M
from oracle import oracle as O
from paper_2011_08697_amd import synth


def _face_vertices(r, fid, nv, tri, edges):
    t, loc = divmod(int(fid), r.S)
    nf, ne = r.nf, r.ne
    if loc < nf:
        a = tri[loc]
        return {(a[0], t), (a[1], t), (a[2], t)}
    if loc < nf + 2 * ne:
        E, up = divmod(loc - nf, 2)
        a, b = edges[E]
        return {(a, t), (a, t + 1), (b, t + 1)} if up else {(a, t), (b, t), (b, t + 1)}
    T, up = divmod(loc - nf - 2 * ne, 2)
    a = tri[T]
    return {(a[0], t), (a[1], t + 1), (a[2], t + 1)} if up else {(a[0], t), (a[1], t), (a[2], t + 1)}


def _grid_face_vertices(fid, nx, ny):
    types = O.kuhn_types(3, 2)
    ty, g = fid % 12, fid // 12
    x, y, t = g % nx, (g // nx) % ny, g // (nx * ny)
    c = [x, y, t]
    out = {(y * nx + x, t)}
    for m in types[ty]:
        for a in range(3):
            if (int(m) >> a) & 1:
                c[a] += 1
        out.add((c[1] * nx + c[0], c[2]))
    return out


@pytest.mark.parametrize("seed,smooth", [(0, False), (1, False), (2, True)])
def test_kuhn_grid_mesh_equals_the_regular_grid(seed, smooth):
    nx, ny, nt = 9, 7, 5
    rng = np.random.default_rng(seed)
    if smooth:
        vec = synth.vortex_sources_2d(nx, ny, nt, 3, sigma=(2.0, 4.0), seed=seed).astype(np.float32)
    else:
        vec = rng.integers(-2, 3, size=(nt, 2, ny, nx)).astype(np.float32) / 2 ** 20
    xy, tri = synth.kuhn_grid_mesh(nx, ny)
    r = M.track_cp_mesh(xy, tri, vec.reshape(nt, 2, ny * nx))
    g = O.track(vec, n=2, kind=1)
    assert r.n_hits == g.n_hits and r.n_traj == g.n_traj
    trs = np.sort(tri, axis=1)
    edges = M.mesh_edges(tri)
    mf = {frozenset(_face_vertices(r, f, nx * ny, trs, edges)): i for i, f in enumerate(r.face_id)}
    gf = {frozenset(_grid_face_vertices(int(f), nx, ny)): i for i, f in enumerate(g.face_id)}
    assert set(mf) == set(gf)
    for k in mf:
        assert np.allclose(r.pos[mf[k]], g.pos[gf[k]], rtol=0, atol=1e-12)
    # the same partition into trajectories
    pairs = {(r.label[mf[k]], g.label[gf[k]]) for k in mf}
    assert len(pairs) == r.n_traj == len({a for a, _ in pairs}) == len({b for _, b in pairs})


@pytest.mark.parametrize("seed", [3, 4])
def test_delaunay_tetrahedra_have_zero_or_two_punctured_faces(seed):
    xy, tri = synth.delaunay_mesh(40, seed=seed)
    rng = np.random.default_rng(seed)
    field = rng.integers(-1, 2, size=(4, 2, len(xy))).astype(np.float32) / 2 ** 20
    r = M.track_cp_mesh(xy, tri, field)
    assert r.n_hits > 0
    assert r.tet_counts[1] == 0 and r.tet_counts[3] == 0 and r.tet_counts[4] == 0


def test_moving_zero_on_a_delaunay_mesh():
    xy, tri = synth.delaunay_mesh(120, seed=5)
    nt = 6
    x0, y0, vx, vy = 3.3, 4.1, 0.6, 0.4
    f = np.zeros((nt, 2, len(xy)), np.float32)
    for t in range(nt):
        f[t, 0] = xy[:, 0] - x0 - vx * t
        f[t, 1] = xy[:, 1] - y0 - vy * t
    r = M.track_cp_mesh(xy, tri, f)
    assert r.n_traj == 1
    tt = r.pos[:, 2]
    assert np.all(np.abs(r.pos[:, 0] - (x0 + vx * tt)) < 1e-5)
    assert np.all(np.abs(r.pos[:, 1] - (y0 + vy * tt)) < 1e-5)
    ordinal = (r.face_id % r.S) < r.nf
    steps = r.face_id[ordinal] // r.S
    assert np.array_equal(np.sort(steps), np.arange(nt))


def _book_mesh():
    """A grid mesh with one more triangle on an interior edge (an edge of three triangles)."""
    xy, tri = synth.kuhn_grid_mesh(7, 6)
    a, b = (int(v) for v in sorted(tri[len(tri) // 2][:2]))
    xy = np.concatenate([xy, (0.5 * (xy[a] + xy[b]) + np.array([0.13, 0.29], np.float32))[None]]).astype(np.float32)
    return xy, np.concatenate([tri, np.array([[a, b, len(xy) - 1]], np.int32)])


@pytest.mark.parametrize("mesh", ["delaunay", "book"])
def test_tetrahedra_reached_from_punctured_faces(mesh):
    """The unions may start from the punctured faces: a face lies in the prisms of its triangle (a mesh triangle: the
    prism above it and the one below), of its edge's triangles (edge faces) or of its triangle (interior faces), and
    the tetrahedra of those prisms that hold it are exactly the tetrahedra with a punctured side (boundary edges
    with one triangle and an edge with three included)."""
    xy, tri = synth.delaunay_mesh(40, seed=6) if mesh == "delaunay" else _book_mesh()
    nt = 4
    rng = np.random.default_rng(11)
    field = rng.integers(-1, 2, size=(nt, 2, len(xy))).astype(np.float32) / 2 ** 20
    r = M.track_cp_mesh(xy, tri, field)
    tri_s = np.sort(np.asarray(tri, np.int64), axis=1)
    edges = M.mesh_edges(tri_s)
    nv, nf, ne = len(xy), r.nf, r.ne
    edge_index = {(int(a), int(b)): i for i, (a, b) in enumerate(edges)}
    edge_tris = [[] for _ in range(ne)]
    for T, (a0, a1, a2) in enumerate(tri_s):
        for e in ((a0, a1), (a1, a2), (a0, a2)):
            edge_tris[edge_index[(int(e[0]), int(e[1]))]].append(T)

    def prism_tets(T, t):
        A = [(int(v), t) for v in tri_s[T]]
        B = [(v, t + 1) for v, _ in A]
        return [frozenset([A[0], A[1], A[2], B[2]]), frozenset([A[0], A[1], B[1], B[2]]),
                frozenset([A[0], B[0], B[1], B[2]])]

    all_tets = {(T, t, k): tet for t in range(nt - 1) for T in range(nf) for k, tet in enumerate(prism_tets(T, t))}
    hit_faces = {frozenset(_face_vertices(r, f, nv, tri_s, edges)) for f in r.face_id}
    every = {key for key, tet in all_tets.items() if any(tet - {p} in hit_faces for p in tet)}
    reached = set()
    for f in r.face_id:
        t, loc = divmod(int(f), r.S)
        if loc < nf:
            prisms = [(loc, t)] * (t < nt - 1) + [(loc, t - 1)] * (t >= 1)
        elif loc < nf + 2 * ne:
            prisms = [(T, t) for T in edge_tris[(loc - nf) // 2]]
        else:
            prisms = [((loc - nf - 2 * ne) // 2, t)]
        face = frozenset(_face_vertices(r, f, nv, tri_s, edges))
        mine = {(T, tp, k) for T, tp in prisms for k, tet in enumerate(prism_tets(T, tp)) if face <= tet}
        # each face by itself: its prisms hold every tetrahedron that has it as a side
        assert mine == {key for key, tet in all_tets.items() if face <= tet}, int(f)
        reached |= mine
    assert len(every) > 0 and reached == every
    if mesh == "book":
        assert max(len(x) for x in edge_tris) == 3
