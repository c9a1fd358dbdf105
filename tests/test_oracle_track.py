"""Pins of the oracle's whole-field tracker: brute force on tiny grids, invariants, closed forms (Sec. 4.5)."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from oracle import ref as R
from paper_2011_08697_amd import synth

ORDINAL_2D = (0, 3)  # triangle types (1,2) and (2,1): no time step inside


def _vec_dict(g, u, n):
    vec = {}
    for gi in range(g.V):
        p = g.coords(gi)
        t = p[-1]
        idx = (t, slice(None)) + tuple(p[:-1][::-1])
        vec[gi] = [int(round(float(x))) for x in u[idx]]
    return vec


@pytest.mark.parametrize("seed,dims,r", [(1, (5, 5, 4), 1), (2, (6, 4, 5), 1), (3, (4, 5, 4), 2)])
def test_tiny_2d_grid_matches_literal_reference(seed, dims, r):
    rng = np.random.default_rng(seed)
    nx, ny, nt = dims
    u = rng.integers(-r, r + 1, size=(nt, 2, ny, nx)).astype(np.float32)
    tr = O.track(u, n=2, kind=1)
    assert tr.status == 0
    g = R.Grid(dims)
    hits, label, hist = R.track(g, _vec_dict(g, u, 2))
    assert list(tr.face_id) == hits
    assert [label[f] for f in tr.face_id] == list(tr.label)
    assert set(hist) <= {0, 2}
    assert tr.n_traj == len(set(label.values()))


def test_tiny_3d_grid_mesh_and_stitching_match_reference():
    """3D: stitching and labels against a breadth-first search over the paper's cell lists; the per-face predicate
    is pinned separately (literal definition, sampled, as it is slow in pure Python)."""
    rng = np.random.default_rng(4)
    dims = (3, 3, 3, 3)
    f = rng.integers(-2, 3, size=(3, 3, 3, 3)).astype(np.float32)  # scalar: the gradient is taken
    tr = O.track(f, n=3, kind=0)
    assert tr.status == 0
    st, q = O.quantise_all(f, n=3, kind=0)
    g = R.Grid(dims)
    vec = {gi: [int(x) for x in q[gi]] for gi in range(g.V)}

    hits, label, hist = _track_with(g, vec, lambda vv: O.face_punctured(np.array(vv)))
    assert list(tr.face_id) == hits
    assert [label[x] for x in tr.face_id] == list(tr.label)
    assert set(hist) <= {0, 2}
    # sampled literal check of the 3D predicate on this grid
    faces = g.faces()
    pick = np.random.default_rng(5).choice(len(faces), 12, replace=False)
    for i in pick:
        vv = [vec[g.g(p)] for p in faces[i]]
        assert O.face_punctured(np.array(vv)) == int(R.punctured(vv))


def _track_with(g, vec, punct):
    import itertools
    hits = {}
    for fc in g.faces():
        if punct([vec[g.g(p)] for p in fc]):
            hits[g.face_id(fc)] = fc
    adj = {h: [] for h in hits}
    hist = {}
    for cell in g.cells():
        ids = [g.face_id(s) for s in itertools.combinations(cell, g.n + 1)]
        pun = [i for i in ids if i in hits]
        hist[len(pun)] = hist.get(len(pun), 0) + 1
        if len(pun) == 2:
            adj[pun[0]].append(pun[1])
            adj[pun[1]].append(pun[0])
    label = {}
    for s in sorted(hits):
        if s in label:
            continue
        comp, i = [s], 0
        while i < len(comp):
            for nb in adj[comp[i]]:
                if nb not in comp:
                    comp.append(nb)
            i += 1
        for c in comp:
            label[c] = min(comp)
    return sorted(hits), label, hist


@pytest.mark.parametrize("n,shape", [(2, (4, 6, 7)), (3, (3, 4, 4, 5))])
def test_all_zero_field_has_no_hits(n, shape):
    tr = O.track(np.zeros(shape, np.float32), n=n, kind=0)
    assert tr.status == 0 and tr.n_hits == 0 and tr.n_traj == 0


def _degrees_equal_cofaces(tr, dims, n):
    """Under SoS every cell holds 0 or 2 punctured sides, so a hit's degree in the trajectory graph equals the
    number of cells containing it: paths end only on boundary faces, everything else is a cycle (Sec. 4.2)."""
    hitset = set(int(x) for x in tr.face_id)
    rng = np.random.default_rng(0)
    sample = tr.face_id if len(tr.face_id) <= 400 else rng.choice(tr.face_id, 400, replace=False)
    for f in sample:
        cof = O.face_cofaces(dims, int(f), n=n)
        sides = O.cell_sides(dims, cof, n=n)
        for row in sides:
            assert sum(1 for s in row if int(s) in hitset) == 2


def test_invariants_on_blob_field():
    f = synth.make("blobs64")
    tr = O.track(f)
    assert tr.status == 0 and tr.invariant_violations == 0
    assert tr.n_hits == 332 and int(np.isin(tr.face_id % 12, ORDINAL_2D).sum()) == 73
    _degrees_equal_cofaces(tr, (64, 64, 10), 2)
    # labels are the smallest face id of each component and belong to it
    assert np.all(tr.label <= tr.face_id)
    assert set(tr.label.tolist()) <= set(tr.face_id.tolist())


def test_invariants_on_degenerate_integer_field():
    f = synth.quantise_levels(synth.moving_gaussians_2d(48, 40, 6, 6, seed=11, noise_std=1e-3))
    tr = O.track(f)
    assert tr.status == 0 and tr.invariant_violations == 0 and tr.n_hits > 0
    _degrees_equal_cofaces(tr, (48, 40, 6), 2)


def test_invariants_3d_random_integer_field():
    rng = np.random.default_rng(9)
    f = rng.integers(0, 4, size=(3, 4, 4, 4)).astype(np.float32)
    tr = O.track(f, n=3)
    assert tr.status == 0 and tr.invariant_violations == 0 and tr.n_hits > 0
    _degrees_equal_cofaces(tr, (4, 4, 4, 3), 3)


def _moving_minimum_check(n, size, direction, nt):
    x0 = [size // 2] * n
    f = synth.moving_minimum(n, size, x0, direction, nt)
    tr = O.track(f, n=n)
    assert tr.status == 0 and tr.invariant_violations == 0
    T = 12 if n == 2 else 60
    types = O.kuhn_types(n + 1, n)
    tbit = 1 << n
    ordinal = [i for i, row in enumerate(types) if not any(int(m) & tbit for m in row)]
    plane = size ** n
    steps = (tr.face_id // T) // plane
    is_ord = np.isin(tr.face_id % T, ordinal)
    # each zero lies in exactly one simplex: one ordinal face per time slice
    for t in range(nt):
        assert int(np.sum(is_ord & (steps == t))) == 1
    # one trajectory from the first to the last step, on the line x0 + d t, every point a minimum
    assert tr.n_traj == 1
    t_pos = tr.pos[:, n]
    for a in range(n):
        assert np.allclose(tr.pos[:, a], x0[a] + direction[a] * t_pos, atol=1e-9)
    assert np.all(tr.type == 1)


def test_moving_minimum_2d_twenty_directions():
    """Sec. 4.5, Eq. 3-4, in 2D: 21^2 grid, x0 = (10, 10), 20 random dyadic directions through grid vertices."""
    rng = np.random.default_rng(2020)
    for it in range(20):
        d = [int(k) / 8 for k in rng.integers(-8, 9, size=2)]
        _moving_minimum_check(2, 21, d, 9)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_moving_minimum_3d(seed):
    """Sec. 4.5, Eq. 3-4: 21^3 grid, x0 = (10, 10, 10), random rational directions through grid vertices."""
    rng = np.random.default_rng(100 + seed)
    d = [int(k) / 4 for k in rng.integers(-4, 5, size=3)]
    _moving_minimum_check(3, 21, d, 5)


def test_birth_death_pair_forms_one_cycle():
    """f = X^3/3 - a(t) X + Y^2 with a(t) > 0 only for t in an inner interval: a minimum and a saddle are born
    together and annihilate, one closed loop in spacetime (Sec. 4.2: trajectories end on the boundary or are
    loops)."""
    nx, ny, nt = 33, 17, 21
    X = np.arange(nx, dtype=np.float64) - 16.0
    Y = np.arange(ny, dtype=np.float64) - 8.0
    f = np.zeros((nt, ny, nx))
    for t in range(nt):
        a = 30.0 - 0.5 * (t - 10.0) ** 2
        f[t] = (X[None, :] ** 3) / 3.0 - a * X[None, :] + (Y[:, None] ** 2)
    f = f.astype(np.float32)
    tr = O.track(f)
    assert tr.status == 0 and tr.invariant_violations == 0
    assert tr.n_traj == 1
    # a cycle: every hit lies in two cells (none on the domain boundary)
    for fid in tr.face_id[::7]:
        assert len(O.face_cofaces((nx, ny, nt), int(fid))) == 2
    t = set(tr.type.tolist())
    assert 1 in t and 3 in t  # MIN and SADDLE
    assert O.trace(f, int(tr.face_id[0]))["closed"] == 1


@pytest.mark.parametrize("A,expect", [
    ([[2, 0], [0, 1]], "SOURCE"), ([[-2, 0], [0, -1]], "SINK"), ([[1, -2], [2, 1]], "REPELLING_FOCUS"),
    ([[-1, -2], [2, -1]], "ATTRACTING_FOCUS"), ([[0, -1], [1, 0]], "CENTER"), ([[1, 0], [0, -1]], "SADDLE")])
def test_linear_vector_field_types(A, expect):
    """v = A (x - c) is exactly linear, so every stencil is exact and the Jacobian is A everywhere."""
    nx, ny, nt = 17, 17, 3
    c = (8.25, 7.5)
    xs = np.arange(nx) - c[0]
    ys = np.arange(ny) - c[1]
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    u = np.zeros((nt, 2, ny, nx), np.float32)
    for t in range(nt):
        u[t, 0] = A[0][0] * X + A[0][1] * Y
        u[t, 1] = A[1][0] * X + A[1][1] * Y
    tr = O.track(u, n=2, kind=1)
    assert tr.status == 0 and tr.n_traj == 1 and tr.n_hits >= nt
    assert set(tr.type.tolist()) == {O.TYPES.index(expect)}
    assert np.allclose(tr.pos[:, 0], c[0], atol=1e-12) and np.allclose(tr.pos[:, 1], c[1], atol=1e-12)


@pytest.mark.parametrize("sx,sy,expect", [(1, 1, "MIN"), (-1, -1, "MAX"), (1, -1, "SADDLE")])
def test_quadratic_scalar_types(sx, sy, expect):
    nx, ny, nt = 17, 15, 3
    X, Y = np.meshgrid(np.arange(nx) - 8.25, np.arange(ny) - 6.5, indexing="xy")
    f = np.stack([sx * X ** 2 + sy * Y ** 2] * nt).astype(np.float32)
    tr = O.track(f)
    assert tr.status == 0 and tr.n_traj == 1
    assert set(tr.type.tolist()) == {O.TYPES.index(expect)}
    assert np.allclose(tr.pos[:, :2], [8.25, 6.5], atol=1e-12)


def test_spiral_woven_critical_points():
    """Sec. 4.5, Eq. 5 (approximate pin): at time t the critical points of cos(x') sin(y'), (x', y') = R(t)(x, y),
    are extrema at x' = k pi, y' = pi/2 + m pi and saddles at x' = pi/2 + k pi, y' = m pi.  The central difference
    of sin/cos vanishes where the derivative does, so the detected points sit on the analytic ones."""
    size, nt, ext, dt = 128, 3, 6.0, 0.25
    f = synth.spiral_woven(size, nt, ext, dt)
    tr = O.track(f)
    assert tr.status == 0 and tr.invariant_violations == 0
    h = 2 * ext / (size - 1)
    plane = size * size
    for t in range(nt):
        tt = t * dt
        sel = np.isin(tr.face_id % 12, ORDINAL_2D) & (((tr.face_id // 12) // plane) == t)
        pts = tr.pos[sel][:, :2] * h - ext
        typ = tr.type[sel]
        expected = []
        for k in range(-4, 5):
            for m in range(-4, 5):
                for (xp, yp, kind) in [(k * math.pi, math.pi / 2 + m * math.pi, "ext"),
                                       (math.pi / 2 + k * math.pi, m * math.pi, "saddle")]:
                    # back-rotate (x', y') = R(t)(x, y)
                    x = xp * math.cos(tt) + yp * math.sin(tt)
                    y = -xp * math.sin(tt) + yp * math.cos(tt)
                    if abs(x) < ext - 3 * h and abs(y) < ext - 3 * h:
                        val = math.cos(xp) * math.sin(yp)
                        ty = "SADDLE" if kind == "saddle" else ("MAX" if val > 0 else "MIN")
                        expected.append((x, y, ty))
        assert len(expected) > 10
        for x, y, ty in expected:
            dist = np.hypot(pts[:, 0] - x, pts[:, 1] - y)
            j = int(np.argmin(dist))
            assert dist[j] < 0.05 * h
            assert O.TYPES[int(typ[j])] == ty


def test_quantisation_rounds_half_to_even_and_checks_range():
    base = np.zeros((2, 2, 3, 3), np.float32)
    for val, q in [(2.5, 2), (3.5, 4), (-2.5, -2), (0.5, 0), (1.25, 1)]:
        u = base.copy()
        u[:, 0] = val * 2.0 ** -20
        st, Q = O.quantise_all(u, n=2, kind=1)
        assert st == 0 and np.all(Q[:, 0] == q)
    u = base.copy()
    u[0, 0, 0, 0] = 2.0 ** 42  # |q| = 2^62: outside the 2D range
    assert O.quantise_all(u, n=2, kind=1)[0] == 3
    u[0, 0, 0, 0] = 2.0 ** 41  # |q| = 2^61: accepted (wide tier)
    assert O.quantise_all(u, n=2, kind=1)[0] == 0
    tr = O.track(u, n=2, kind=1)
    assert tr.status == 0
    u[0, 0, 0, 0] = np.nan
    assert O.track(u, n=2, kind=1).status == 2
    u[0, 0, 0, 0] = np.inf
    assert O.track(u, n=2, kind=1).status == 2


def test_stencil_on_linear_and_quadratic_fields():
    nx, ny, nt = 9, 7, 2
    X, Y = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64), indexing="xy")
    f = np.stack([0.75 * X - 0.5 * Y] * nt).astype(np.float32)
    st, q = O.quantise_all(f)
    assert st == 0 and np.all(q[:, 0] == int(0.75 * 2 ** 20)) and np.all(q[:, 1] == -(2 ** 19))
    f = np.stack([X ** 2 + 3 * Y ** 2 + X * Y] * nt).astype(np.float32)
    st, J = O.jacobian_all(f)
    J = J.reshape(nt, ny, nx, 2, 2)
    inner = J[:, 2:-2, 2:-2]
    assert np.all(inner[..., 0, 0] == 2) and np.all(inner[..., 1, 1] == 6)
    assert np.all(inner[..., 0, 1] == 1) and np.all(inner[..., 1, 0] == 1)


def test_sublocation_matches_exact_rationals():
    """mu from the oracle (binary64) against the exact rational solution of Eq. 2 on the quantised vectors."""
    f = synth.make("blobs64")
    tr = O.track(f)
    st, q = O.quantise_all(f)
    g = R.Grid((64, 64, 10))
    rng = np.random.default_rng(1)
    for i in rng.choice(tr.n_hits, 60, replace=False):
        fid = int(tr.face_id[i])
        anchor = g.coords(fid // 12)
        masks = g.face_types[fid % 12]
        verts = [anchor]
        for m in masks:
            verts.append(tuple(c + ((m >> a) & 1) for a, c in enumerate(verts[-1])))
        V = [[int(x) for x in q[g.g(p)]] for p in verts]
        M = [[Fraction(V[k][j]) for k in range(3)] for j in range(2)] + [[Fraction(1)] * 3]
        D = R.det(M)
        assert D != 0
        for k in range(3):
            Mi = [row[:] for row in M]
            for r in range(3):
                Mi[r][k] = Fraction(1 if r == 2 else 0)
            mu = R.det(Mi) / D
            assert abs(tr.mu[i, k] - float(mu)) <= 4e-16
        pos = [sum(float(R.det([[M[r][c] if c != k else Fraction(1 if r == 2 else 0) for c in range(3)]
                                for r in range(3)]) / D) * verts[k][a] for k in range(3)) for a in range(3)]
        assert np.allclose(tr.pos[i], pos, rtol=0, atol=1e-12)


def test_point_queries_agree_with_whole_field_run():
    f = synth.make("blobs64")
    tr = O.track(f)
    rng = np.random.default_rng(2)
    fids = np.concatenate([tr.face_id[rng.choice(tr.n_hits, 50, replace=False)],
                           rng.integers(0, 64 * 64 * 10 * 12, 300)])
    ev = O.eval_faces(f, fids)
    hitset = {int(x): i for i, x in enumerate(tr.face_id)}
    for k, fid in enumerate(fids):
        if ev["punctured"][k] == 255:
            continue
        assert bool(ev["punctured"][k]) == (int(fid) in hitset)
        if int(fid) in hitset:
            i = hitset[int(fid)]
            assert np.array_equal(ev["pos"][k], tr.pos[i]) and ev["type"][k] == tr.type[i]
    # following a trajectory through its cells reaches the component's smallest face id
    for i in rng.choice(tr.n_hits, 20, replace=False):
        r = O.trace(f, int(tr.face_id[i]))
        assert r["min_face"] == tr.label[i]
        assert r["length"] == int(np.sum(tr.label == tr.label[i]))


# Quadratic forms f = (x - c)^T A (x - c) in 3D with an off-grid centre.  Central differences of a quadratic are
# exact, so the gradient is exactly the linear field 2 A (x - c) (dyadic values, exact in binary32), the zero sits
# exactly at c, and the Jacobian stencil of that linear gradient is exactly 2 A.  The type is the inertia of A
# (Sec. 4.1: types from the eigenvalues of the Jacobian): the number of negative eigenvalues picks MIN, SADDLE1,
# SADDLE2 or MAX.  The non-diagonal forms make every term of the Descartes sequence (trace, sum of principal 2x2
# minors, determinant) decide a case: diag(-1, -1, 5) has trace 3, minors -9 and determinant 5, so a sign slip in
# the minors would read MIN instead of SADDLE2.
QUAD3_CASES = [
    ([[1, 0, 0], [0, 1, 0], [0, 0, 1]], "MIN"),
    ([[-1, 0, 0], [0, -1, 0], [0, 0, -1]], "MAX"),
    ([[-1, 0, 0], [0, 1, 0], [0, 0, 1]], "SADDLE1"),
    ([[1, 0, 0], [0, -1, 0], [0, 0, 1]], "SADDLE1"),
    ([[1, 0, 0], [0, 1, 0], [0, 0, -1]], "SADDLE1"),
    ([[-1, 0, 0], [0, -1, 0], [0, 0, 1]], "SADDLE2"),
    ([[1, 0, 0], [0, -1, 0], [0, 0, -1]], "SADDLE2"),
    ([[-1, 0, 0], [0, 1, 0], [0, 0, -1]], "SADDLE2"),
    ([[-1, 0, 0], [0, -1, 0], [0, 0, 5]], "SADDLE2"),
    ([[1, 2, 0], [2, 1, 0], [0, 0, 1]], "SADDLE1"),   # eigenvalues 3, -1, 1
    ([[2, 1, 1], [1, 2, 1], [1, 1, 2]], "MIN"),       # 4, 1, 1
    ([[-2, 1, 1], [1, -2, 1], [1, 1, 1]], "SADDLE2"),  # -3, -sqrt 3, sqrt 3
    ([[-3, 1, 1], [1, -3, 1], [1, 1, -3]], "MAX"),  # -4, -4, -1
    ([[-3, 1, 0], [1, -3, 1], [0, 1, -3]], "MAX"),    # all negative (diagonally dominant)
    ([[0, 1, 1], [1, 0, 1], [1, 1, 0]], "SADDLE2"),   # 2, -1, -1 with a zero diagonal
]
QUAD3_CENTRE = (8.25, 7.5, 6.75)


def quadratic_field_3d(A, c=QUAD3_CENTRE, dims=(17, 15, 14), nt=3):
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz) - c[2], np.arange(ny) - c[1], np.arange(nx) - c[0], indexing="ij")
    X = (x, y, z)
    f = sum(A[a][b] * X[a] * X[b] for a in range(3) for b in range(3))
    return np.stack([f] * nt).astype(np.float32)


def test_quadratic_field_3d_is_exact_in_binary32():
    for A, _ in QUAD3_CASES:
        nx, ny, nz = 17, 15, 14
        z, y, x = np.meshgrid(np.arange(nz) - 6.75, np.arange(ny) - 7.5, np.arange(nx) - 8.25, indexing="ij")
        X = (x, y, z)
        f64 = sum(A[a][b] * X[a] * X[b] for a in range(3) for b in range(3))
        assert np.array_equal(quadratic_field_3d(A)[0].astype(np.float64), f64)


@pytest.mark.parametrize("A,expect", QUAD3_CASES)
def test_quadratic_scalar_types_3d(A, expect):
    """Sec. 4.1 types in 3D on quadratic forms of known inertia: one vertical trajectory through the centre, every
    point of the expected type, positions exactly at the centre."""
    ev = np.linalg.eigvalsh(np.array(A, np.float64))
    n_neg = int(np.sum(ev < 0))
    assert np.all(np.abs(ev) > 0.5)
    assert expect == ["MIN", "SADDLE1", "SADDLE2", "MAX"][n_neg]
    f = quadratic_field_3d(A)
    tr = O.track(f, n=3)
    assert tr.status == 0 and tr.invariant_violations == 0
    assert tr.n_traj == 1 and tr.n_hits >= 3
    assert set(tr.type.tolist()) == {O.TYPES.index(expect)}
    assert np.allclose(tr.pos[:, :3], QUAD3_CENTRE, atol=1e-12)
    # a vertical line: the trajectory reaches the first and the last step
    assert tr.pos[:, 3].min() == 0.0 and tr.pos[:, 3].max() == 2.0
