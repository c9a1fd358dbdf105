"""Critical-point tracking on an unstructured triangle mesh extruded in time (test infrastructure only, like the rest
of oracle/): plain numpy and the oracle's exact predicate, one face at a time.

Written from the prismatic subdivision (Sec. 3.2): every mesh triangle with vertices v0 < v1 < v2 (global vertex
order g = t nv + v) becomes, between steps t and t + 1, a prism a0 a1 a2 - b0 b1 b2 split by the staircase into the
tetrahedra a0 a1 a2 b2, a0 a1 b1 b2 and a0 b0 b1 b2; the quadrilateral of a mesh edge (a < b) is split along the
monotone diagonal a - b'.  Faces of step t, numbered t * S + local with S = nf + 2 ne + 2 nf:
  * ordinal (the mesh triangle T at step t): local T;
  * edge faces of mesh edge E = (a < b): lower (a, b, b') at nf + 2E, upper (a, a', b') at nf + 2E + 1;
  * interior faces of triangle T: lower (v0, v1, v2') at nf + 2 ne + 2T, upper (v0, v1', v2') one more;
interval faces exist for t < nt - 1.  A face is punctured when the 2D vector field, quantised like the regular
path, has a zero in it under the symbolic perturbation (the puncture test of Sec. 4.3 with the vertices in global
order); its point comes from the exact cofactors (Eq. 2); the punctured faces of every tetrahedron (0 or 2) are
united (Alg. 1), labels = smallest face id.
"""
import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

from . import oracle as O


class MeshResult:
    pass


def mesh_edges(tri):
    """Sorted unique edges (a < b) of the triangles (rows sorted ascending)."""
    t = np.sort(np.asarray(tri, np.int64), axis=1)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [0, 2]]])
    return np.unique(e, axis=0)


def track_cp_mesh(xy, tri, field, qshift=20):
    """xy [nv][2], tri [nf][3] vertex indices, field float32 [nt][2][nv] (vector components per step)."""
    tri = np.sort(np.asarray(tri, np.int64), axis=1)
    xy = np.asarray(xy, np.float64)
    v = np.asarray(field, np.float32) * np.float32(2.0 ** qshift)
    if not np.all(np.isfinite(v)) or np.any(np.abs(v) >= 2.0 ** 31):
        raise ValueError("non-finite or out-of-range value")
    q = np.rint(v).astype(np.int64)              # [nt][2][nv]
    nt, nv, nf = q.shape[0], xy.shape[0], tri.shape[0]
    edges = mesh_edges(tri)
    ne = len(edges)
    S = nf + 2 * ne + 2 * nf
    key_to_id = {}
    faces = []  # (id, [(v, t) x 3] in global order)
    for t in range(nt):
        for T, (a0, a1, a2) in enumerate(tri):
            faces.append((t * S + T, [(a0, t), (a1, t), (a2, t)]))
        if t == nt - 1:
            continue
        for E, (a, b) in enumerate(edges):
            faces.append((t * S + nf + 2 * E, [(a, t), (b, t), (b, t + 1)]))
            faces.append((t * S + nf + 2 * E + 1, [(a, t), (a, t + 1), (b, t + 1)]))
        for T, (a0, a1, a2) in enumerate(tri):
            base = t * S + nf + 2 * ne + 2 * T
            faces.append((base, [(a0, t), (a1, t), (a2, t + 1)]))
            faces.append((base + 1, [(a0, t), (a1, t + 1), (a2, t + 1)]))
    ids, pos = [], []
    for fid, vs in faces:
        key_to_id[tuple(sorted(tt * nv + vv for vv, tt in vs))] = fid
        V = np.array([[q[tt, 0, vv], q[tt, 1, vv]] for vv, tt in vs], np.int64)
        if not O.face_punctured(V):
            continue
        d = lambda A, B: int(A[0]) * int(B[1]) - int(A[1]) * int(B[0])
        C = [d(V[1], V[2]), -d(V[0], V[2]), d(V[0], V[1])]
        D = sum(C)
        mu = [1.0 / 3.0] * 3 if D == 0 else [c / D for c in C]
        P = [np.array([xy[vv, 0], xy[vv, 1], float(tt)]) for vv, tt in vs]
        pos.append(mu[0] * P[0] + mu[1] * P[1] + mu[2] * P[2])
        ids.append(fid)
    ids = np.array(ids, np.int64)
    pos = np.array(pos, np.float64).reshape(-1, 3)
    o = np.argsort(ids)
    ids, pos = ids[o], pos[o]
    index = {int(e): i for i, e in enumerate(ids)}
    rows, cols, per_tet = [], [], []
    for t in range(nt - 1):
        for a0, a1, a2 in tri:
            A = [t * nv + a0, t * nv + a1, t * nv + a2]
            B = [x + nv for x in A]
            for tet in ([A[0], A[1], A[2], B[2]], [A[0], A[1], B[1], B[2]], [A[0], B[0], B[1], B[2]]):
                hit = [index[key_to_id[tuple(sorted(tet[:k] + tet[k + 1:]))]] for k in range(4)
                       if key_to_id[tuple(sorted(tet[:k] + tet[k + 1:]))] in index]
                per_tet.append(len(hit))
                if len(hit) == 2:
                    rows.append(hit[0])
                    cols.append(hit[1])
    n = len(ids)
    if n:
        ncomp, comp = connected_components(coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n)),
                                           directed=False)
        first = np.full(ncomp, np.iinfo(np.int64).max, np.int64)
        np.minimum.at(first, comp, ids)
        label = first[comp]
    else:
        ncomp, label = 0, np.zeros(0, np.int64)
    r = MeshResult()
    r.face_id, r.pos, r.label, r.n_traj, r.n_hits = ids, pos, label, ncomp, n
    r.tet_counts = np.bincount(np.array(per_tet, np.int64), minlength=5)
    r.S, r.nf, r.ne = S, nf, ne
    return r
