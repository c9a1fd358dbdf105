"""Quantum vortex surface tracking oracle (test infrastructure only, like the rest of oracle/): plain numpy and the
oracle's exact predicate, one triangle at a time.

Written from the two-pass vortex surface reconstruction (Sec. 5.1, Alg. 1 middle column) on the regular simplicial
spacetime mesh of a 3D complex series (Sec. 3.3):
  * a spacetime triangle (2-simplex of the 4D mesh) anchored at p with axis masks (M1, M2) has the vertices p,
    p + e(M1), p + e(M1|M2) (bits x = 1, y = 2, z = 4, t = 8); its id is g(p) * 50 + type, types in lexicographic
    order of (M1, M2), g the t-major vertex index;
  * the contour-integral test (Eq. 1 and Sec. 5.1): the sum of the phase changes along the three edges, each taken
    modulo 2 pi into (-pi, pi], is +-2 pi.  A straight segment from psi_i to psi_j in the complex plane that misses
    0 turns by exactly that wrapped phase change as seen from 0, so the sum is 2 pi times the winding number of the
    image triangle (psi_0, psi_1, psi_2) around 0: the test asks whether 0 lies inside the image triangle, i.e. the
    puncture test of the 2-component field (Re psi, Im psi) on the triangle, decided exactly on quantised values
    with the symbolic perturbation (Sec. 4.3) like the critical-point test;
  * the vortex point on a positive triangle: barycentric weights from the exact cofactors (Eq. 2);
  * surface pass: the positive triangles of every pentachoron are united; labels are the smallest triangle id of
    each vortex surface.
"""
import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

from . import oracle as O


class VortexResult:
    pass


def quantise(psi, qshift=20):
    """psi: float32 [nt][2][nz][ny][nx] (real and imaginary planes) -> int64 [nt][nz][ny][nx][2],
    rint half-even of fl32(v * 2^qshift) (the scaling is exact)."""
    v = np.asarray(psi, dtype=np.float32) * np.float32(2.0 ** qshift)
    if not np.all(np.isfinite(v)):
        raise ValueError("non-finite value")
    if np.any(np.abs(v) >= 2.0 ** 31):
        raise ValueError("quantised value out of range")
    return np.moveaxis(np.rint(v).astype(np.int64), 1, -1)


def _det(a, b):
    return int(a[0]) * int(b[1]) - int(a[1]) * int(b[0])


def track_vortex(psi, qshift=20):
    q = quantise(psi, qshift)
    nt, nz, ny, nx = q.shape[:4]
    dims = (nx, ny, nz, nt)

    def g(c):
        return ((c[3] * nz + c[2]) * ny + c[1]) * nx + c[0]

    def at(c):
        return q[c[3], c[2], c[1], c[0]]

    def step(c, m):
        return tuple(c[k] + ((m >> k) & 1) for k in range(4))

    tri_types = [tuple(int(x) for x in r) for r in O.kuhn_types(4, 2)]
    tri_index = {t: i for i, t in enumerate(tri_types)}
    ids, pos = [], []
    for ty, (m1, m2) in enumerate(tri_types):
        span = [(m1 | m2) >> k & 1 for k in range(4)]
        for t in range(nt - span[3]):
            for z in range(nz - span[2]):
                for y in range(ny - span[1]):
                    for x in range(nx - span[0]):
                        p0 = (x, y, z, t)
                        p1 = step(p0, m1)
                        p2 = step(p1, m2)
                        V = [at(p0), at(p1), at(p2)]
                        if not O.face_punctured(np.array(V)):
                            continue
                        C = [_det(V[1], V[2]), -_det(V[0], V[2]), _det(V[0], V[1])]
                        D = sum(C)
                        mu = [1.0 / 3.0] * 3 if D == 0 else [c / D for c in C]
                        P = np.array([p0, p1, p2], np.float64)
                        pos.append(mu[0] * P[0] + mu[1] * P[1] + mu[2] * P[2])
                        ids.append(g(p0) * 50 + ty)
    ids = np.array(ids, np.int64)
    pos = np.array(pos, np.float64).reshape(-1, 4)
    o = np.argsort(ids)
    ids, pos = ids[o], pos[o]
    index = {int(e): i for i, e in enumerate(ids)}

    # surface pass: unite the positive triangle sides of every pentachoron
    rows, cols, per_penta = [], [], []
    for perm in O.kuhn_types(4, 4):
        corners = [0]
        for m in perm:
            corners.append(corners[-1] | int(m))
        for t in range(nt - 1):
            for z in range(nz - 1):
                for y in range(ny - 1):
                    for x in range(nx - 1):
                        sides = []
                        for i in range(5):
                            for j in range(i + 1, 5):
                                for k in range(j + 1, 5):
                                    a = step((x, y, z, t), corners[i])
                                    tid = g(a) * 50 + tri_index[(corners[j] ^ corners[i], corners[k] ^ corners[j])]
                                    if tid in index:
                                        sides.append(index[tid])
                        per_penta.append(len(sides))
                        for s in sides[1:]:
                            rows.append(sides[0])
                            cols.append(s)
    n = len(ids)
    if n:
        ncomp, comp = connected_components(coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n)),
                                           directed=False)
        first = np.full(ncomp, np.iinfo(np.int64).max, np.int64)
        np.minimum.at(first, comp, ids)
        label = first[comp]
    else:
        ncomp, label = 0, np.zeros(0, np.int64)
    r = VortexResult()
    r.tri_id, r.pos, r.label, r.n_components, r.n_hits = ids, pos, label, ncomp, n
    r.penta_counts = np.bincount(np.array(per_penta, np.int64), minlength=11)
    return r
