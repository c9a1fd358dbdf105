"""Isovolume tracking oracle (test infrastructure only, like the rest of oracle/): plain numpy, binary64.

Written from the two-pass isovolume reconstruction (Sec. 6.1, Alg. 1 right column) on the regular simplicial
spacetime mesh of a 3D scalar series (Sec. 3.3), with the robustness rule of Sec. 6.2:
  * mesh: vertices (x, y, z, t), t-major index g = ((t nz + z) ny + y) nx + x; an edge anchored at p with axis mask
    M (1..15; bits x = 1, y = 2, z = 4, t = 8) joins p and p + e(M); its id is g(p) * 15 + (M - 1) (edge types in
    increasing mask order); a pentachoron anchored at p with axis order (s1, s2, s3, s4) has the chain vertices
    p, p + e(s1), p + e(s1|s2), p + e(s1|s2|s3), p + e(1111);
  * edge pass: the edge crosses the level set f = c when its two vertices fall on different sides; as a 1D
    critical-point test under the symbolic perturbation, a vertex value exactly equal to c counts as above it
    (the perturbation of a single entry is positive);
  * intersection point: p + mu e(M) with mu = (c - f(p)) / (f(q) - f(p));
  * pentachoron pass: the crossed edges of every pentachoron are united; labels are the smallest edge id of each
    component;
  * tessellation (Sec. 6.1 case analysis): with one vertex on its side (case I) the crossed edges are the four
    edges from that vertex and form one tetrahedron; with two (case II) the six crossed edges form a prism
    (pair x triple), split into three tetrahedra along monotone paths of the pair and triple in chain order
    (staircase triangulation).
"""
import itertools

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

AXES = 4


def _perms():
    return [tuple(1 << a for a in p) for p in itertools.permutations(range(AXES))]


def _gindex(c, dims):
    nx, ny, nz, nt = dims
    return ((c[3] * nz + c[2]) * ny + c[1]) * nx + c[0]


class IsoResult:
    pass


def track_iso(field, c):
    """field: float32 [nt][nz][ny][nx]; c: isovalue (float32).  Returns an IsoResult with edge_id (ascending),
    pos [n][4] (x, y, z, t), label, n_components, tets [m][4] (indices into the hits, ordered by pentachoron id
    g * 24 + type and by tetrahedron within it)."""
    f = np.ascontiguousarray(field, dtype=np.float32)
    nt, nz, ny, nx = f.shape
    dims = (nx, ny, nz, nt)
    c32 = np.float32(c)
    above = f >= c32                       # exact comparison of binary32 values
    grid = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), np.arange(nt), indexing="ij"), 0)
    grid = np.transpose(grid, (0, 4, 3, 2, 1))  # [4][nt][nz][ny][nx] coordinates (x, y, z, t)

    def shifted(a, M):
        """a at p + e(M), and whether that vertex is in the grid (arrays over anchors p)."""
        d = [(M >> k) & 1 for k in range(AXES)]   # x, y, z, t
        out = np.zeros_like(a)
        ok = np.zeros(a.shape, bool)
        sl_src = (slice(d[3], None), slice(d[2], None), slice(d[1], None), slice(d[0], None))
        sl_dst = (slice(0, nt - d[3]), slice(0, nz - d[2]), slice(0, ny - d[1]), slice(0, nx - d[0]))
        out[sl_dst] = a[sl_src]
        ok[sl_dst] = True
        return out, ok

    ids, pos = [], []
    g_all = _gindex(grid, dims)
    for M in range(1, 16):
        aq, ok = shifted(above, M)
        fq, _ = shifted(f, M)
        hit = ok & (above != aq)
        if not hit.any():
            continue
        fa = f[hit].astype(np.float64)
        fb = fq[hit].astype(np.float64)
        mu = (np.float64(c32) - fa) / (fb - fa)
        p = np.stack([grid[k][hit] for k in range(AXES)], 1).astype(np.float64)
        e = np.array([(M >> k) & 1 for k in range(AXES)], np.float64)
        pos.append(p + mu[:, None] * e[None, :])
        ids.append(g_all[hit] * 15 + (M - 1))
    if ids:
        ids = np.concatenate(ids)
        pos = np.concatenate(pos)
        o = np.argsort(ids)
        ids, pos = ids[o], pos[o]
    else:
        ids, pos = np.zeros(0, np.int64), np.zeros((0, 4))
    index = {int(e): i for i, e in enumerate(ids)}

    # pentachoron pass: unite crossed edges, tessellate
    rows, cols, tets, tet_key = [], [], [], []
    valid = np.ones(f.shape, bool)
    valid[nt - 1, :, :, :] = False
    valid[:, nz - 1, :, :] = False
    valid[:, :, ny - 1, :] = False
    valid[:, :, :, nx - 1] = False
    anchors = np.argwhere(valid)  # (t, z, y, x)
    for ty, perm in enumerate(_perms()):
        corners = [0]
        for m in perm:
            corners.append(corners[-1] | m)
        for (t, z, y, x) in anchors:
            vs = [(x + (cm & 1), y + ((cm >> 1) & 1), z + ((cm >> 2) & 1), t + ((cm >> 3) & 1)) for cm in corners]
            sg = [bool(above[v[3], v[2], v[1], v[0]]) for v in vs]
            k = sum(sg)
            if k in (0, 5):
                continue

            def edge(i, j):  # hit index of the edge between chain vertices i < j
                return index[_gindex(vs[i], dims) * 15 + ((corners[j] ^ corners[i]) - 1)]

            crossed = [edge(i, j) for i in range(5) for j in range(i + 1, 5) if sg[i] != sg[j]]
            assert len(crossed) == k * (5 - k)
            for e in crossed[1:]:
                rows.append(crossed[0])
                cols.append(e)
            key = _gindex((x, y, z, t), dims) * 24 + ty
            minority = [i for i in range(5) if sg[i] == (k <= 2)]
            majority = [i for i in range(5) if sg[i] != (k <= 2)]
            if len(minority) == 1:
                L = minority[0]
                tets.append([edge(min(L, o), max(L, o)) for o in majority])
                tet_key.append((key, 0))
            else:
                p1, p2 = minority
                m1, m2, m3 = majority

                def pe(p, m):
                    return edge(min(p, m), max(p, m))
                tets.append([pe(p1, m1), pe(p1, m2), pe(p1, m3), pe(p2, m3)])
                tets.append([pe(p1, m1), pe(p1, m2), pe(p2, m2), pe(p2, m3)])
                tets.append([pe(p1, m1), pe(p2, m1), pe(p2, m2), pe(p2, m3)])
                tet_key += [(key, 0), (key, 1), (key, 2)]
    n = len(ids)
    if n:
        A = coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
        ncomp, comp = connected_components(A, directed=False)
        first = np.full(ncomp, np.iinfo(np.int64).max, np.int64)
        np.minimum.at(first, comp, ids)
        label = first[comp]
    else:
        ncomp, label = 0, np.zeros(0, np.int64)
    if tets:
        o = sorted(range(len(tets)), key=lambda i: tet_key[i])
        tets = np.array([tets[i] for i in o], np.int64)
    else:
        tets = np.zeros((0, 4), np.int64)
    r = IsoResult()
    r.edge_id, r.pos, r.label, r.n_components, r.tets, r.n_hits = ids, pos, label, ncomp, tets, n
    return r


def tet_volume(P):
    """3-volume of the tetrahedron with 4D vertices P[4][4] (Gram determinant)."""
    E = P[1:] - P[0]
    G = E @ E.T
    return float(np.sqrt(max(np.linalg.det(G), 0.0)) / 6.0)
