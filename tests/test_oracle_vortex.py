"""Pins of the vortex oracle (oracle/vortex.py) against what the paper and geometry fix: the paper's contour-integral
test (wrapped phase changes summing to +-2 pi) agrees with the exact puncture test on random triangles; a moving
straight vortex line gives one surface whose points lie on the line and one positive triangle per spatial plane and
step; on fields with ties everywhere every tetrahedron has 0 or 2 positive faces and every pentachoron 0, 3, 4 or 5
(the cases of Sec. 5.1); a ring is one surface and two rings two."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import vortex as Vx


def _field(nx, ny, nz, nt, fn):
    X, Y, Z, T = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64),
                             np.arange(nz, dtype=np.float64), np.arange(nt, dtype=np.float64), indexing="ij")
    re, im = fn(X, Y, Z, T)
    return np.stack([np.transpose(re, (3, 2, 1, 0)), np.transpose(im, (3, 2, 1, 0))], 1).astype(np.float32)


def test_phase_sum_definition_equals_the_exact_test():
    """Sum over the three edges of the phase change wrapped into (-pi, pi] is +-2 pi exactly when the exact test
    fires (random integer triangles away from the wrap point)."""
    rng = np.random.default_rng(0)
    checked = 0
    while checked < 3000:
        V = rng.integers(-50, 51, size=(3, 2))
        th = np.arctan2(V[:, 1].astype(float), V[:, 0].astype(float))
        d = [(th[(i + 1) % 3] - th[i] + np.pi) % (2 * np.pi) - np.pi for i in range(3)]
        if np.any(np.abs(np.abs(d) - np.pi) < 1e-6) or np.any(np.all(V == 0, axis=1)):
            continue
        k = int(np.rint(sum(d) / (2 * np.pi)))
        assert (k != 0) == bool(O.face_punctured(V))
        checked += 1


def test_moving_straight_line():
    x0, y0, vx, vy = 4.3, 3.6, 0.5, -0.25
    psi = _field(9, 9, 4, 5, lambda X, Y, Z, T: (X - x0 - vx * T, Y - y0 - vy * T))
    r = Vx.track_vortex(psi)
    assert r.n_components == 1
    t = r.pos[:, 3]
    assert np.all(np.abs(r.pos[:, 0] - (x0 + vx * t)) < 2e-6)
    assert np.all(np.abs(r.pos[:, 1] - (y0 + vy * t)) < 2e-6)
    # one positive triangle with all vertices in one (z, t) plane per plane
    types = O.kuhn_types(4, 2)
    planar = [i for i, (a, b) in enumerate(types) if not ((int(a) | int(b)) & 12)]
    ty = r.tri_id % 50
    gv = r.tri_id // 50
    z = (gv // 81) % 4
    tt = gv // (81 * 4)
    sel = np.isin(ty, planar)
    counts = np.zeros((5, 4), int)
    np.add.at(counts, (tt[sel], z[sel]), 1)
    assert np.all(counts == 1)
    assert set(np.nonzero(r.penta_counts)[0].tolist()) <= {0, 3, 4, 5}


@pytest.mark.parametrize("seed", [0, 1])
def test_tied_fields_tetrahedra_have_zero_or_two_positive_faces(seed):
    rng = np.random.default_rng(seed)
    psi = rng.integers(-1, 2, size=(3, 2, 3, 4, 4)).astype(np.float32) / np.float32(2 ** 20)
    r = Vx.track_vortex(psi)
    assert r.n_hits > 0
    assert set(np.nonzero(r.penta_counts)[0].tolist()) <= {0, 3, 4, 5}
    nt, nz, ny, nx = 3, 3, 4, 4
    pos = set(int(e) for e in r.tri_id)
    tri = {tuple(int(x) for x in row): i for i, row in enumerate(O.kuhn_types(4, 2))}
    for m1, m2, m3 in O.kuhn_types(4, 3):
        m1, m2, m3 = int(m1), int(m2), int(m3)
        span = m1 | m2 | m3
        for t in range(nt - (span >> 3 & 1)):
            for z in range(nz - (span >> 2 & 1)):
                for y in range(ny - (span >> 1 & 1)):
                    for x in range(nx - (span & 1)):
                        def gid(c):
                            return ((c[3] * nz + c[2]) * ny + c[1]) * nx + c[0]
                        p = (x, y, z, t)
                        p1 = tuple(p[k] + (m1 >> k & 1) for k in range(4))
                        faces = [gid(p1) * 50 + tri[(m2, m3)], gid(p) * 50 + tri[(m1 | m2, m3)],
                                 gid(p) * 50 + tri[(m1, m2 | m3)], gid(p) * 50 + tri[(m1, m2)]]
                        assert sum(f in pos for f in faces) in (0, 2)


def _rings(centres):
    def fn(X, Y, Z, T):
        re = np.ones_like(X) * 10.0
        im = np.zeros_like(X)
        for cx, cy, cz, R in centres:
            rho = np.sqrt((X - cx) ** 2 + (Y - cy) ** 2)
            near = (np.abs(X - cx) < R + 2.5) & (np.abs(Y - cy) < R + 2.5) & (np.abs(Z - cz) < 2.5)
            re = np.where(near, rho - R, re)
            im = np.where(near, Z - cz, im)
        return re, im
    return fn


def test_rings_are_closed_surfaces():
    r = Vx.track_vortex(_field(10, 10, 6, 3, _rings([(4.5, 4.5, 2.5, 2.2)])))
    assert r.n_components == 1
    r = Vx.track_vortex(_field(18, 9, 6, 3, _rings([(4.2, 4.5, 2.5, 2.2), (13.1, 4.4, 2.6, 2.0)])))
    assert r.n_components == 2
