"""Pins of the isovolume oracle (oracle/iso.py) against what the paper and geometry fix: the paper's moving plane
f = x - alpha t (Sec. 6.3) with its closed-form trajectory x = alpha t, the total 3-volume of the tessellation for
planes whose section of the grid box has a closed-form volume, the tessellation as a 3-manifold whose faces are
shared by two tetrahedra except on the grid boundary (conforming case II splits), and the tie rule (a vertex
exactly at the isovalue counts as above it)."""
import collections

import numpy as np
import pytest

from oracle import iso


def _linear(nx, ny, nz, nt, fn):
    X, Y, Z, T = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64),
                             np.arange(nz, dtype=np.float64), np.arange(nt, dtype=np.float64), indexing="ij")
    return np.transpose(fn(X, Y, Z, T), (3, 2, 1, 0)).astype(np.float32)


def _volume(r):
    return sum(iso.tet_volume(r.pos[t]) for t in r.tets)


def _decode(eid, dims):
    nx, ny, nz, nt = dims
    M = eid % 15 + 1
    g = eid // 15
    a = (g % nx, (g // nx) % ny, (g // (nx * ny)) % nz, g // (nx * ny * nz))
    return a, tuple(a[k] + ((M >> k) & 1) for k in range(4))


def test_moving_plane_closed_form():
    """f = x - 0.9 t on 21^3 x 12 (the paper's synthetic case): one isovolume, every point on x = alpha t, and its
    3-volume is that of the plane's section of the box, 20 * 20 * 11 * sqrt(1 + alpha^2)."""
    alpha = 0.9
    f = _linear(21, 21, 21, 12, lambda X, Y, Z, T: X - alpha * T)
    r = iso.track_iso(f, 0.0)
    assert r.n_components == 1
    assert np.all(np.abs(r.pos[:, 0] - alpha * r.pos[:, 3]) < 1e-6)  # field stored in binary32
    assert abs(_volume(r) - 20 * 20 * 11 * np.sqrt(1 + alpha ** 2)) < 1e-8 * 6000


@pytest.mark.parametrize("case", ["diagonal", "tilted_in_time"])
def test_tessellation_volume(case):
    if case == "diagonal":   # x + y = 8 in [0, 8]^2: a segment of length 8 sqrt 2, times z in [0, 8], t in [0, 3]
        f = _linear(9, 9, 9, 4, lambda X, Y, Z, T: X + Y - 8.0)
        want = 8 * np.sqrt(2) * 8 * 3
    else:                    # z = 4 - t / 2 over x, y in [0, 6], t in [0, 4]: area element sqrt(1 + 1/4)
        f = _linear(7, 7, 9, 5, lambda X, Y, Z, T: Z + 0.5 * T - 4.0)
        want = 6 * 6 * 4 * np.sqrt(1.25)
    r = iso.track_iso(f, 0.0)
    assert r.n_components == 1
    assert abs(_volume(r) - want) < 1e-9 * want


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tessellation_is_a_manifold_on_tied_fields(seed):
    """Values in {-1, 0, 1} at isovalue 0 (every zero vertex a tie): every triangle of the tessellation bounds two
    tetrahedra, or one when it lies in a boundary hyperplane of the grid."""
    rng = np.random.default_rng(seed)
    f = rng.integers(-1, 2, size=(4, 4, 5, 5)).astype(np.float32)
    nt, nz, ny, nx = f.shape
    dims = (nx, ny, nz, nt)
    r = iso.track_iso(f, 0.0)
    assert len(r.tets) > 1000
    cnt = collections.Counter()
    for tet in r.tets:
        for drop in range(4):
            cnt[tuple(sorted(int(tet[i]) for i in range(4) if i != drop))] += 1
    for face, k in cnt.items():
        assert k in (1, 2)
        if k == 1:
            verts = [v for h in face for v in _decode(int(r.edge_id[h]), dims)]
            assert any(all(v[a] == 0 for v in verts) or all(v[a] == dims[a] - 1 for v in verts) for a in range(4))


def test_tie_counts_as_above():
    """A vertex exactly at the isovalue lies above it: among values above, no edge crosses; among values below,
    each of the 30 edges at an interior tied vertex crosses, at the vertex itself."""
    f = np.ones((5, 5, 5, 5), np.float32)
    f[2, 2, 2, 2] = 0.0
    assert iso.track_iso(f, 0.0).n_hits == 0
    f = -np.ones((5, 5, 5, 5), np.float32)
    f[2, 2, 2, 2] = 0.0
    r = iso.track_iso(f, 0.0)
    assert r.n_hits == 30 and r.n_components == 1
    assert np.all(r.pos == 2.0)


def test_two_separate_blobs_are_two_isovolumes():
    def fn(X, Y, Z, T):
        a = np.exp(-((X - 3 - 0.3 * T) ** 2 + (Y - 4) ** 2 + (Z - 4) ** 2) / 4.0)
        b = np.exp(-((X - 12) ** 2 + (Y - 4) ** 2 + (Z - 4 + 0.2 * T) ** 2) / 4.0)
        return a + b
    r = iso.track_iso(_linear(16, 9, 9, 4, fn), 0.5)
    assert r.n_components == 2
    assert len(np.unique(r.label)) == 2
