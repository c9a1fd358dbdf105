"""Shared comparison helpers for the GPU parity tests (HIP path vs the oracle)."""
import numpy as np

# Sublocation tolerance: |x32 - x64| <= 1e-5 * max(1, |x64|) per component (FP32 result vs binary64 reference).
POS_RTOL = 1e-5
FLAG_FP64 = 2  # implementation-only flag (which precision decided the type); not part of parity


def to_np(gpu):
    out = {}
    for k, v in gpu.items():
        if hasattr(v, "cpu"):
            out[k] = v.cpu().numpy()
        else:
            out[k] = v
    return out


def assert_pos_close(pos32, pos64):
    pos32 = np.asarray(pos32, np.float64)
    err = np.abs(pos32 - pos64)
    tol = POS_RTOL * np.maximum(1.0, np.abs(pos64))
    bad = np.argwhere(err > tol)
    assert bad.size == 0, f"{len(bad)} position components beyond tolerance, worst {err.max():.3g}"


def assert_full_parity(gpu, orc):
    g = to_np(gpu)
    assert g["n_hits"] == orc.n_hits, (g["n_hits"], orc.n_hits)
    assert np.array_equal(g["face_id"], orc.face_id)
    assert np.array_equal(g["type"], orc.type)
    assert np.array_equal(g["flags"] & np.uint8(0xFF ^ FLAG_FP64), orc.flags)
    assert np.array_equal(g["label"], orc.label)
    assert g["n_trajectories"] == orc.n_traj
    assert_pos_close(g["pos"], orc.pos)
    if g.get("mu") is not None:
        assert np.all(np.abs(g["mu"] - orc.mu) <= 1e-5)


def face_vertices(fid, n, dims):
    """Vertex coordinates (x, y, [z], t) of a face, decoded from its id (t-major anchor index times the type count
    plus the type) and the type's axis masks."""
    from oracle import oracle as O
    T = 12 if n == 2 else 60
    masks = O.kuhn_types(n + 1, n)[fid % T]
    g = fid // T
    c = []
    for a in range(n):
        c.append(g % dims[a])
        g //= dims[a]
    c.append(g)
    vs = [tuple(c)]
    for m in masks:
        v = list(vs[-1])
        for a in range(n + 1):
            if (int(m) >> a) & 1:
                v[a] += 1
        vs.append(tuple(v))
    return vs


def share_a_cell(f1, f2, n, dims):
    """Two faces are sides of one cell: their vertices together form a unit-step chain across one unit cube."""
    vs = sorted(set(face_vertices(f1, n, dims)) | set(face_vertices(f2, n, dims)), key=sum)
    if len(vs) != n + 2:
        return False
    steps = [np.subtract(vs[k + 1], vs[k]) for k in range(n + 1)]
    return all(s.min() == 0 and s.sum() == 1 for s in steps) and np.array_equal(np.subtract(vs[-1], vs[0]),
                                                                                np.ones(n + 1))
