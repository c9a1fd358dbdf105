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
