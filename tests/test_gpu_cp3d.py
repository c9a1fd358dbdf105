"""GPU parity of the 3D path (ftk_track_cp3d through the C ABI) against the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_08697_amd import synth
from tests.parity import assert_full_parity, assert_pos_close, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2011_08697_amd as F  # noqa: E402

DEV = torch.device("cuda", 0)


def run(field, **kw):
    t = torch.from_numpy(np.ascontiguousarray(field)).to(DEV)
    r = F.track_cp3d(t, **kw)
    torch.cuda.synchronize()
    return r


@pytest.mark.parametrize("shape,seed,r", [((4, 4, 4, 3), 1, 2), ((17, 9, 5, 4), 2, 3), ((18, 10, 6, 3), 3, 1),
                                          ((2, 2, 2, 2), 4, 2), ((33, 3, 9, 5), 5, 2)])
def test_random_integer_scalar_fields(shape, seed, r):
    """Random small-integer scalars: gradients with many zero and equal components (SoS decides), ragged tiles."""
    nx, ny, nz, nt = shape
    rng = np.random.default_rng(seed)
    f = rng.integers(0, r + 1, size=(nt, nz, ny, nx)).astype(np.float32) * 2.0 ** -19
    assert_full_parity(run(f), O.track(f, n=3))


def test_blob_field_crop():
    f = synth.moving_gaussians_3d(40, 36, 20, 5, 24, seed=2)
    assert_full_parity(run(f), O.track(f, n=3))


def test_moving_minimum_3d():
    f = synth.moving_minimum(3, 21, [10, 10, 10], [0.25, -0.5, 0.75], 5)
    g = to_np(run(f))
    assert_full_parity(run(f), O.track(f, n=3))
    assert g["n_trajectories"] == 1 and np.all(g["type"] == 1)


def test_wide_path_3d():
    rng = np.random.default_rng(7)
    f = rng.integers(-3, 4, size=(3, 6, 7, 9)).astype(np.float32)  # gradient components up to 6: |q| >= 2^20
    g = run(f)
    assert g["stats"]["wide_path"] == 1
    assert_full_parity(g, O.track(f, n=3))


def test_precision_fp64_3d():
    f = synth.moving_gaussians_3d(24, 20, 18, 4, 10, seed=3)
    assert_full_parity(run(f, precision=1), O.track(f, n=3))


def test_errors_3d():
    f = np.zeros((3, 4, 4, 4), np.float32)
    f[1, 2, 2, 2] = np.inf
    with pytest.raises(F.FtkError) as e:
        run(f)
    assert e.value.status == 2


def test_full_size_blobs3d256_sampled():
    """256^3 x 16: sampled anchors (all 60 tetrahedra) and sampled hits against point queries of the oracle;
    labels of sampled hits by walking the trajectory through the pentachora."""
    f = synth.make("blobs3d256", device=DEV)
    g = to_np(run(f))
    fid = g["face_id"]
    assert g["n_hits"] > 0 and np.all(np.diff(fid) > 0)
    rng = np.random.default_rng(0)
    V = 256 * 256 * 256 * 16
    verts = rng.integers(0, V, 60)
    # anchors next to hits too (hits are sparse)
    verts = np.concatenate([verts, fid[rng.choice(len(fid), 40, replace=False)] // 60])
    cand = (verts[:, None] * 60 + np.arange(60)[None, :]).ravel()
    ev = O.eval_faces(f, cand, n=3)
    gpu_hit = np.isin(cand, fid)
    valid = ev["punctured"] != 255
    assert np.array_equal(gpu_hit[valid], ev["punctured"][valid].astype(bool))
    assert not np.any(gpu_hit[~valid])
    idx = rng.choice(len(fid), min(500, len(fid)), replace=False)
    ev = O.eval_faces(f, fid[idx], n=3)
    assert np.all(ev["punctured"] == 1)
    assert np.array_equal(g["type"][idx], ev["type"])
    assert np.array_equal(g["flags"][idx] & np.uint8(0xFD), ev["flags"])
    assert_pos_close(g["pos"][idx], ev["pos"])
    for i in rng.choice(len(fid), 10, replace=False):
        r = O.trace(f, int(fid[i]), n=3, max_steps=100000)
        assert r["closed"] != -1
        assert r["min_face"] == g["label"][i]


@pytest.mark.parametrize("case", range(15))
def test_quadratic_types_3d(case):
    """Quadratic forms of known inertia (Sec. 4.1): MIN, SADDLE1, SADDLE2 and MAX, with off-diagonal terms; full
    parity with the oracle and the expected type everywhere on the one trajectory."""
    from tests.test_oracle_track import QUAD3_CASES, quadratic_field_3d
    A, expect = QUAD3_CASES[case]
    f = quadratic_field_3d(A)
    g = to_np(run(f))
    assert_full_parity(run(f), O.track(f, n=3))
    assert g["n_trajectories"] == 1 and set(g["type"].tolist()) == {O.TYPES.index(expect)}
