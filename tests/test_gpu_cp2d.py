"""GPU parity of the 2D path (ftk_track_cp2d through the C ABI) against the oracle."""
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


def run(field, kind=0, **kw):
    t = torch.from_numpy(np.ascontiguousarray(field)).to(DEV)
    r = F.track_cp2d(t, kind=kind, **kw)
    torch.cuda.synchronize()
    return r


def test_blobs64_full_parity():
    f = synth.make("blobs64")
    assert_full_parity(run(f), O.track(f))


@pytest.mark.parametrize("shape,seed,r", [((5, 5, 4), 1, 1), ((70, 9, 5), 2, 1), ((130, 37, 7), 3, 2),
                                          ((64, 16, 17), 4, 1), ((65, 17, 18), 5, 3), ((2, 2, 2), 6, 1),
                                          ((3, 100, 3), 7, 1)])
def test_degenerate_integer_vectors(shape, seed, r):
    """Random small-integer vector fields: most determinants vanish, SoS decides; ragged tiles in x, y and t."""
    nx, ny, nt = shape
    rng = np.random.default_rng(seed)
    u = rng.integers(-r, r + 1, size=(nt, 2, ny, nx)).astype(np.float32)
    assert_full_parity(run(u, kind=1), O.track(u, n=2, kind=1))


@pytest.mark.parametrize("tile_y,slab", [(8, 3), (16, 0), (32, 5)])
def test_noise_crop_tilings(tile_y, slab):
    """Noisy blob field (the large benchmark's recipe on a crop): dense hits, long and short trajectories."""
    f = synth.moving_gaussians_2d(200, 150, 12, 12, seed=1, noise_std=1e-3)
    assert_full_parity(run(f, tile_y=tile_y, slab_depth=slab), O.track(f))


def test_sixteen_level_degenerate_crop():
    f = synth.quantise_levels(synth.moving_gaussians_2d(257, 131, 9, 16, seed=1, noise_std=1e-3))
    assert_full_parity(run(f), O.track(f))


def test_vector_field_sources_vortices_crop():
    u = synth.vortex_sources_2d(300, 220, 6, 24, seed=4)
    assert_full_parity(run(u, kind=1), O.track(u, n=2, kind=1))


def test_moving_minimum_2d():
    f = synth.moving_minimum(2, 21, [10, 10], [0.375, -0.625], 9)
    g = to_np(run(f))
    tr = O.track(f)
    assert_full_parity(run(f), tr)
    assert g["n_trajectories"] == 1 and np.all(g["type"] == 1)


def test_precision_fp64_mode():
    f = synth.moving_gaussians_2d(96, 80, 8, 10, seed=5, noise_std=1e-3)
    assert_full_parity(run(f, precision=1), O.track(f))


def test_wide_path_and_range_error():
    rng = np.random.default_rng(11)
    u = (rng.integers(-3, 4, size=(4, 2, 20, 70)) * 2.0 ** 12).astype(np.float32)  # |q| up to 3 * 2^32
    g = run(u, kind=1)
    assert g["stats"]["wide_path"] == 1
    assert_full_parity(g, O.track(u, n=2, kind=1))
    u[1, 0, 3, 5] = 2.0 ** 43  # |q| = 2^63 > 2^62
    with pytest.raises(F.FtkError) as e:
        run(u, kind=1)
    assert e.value.status == 3


def test_errors():
    f = synth.make("blobs64")
    f[3, 10, 10] = np.nan
    with pytest.raises(F.FtkError) as e:
        run(f)
    assert e.value.status == 2
    with pytest.raises(F.FtkError) as e:
        run(np.zeros((4, 1, 8), np.float32))
    assert e.value.status == 1


def test_all_zero_and_constant_fields():
    g = to_np(run(np.zeros((5, 33, 70), np.float32)))
    assert g["n_hits"] == 0 and g["n_trajectories"] == 0


def test_outputs_subset():
    f = synth.make("blobs64")
    g = run(f, outputs=F.OUT_POS)
    assert g["type"] is None and g["label"] is None and g["pos"] is not None
    tr = O.track(f)
    assert np.array_equal(g["face_id"].cpu().numpy(), tr.face_id)


def test_determinism_repeated_runs():
    f = synth.moving_gaussians_2d(256, 200, 10, 16, seed=9, noise_std=1e-3)
    a = to_np(run(f))
    for _ in range(3):
        b = to_np(run(f))
        for k in ("face_id", "pos", "type", "flags", "label"):
            assert np.array_equal(a[k], b[k])


def test_full_size_noise1024_sampled():
    """1024 x 1024 x 100 (the benchmark workload): every GPU output checked at sampled vertices and hits against
    point queries of the oracle, plus the trajectory of sampled hits traced through the cells."""
    f = synth.make("noise1024")
    g = to_np(run(f))
    fid = g["face_id"]
    assert np.all(np.diff(fid) > 0)
    rng = np.random.default_rng(0)
    # completeness and exactness at sampled anchors: all 12 triangles of each sampled vertex
    V = 1024 * 1024 * 100
    verts = rng.integers(0, V, 400)
    cand = (verts[:, None] * 12 + np.arange(12)[None, :]).ravel()
    ev = O.eval_faces(f, cand)
    gpu_hit = np.isin(cand, fid)
    valid = ev["punctured"] != 255
    assert np.array_equal(gpu_hit[valid], ev["punctured"][valid].astype(bool))
    assert not np.any(gpu_hit[~valid])
    # sampled hits: position, type, flags
    idx = rng.choice(len(fid), 3000, replace=False)
    ev = O.eval_faces(f, fid[idx])
    assert np.all(ev["punctured"] == 1)
    assert np.array_equal(g["type"][idx], ev["type"])
    assert np.array_equal(g["flags"][idx] & np.uint8(0xFD), ev["flags"])
    assert_pos_close(g["pos"][idx], ev["pos"])
    # labels: smallest face id on the component reached by walking the cells
    for i in rng.choice(len(fid), 40, replace=False):
        r = O.trace(f, int(fid[i]), max_steps=200000)
        assert r["closed"] != -1
        assert r["min_face"] == g["label"][i]


def test_full_size_vortex4096_sampled():
    """4096 x 4096 x 50 vector field (the precision workload) in the benchmark's launch configuration: completeness
    at sampled vertices, outputs of sampled hits and labels of sampled trajectories against the oracle."""
    u = synth.make("vortex4096", device=DEV)
    g = to_np(run(u, kind=1))
    fid = g["face_id"]
    assert len(fid) > 0 and np.all(np.diff(fid) > 0)
    rng = np.random.default_rng(4)
    V = 4096 * 4096 * 50
    verts = rng.integers(0, V, 400)
    cand = (verts[:, None] * 12 + np.arange(12)[None, :]).ravel()
    ev = O.eval_faces(u, cand, kind=1)
    gpu_hit = np.isin(cand, fid)
    valid = ev["punctured"] != 255
    assert np.array_equal(gpu_hit[valid], ev["punctured"][valid].astype(bool))
    assert not np.any(gpu_hit[~valid])
    idx = rng.choice(len(fid), min(3000, len(fid)), replace=False)
    ev = O.eval_faces(u, fid[idx], kind=1)
    assert np.all(ev["punctured"] == 1)
    assert np.array_equal(g["type"][idx], ev["type"])
    assert np.array_equal(g["flags"][idx] & np.uint8(0xFD), ev["flags"])
    assert_pos_close(g["pos"][idx], ev["pos"])
    for i in rng.choice(len(fid), 20, replace=False):
        r = O.trace(u, int(fid[i]), kind=1, max_steps=400000)
        assert r["closed"] != -1
        assert r["min_face"] == g["label"][i]


def test_all_outputs_with_mu():
    f = synth.moving_gaussians_2d(150, 90, 7, 9, seed=12, noise_std=1e-3)
    g = run(f, outputs=F.OUT_ALL)
    assert g["mu"] is not None
    assert_full_parity(g, O.track(f))


def test_autotune_picks_a_candidate_and_keeps_parity():
    """The tuned tiling (remembered for the shape and used by the default call) changes no result."""
    f = synth.moving_gaussians_2d(150, 90, 10, 10, seed=5, noise_std=1e-3)
    t = torch.from_numpy(np.ascontiguousarray(f)).to(DEV)
    ty, tt = F.autotune_cp2d(t)
    assert ty in (8, 16, 32) and tt in (8, 10)  # slab depths clamp to nt = 10
    assert_full_parity(run(f), O.track(f))
