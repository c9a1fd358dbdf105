"""Whole-configuration parity of the HIP path against the oracle (Alg. 1, Sec. 4.1-4.3, Eq. 2): every output of
the full-size workloads compared element by element, not sampled.

* 1024 x 1024 x 100 noisy blob series and its 16-level degenerate variant: every face id, type, flag and label,
  positions within 1e-5 relative.
* 4096 x 4096 x 50 vector series: every face whose vertices lie in steps 0-2 (the full spatial extent) against the
  oracle on those three steps (face set, positions, types, flags; a simplex's results depend only on its own
  vertices and their spatial stencils), labels of 200 sampled hits by walking their trajectories through the cells.
* 256^3 x 16 3D series: every face anchored in an interior 64^3 x 16 box against the oracle on the box plus a
  two-cell margin (the reach of the gradient and Jacobian stencils), labels of sampled hits by walking.
* The 96-series batch at full size in one batched call: 16 series spanning the size range against the oracle.
"""
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
FLAG_FP64 = 2
ORDINAL_2D = (0, 3)  # triangle types (x, y) and (y, x): no time axis


def gpu(field, n=2, kind=0):
    t = torch.from_numpy(np.ascontiguousarray(field)).to(DEV)
    r = F.track_cp2d(t, kind=kind) if n == 2 else F.track_cp3d(t)
    torch.cuda.synchronize()
    del t
    return to_np(r)


@pytest.mark.parametrize("name", ["noise1024", "levels1024"])
def test_full_config_2d_every_output(name):
    f = synth.make(name)
    g = gpu(f)
    ref = O.track(f)
    assert ref.status == 0 and ref.invariant_violations == 0
    assert_full_parity(g, ref)


def test_full_config_vortex4096_first_three_steps_and_traced_labels():
    u = synth.make("vortex4096", device=DEV)
    g = gpu(u, kind=1)
    fid = g["face_id"]
    nx = ny = 4096
    plane = nx * ny
    t = fid // 12 // plane
    ty = fid % 12
    sel = (t <= 1) | ((t == 2) & np.isin(ty, ORDINAL_2D))
    ref = O.track(np.ascontiguousarray(u[:3]), n=2, kind=1)
    assert ref.status == 0
    assert np.array_equal(fid[sel], ref.face_id)
    assert np.array_equal(g["type"][sel], ref.type)
    assert np.array_equal(g["flags"][sel] & np.uint8(0xFF ^ FLAG_FP64), ref.flags)
    assert_pos_close(g["pos"][sel], ref.pos)
    rng = np.random.default_rng(40)
    for i in rng.choice(len(fid), 200, replace=False):
        r = O.trace(u, int(fid[i]), kind=1, max_steps=1 << 22)
        assert r["closed"] != -1
        assert r["min_face"] == g["label"][i]


def _decode3(fid, dims):
    g = fid // 60
    x = g % dims[0]
    g //= dims[0]
    y = g % dims[1]
    g //= dims[1]
    z = g % dims[2]
    return x, y, z, g // dims[2], fid % 60


def test_full_config_blobs3d256_interior_box():
    f = synth.make("blobs3d256", device=DEV)
    g = gpu(f, n=3)
    B, M = 64, 2          # box of anchors, stencil margin
    lo = 96               # first anchor of the box on every spatial axis
    off = lo - M          # crop origin
    C = B + 2 * M         # crop width (vertices off .. off + C - 1)
    crop = np.ascontiguousarray(f[:, off:off + C, off:off + C, off:off + C])
    ref = O.track(crop, n=3)
    assert ref.status == 0
    # faces anchored at crop coordinates [M, M + B - 1]: their vertices (anchor + 0/1) have central stencils in
    # the crop for the gradient (reach 1) and the Jacobian (reach 2), identical to the full field's
    x, y, z, t, ty = _decode3(g["face_id"], (256, 256, 256))
    gs = (x >= lo) & (x < lo + B) & (y >= lo) & (y < lo + B) & (z >= lo) & (z < lo + B)
    cx, cy, cz, ct, cty = _decode3(ref.face_id, (C, C, C))
    cs = (cx >= M) & (cx < M + B) & (cy >= M) & (cy < M + B) & (cz >= M) & (cz < M + B)
    assert cs.sum() > 500
    mapped = ((((t[gs] * C + (z[gs] - off)) * C + (y[gs] - off)) * C + (x[gs] - off)) * 60 + ty[gs])
    assert np.array_equal(mapped, ref.face_id[cs])
    assert np.array_equal(g["type"][gs], ref.type[cs])
    assert np.array_equal(g["flags"][gs] & np.uint8(0xFF ^ FLAG_FP64), ref.flags[cs])
    shifted = ref.pos[cs] + np.array([off, off, off, 0], np.float64)
    assert_pos_close(g["pos"][gs], shifted)
    rng = np.random.default_rng(2)
    idx = np.flatnonzero(gs)
    for i in rng.choice(idx, 30, replace=False):
        r = O.trace(f, int(g["face_id"][i]), n=3, max_steps=1 << 20)
        assert r["closed"] != -1
        assert r["min_face"] == g["label"][i]


def test_full_config_batch96_spanning_series():
    fields = synth.batch_series(count=96, seed0=3, device=DEV)
    ts = [torch.from_numpy(f).to(DEV) for f in fields]
    res = F.track_cp2d_batched(ts)
    torch.cuda.synchronize()
    del ts
    order = np.argsort([f.size for f in fields])
    for i in order[::6]:  # 16 series from 0.5M to 74M vertices
        assert_full_parity(res[i], O.track(fields[i]))
