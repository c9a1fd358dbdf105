"""GPU parity of the streaming form (ftk_cp_create / push / finish): identical to the one-shot call."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_08697_amd import synth
from tests.parity import assert_full_parity, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2011_08697_amd as F  # noqa: E402

DEV = torch.device("cuda", 0)
KEYS = ("face_id", "pos", "type", "flags", "label")


def _stream(field, n, kind=0, **kw):
    f = torch.from_numpy(np.ascontiguousarray(field)).to(DEV)
    dims = list(field.shape[::-1][: n]) if kind == 0 else list(field.shape[2:][::-1])
    tr = F.Tracker(n, dims, kind=kind, **kw)
    for t in range(field.shape[0]):
        tr.push(f[t].contiguous())
    r = tr.finish()
    tr.close()
    return r


def _same(a, b):
    a, b = to_np(a), to_np(b)
    assert a["n_hits"] == b["n_hits"] and a["n_trajectories"] == b["n_trajectories"]
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("shape,seed", [((130, 70, 9), 1), ((64, 64, 2), 2), ((200, 33, 17), 3)])
def test_stream_2d_equals_one_shot_and_oracle(shape, seed):
    nx, ny, nt = shape
    f = synth.moving_gaussians_2d(nx, ny, nt, 10, seed=seed, noise_std=1e-3)
    r = _stream(f, 2)
    _same(r, F.track_cp2d(torch.from_numpy(f).to(DEV)))
    assert_full_parity(r, O.track(f))


def test_stream_2d_vector_and_degenerate():
    u = synth.vortex_sources_2d(96, 80, 7, 12, seed=5)
    _same(_stream(u, 2, kind=1), F.track_cp2d(torch.from_numpy(u).to(DEV), kind=1))
    rng = np.random.default_rng(3)
    v = rng.integers(-1, 2, size=(6, 2, 20, 70)).astype(np.float32)
    r = _stream(v, 2, kind=1)
    assert_full_parity(r, O.track(v, n=2, kind=1))


def test_stream_3d():
    f = synth.moving_gaussians_3d(30, 20, 18, 5, 8, seed=4)
    r = _stream(f, 3)
    _same(r, F.track_cp3d(torch.from_numpy(f).to(DEV)))
    assert_full_parity(r, O.track(f, n=3))


def test_stream_3d_longer_than_the_window():
    """The 3D tracker keeps a window of three steps (Sec. 3.2: every simplex lies within two consecutive steps):
    a series several times longer than the window, with ragged tiles and integer-valued ties, equals the one-shot
    call and the oracle, and the tracker's device memory does not grow with the number of steps pushed."""
    f = synth.moving_gaussians_3d(19, 13, 10, 11, 6, seed=8)
    r = _stream(f, 3)
    _same(r, F.track_cp3d(torch.from_numpy(f).to(DEV)))
    assert_full_parity(r, O.track(f, n=3))
    rng = np.random.default_rng(9)
    g = (rng.integers(0, 3, size=(9, 5, 6, 7)) * 2.0 ** -19).astype(np.float32)
    assert_full_parity(_stream(g, 3), O.track(g, n=3))
    # memory held by the tracker itself (window, masks, offsets) after 3 and after 12 pushed steps of a field
    # without hits: equal (outputs grow only with the hits)
    z = torch.zeros((10, 12, 16), device=DEV)  # one step [nz][ny][nx]
    tr = F.Tracker(3, [16, 12, 10])
    held = []
    for t in range(12):
        tr.push(z)
        if t in (2, 11):
            torch.cuda.synchronize()
            held.append(sum(v.numel() for v in tr.pool.live.values()))
    tr.finish()
    tr.close()
    assert held[0] == held[1]


def test_stream_state_errors():
    tr = F.Tracker(2, [16, 16])
    tr.push(torch.zeros((16, 16), device=DEV))
    with pytest.raises(F.FtkError) as e:
        tr.finish()  # a single step
    assert e.value.status == 8
    tr.close()
    tr = F.Tracker(2, [16, 16])
    for _ in range(3):
        tr.push(torch.rand((16, 16), device=DEV))
    tr.finish()
    with pytest.raises(F.FtkError) as e:
        tr.push(torch.zeros((16, 16), device=DEV))
    assert e.value.status == 8
    tr.close()
