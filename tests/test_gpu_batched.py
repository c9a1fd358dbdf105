"""GPU parity of the batched form (ftk_track_cp2d_batched): every series equals its plain call bit for bit and
matches the oracle."""
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


def _same(a, b):
    a, b = to_np(a), to_np(b)
    assert a["n_hits"] == b["n_hits"] and a["n_trajectories"] == b["n_trajectories"]
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k


def test_small_batch_matches_oracle_and_plain_calls():
    # uneven sizes (ragged tiles), lengths 2..9, the batch recipe on small grids
    fields = synth.batch_series(count=9, seed0=100, size_range=(24, 150), nt_range=(2, 9), k_range=(2, 12))
    fields.append(np.zeros((3, 5, 7), np.float32))  # a series without hits
    ts = [torch.from_numpy(f).to(DEV) for f in fields]
    res = F.track_cp2d_batched(ts)
    torch.cuda.synchronize()
    for f, t, r in zip(fields, ts, res):
        assert_full_parity(r, O.track(f))
        _same(r, F.track_cp2d(t))


def test_vector_batch():
    fields = [synth.vortex_sources_2d(n, m, k, 6, seed=s) for n, m, k, s in [(40, 33, 4, 1), (90, 70, 3, 2),
                                                                          (65, 64, 5, 3)]]
    ts = [torch.from_numpy(f).to(DEV) for f in fields]
    res = F.track_cp2d_batched(ts, kind=F.VECTOR)
    for f, r in zip(fields, res):
        assert_full_parity(r, O.track(f, n=2, kind=1))


def test_batch_of_96_uneven_series_equals_plain_calls():
    """The batched workload's shape recipe (96 series, 128-2048 squared, 8-64 steps) with sizes divided by 4 so the
    test stays short; every series must equal its plain call."""
    fields = synth.batch_series(count=96, seed0=3, size_range=(32, 512), nt_range=(8, 64), k_range=(4, 128),
                                device=DEV)
    ts = [torch.from_numpy(f).to(DEV) for f in fields]
    res = F.track_cp2d_batched(ts)
    torch.cuda.synchronize()
    for t, r in zip(ts, res):
        _same(r, F.track_cp2d(t))
    # and a few against the oracle
    for i in (0, 17, 63):
        assert_full_parity(res[i], O.track(fields[i]))
