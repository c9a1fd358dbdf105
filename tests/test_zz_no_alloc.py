"""The 2D call that allocates nothing (ftk_track_cp2d_into, for callers that cannot allocate): through the C ABI,
its results equal ftk_track_cp2d's on consecutive calls that share the library's static scratch region (the second
call smaller than the first, so stale scratch of the first must not leak into it), and sizes beyond the region or
the caller's capacity are refused with FTK_ERR_CAPACITY."""
import numpy as np
import pytest

from paper_2011_08697_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2011_08697_amd as F  # noqa: E402

DEV = torch.device("cuda", 0)
KEYS = ("face_id", "pos", "mu", "type", "flags", "label")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def assert_same(a, b):
    assert a["n_hits"] == b["n_hits"] and a["n_trajectories"] == b["n_trajectories"]
    for k in KEYS:
        x, y = a[k], b[k]
        assert (x is None) == (y is None), k
        if x is not None:
            assert torch.equal(x.cpu(), y.cpu()), k
    for k in ("simplices_tested", "cells_linked", "fp64_fallbacks", "degenerate_sublocations", "wide_path"):
        assert a["stats"][k] == b["stats"][k], k


CASES = [
    # (field, kind): a large noisy scalar series first, then smaller ones
    lambda: (synth.moving_gaussians_2d(300, 260, 14, 16, seed=1, noise_std=1e-3), 0),
    lambda: (synth.moving_gaussians_2d(97, 70, 9, 6, seed=5), 0),
    lambda: (synth.vortex_sources_2d(150, 110, 7, 10, seed=4), 1),
    lambda: (synth.quantise_levels(synth.moving_gaussians_2d(130, 90, 8, 9, seed=2, noise_std=1e-3)), 0),
]


def test_two_calls_in_a_row_match_the_allocating_call():
    for first, second in [(0, 1), (0, 3), (2, 1)]:
        fa, ka = CASES[first]()
        fb, kb = CASES[second]()
        assert fb.size < fa.size
        ra, rb = F.track_cp2d(dev(fa), kind=ka, outputs=F.OUT_ALL), F.track_cp2d(dev(fb), kind=kb, outputs=F.OUT_ALL)
        cap = max(ra["n_hits"], rb["n_hits"]) + 5
        out = dict(face_id=torch.empty(cap, dtype=torch.int64, device=DEV),
                   pos=torch.full((cap, 3), -1.0, dtype=torch.float32, device=DEV),
                   mu=torch.full((cap, 3), -1.0, dtype=torch.float32, device=DEV),
                   type=torch.full((cap,), 255, dtype=torch.uint8, device=DEV),
                   flags=torch.full((cap,), 255, dtype=torch.uint8, device=DEV),
                   label=torch.full((cap,), -1, dtype=torch.int64, device=DEV))
        for f, k, ref in ((fa, ka, ra), (fb, kb, rb)):  # the same caller arrays and scratch region twice
            g = F.track_cp2d_into(dev(f), kind=k, out=out, outputs=F.OUT_ALL)
            torch.cuda.synchronize()
            assert_same(g, ref)


def test_default_outputs_and_reused_arrays():
    f, k = CASES[1]()
    ref = F.track_cp2d(dev(f), kind=k)
    cap = ref["n_hits"] + 100
    out = dict(face_id=torch.empty(cap, dtype=torch.int64, device=DEV),
               pos=torch.empty((cap, 3), dtype=torch.float32, device=DEV),
               type=torch.empty(cap, dtype=torch.uint8, device=DEV),
               flags=torch.empty(cap, dtype=torch.uint8, device=DEV),
               label=torch.empty(cap, dtype=torch.int64, device=DEV))
    for _ in range(2):
        g = F.track_cp2d_into(dev(f), kind=k, out=out)
        torch.cuda.synchronize()
        assert g["mu"] is None
        assert_same(g, ref)


def test_capacity_and_region_limits():
    f, k = CASES[1]()
    ref = F.track_cp2d(dev(f), kind=k)
    with pytest.raises(F.FtkError) as e:
        F.track_cp2d_into(dev(f), kind=k, capacity=ref["n_hits"] - 1)
    assert e.value.status == 4 and f"n_hits {ref['n_hits']}" in str(e.value)
    # 2 bytes of puncture mask per vertex alone exceed the region: refused before any device work
    big = torch.zeros((9, 4096, 4096), dtype=torch.float32, device=DEV)
    assert 2 * big.numel() > F.STATIC_SCRATCH_BYTES
    with pytest.raises(F.FtkError) as e:
        F.track_cp2d_into(big, capacity=16)
    assert e.value.status == 4 and "static region" in str(e.value)
    # the region is usable again afterwards
    assert_same(F.track_cp2d_into(dev(f), kind=k, capacity=ref["n_hits"]), ref)
