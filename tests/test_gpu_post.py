"""GPU parity of the trajectory post-processing (ftk_traj_table_build, ftk_cp_slice, ftk_cp_filter_loops through the
C ABI) against the oracle's post-processing of the oracle's own run on the same fields."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import post as P
from paper_2011_08697_amd import synth
from parity import share_a_cell

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2011_08697_amd as F  # noqa: E402

DEV = torch.device("cuda", 0)


def _track(f, n, kind=0):
    t = torch.from_numpy(np.ascontiguousarray(f)).to(DEV)
    r = F.track_cp2d(t, kind=kind) if n == 2 else F.track_cp3d(t)
    torch.cuda.synchronize()
    return r


def _dims(f, n, kind=0):
    if n == 2:
        return (f.shape[-1], f.shape[-2], f.shape[0])
    return (f.shape[3], f.shape[2], f.shape[1], f.shape[0])


def _check_table(g, o):
    assert g["n"] == o["n"]
    assert np.array_equal(g["label"].cpu().numpy(), o["label"])
    assert np.array_equal(g["n_points"].cpu().numpy(), o["n_points"])
    assert np.array_equal(g["n_ends"].cpu().numpy(), o["n_ends"])
    for k in ("t_min", "t_max"):  # FP32 positions against the oracle's binary64 ones
        gv = g[k].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(gv - o[k]) <= 1e-5 * np.maximum(1.0, np.abs(o[k]))), k


CASES = {
    "blobs64": lambda: (synth.make("blobs64"), 2, 0),
    "noise_crop": lambda: (synth.moving_gaussians_2d(200, 150, 12, 12, seed=1, noise_std=1e-3), 2, 0),
    "vector": lambda: (synth.vortex_sources_2d(96, 80, 9, 12, seed=4), 2, 1),
    "3d": lambda: (synth.moving_gaussians_3d(24, 20, 18, 5, 6, seed=2), 3, 0),
}


@pytest.mark.parametrize("case", list(CASES))
def test_table_slices_and_filter_match_oracle(case):
    f, n, kind = CASES[case]()
    dims = _dims(f, n, kind)
    g = _track(f, n, kind)
    tr = O.track(f, n=n, kind=kind)
    assert g["n_hits"] == tr.n_hits and g["n_trajectories"] == tr.n_traj
    tab_o = P.traj_table(tr, n, dims)
    tab_g = F.trajectory_table(g, dims)
    _check_table(tab_g, tab_o)
    assert set(np.unique(tab_o["n_ends"]).tolist()) <= {0, 2}
    for t0 in range(dims[-1]):
        gi = F.slice_at(g, dims, t0).cpu().numpy()
        assert np.array_equal(gi, P.slice_at(tr, n, dims, t0)), t0
    # loop filter at thresholds that fall between loop durations (FP32 vs binary64 extents cannot straddle them)
    dur = np.unique(np.round((tab_o["t_max"] - tab_o["t_min"])[tab_o["n_ends"] == 0], 6))
    cuts = [0.0, 1e9] + ([float(dur[len(dur) // 2]) + 1e-3] if len(dur) else [])
    for c in cuts:
        assert np.array_equal(F.filter_loops(g, tab_g, c).cpu().numpy(), P.filter_loops(tr, tab_o, c)), c


def test_birth_death_loop_is_filtered():
    nx, ny, nt = 33, 17, 21
    X = np.arange(nx, dtype=np.float64) - 16.0
    Y = np.arange(ny, dtype=np.float64) - 8.0
    f = np.zeros((nt, ny, nx))
    for t in range(nt):
        f[t] = (X[None, :] ** 3) / 3.0 - (30.0 - 0.5 * (t - 10.0) ** 2) * X[None, :] + (Y[:, None] ** 2)
    f = f.astype(np.float32)
    g = _track(f, 2)
    tab = F.trajectory_table(g, (nx, ny, nt))
    assert tab["n"] == 1 and int(tab["n_ends"][0]) == 0
    dur = float(tab["t_max"][0] - tab["t_min"][0])
    assert int(F.filter_loops(g, tab, dur + 0.5).sum()) == 0
    assert int(F.filter_loops(g, tab, dur - 0.5).sum()) == g["n_hits"]


def test_empty_result_and_argument_errors():
    f = np.zeros((4, 9, 10), np.float32)
    g = _track(f, 2)
    assert g["n_hits"] == 0
    tab = F.trajectory_table(g, (10, 9, 4))
    assert tab["n"] == 0
    assert F.slice_at(g, (10, 9, 4), 2).numel() == 0
    assert F.filter_loops(g, tab, 1.0).numel() == 0
    with pytest.raises(F.FtkError):
        F.slice_at(g, (10, 9, 4), 4)  # t0 outside [0, nt)
    with pytest.raises(ValueError):
        F.trajectory_table(g, (10, 9))  # wrong dimension count


def _check_simplified(got, order, offsets, is_loop, types, t, theta, delta=1e-3):
    """Device runs have FP32 time extents, the oracle's binary64 ones (positions agree to 1e-5 relative, so extents
    to about 2.4e-4 at t <= 12).  Where the oracle's decision is the same at theta - delta, theta and theta + delta
    the device must agree with it; where a run extent lies within delta of the threshold either side is accepted."""
    outs = [P.simplify_types(order, offsets, is_loop, types, t, x) for x in (theta - delta, theta, theta + delta)]
    ok = (got == outs[0]) | (got == outs[1]) | (got == outs[2])
    assert np.all(ok), int((~ok).sum())
    firm = (outs[0] == outs[1]) & (outs[1] == outs[2])
    assert np.array_equal(got[firm], outs[1][firm])
    assert firm.mean() > 0.95  # the comparison still covers nearly every point


@pytest.mark.parametrize("case", list(CASES))
def test_order_smoothing_and_simplification_match_oracle(case):
    f, n, kind = CASES[case]()
    dims = _dims(f, n, kind)
    g = _track(f, n, kind)
    tr = O.track(f, n=n, kind=kind)
    tab_o = P.traj_table(tr, n, dims)
    tab_g = F.trajectory_table(g, dims)
    order_o, off_o = P.traj_order(tr, n, dims, tab_o)
    order_g, off_g = F.trajectory_order(g, dims, tab_g)
    assert np.array_equal(off_g.cpu().numpy(), off_o)
    assert np.array_equal(order_g.cpu().numpy(), order_o)
    loop = tab_o["n_ends"] == 0
    t = tr.pos[:, n]
    rng = np.random.default_rng(17)
    planted = rng.integers(1, 3, size=tr.n_hits).astype(np.uint8)  # two types at random: many runs and changes
    for types in (tr.type, planted):
        tg = torch.from_numpy(types).to(DEV)
        for w in (1, 2, 3):
            want = P.smooth_types(order_o, off_o, loop, types, w)
            got = F.smooth_types(g, tab_g, order_g, off_g, w, types=tg).cpu().numpy()
            assert np.array_equal(got, want), w
        for th in (0.3, 1.0, 2.5):
            got = F.simplify_types(g, tab_g, order_g, off_g, th, types=tg).cpu().numpy()
            _check_simplified(got, order_o, off_o, loop, types, t, th)


def test_birth_death_loop_order_and_simplification():
    """The loop is walked from its label face; a persistence threshold above the whole loop's extent leaves both
    branches (neither run has a persistent neighbour), one below the shorter branch changes nothing either."""
    nx, ny, nt = 33, 17, 21
    X = np.arange(nx, dtype=np.float64) - 16.0
    Y = np.arange(ny, dtype=np.float64) - 8.0
    f = np.zeros((nt, ny, nx))
    for t in range(nt):
        f[t] = (X[None, :] ** 3) / 3.0 - (30.0 - 0.5 * (t - 10.0) ** 2) * X[None, :] + (Y[:, None] ** 2)
    f = f.astype(np.float32)
    dims = (nx, ny, nt)
    g = _track(f, 2)
    tab = F.trajectory_table(g, dims)
    order, off = F.trajectory_order(g, dims, tab)
    o = order.cpu().numpy()
    assert off.cpu().numpy().tolist() == [0, g["n_hits"]]
    assert int(g["face_id"][o[0]]) == int(tab["label"][0])
    assert int(g["face_id"][o[1]]) < int(g["face_id"][o[-1]])
    assert np.array_equal(F.simplify_types(g, tab, order, off, 100.0).cpu().numpy(), g["type"].cpu().numpy())


def test_order_and_walk_errors():
    f = np.zeros((4, 9, 10), np.float32)
    g = _track(f, 2)
    tab = F.trajectory_table(g, (10, 9, 4))
    order, off = F.trajectory_order(g, (10, 9, 4), tab)
    assert order.numel() == 0 and off.cpu().numpy().tolist() == [0]
    f = synth.make("blobs64")
    g = _track(f, 2)
    dims = (f.shape[-1], f.shape[-2], f.shape[0])
    tab = F.trajectory_table(g, dims)
    order, off = F.trajectory_order(g, dims, tab)
    with pytest.raises(F.FtkError):
        F.smooth_types(g, tab, order, off, -1)
    with pytest.raises(ValueError):
        F.smooth_types(g, tab, order, off, 2, types=g["type"][:-1].contiguous())


def test_full_size_noise1024_order_properties():
    """The order on the full 1024^2 x 100 noise result (1.8e8 points): a permutation grouped by trajectory in label
    order with the table's offsets, one label per group, paths from their smaller-id end and loops from their
    label face, and consecutive points that are two sides of one cell (sampled, decoded on the host)."""
    f = synth.make("noise1024")
    dims = (f.shape[-1], f.shape[-2], f.shape[0])
    g = _track(f, 2)
    del f
    tab = F.trajectory_table(g, dims)
    order, off = F.trajectory_order(g, dims, tab)
    nh = g["n_hits"]
    assert torch.equal(torch.sort(order).values, torch.arange(nh, device=DEV))
    cnt = tab["n_points"]
    assert torch.equal(off[1:] - off[:-1], cnt) and int(off[0]) == 0 and int(off[-1]) == nh
    traj = torch.repeat_interleave(torch.arange(tab["n"], device=DEV), cnt)
    assert torch.equal(g["label"][order], tab["label"][traj])
    fid = g["face_id"]
    first, last = fid[order[off[:-1]]], fid[order[off[1:] - 1]]
    loop = tab["n_ends"] == 0
    assert torch.equal(first[loop], tab["label"][loop])
    assert bool((first[~loop] < last[~loop]).all())
    rng = np.random.default_rng(5)
    ks = rng.integers(0, nh - 1, size=3000)
    same = (traj[ks] == traj[ks + 1]).cpu().numpy()
    a = fid[order[ks]].cpu().numpy()
    b = fid[order[ks + 1]].cpu().numpy()
    checked = 0
    for x, y, s in zip(a, b, same):
        if s:
            assert share_a_cell(int(x), int(y), 2, dims)
            checked += 1
    assert checked > 2000


def test_full_size_blobs3d256_order_properties():
    """The order on the full 256^3 x 16 blob result: a permutation grouped by trajectory with the table's offsets,
    one label per group, paths from their smaller-id end and loops from their label face, consecutive points two
    sides of one pentachoron (sampled, decoded on the host)."""
    t = torch.from_numpy(synth.make("blobs3d256", device=DEV)).to(DEV)
    nt, nz, ny, nx = t.shape
    dims = (nx, ny, nz, nt)
    g = F.track_cp3d(t)
    torch.cuda.synchronize()
    del t
    tab = F.trajectory_table(g, dims)
    order, off = F.trajectory_order(g, dims, tab)
    nh = g["n_hits"]
    assert torch.equal(torch.sort(order).values, torch.arange(nh, device=DEV))
    assert torch.equal(off[1:] - off[:-1], tab["n_points"]) and int(off[-1]) == nh
    traj = torch.repeat_interleave(torch.arange(tab["n"], device=DEV), tab["n_points"])
    assert torch.equal(g["label"][order], tab["label"][traj])
    fid = g["face_id"]
    first, last = fid[order[off[:-1]]], fid[order[off[1:] - 1]]
    loop = tab["n_ends"] == 0
    assert torch.equal(first[loop], tab["label"][loop])
    assert bool((first[~loop] < last[~loop]).all())
    rng = np.random.default_rng(6)
    ks = rng.integers(0, nh - 1, size=2000)
    same = (traj[ks] == traj[ks + 1]).cpu().numpy()
    a = fid[order[ks]].cpu().numpy()
    b = fid[order[ks + 1]].cpu().numpy()
    checked = 0
    for x, y, s in zip(a, b, same):
        if s:
            assert share_a_cell(int(x), int(y), 3, dims)
            checked += 1
    assert checked > 1000
