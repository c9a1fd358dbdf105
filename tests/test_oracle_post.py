"""Pins of the oracle's trajectory post-processing (slicing at a time step, per-trajectory table, loop filter)
against what the paper and the mesh fix: one critical point per slice for a single moving zero at its analytic
position, a birth-death pair as one closed loop of the right time extent, every trajectory a path with two ends
or a loop with none, and the slice equal to a face-by-face test of every ordinal face of the step."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import post as P
from paper_2011_08697_amd import synth


def _birth_death_field():
    nx, ny, nt = 33, 17, 21
    X = np.arange(nx, dtype=np.float64) - 16.0
    Y = np.arange(ny, dtype=np.float64) - 8.0
    f = np.zeros((nt, ny, nx))
    for t in range(nt):
        a = 30.0 - 0.5 * (t - 10.0) ** 2
        f[t] = (X[None, :] ** 3) / 3.0 - a * X[None, :] + (Y[:, None] ** 2)
    return f.astype(np.float32), (nx, ny, nt)


@pytest.mark.parametrize("n,size,direction,nt", [(2, 21, (0.5, -0.25), 9), (2, 21, (0.0, 0.0), 6),
                                                 (3, 13, (0.25, 0.0, -0.5), 5)])
def test_moving_minimum_slices_and_table(n, size, direction, nt):
    """Sec. 4.5 moving minimum: each time slice holds exactly one critical point, at x0 + d t0; the one trajectory
    runs from the first to the last step with its two ends on the t = 0 and t = nt - 1 planes."""
    x0 = [size // 2] * n
    f = synth.moving_minimum(n, size, x0, list(direction), nt)
    tr = O.track(f, n=n)
    dims = tuple([size] * n + [nt])
    for t0 in range(nt):
        idx = P.slice_at(tr, n, dims, t0)
        assert len(idx) == 1
        for a in range(n):
            assert abs(tr.pos[idx[0], a] - (x0[a] + direction[a] * t0)) < 1e-9
        assert tr.pos[idx[0], n] == t0
    tab = P.traj_table(tr, n, dims)
    assert tab["n"] == 1 and tab["n_points"][0] == tr.n_hits
    assert tab["t_min"][0] == 0.0 and tab["t_max"][0] == nt - 1
    assert tab["n_ends"][0] == 2


def test_birth_death_pair_is_one_loop_with_its_time_extent():
    """A minimum and a saddle born together and annihilating: one closed loop (no ends) between the birth and
    death times, t = 10 -+ sqrt(60) where a(t) = 30 - (t - 10)^2 / 2 vanishes; the loop filter drops it below that
    extent and keeps it above."""
    f, dims = _birth_death_field()
    tr = O.track(f)
    tab = P.traj_table(tr, 2, dims)
    assert tab["n"] == 1 and tab["n_ends"][0] == 0
    dur = tab["t_max"][0] - tab["t_min"][0]
    exact = 2.0 * np.sqrt(60.0)
    assert abs(dur - exact) < 1.0  # the extremes of a PL loop lie within one step of the analytic ones
    assert np.all(P.filter_loops(tr, tab, dur + 0.5) == 0)
    assert np.all(P.filter_loops(tr, tab, dur - 0.5) == 1)


@pytest.mark.parametrize("case", ["blob", "degenerate", "3d"])
def test_every_trajectory_is_a_path_or_a_loop(case):
    """Under SoS the trajectories form a 1-manifold: a component has two ends on the grid boundary or none."""
    if case == "blob":
        f, n = synth.make("blobs64"), 2
    elif case == "degenerate":
        f, n = synth.quantise_levels(synth.moving_gaussians_2d(48, 40, 6, 6, seed=11, noise_std=1e-3)), 2
    else:
        rng = np.random.default_rng(9)
        f, n = rng.integers(0, 4, size=(3, 5, 4, 4)).astype(np.float32), 3
    tr = O.track(f, n=n)
    dims = tuple(reversed(f.shape)) if n == 2 else (f.shape[3], f.shape[2], f.shape[1], f.shape[0])
    tab = P.traj_table(tr, n, dims)
    assert tab["n"] == tr.n_traj and int(tab["n_points"].sum()) == tr.n_hits
    assert set(np.unique(tab["n_ends"]).tolist()) <= {0, 2}
    assert np.all(tab["t_min"] <= tab["t_max"])


def test_slice_equals_facewise_test_of_the_step():
    """The slice at t0 from a whole-field run equals the punctured set among all ordinal faces of step t0 tested
    one by one."""
    f = synth.moving_gaussians_2d(24, 20, 5, 4, seed=3)
    nt, ny, nx = f.shape
    dims = (nx, ny, nt)
    tr = O.track(f)
    ords = P.ordinal_types(2)
    types = O.kuhn_types(3, 2)
    used = {int(ty): int(types[ty][0]) | int(types[ty][1]) for ty in ords}
    for t0 in range(nt):
        # every ordinal face of the step whose vertices lie in the grid
        fids = np.array([((t0 * ny + y) * nx + x) * 12 + ty for y in range(ny) for x in range(nx) for ty in ords
                         if not ((used[ty] & 1 and x == nx - 1) or (used[ty] & 2 and y == ny - 1))], dtype=np.int64)
        ev = O.eval_faces(f, fids)
        assert ev["status"] == 0
        expect = np.sort(fids[ev["punctured"] == 1])
        got = tr.face_id[P.slice_at(tr, 2, dims, t0)]
        assert np.array_equal(got, expect)
