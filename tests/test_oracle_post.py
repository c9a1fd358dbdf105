"""Pins of the oracle's trajectory post-processing (slicing at a time step, per-trajectory table, loop filter)
against what the paper and the mesh fix: one critical point per slice for a single moving zero at its analytic
position, a birth-death pair as one closed loop of the right time extent, every trajectory a path with two ends
or a loop with none, and the slice equal to a face-by-face test of every ordinal face of the step."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import post as P
from paper_2011_08697_amd import synth
from parity import share_a_cell


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


# ---------------------------------------------------------------------------------------------------------------
# Order along the trajectories, type smoothing and simplification (Sec. 4.4).
# ---------------------------------------------------------------------------------------------------------------

def _check_order(tr, n, dims, tab, order, offsets):
    assert np.array_equal(np.sort(order), np.arange(tr.n_hits))
    assert offsets[0] == 0 and offsets[-1] == tr.n_hits and len(offsets) == tab["n"] + 1
    for j in range(tab["n"]):
        seq = order[offsets[j]:offsets[j + 1]]
        assert np.all(tr.label[seq] == tab["label"][j])
        assert len(seq) == tab["n_points"][j]
        links = list(zip(seq[:-1], seq[1:])) + ([(seq[-1], seq[0])] if tab["n_ends"][j] == 0 else [])
        for a, b in links:
            assert share_a_cell(int(tr.face_id[a]), int(tr.face_id[b]), n, dims)
            # the curve's piece in a cell is a segment inside that unit cube
            assert np.all(np.abs(tr.pos[a] - tr.pos[b]) <= 1.0 + 1e-12)
        if tab["n_ends"][j] == 0:
            assert tr.face_id[seq[0]] == tab["label"][j]
            assert tr.face_id[seq[1]] < tr.face_id[seq[-1]]
        else:
            assert tr.face_id[seq[0]] < tr.face_id[seq[-1]]


@pytest.mark.parametrize("n,size,direction,nt", [(2, 21, (0.5, -0.25), 9), (3, 13, (0.25, 0.0, -0.5), 5)])
def test_moving_minimum_is_ordered_forward_in_time(n, size, direction, nt):
    """The single trajectory of a moving minimum starts on the t = 0 plane and its time coordinate never decreases
    along the order; consecutive points are two sides of one cell."""
    f = synth.moving_minimum(n, size, [size // 2] * n, list(direction), nt)
    tr = O.track(f, n=n)
    dims = tuple([size] * n + [nt])
    tab = P.traj_table(tr, n, dims)
    order, offsets = P.traj_order(tr, n, dims, tab)
    _check_order(tr, n, dims, tab, order, offsets)
    t = tr.pos[order, n]
    assert t[0] == 0.0 and t[-1] == nt - 1 and np.all(np.diff(t) >= 0)


def test_birth_death_loop_order_crosses_the_fold_twice():
    """The birth-death loop is one cycle whose consecutive points share a cell; the minimum branch (x > 0 about the
    centre) and the saddle branch (x < 0) meet at the two folds, so the sign of x changes exactly twice around it."""
    f, dims = _birth_death_field()
    tr = O.track(f)
    tab = P.traj_table(tr, 2, dims)
    order, offsets = P.traj_order(tr, 2, dims, tab)
    _check_order(tr, 2, dims, tab, order, offsets)
    side = np.sign(tr.pos[order, 0] - 16.0)
    side = side[side != 0]
    assert int(np.sum(side != np.roll(side, 1))) == 2


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_degenerate_grid_orders_are_curves(seed):
    """On integer fields with many exact zeros every trajectory is walked as one curve: consecutive points share a
    cell, a path runs between its two boundary ends, a loop closes."""
    rng = np.random.default_rng(seed)
    f = rng.integers(-1, 2, size=(5, 7, 6)).astype(np.float32)
    tr = O.track(f)
    dims = (6, 7, 5)
    tab = P.traj_table(tr, 2, dims)
    order, offsets = P.traj_order(tr, 2, dims, tab)
    _check_order(tr, 2, dims, tab, order, offsets)


def _one(types, loop=False):
    m = len(types)
    return np.arange(m, dtype=np.int64), np.array([0, m], np.int64), np.array([loop]), np.array(types, np.uint8)


@pytest.mark.parametrize("types,loop,w,expect", [
    ([1, 1, 3, 1, 1], False, 2, [1, 1, 1, 1, 1]),
    ([1, 1, 3, 1, 1], False, 1, [1, 1, 1, 1, 1]),
    ([1, 3, 1, 1, 1], False, 2, [1, 3, 1, 1, 1]),   # too close to the end for a half window of 2
    ([1, 3, 1, 1, 1], False, 1, [1, 1, 1, 1, 1]),
    ([1, 1, 3, 3, 1, 1], False, 1, [1, 1, 3, 3, 1, 1]),
    ([1, 1, 3, 1, 3, 1, 1], False, 1, [1, 1, 1, 3, 1, 1, 1]),  # decisions read the input types only
    ([2, 1, 1, 1, 1], True, 2, [1, 1, 1, 1, 1]),    # a loop wraps around
    ([2, 1, 1, 1], True, 2, [2, 1, 1, 1]),          # loop shorter than the window
    ([1, 2, 1, 2, 1, 2], True, 1, [2, 1, 2, 1, 2, 1]),
])
def test_smoothing_worked_examples(types, loop, w, expect):
    order, offsets, is_loop, ty = _one(types, loop)
    assert P.smooth_types(order, offsets, is_loop, ty, w).tolist() == expect


A, B, C = 1, 3, 4


@pytest.mark.parametrize("types,t,loop,theta,expect", [
    # a short saddle run between two persistent runs of one type merges into them (Sec. 4.4 example)
    ([A, A, A, B, B, A, A, A], [0, 1, 2, 2.2, 2.4, 2.6, 3.6, 4.6], False, 1.0, [A] * 8),
    ([A, A, A, B, B, A, A, A], [0, 1, 2, 2.2, 2.4, 2.6, 3.6, 4.6], False, 0.1, [A, A, A, B, B, A, A, A]),
    ([A, A, A, B, B, A, A, A], [0, 1, 2, 2.2, 2.4, 2.6, 3.6, 4.6], False, 2.5, [A, A, A, B, B, A, A, A]),
    ([A, B, B, C, C], [0, 1, 1.1, 2, 3], False, 0.5, [A, B, B, C, C]),       # neighbours of different types
    ([B, A, A, A], [0, 1, 2, 3], False, 0.5, [B, A, A, A]),                  # a run at a path end stays
    ([A, A, B, A], [0, 1, 1.1, 0.5], True, 0.5, [A, A, A, A]),               # on a loop the run wraps around
    ([A, A, B, B], [0, 0.1, 0.2, 0.3], True, 1.0, [A, A, B, B]),             # both runs short: neither changes
])
def test_simplification_worked_examples(types, t, loop, theta, expect):
    order, offsets, is_loop, ty = _one(types, loop)
    assert P.simplify_types(order, offsets, is_loop, ty, np.array(t, float), theta).tolist() == expect
