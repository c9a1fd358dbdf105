"""Trajectory post-processing on the oracle's results (test infrastructure only, like the rest of oracle/).

Plain numpy over the host arrays of an oracle run, written from the definitions:
  * slicing at a time step (Sec. 3.2, "Ordinal and interval mesh elements"): the critical points of step t0 are the
    punctured faces anchored at t0 whose vertices all lie in that step (no time axis in their type);
  * per-trajectory attributes for filtering (Sec. 4.4, "Filtering"): number of points, time extent of their
    positions, and the number of points that lie in only one cell of the grid (the trajectory's ends, counted
    with the oracle's own coface enumeration);
  * the loop filter (Sec. 4.4): the points of closed trajectories (no ends) shorter in time than a threshold.
"""
import numpy as np

from . import oracle as O


def ordinal_types(n):
    """Indices of the face types (n-simplices of the (n+1)-D Kuhn mesh) that do not use the time axis."""
    types = O.kuhn_types(n + 1, n)
    tbit = 1 << n
    return np.array([i for i, row in enumerate(types) if not any(int(m) & tbit for m in row)], dtype=np.int64)


def slice_at(tr, n, dims_with_t, t0):
    """Ascending indices of the punctured ordinal faces anchored at step t0."""
    T = 12 if n == 2 else 60
    plane = int(np.prod(dims_with_t[:n]))
    steps = (tr.face_id // T) // plane
    sel = (steps == t0) & np.isin(tr.face_id % T, ordinal_types(n))
    return np.nonzero(sel)[0].astype(np.int64)


def cells_holding(dims_with_t, fid, n):
    """Number of grid cells that contain the face (1 on a boundary hyperplane, else 2)."""
    return len(O.face_cofaces(tuple(dims_with_t), int(fid), n=n))


def traj_table(tr, n, dims_with_t):
    labels = np.unique(tr.label)
    j = np.searchsorted(labels, tr.label)
    n_points = np.bincount(j, minlength=len(labels)).astype(np.int64)
    t = tr.pos[:, n]
    t_min = np.full(len(labels), np.inf)
    t_max = np.full(len(labels), -np.inf)
    np.minimum.at(t_min, j, t)
    np.maximum.at(t_max, j, t)
    ends = np.array([cells_holding(dims_with_t, f, n) == 1 for f in tr.face_id], dtype=np.int64)
    n_ends = np.bincount(j, weights=ends, minlength=len(labels)).astype(np.int64)
    return dict(n=len(labels), label=labels, n_points=n_points, t_min=t_min, t_max=t_max, n_ends=n_ends)


def filter_loops(tr, table, min_duration):
    """uint8 keep mask: 0 for the points of closed loops whose time extent is below min_duration."""
    j = np.searchsorted(table["label"], tr.label)
    loop = table["n_ends"][j] == 0
    short = (table["t_max"] - table["t_min"])[j] < min_duration
    return (~(loop & short)).astype(np.uint8)
