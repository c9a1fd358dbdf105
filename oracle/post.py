"""Trajectory post-processing on the oracle's results (test infrastructure only, like the rest of oracle/).

Plain numpy over the host arrays of an oracle run, written from the definitions:
  * slicing at a time step (Sec. 3.2, "Ordinal and interval mesh elements"): the critical points of step t0 are the
    punctured faces anchored at t0 whose vertices all lie in that step (no time axis in their type);
  * per-trajectory attributes for filtering (Sec. 4.4, "Filtering"): number of points, time extent of their
    positions, and the number of points that lie in only one cell of the grid (the trajectory's ends, counted
    with the oracle's own coface enumeration);
  * the loop filter (Sec. 4.4): the points of closed trajectories (no ends) shorter in time than a threshold;
  * the order of the points along each trajectory, and the type smoothing and simplification over it (Sec. 4.4).
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


# ---------------------------------------------------------------------------------------------------------------
# Order of the points along each trajectory, and the type smoothing and simplification that walk it (Sec. 4.4,
# "Simplification" and "Smoothing").  A trajectory is a PL curve whose piece in each cell is the segment between
# the cell's two punctured sides (Sec. 3.1, Alg. 1 pass 2), so the points of a trajectory are ordered by walking
# from cell to cell.
# ---------------------------------------------------------------------------------------------------------------

def neighbours(tr, n, dims_with_t):
    """[n_hits][2] int64: for every hit, the other punctured side of each cell that holds it (smaller index
    first, -1 where the hit lies in only one cell).  Every cell holds 0 or 2 punctured sides."""
    dims = tuple(int(v) for v in dims_with_t)
    index = {int(f): i for i, f in enumerate(tr.face_id)}
    nb = np.full((tr.n_hits, 2), -1, np.int64)
    for i, f in enumerate(tr.face_id):
        found = []
        for c in O.face_cofaces(dims, int(f), n=n):
            sides = O.cell_sides(dims, [int(c)], n=n)[0]
            other = [index[int(s)] for s in sides if int(s) != int(f) and int(s) in index]
            if len(other) != 1:
                raise AssertionError("cell %d holds %d punctured sides besides face %d" % (c, len(other), f))
            found.append(other[0])
        found.sort()
        nb[i, :len(found)] = found
    return nb


def traj_order(tr, n, dims_with_t, table):
    """(order, offsets): hit indices grouped by trajectory in ascending label order, each trajectory in curve
    order.  A path starts at its end with the smaller face id; a closed loop starts at its label face (its smallest
    face id) and steps first to the neighbour with the smaller face id.  offsets[j] is the start of trajectory j,
    offsets[-1] = n_hits."""
    nb = neighbours(tr, n, dims_with_t)
    fid = tr.face_id
    members = {}
    for i, lab in enumerate(tr.label):
        members.setdefault(int(lab), []).append(i)
    order, offsets = [], [0]
    for j, lab in enumerate(table["label"]):
        pts = members[int(lab)]
        if table["n_ends"][j] == 0:
            start = pts[int(np.argmin(fid[pts]))]
            first = min((int(k) for k in nb[start] if k >= 0), key=lambda k: fid[k])
        else:
            ends = [p for p in pts if int((nb[p] >= 0).sum()) == 1]
            assert len(ends) == 2
            start = min(ends, key=lambda p: fid[p])
            first = int(nb[start][0])
        seq, prev, cur = [start], start, first
        while cur != start and cur >= 0:
            seq.append(cur)
            nxt = [int(k) for k in nb[cur] if k >= 0 and k != prev]
            prev, cur = cur, (nxt[0] if nxt else -1)
        assert sorted(seq) == sorted(pts), "trajectory %d is not one curve" % j
        order.extend(seq)
        offsets.append(len(order))
    return np.array(order, np.int64), np.array(offsets, np.int64)


def smooth_types(order, offsets, is_loop, types, half_window):
    """Window-shifting type smoothing: a point whose half_window predecessors and half_window successors along
    its trajectory all share one type different from its own takes that type.  Decisions read the input types
    only (marks first, changes after the pass).  Loops wrap around; a loop shorter than 2 * half_window + 1 points
    and the points of a path closer than half_window to an end keep their types."""
    types = np.asarray(types)
    out = types.copy()
    w = int(half_window)
    for j in range(len(offsets) - 1):
        seq = order[offsets[j]:offsets[j + 1]]
        m = len(seq)
        for r in range(m):
            if is_loop[j]:
                if m < 2 * w + 1:
                    continue
                around = [seq[(r + d) % m] for d in range(-w, w + 1) if d != 0]
            else:
                if r - w < 0 or r + w > m - 1:
                    continue
                around = [seq[r + d] for d in range(-w, w + 1) if d != 0]
            vals = set(int(types[k]) for k in around)
            if len(vals) == 1 and vals != {int(types[seq[r]])}:
                out[seq[r]] = vals.pop()
    return out


def _runs(seq_types, loop):
    """Maximal runs of equal consecutive values as lists of positions; on a loop a run may wrap around."""
    m = len(seq_types)
    if loop:
        starts = [r for r in range(m) if seq_types[r] != seq_types[r - 1]]
        if not starts:
            return [list(range(m))]
        runs = []
        for a, s in enumerate(starts):
            e = starts[(a + 1) % len(starts)]
            runs.append([(s + k) % m for k in range((e - s) % m or m)])
        return runs
    runs, cur = [], [0]
    for r in range(1, m):
        if seq_types[r] == seq_types[r - 1]:
            cur.append(r)
        else:
            runs.append(cur)
            cur = [r]
    runs.append(cur)
    return runs


def simplify_types(order, offsets, is_loop, types, t, min_persistence):
    """Run simplification: a run (maximal stretch of one type along a trajectory) whose time extent is below
    min_persistence, lying between two runs of one common type whose extents are both at least min_persistence,
    takes that type.  Decisions read the input types only.  Runs at the ends of a path have one neighbour and stay;
    on a loop the neighbours wrap around (with two runs, both neighbours are the other run)."""
    types = np.asarray(types)
    out = types.copy()
    for j in range(len(offsets) - 1):
        seq = order[offsets[j]:offsets[j + 1]]
        st = [int(types[k]) for k in seq]
        runs = _runs(st, bool(is_loop[j]))
        if len(runs) < 2:
            continue
        ext = [max(t[seq[r]] for r in R) - min(t[seq[r]] for r in R) for R in runs]
        typ = [st[R[0]] for R in runs]
        for a, R in enumerate(runs):
            if is_loop[j]:
                p, q = (a - 1) % len(runs), (a + 1) % len(runs)
            else:
                if a == 0 or a == len(runs) - 1:
                    continue
                p, q = a - 1, a + 1
            if ext[a] < min_persistence and typ[p] == typ[q] and ext[p] >= min_persistence and \
                    ext[q] >= min_persistence:
                for r in R:
                    out[seq[r]] = typ[p]
    return out
