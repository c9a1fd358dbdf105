"""Pins of the oracle's mesh (Sec. 3.2-3.3) against what the paper prints and what combinatorics fixes."""
import itertools
import os

import numpy as np
import pytest

from oracle import oracle as O
from oracle import ref as R

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]


@pytest.mark.parametrize("d,counts", [(3, [1, 7, 12, 6]), (4, [1, 15, 50, 60, 24])])
def test_types_per_vertex_counts_and_euler(d, counts):
    got = [1] + [len(O.kuhn_types(d, k)) for k in range(1, d + 1)]
    assert got == counts
    # the star of a vertex tiles space: alternating sum of simplex types per vertex is 0
    assert sum((-1) ** k * c for k, c in enumerate(got)) == 0


@pytest.mark.parametrize("d", [2, 3, 4])
def test_oracle_types_equal_monotone_path_faces(d):
    """Mask-tuple enumeration (oracle) == faces of the paper's monotone vertex lists (Python reference)."""
    for k in range(1, d + 1):
        masks = [tuple(int(x) for x in row) for row in O.kuhn_types(d, k)]
        assert masks == sorted(masks), "type ids must follow lexicographic mask order"
        assert sorted(masks) == R.type_order(d, k)


def test_triangle_type_list_2d():
    assert [tuple(r) for r in O.kuhn_types(3, 2).tolist()] == [
        (1, 2), (1, 4), (1, 6), (2, 1), (2, 4), (2, 5), (3, 4), (4, 1), (4, 2), (4, 3), (5, 2), (6, 1)]


def test_unit_cube_lists_printed_in_paper():
    rows = _rows("unit_cube_subdivisions.txt")
    for row in rows:
        d, total = int(row[0]), int(row[1])
        verts = [tuple(int(c) for c in v) for v in row[2:]]
        cells = set(R.unit_cube_cells(d))
        assert len(cells) == total == len(O.kuhn_types(d, d))
        # every printed list is a monotone path (each step raises exactly one coordinate)
        for u, v in zip(verts, verts[1:]):
            assert sum(b - a for a, b in zip(u, v)) == 1 and all(b >= a for a, b in zip(u, v))
        # the full cell set is symmetric under axis permutations, so membership holds whatever the digit order
        assert tuple(verts) in cells


def test_table1_staircases_are_kuhn_cells_of_the_prism():
    """Table 1: the (n+1)-simplices of the prism over a_0..a_n are the monotone staircases.  In the regular mesh the
    prism over one spatial Kuhn simplex is tiled by exactly the Kuhn cells of the (n+1)-cube whose spatial axis
    order matches the simplex, i.e. time inserted at any position."""
    rows = _rows("table1_staircase.txt")
    by_dim = {}
    for dim, lst in rows:
        by_dim.setdefault(int(dim), set()).add(lst)
    for dim, expected in by_dim.items():
        n = dim - 1  # spatial simplex dimension; the spatial axes are 0..n-1, time is axis n
        got = set()
        for chain in R.unit_cube_cells(dim):
            # vertex v = (spatial part, t); spatial part must be a_i (first i axes raised, in order)
            names = []
            ok = True
            for v in chain:
                sp, t = v[:n], v[n]
                i = sum(sp)
                if tuple(sp) != tuple([1] * i + [0] * (n - i)):
                    ok = False
                    break
                names.append(("b" if t else "a") + str(i))
            if ok:
                got.add("".join(names))
        assert got == expected


@pytest.mark.parametrize("dims", [(3, 4, 3), (5, 2, 4), (3, 3, 2, 2), (2, 3, 2, 3)])
def test_simplex_count_formula_vs_brute_force(dims):
    n = len(dims) - 1
    g = R.Grid(dims)
    assert O.simplex_count(n, dims) == len(g.faces())


def test_simplex_count_named_workloads():
    # sum over types of prod_a (N_a - [axis a used]) at the benchmark sizes
    assert O.simplex_count(2, (64, 64, 10)) == 438858
    assert O.simplex_count(2, (1024, 1024, 100)) == 1245774618
    assert O.simplex_count(2, (4096, 4096, 50)) == 9894527370
    assert O.simplex_count(3, (256, 256, 256, 16)) == 15040282500


@pytest.mark.parametrize("dims", [(4, 3, 3), (3, 3, 2, 2)])
def test_faces_in_one_or_two_cells(dims):
    """Each n-face lies in exactly two (n+1)-simplices, one if it is on the domain boundary (Sec. 3.2)."""
    n = len(dims) - 1
    g = R.Grid(dims)
    owners, verts = {}, {}
    for c in g.cells():
        for s in itertools.combinations(c, n + 1):
            owners.setdefault(g.face_id(s), []).append(c)
            verts[g.face_id(s)] = s
    for fid, lst in owners.items():
        assert len(lst) in (1, 2)
        assert len(O.face_cofaces(dims, fid, n=n)) == len(lst)
        on_boundary = any(all(v[a] == 0 for v in verts[fid]) or all(v[a] == dims[a] - 1 for v in verts[fid])
                          for a in range(n + 1))
        assert (len(lst) == 1) == on_boundary


@pytest.mark.parametrize("dims", [(3, 3, 3), (3, 2, 2, 3)])
def test_cell_sides_match_reference(dims):
    n = len(dims) - 1
    g = R.Grid(dims)
    ncell = len(O.kuhn_types(n + 1, n + 1))
    ref = {}
    for c in g.cells():
        masks = R.mask_tuple(c)
        cid = g.g(c[0]) * ncell + g.cell_types.index(masks)
        ref[cid] = sorted(g.face_id(s) for s in itertools.combinations(c, n + 1))
    ids = np.array(sorted(ref), np.int64)
    sides = O.cell_sides(dims, ids, n=n)
    for cid, row in zip(ids, sides):
        assert sorted(row.tolist()) == ref[int(cid)]
