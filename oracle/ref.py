"""Tiny exact reference (TEST INFRASTRUCTURE ONLY), pure Python, for small grids.

It restates the definitions a second way, to pin the C oracle:
  * the mesh is built from the paper's monotone vertex lists of the unit cube (Sec. 3.3, "Precomputation of the
    subdivision for n-D unit cube"), not from mask tuples: cells are the d! lists, k-simplices are their
    (k+1)-vertex subsets;
  * the symbolic perturbation is evaluated numerically at one concrete, sufficiently small rational eps instead of
    being expanded symbolically (Sec. 2.4, Sec. 4.3);
  * the puncture test is the literal statement "the origin is interior to the simplex of the perturbed vectors",
    decided by solving Eq. 2 with Cramer's rule in exact rationals and checking every mu_i > 0;
  * trajectories are connected components found by breadth-first search over cells (Alg. 1, pass 2).
Only tests import it.
"""
from fractions import Fraction
from itertools import combinations, permutations, product


def unit_cube_cells(d):
    """Sec. 3.3: the d! monotone vertex lists from 0..0 to 1..1 (one per order in which the axes are raised)."""
    cells = []
    for order in permutations(range(d)):
        v = [0] * d
        chain = [tuple(v)]
        for a in order:
            v[a] = 1
            chain.append(tuple(v))
        cells.append(tuple(chain))
    return cells


def simplices_at_origin(d, k):
    """k-simplices of the regular mesh whose lowest vertex is the origin (the per-vertex "unique types")."""
    out = set()
    for chain in unit_cube_cells(d):
        for sub in combinations(chain, k + 1):
            if sub[0] == (0,) * d:
                out.add(sub)
    return out


def mask_tuple(simplex):
    """Axis masks between consecutive vertices of a chain (bit a = axis a)."""
    masks = []
    for u, v in zip(simplex, simplex[1:]):
        masks.append(sum(1 << a for a in range(len(u)) if v[a] != u[a]))
    return tuple(masks)


def type_order(d, k):
    """Type list: mask tuples sorted lexicographically (the indexing reading shared with the oracle)."""
    return sorted(mask_tuple(s) for s in simplices_at_origin(d, k))


class Grid:
    def __init__(self, dims):
        self.dims = tuple(dims)  # (nx, ny, [nz], nt)
        self.d = len(dims)
        self.n = self.d - 1
        self.stride = []
        s = 1
        for N in dims:
            self.stride.append(s)
            s *= N
        self.V = s
        self.face_types = type_order(self.d, self.n)
        self.cell_types = type_order(self.d, self.d)

    def g(self, p):
        return sum(c * s for c, s in zip(p, self.stride))

    def coords(self, g):
        p = []
        for N in self.dims:
            p.append(g % N)
            g //= N
        return tuple(p)

    def cells(self):
        """Every (n+1)-simplex as a tuple of vertex coordinates in chain order."""
        out = []
        for c in product(*[range(N - 1) for N in self.dims]):
            for chain in unit_cube_cells(self.d):
                out.append(tuple(tuple(ci + vi for ci, vi in zip(c, v)) for v in chain))
        return out

    def faces(self):
        out = set()
        for cell in self.cells():
            for sub in combinations(cell, self.n + 1):
                out.add(sub)
        return sorted(out, key=self.face_id)

    def face_id(self, simplex):
        T = len(self.face_types)
        return self.g(simplex[0]) * T + self.face_types.index(mask_tuple(simplex))


def det(M):
    """Leibniz determinant (exact for integers or Fractions)."""
    n = len(M)
    total = 0
    for perm in permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        term = -1 if inv % 2 else 1
        for r in range(n):
            term *= M[r][perm[r]]
            if term == 0:
                break
        total += term
    return total


def eps_bits(vecs):
    """eps = 2^-bits, small enough that every perturbed minor has the sign of its lowest-order eps term: the
    coefficients are integers bounded by n! * (max|v| + 1)^n and there are fewer than 2^(n*(n+1)) of them."""
    n = len(vecs[0])
    mx = max(1, max(abs(int(x)) for v in vecs for x in v)) + 1
    return (n * mx.bit_length()) + 3 + n * (n + 1) + 4


def perturbed_vectors(vecs, bits):
    """Vertex k (k-th in increasing global index), component j gets + eps^(2^(k*n + j)), eps = 2^-bits.
    Every entry is multiplied by the common factor 2^(bits*W), W = 2^(max weight), to stay in integers; a
    common positive factor on the vector rows changes no sign and no barycentric coordinate."""
    n = len(vecs[0])
    wmax = len(vecs) * n - 1
    W = 2 ** wmax
    return [[int(vecs[k][j]) * 2 ** (bits * W) + 2 ** (bits * (W - 2 ** (k * n + j))) for j in range(n)]
            for k in range(len(vecs))]


def barycentric(vecs):
    """Eq. 2 solved by Cramer's rule for the perturbed vectors: returns mu (Fractions)."""
    n = len(vecs[0])
    P = perturbed_vectors(vecs, eps_bits(vecs))
    M = [[P[k][j] for k in range(n + 1)] for j in range(n)] + [[1] * (n + 1)]
    D = det(M)
    rhs = [0] * n + [1]
    mu = []
    for i in range(n + 1):
        Mi = [row[:] for row in M]
        for r in range(n + 1):
            Mi[r][i] = rhs[r]
        mu.append(Fraction(det(Mi), D))
    return mu


def punctured(vecs):
    """Origin strictly inside the simplex of the perturbed vectors (Sec. 4.3)."""
    return all(m > 0 for m in barycentric(vecs))


def perturbed_det_sign(M):
    """Sign of det(M + E) at a concrete tiny eps, columns = vertices in index order (Sec. 2.4)."""
    n = len(M)
    cols = [[M[j][k] for j in range(n)] for k in range(n)]
    P = perturbed_vectors(cols, eps_bits(cols))
    D = det([[P[k][j] for k in range(n)] for j in range(n)])
    return (D > 0) - (D < 0)


def track(grid, vec):
    """vec: dict or list indexed by global vertex index -> integer n-vector.
    Returns (sorted face ids of punctured faces, {face_id: label}, histogram of punctured sides per cell)."""
    hits = {}
    for f in grid.faces():
        vv = [vec[grid.g(p)] for p in f]
        if punctured(vv):
            hits[grid.face_id(f)] = f
    adj = {fid: [] for fid in hits}
    hist = {}
    for cell in grid.cells():
        ids = [grid.face_id(s) for s in combinations(cell, grid.n + 1)]
        pun = [i for i in ids if i in hits]
        hist[len(pun)] = hist.get(len(pun), 0) + 1
        if len(pun) == 2:
            adj[pun[0]].append(pun[1])
            adj[pun[1]].append(pun[0])
    label = {}
    for start in sorted(hits):
        if start in label:
            continue
        comp = [start]
        seen = {start}
        i = 0
        while i < len(comp):
            for nb in adj[comp[i]]:
                if nb not in seen:
                    seen.add(nb)
                    comp.append(nb)
            i += 1
        m = min(comp)
        for c in comp:
            label[c] = m
    return sorted(hits), label, hist
