"""Pins of the oracle's robust predicate (Sec. 2.4, Sec. 4.3, Eq. 2) by means other than the oracle itself."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from oracle import ref as R


def _rng(seed):
    return np.random.default_rng(seed)


@pytest.mark.parametrize("n", [2, 3])
def test_sos_sign_matches_concrete_eps_evaluation(n):
    """Symbolic expansion (oracle) == sign of the perturbed determinant evaluated at a concrete tiny eps."""
    rng = _rng(10 + n)
    for it in range(1500):
        r = int(rng.choice([1, 2, 5]))
        M = rng.integers(-r, r + 1, size=(n, n))
        if n == 3 and rng.random() < 0.3:  # force rank deficiency
            M[:, 2] = M[:, 0] * rng.integers(-2, 3) + M[:, 1] * rng.integers(-2, 3)
        if rng.random() < 0.1:
            M[:, rng.integers(n)] = 0
        assert O.sos_sign(M) == R.perturbed_det_sign(M.tolist())


@pytest.mark.parametrize("n", [2, 3])
def test_sos_sign_is_det_sign_when_nonzero(n):
    rng = _rng(20 + n)
    for it in range(2000):
        M = rng.integers(-(1 << 20), 1 << 20, size=(n, n))
        d = R.det([[int(x) for x in row] for row in M])
        if d != 0:
            assert O.sos_sign(M) == (1 if d > 0 else -1)


def test_sos_sign_2x2_hand_expansion():
    """det([[A0+e^1, B0+e^4], [A1+e^2, B1+e^8]]) = (A0B1-A1B0) + B1 e - B0 e^2 - A1 e^4 - e^6 + A0 e^8 + e^9:
    the first nonzero of (det, B1, -B0, -A1, -1) decides."""
    rng = _rng(3)
    for it in range(3000):
        A = rng.integers(-2, 3, size=2)
        B = rng.integers(-2, 3, size=2)
        seq = [A[0] * B[1] - A[1] * B[0], B[1], -B[0], -A[1], -1]
        expect = next(int(np.sign(s)) for s in seq if s != 0)
        assert O.sos_sign(np.array([[A[0], B[0]], [A[1], B[1]]])) == expect


def test_sos_sign_3x3_sequence():
    """Closed-form decision sequence for n = 3 (first nonzero decides), with M_jk the 2x2 minor without row j and
    column k and C_jk = (-1)^(j+k) M_jk."""
    rng = _rng(4)
    for it in range(3000):
        m = rng.integers(-1, 2, size=(3, 3))
        if rng.random() < 0.5:
            m[:, 2] = m[:, 0] + m[:, 1] * rng.integers(-1, 2)

        def C(j, k):
            rows = [r for r in range(3) if r != j]
            cols = [c for c in range(3) if c != k]
            mm = m[rows][:, cols]
            return (-1) ** (j + k) * (mm[0, 0] * mm[1, 1] - mm[0, 1] * mm[1, 0])

        dm = R.det(m.tolist())
        seq = [dm, C(0, 0), C(1, 0), C(2, 0), C(0, 1), -m[2, 2], m[1, 2], C(1, 1), m[2, 2], -m[0, 2], C(2, 1),
               -m[1, 2], m[0, 2], C(0, 2), m[2, 1], -m[1, 1], -m[2, 0], -1]
        expect = next(int(np.sign(s)) for s in seq if s != 0)
        assert O.sos_sign(m) == expect


@pytest.mark.parametrize("n", [2, 3])
def test_predicate_generic_equals_exact_barycentric(n):
    """On generic inputs (no zero cofactor) the robust test is the textbook one: solve Eq. 2 exactly and check
    every mu_i > 0."""
    rng = _rng(30 + n)
    for it in range(1500 if n == 2 else 600):
        V = rng.integers(-(1 << 20), 1 << 20, size=(n + 1, n))
        M = [[Fraction(int(V[k][j])) for k in range(n + 1)] for j in range(n)] + [[Fraction(1)] * (n + 1)]
        D = R.det(M)
        mus = []
        for i in range(n + 1):
            Mi = [row[:] for row in M]
            for r in range(n + 1):
                Mi[r][i] = Fraction(1 if r == n else 0)
            mus.append(R.det(Mi))
        if D == 0 or any(x == 0 for x in mus):
            continue
        expect = all((x / D) > 0 for x in mus)
        assert bool(O.face_punctured(V)) == expect


def test_predicate_degenerate_2d_matches_literal_definition():
    rng = _rng(5)
    for it in range(1500):
        V = rng.integers(-1, 2, size=(3, 2))
        assert O.face_punctured(V) == int(R.punctured(V.tolist()))


def test_predicate_degenerate_3d_matches_literal_definition():
    rng = _rng(6)
    for it in range(30):
        V = rng.integers(-1, 2, size=(4, 3))
        assert O.face_punctured(V) == int(R.punctured(V.tolist()))


def test_zero_at_shared_vertex_goes_to_exactly_one_triangle():
    """A zero sitting exactly on a vertex shared by a fan of triangles is assigned to exactly one of them: the 2D
    triangles of one time slice around an interior vertex with a radial field."""
    rng = _rng(7)
    for it in range(50):
        # a 3x3 slice whose centre vertex carries the zero vector, neighbours random nonzero vectors around it
        u = np.zeros((2, 2, 3, 3), np.float32)
        for y in range(3):
            for x in range(3):
                if (x, y) != (1, 1):
                    u[:, 0, y, x] = x - 1 + 0.25 * rng.integers(-1, 2)
                    u[:, 1, y, x] = y - 1 + 0.25 * rng.integers(-1, 2)
        tr = O.track(u, n=2, kind=1)
        ordinal = [f for f in tr.face_id if f % 12 in (0, 3) and (f // 12) // 9 == 0]
        assert len(ordinal) == 1


@pytest.mark.parametrize("n", [2, 3])
def test_strictly_signed_component_or_all_zero_is_never_punctured(n):
    """The facts the detection kernels use to skip a tile-step: if one component has the same strict sign at every
    vertex of a simplex, the perturbed vectors keep that sign and the origin is outside; if every vector is zero,
    the cofactor signs never agree.  Checked on the oracle's predicate (the SoS expansion) with ties everywhere in
    the other components."""
    rng = np.random.default_rng(20 + n)
    for _ in range(3000):
        V = rng.integers(-2, 3, size=(n + 1, n)).astype(np.int64)
        c = rng.integers(0, n)
        sign = 1 if rng.random() < 0.5 else -1
        V[:, c] = sign * rng.integers(1, 3, size=n + 1)
        assert O.face_punctured(V) == 0
    assert O.face_punctured(np.zeros((n + 1, n), np.int64)) == 0
