/*
 * ftk_oracle.c -- TEST INFRASTRUCTURE ONLY (the oracle).
 *
 * A plain, slow, exact CPU implementation of robust critical-point tracking on the regular simplicial
 * spacetime mesh of Guo et al., "FTK: A Simplicial Spacetime Meshing Framework for Robust and Scalable
 * Feature Tracking" (IEEE TVCG).  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  The product path (the HIP library) never calls it and shares no code,
 * header, table or helper with it.
 *
 * What it computes, in the paper's order:
 *   - Sec. 3.3 "Simplicial subdivision of (n+1)-D regular mesh": every d-cube of the spacetime grid is split
 *     into d! simplices whose vertex lists are the monotone paths from corner 0..0 to corner 1..1; k-simplices
 *     are indexed by (corner, unique type), so no mesh is stored ("Mesh element indexing", "Complexity").
 *   - Sec. 4.1: the field is a PL vector field on that mesh; a scalar field enters through its gradient
 *     (Sec. 2.1; limitations in Sec. 4.7).  Central differences (Sec. 4.3) give the gradient.
 *   - Sec. 4.3 with Sec. 2.4: an n-simplex is punctured iff the origin lies in the interior of the convex hull of
 *     its vertex vectors, decided by determinant signs of (v_0..v_n, 1) under Simulation of Simplicity.
 *   - Eq. 2: barycentric coordinates of the zero give its spacetime location.
 *   - Alg. 1 (left column): pass 1 tests every n-simplex; pass 2 unites the punctured sides of every
 *     (n+1)-simplex with union-find.
 *   - Sec. 4.1: critical-point types from the spatial Jacobian.
 * Readings where the paper is silent (vertex order, SoS exponents, stencil at the boundary, quantisation,
 * type ties, trajectory identity) are stated at each function.
 *
 * Exactness: vectors are quantised to integers; every determinant is computed exactly in 128-bit integers
 * (the accepted value ranges keep all products in range).  Floating point appears only in the stencils
 * (fixed IEEE binary32 operation order, no contraction) and in the binary64 reference semantics of
 * sublocation and classification.
 *
 * Build: gcc -O2 -std=gnu11 -ffp-contract=off -fno-fast-math -fPIC -shared -pthread (see build_oracle.py).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#include <unistd.h>

typedef __int128 i128;

/* Status codes (numerically the same meaning as the library's, defined here independently). */
enum { ORC_OK = 0, ORC_ERR_ARG = 1, ORC_ERR_NONFINITE = 2, ORC_ERR_RANGE = 3, ORC_ERR_OOM = 5,
       ORC_ERR_INVARIANT = 7 };

/* Critical-point types. */
enum { T_DEGENERATE = 0, T_MIN, T_MAX, T_SADDLE, T_SADDLE1, T_SADDLE2, T_SOURCE, T_SINK,
       T_REPELLING_FOCUS, T_ATTRACTING_FOCUS, T_CENTER };

/* Flags per punctured face. */
enum { F_DEGENERATE_SUBLOC = 1, F_WIDE = 4 };

#define MAXD 4 /* spacetime dimension d = n + 1 <= 4 */

/* ------------------------------------------------------------------------------------------------------------
 * Mesh: axes 0..n-1 are space (x, y, [z]), axis n is time.  Vertex p has global index
 * g = sum_a p_a * stride_a with stride_x = 1 and time slowest (the global vertex order used by SoS).
 * ---------------------------------------------------------------------------------------------------------- */
typedef struct {
  int n, d;
  int64_t N[MAXD];
  int64_t stride[MAXD];
  int64_t V;
  int nface, ncell;             /* number of n-simplex and (n+1)-simplex types */
  int8_t face[64][MAXD];        /* masks of the n-simplex types (n masks each) */
  int8_t cell[24][MAXD];        /* masks of the (n+1)-simplex types (d singleton masks each) */
  int kind;                     /* 0 = scalar (gradient taken), 1 = vector */
  int qshift;                   /* quantisation exponent */
  const float* field;
} mesh_t;

/* Sec. 3.3: a k-simplex inside a d-cube is a sub-list of a monotone vertex list from 0..0 to 1..1, so anchored
 * at its lowest vertex p it is p, p+e(M_1), p+e(M_1|M_2), ... for nonempty, pairwise disjoint axis masks
 * M_1..M_k.  Such tuples are the unique type IDs of the paper's indexing; enumerated here in lexicographic order
 * of the mask tuple (our reading: the paper does not fix an order). */
static void enum_rec(int d, int k, int depth, int used, int8_t* cur, int8_t (*out)[MAXD], int* count) {
  if (depth == k) {
    if (out) memcpy(out[*count], cur, MAXD);
    (*count)++;
    return;
  }
  for (int m = 1; m < (1 << d); ++m) {
    if (m & used) continue;
    cur[depth] = (int8_t)m;
    enum_rec(d, k, depth + 1, used | m, cur, out, count);
  }
}

int orc_kuhn_types(int d, int k, int8_t* out /* [count][4], may be NULL */) {
  if (d < 1 || d > MAXD || k < 0 || k > d) return -1;
  int8_t cur[MAXD] = {0, 0, 0, 0};
  int count = 0;
  enum_rec(d, k, 0, 0, cur, (int8_t(*)[MAXD])out, &count);
  return count;
}

static int mesh_init(mesh_t* m, int n, const int64_t* dims, int kind, int qshift, const float* field) {
  if (n < 2 || n > 3) return ORC_ERR_ARG;
  memset(m, 0, sizeof(*m));
  m->n = n;
  m->d = n + 1;
  m->V = 1;
  for (int a = 0; a < m->d; ++a) {
    if (dims[a] < 2) return ORC_ERR_ARG;
    m->N[a] = dims[a];
    m->stride[a] = m->V;
    m->V *= dims[a];
  }
  m->nface = orc_kuhn_types(m->d, n, &m->face[0][0]);
  int8_t tmp[24][MAXD];
  m->ncell = 0;
  /* cells: d-simplex types, i.e. d singleton masks (orderings of the axes) */
  int cnt = orc_kuhn_types(m->d, m->d, &tmp[0][0]);
  for (int i = 0; i < cnt; ++i) memcpy(m->cell[m->ncell++], tmp[i], MAXD);
  m->kind = kind;
  m->qshift = qshift;
  m->field = field;
  return ORC_OK;
}

static void coords_of(const mesh_t* m, int64_t g, int64_t* p) {
  for (int a = 0; a < MAXD; ++a) p[a] = 0;
  for (int a = 0; a < m->d; ++a) {
    p[a] = g % m->N[a];
    g /= m->N[a];
  }
}

static int64_t index_of(const mesh_t* m, const int64_t* p) {
  int64_t g = 0;
  for (int a = 0; a < m->d; ++a) g += p[a] * m->stride[a];
  return g;
}

/* Vertices of the simplex anchored at p with masks M_1..M_k, in chain order (increasing global index).
 * Returns 0 if a vertex falls outside the grid. */
static int simplex_vertices(const mesh_t* m, const int64_t* p, const int8_t* masks, int k, int64_t (*v)[MAXD]) {
  memcpy(v[0], p, sizeof(int64_t) * MAXD);
  for (int i = 1; i <= k; ++i) {
    memcpy(v[i], v[i - 1], sizeof(int64_t) * MAXD);
    for (int a = 0; a < m->d; ++a)
      if (masks[i - 1] & (1 << a)) v[i][a] += 1;
  }
  for (int a = 0; a < m->d; ++a)
    if (v[k][a] >= m->N[a]) return 0;
  return 1;
}

/* ------------------------------------------------------------------------------------------------------------
 * Field access and stencils (binary32, fixed order, no contraction).
 * Scalar layout f[t][(z)][y][x]; vector layout u[t][c][(z)][y][x] (planar components).
 * ---------------------------------------------------------------------------------------------------------- */
static float scalar_at(const mesh_t* m, const int64_t* p) { return m->field[index_of(m, p)]; }

static float vector_comp_at(const mesh_t* m, const int64_t* p, int c) {
  int64_t plane = m->V / m->N[m->n]; /* vertices per time step */
  int64_t t = p[m->n];
  int64_t sp = index_of(m, p) - t * plane;
  return m->field[(t * m->n + c) * plane + sp];
}

/* Central difference in the interior, one-sided difference at the first and last index of the axis.
 * Sec. 4.3 names central differences; the boundary rule is our reading.  sample(k) returns the sampled
 * quantity at p + k*e_a for k in {-1, 0, 1}. */
typedef float (*sample_fn)(const mesh_t* m, const int64_t* p, int arg);

static float stencil(const mesh_t* m, sample_fn fn, int arg, const int64_t* p, int a) {
  int64_t lo[MAXD], hi[MAXD];
  memcpy(lo, p, sizeof(lo));
  memcpy(hi, p, sizeof(hi));
  if (p[a] == 0) {
    hi[a] += 1;
    float r = fn(m, hi, arg) - fn(m, p, arg);
    return r;
  }
  if (p[a] == m->N[a] - 1) {
    lo[a] -= 1;
    float r = fn(m, p, arg) - fn(m, lo, arg);
    return r;
  }
  hi[a] += 1;
  lo[a] -= 1;
  float dlt = fn(m, hi, arg) - fn(m, lo, arg);
  float r = dlt * 0.5f;
  return r;
}

static float sample_scalar(const mesh_t* m, const int64_t* p, int unused) {
  (void)unused;
  return scalar_at(m, p);
}

/* Component c of the vector field at p: the gradient along spatial axis c (scalar input), or u_c (vector). */
static float vec_at(const mesh_t* m, const int64_t* p, int c) {
  if (m->kind == 0) return stencil(m, sample_scalar, 0, p, c);
  return vector_comp_at(m, p, c);
}

/* Spatial Jacobian J[a][b] = d(v_a)/d(x_b), the same stencil applied to the binary32 vector components. */
static void jacobian_at(const mesh_t* m, const int64_t* p, float J[3][3]) {
  for (int a = 0; a < m->n; ++a)
    for (int b = 0; b < m->n; ++b) J[a][b] = stencil(m, vec_at, a, p, b);
}

/* Fixed-point quantisation (our reading; the paper's robustness needs exact arithmetic on the vectors):
 * q = round-half-even(v * 2^s) computed in binary32 (the scaling by a power of two is exact).  Accepted
 * magnitudes keep every determinant inside 128 bits: 2D |q| < 2^62, 3D |q| < 2^41. */
static int quantise(const mesh_t* m, float v, int64_t* q) {
  float x = v * ldexpf(1.0f, m->qshift);
  if (!isfinite(x)) return ORC_ERR_RANGE;
  float r = rintf(x);
  float lim = (m->n == 2) ? 0x1p62f : 0x1p41f;
  if (fabsf(r) >= lim) return ORC_ERR_RANGE;
  *q = (int64_t)r;
  return ORC_OK;
}

static int vertex_q(const mesh_t* m, const int64_t* p, int64_t* q /* [n] */) {
  for (int c = 0; c < m->n; ++c) {
    int st = quantise(m, vec_at(m, p, c), &q[c]);
    if (st) return st;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------------------------------------------
 * Simulation of Simplicity (Sec. 2.4, Sec. 4.3).  Our reading of the perturbation ("determined by the vertex
 * and dimension ordering"): entry (component j, column k) of an n x n matrix whose columns are vertex vectors in
 * increasing global index is replaced by m[j][k] + eps^(2^(k*n+j)); a lower global index therefore carries the
 * larger perturbation.  The perturbed determinant is a polynomial in eps; its sign for eps -> 0+ is the sign of
 * the nonzero coefficient with the smallest exponent.  The polynomial is expanded literally (Leibniz formula,
 * every choice of perturbed factors), so this routine is the definition itself.
 * ---------------------------------------------------------------------------------------------------------- */
static int nperms(int n, int perm[6][3], int sgn[6]) {
  int count = 0;
  int tot = 1;
  for (int i = 0; i < n; ++i) tot *= n;
  for (int code = 0; code < tot; ++code) {
    int p[3], c = code, ok = 1, seen = 0;
    for (int i = 0; i < n; ++i) {
      p[i] = c % n;
      c /= n;
      if (seen & (1 << p[i])) ok = 0;
      seen |= 1 << p[i];
    }
    if (!ok) continue;
    int inv = 0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j)
        if (p[i] > p[j]) inv++;
    for (int i = 0; i < n; ++i) perm[count][i] = p[i];
    sgn[count] = (inv & 1) ? -1 : 1;
    count++;
  }
  return count;
}

/* m[j][k]: row j = component, column k = vertex.  Returns -1 or +1 (never 0). */
int orc_sos_sign_i128(int n, i128 m[3][3]) {
  i128 coef[512];
  memset(coef, 0, sizeof(coef));
  int perm[6][3], sgn[6];
  int np = nperms(n, perm, sgn);
  for (int pi = 0; pi < np; ++pi) {
    /* term: sgn * prod_k m[perm[k]][k]; column k takes row perm[k] */
    for (int S = 0; S < (1 << n); ++S) { /* S: columns whose factor is the perturbation */
      i128 c = sgn[pi];
      unsigned E = 0;
      for (int k = 0; k < n; ++k) {
        int j = perm[pi][k];
        if (S & (1 << k))
          E |= 1u << (k * n + j);
        else
          c *= m[j][k];
      }
      coef[E] += c;
    }
  }
  for (unsigned E = 0; E < (1u << (n * n)); ++E) {
    if (coef[E] > 0) return 1;
    if (coef[E] < 0) return -1;
  }
  return 0; /* unreachable: the all-perturbed term of each permutation has a distinct exponent */
}

/* Exact unperturbed determinant (Leibniz). */
static i128 det_exact(int n, i128 m[3][3]) {
  int perm[6][3], sgn[6];
  int np = nperms(n, perm, sgn);
  i128 s = 0;
  for (int pi = 0; pi < np; ++pi) {
    i128 c = sgn[pi];
    for (int k = 0; k < n; ++k) c *= m[perm[pi][k]][k];
    s += c;
  }
  return s;
}

/* Test hook: direct SoS sign of an n x n int64 matrix given column-major (cols[k*n + j]). */
int orc_sos_sign(int n, const int64_t* cols) {
  if (n < 1 || n > 3) return 0;
  i128 m[3][3];
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j) m[j][k] = cols[k * n + j];
  return orc_sos_sign_i128(n, m);
}

/* Matrix of the vectors of all vertices but `skip` (columns in chain order). */
static void minor_matrix(int n, const int64_t (*Q)[3], int skip, i128 m[3][3]) {
  int k = 0;
  for (int i = 0; i <= n; ++i) {
    if (i == skip) continue;
    for (int j = 0; j < n; ++j) m[j][k] = Q[i][j];
    k++;
  }
}

/* Sec. 4.3 / Eq. 2: with C_i = (-1)^(n+i) det(V without column i) the cofactors of the last row of
 * (v_0..v_n ; 1 .. 1), the barycentric coordinates are mu_i = C_i / sum C.  The origin is interior iff all C_i
 * have one sign; with SoS every sign is nonzero.  Q[i] are the quantised vectors of the vertices in chain
 * order. */
static int face_punctured(int n, const int64_t (*Q)[3]) {
  int first = 0;
  for (int i = 0; i <= n; ++i) {
    i128 mm[3][3];
    minor_matrix(n, Q, i, mm);
    int s = orc_sos_sign_i128(n, mm);
    if ((n + i) & 1) s = -s;
    if (i == 0)
      first = s;
    else if (s != first)
      return 0;
  }
  return 1;
}

/* Test hook: puncture predicate on explicit integer vectors (row-major [n+1][n], chain order). */
int orc_face_punctured(int n, const int64_t* vecs) {
  int64_t Q[4][3];
  for (int i = 0; i <= n; ++i)
    for (int j = 0; j < n; ++j) Q[i][j] = vecs[i * n + j];
  return face_punctured(n, (const int64_t(*)[3])Q);
}

/* ------------------------------------------------------------------------------------------------------------
 * Sublocation (Eq. 2) and classification (Sec. 4.1), binary64 reference semantics.
 * ---------------------------------------------------------------------------------------------------------- */
static i128 cofactor(int n, const int64_t (*Q)[3], int i) {
  i128 mm[3][3];
  minor_matrix(n, Q, i, mm);
  i128 dd = det_exact(n, mm);
  return ((n + i) & 1) ? -dd : dd;
}

/* Exact cofactors, then mu_i = fl64(C_i) / fl64(D) with D = sum C_i (exact).  When D = 0 every C_i is 0 and the
 * simplex is punctured only through the perturbation; the centroid is used and flagged. */
static int sublocate(int n, const int64_t (*Q)[3], const int64_t (*verts)[MAXD], double* mu, double* pos) {
  i128 C[4], D = 0;
  for (int i = 0; i <= n; ++i) {
    C[i] = cofactor(n, Q, i);
    D += C[i];
  }
  int flags = 0;
  if (D != 0) {
    double dD = (double)D;
    for (int i = 0; i <= n; ++i) mu[i] = (double)C[i] / dD;
  } else {
    for (int i = 0; i <= n; ++i) mu[i] = 1.0 / (double)(n + 1);
    flags |= F_DEGENERATE_SUBLOC;
  }
  for (int a = 0; a <= n; ++a) {
    double s = 0.0;
    for (int i = 0; i <= n; ++i) {
      double term = mu[i] * (double)verts[i][a];
      s = (i == 0) ? term : s + term;
    }
    pos[a] = s;
  }
  return flags;
}

static int classify2_gradient(const double J[3][3]) {
  double p1 = J[0][0] * J[1][1];
  double p2 = J[0][1] * J[1][0];
  double det = p1 - p2;
  double tr = J[0][0] + J[1][1];
  if (det < 0) return T_SADDLE;
  if (det > 0 && tr < 0) return T_MAX;
  if (det > 0 && tr > 0) return T_MIN;
  return T_DEGENERATE;
}

static int classify2_vector(const double J[3][3]) {
  double p1 = J[0][0] * J[1][1];
  double p2 = J[0][1] * J[1][0];
  double det = p1 - p2;
  double tr = J[0][0] + J[1][1];
  if (det < 0) return T_SADDLE;
  if (det == 0) return T_DEGENERATE;
  if (tr == 0) return T_CENTER;
  double t2 = tr * tr;
  double d4 = 4.0 * det;
  double disc = t2 - d4;
  if (tr < 0) return (disc >= 0) ? T_SINK : T_ATTRACTING_FOCUS;
  return (disc >= 0) ? T_SOURCE : T_REPELLING_FOCUS;
}

/* 3D gradient: H = (J + J^T)/2 is symmetric, so its characteristic polynomial has real roots and Descartes'
 * rule on (1, s1, s2, s3) counts its negative eigenvalues exactly (s3 != 0). */
static int classify3_gradient(const double J[3][3]) {
  double H[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double s = J[a][b] + J[b][a];
      H[a][b] = s * 0.5;
    }
  double s1 = (H[0][0] + H[1][1]) + H[2][2];
  double m01 = H[0][0] * H[1][1] - H[0][1] * H[1][0];
  double m02 = H[0][0] * H[2][2] - H[0][2] * H[2][0];
  double m12 = H[1][1] * H[2][2] - H[1][2] * H[2][1];
  double s2 = (m01 + m02) + m12;
  double c0 = H[1][1] * H[2][2] - H[1][2] * H[2][1];
  double c1 = H[1][0] * H[2][2] - H[1][2] * H[2][0];
  double c2 = H[1][0] * H[2][1] - H[1][1] * H[2][0];
  double s3 = (H[0][0] * c0 - H[0][1] * c1) + H[0][2] * c2;
  if (s3 == 0) return T_DEGENERATE;
  double seq[4] = {1.0, s1, s2, s3};
  int changes = 0;
  double prev = 1.0;
  for (int i = 1; i < 4; ++i) {
    if (seq[i] == 0) continue;
    if ((seq[i] < 0) != (prev < 0)) changes++;
    prev = seq[i];
  }
  static const int by_count[4] = {T_MIN, T_SADDLE1, T_SADDLE2, T_MAX};
  return by_count[changes];
}

static int classify(const mesh_t* m, const int64_t (*verts)[MAXD], const double* mu) {
  double Jc[3][3];
  float Jv[4][3][3];
  for (int i = 0; i <= m->n; ++i) jacobian_at(m, verts[i], Jv[i]);
  for (int a = 0; a < m->n; ++a)
    for (int b = 0; b < m->n; ++b) {
      double s = 0.0;
      for (int i = 0; i <= m->n; ++i) {
        double term = mu[i] * (double)Jv[i][a][b];
        s = (i == 0) ? term : s + term;
      }
      Jc[a][b] = s;
    }
  if (m->n == 2) return m->kind == 0 ? classify2_gradient(Jc) : classify2_vector(Jc);
  return classify3_gradient(Jc);
}

/* ------------------------------------------------------------------------------------------------------------
 * Per-face evaluation.
 * ---------------------------------------------------------------------------------------------------------- */
typedef struct {
  int valid;
  int punctured;
  int status;
  double mu[4];
  double pos[4];
  int type;
  int flags;
} face_eval_t;

static int64_t wide_limit(const mesh_t* m) { return m->n == 2 ? ((int64_t)1 << 31) : ((int64_t)1 << 20); }

static void eval_face(const mesh_t* m, int64_t fid, int want_details, face_eval_t* r) {
  memset(r, 0, sizeof(*r));
  int64_t g = fid / m->nface;
  int ty = (int)(fid % m->nface);
  int64_t p[MAXD], v[MAXD + 1][MAXD];
  coords_of(m, g, p);
  if (!simplex_vertices(m, p, m->face[ty], m->n, v)) return;
  r->valid = 1;
  int64_t Q[4][3];
  for (int i = 0; i <= m->n; ++i) {
    int st = vertex_q(m, v[i], Q[i]);
    if (st) {
      r->status = st;
      return;
    }
  }
  r->punctured = face_punctured(m->n, (const int64_t(*)[3])Q);
  if (!r->punctured || !want_details) return;
  r->flags = sublocate(m->n, (const int64_t(*)[3])Q, (const int64_t(*)[MAXD])v, r->mu, r->pos);
  int64_t lim = wide_limit(m);
  for (int i = 0; i <= m->n; ++i)
    for (int j = 0; j < m->n; ++j)
      if (Q[i][j] >= lim || Q[i][j] <= -lim) r->flags |= F_WIDE;
  r->type = classify(m, (const int64_t(*)[MAXD])v, r->mu);
}

/* Sides of a cell (its 2-simplex faces, Alg. 1 pass 2; the sides query of Sec. 3.2): drop one vertex of the chain
 * and re-anchor at the lowest remaining vertex; the masks are the differences of consecutive remaining vertices.
 * Returns face ids, or -1 for a side that leaves the grid (cannot happen for a valid cell). */
static int face_type_of(const mesh_t* m, const int8_t* masks) {
  for (int t = 0; t < m->nface; ++t) {
    int same = 1;
    for (int i = 0; i < m->n; ++i)
      if (m->face[t][i] != masks[i]) same = 0;
    if (same) return t;
  }
  return -1;
}

static int cell_sides(const mesh_t* m, int64_t cid, int64_t* fids) {
  int64_t g = cid / m->ncell;
  int ct = (int)(cid % m->ncell);
  int64_t p[MAXD], w[MAXD + 2][MAXD];
  coords_of(m, g, p);
  if (!simplex_vertices(m, p, m->cell[ct], m->d, w)) return 0;
  for (int drop = 0; drop <= m->d; ++drop) {
    int64_t rest[MAXD + 1][MAXD];
    int k = 0;
    for (int i = 0; i <= m->d; ++i)
      if (i != drop) memcpy(rest[k++], w[i], sizeof(int64_t) * MAXD);
    int8_t masks[MAXD] = {0, 0, 0, 0};
    for (int i = 1; i <= m->n; ++i) {
      int mk = 0;
      for (int a = 0; a < m->d; ++a)
        if (rest[i][a] != rest[i - 1][a]) mk |= 1 << a;
      masks[i - 1] = (int8_t)mk;
    }
    int ty = face_type_of(m, masks);
    fids[drop] = ty < 0 ? -1 : index_of(m, rest[0]) * m->nface + ty;
  }
  return 1;
}

/* Cells that contain a face (the side-of query of Sec. 3.2): brute force over the cells anchored at the face's anchor or
 * one step below it along any axis, keeping those whose side list holds the face. */
static int face_cofaces(const mesh_t* m, int64_t fid, int64_t* cids) {
  int64_t g = fid / m->nface;
  int64_t p[MAXD];
  coords_of(m, g, p);
  int cnt = 0;
  for (int a = -1; a < m->d; ++a) {
    int64_t c[MAXD];
    memcpy(c, p, sizeof(c));
    if (a >= 0) {
      if (c[a] == 0) continue;
      c[a] -= 1;
    }
    int64_t cg = index_of(m, c);
    for (int ct = 0; ct < m->ncell; ++ct) {
      int64_t sides[MAXD + 1];
      if (!cell_sides(m, cg * m->ncell + ct, sides)) continue;
      for (int i = 0; i <= m->d; ++i)
        if (sides[i] == fid) cids[cnt++] = cg * m->ncell + ct;
    }
  }
  return cnt;
}

/* ------------------------------------------------------------------------------------------------------------
 * Whole-field tracking (Alg. 1, left column), threaded over time steps.
 * ---------------------------------------------------------------------------------------------------------- */
typedef struct {
  int64_t n_hits, n_traj;
  int64_t* face_id;
  double* pos; /* [n_hits][n+1] */
  double* mu;  /* [n_hits][n+1] */
  uint8_t* type;
  uint8_t* flags;
  int64_t* label;
  int64_t simplices_tested;
  int64_t cells_with_hits;
  int64_t invariant_violations;
  double t_quantise, t_detect, t_subloc, t_stitch;
} orc_result;

typedef struct {
  int64_t* v;
  int64_t n, cap;
} vec64;

static int vec_push(vec64* a, int64_t x) {
  if (a->n == a->cap) {
    int64_t nc = a->cap ? a->cap * 2 : 1024;
    int64_t* nv = (int64_t*)realloc(a->v, (size_t)nc * sizeof(int64_t));
    if (!nv) return 0;
    a->v = nv;
    a->cap = nc;
  }
  a->v[a->n++] = x;
  return 1;
}

typedef struct {
  const mesh_t* m;
  int64_t* q;          /* [V][n] quantised vectors */
  int64_t nt;          /* time steps */
  int64_t next;        /* work counter (protected by lock) */
  pthread_mutex_t lock;
  vec64* per_step;     /* hits per time step (detect) or edges per time step (stitch) */
  int64_t* viol;       /* invariant violations per time step */
  int status;
  /* for stitching */
  const int64_t* hits;
  int64_t n_hits;
  /* for sublocation */
  orc_result* res;
} job_t;

static int64_t take(job_t* j) {
  pthread_mutex_lock(&j->lock);
  int64_t t = j->next++;
  pthread_mutex_unlock(&j->lock);
  return t;
}

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

static void* quantise_worker(void* arg) {
  job_t* j = (job_t*)arg;
  const mesh_t* m = j->m;
  int64_t plane = m->V / m->N[m->n];
  for (;;) {
    int64_t t = take(j);
    if (t >= j->nt) break;
    for (int64_t g = t * plane; g < (t + 1) * plane; ++g) {
      int64_t p[MAXD];
      coords_of(m, g, p);
      int st = vertex_q(m, p, &j->q[g * m->n]);
      if (st) {
        pthread_mutex_lock(&j->lock);
        j->status = st;
        pthread_mutex_unlock(&j->lock);
      }
    }
  }
  return NULL;
}

static int punctured_q(const mesh_t* m, const int64_t* q, int64_t fid) {
  int64_t g = fid / m->nface;
  int ty = (int)(fid % m->nface);
  int64_t p[MAXD], v[MAXD + 1][MAXD];
  coords_of(m, g, p);
  if (!simplex_vertices(m, p, m->face[ty], m->n, v)) return -1;
  int64_t Q[4][3];
  for (int i = 0; i <= m->n; ++i) {
    int64_t vg = index_of(m, v[i]);
    for (int c = 0; c < m->n; ++c) Q[i][c] = q[vg * m->n + c];
  }
  return face_punctured(m->n, (const int64_t(*)[3])Q);
}

/* Pass 1: every n-simplex, in increasing face id (anchor index, then type), so the hit list comes out sorted. */
static void* detect_worker(void* arg) {
  job_t* j = (job_t*)arg;
  const mesh_t* m = j->m;
  int64_t plane = m->V / m->N[m->n];
  for (;;) {
    int64_t t = take(j);
    if (t >= j->nt) break;
    for (int64_t g = t * plane; g < (t + 1) * plane; ++g)
      for (int ty = 0; ty < m->nface; ++ty) {
        int64_t fid = g * m->nface + ty;
        if (punctured_q(m, j->q, fid) == 1 && !vec_push(&j->per_step[t], fid)) {
          pthread_mutex_lock(&j->lock);
          j->status = ORC_ERR_OOM;
          pthread_mutex_unlock(&j->lock);
        }
      }
  }
  return NULL;
}

static int64_t find_hit(const int64_t* hits, int64_t n, int64_t fid) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (hits[mid] < fid)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < n && hits[lo] == fid) ? lo : -1;
}

/* Pass 2: every (n+1)-simplex; T = S intersected with its sides; under SoS |T| is 0 or 2. */
static void* stitch_worker(void* arg) {
  job_t* j = (job_t*)arg;
  const mesh_t* m = j->m;
  int64_t plane = m->V / m->N[m->n];
  for (;;) {
    int64_t t = take(j);
    if (t >= j->nt) break;
    for (int64_t g = t * plane; g < (t + 1) * plane; ++g)
      for (int ct = 0; ct < m->ncell; ++ct) {
        int64_t sides[MAXD + 1];
        if (!cell_sides(m, g * m->ncell + ct, sides)) continue;
        int64_t idx[MAXD + 1];
        int cnt = 0;
        for (int i = 0; i <= m->d; ++i) {
          int64_t h = find_hit(j->hits, j->n_hits, sides[i]);
          if (h >= 0) idx[cnt++] = h;
        }
        if (cnt == 2) {
          vec_push(&j->per_step[t], idx[0]);
          vec_push(&j->per_step[t], idx[1]);
        } else if (cnt != 0) {
          j->viol[t]++;
        }
      }
  }
  return NULL;
}

static void* subloc_worker(void* arg) {
  job_t* j = (job_t*)arg;
  const mesh_t* m = j->m;
  orc_result* r = j->res;
  const int64_t chunk = 4096;
  for (;;) {
    int64_t c = take(j);
    int64_t b = c * chunk;
    if (b >= r->n_hits) break;
    int64_t e = b + chunk < r->n_hits ? b + chunk : r->n_hits;
    for (int64_t i = b; i < e; ++i) {
      face_eval_t fe;
      eval_face(m, r->face_id[i], 1, &fe);
      for (int a = 0; a <= m->n; ++a) {
        r->mu[i * (m->n + 1) + a] = fe.mu[a];
        r->pos[i * (m->n + 1) + a] = fe.pos[a];
      }
      r->type[i] = (uint8_t)fe.type;
      r->flags[i] = (uint8_t)fe.flags;
    }
  }
  return NULL;
}

static int run_threads(int nthreads, void* (*fn)(void*), job_t* j) {
  pthread_t th[256];
  if (nthreads > 256) nthreads = 256;
  j->next = 0;
  int started = 0;
  for (int i = 0; i < nthreads; ++i)
    if (pthread_create(&th[i], NULL, fn, j) == 0) started++;
  if (started == 0) fn(j);
  for (int i = 0; i < started; ++i) pthread_join(th[i], NULL);
  return ORC_OK;
}

static int64_t uf_find(int64_t* parent, int64_t x) {
  int64_t r = x;
  while (parent[r] != r) r = parent[r];
  while (parent[x] != r) {
    int64_t nx = parent[x];
    parent[x] = r;
    x = nx;
  }
  return r;
}

/* Union keeps the smaller index as root, so every root is the first hit (smallest face id) of its set. */
static void uf_unite(int64_t* parent, int64_t a, int64_t b) {
  int64_t ra = uf_find(parent, a), rb = uf_find(parent, b);
  if (ra == rb) return;
  if (ra < rb)
    parent[rb] = ra;
  else
    parent[ra] = rb;
}

void orc_result_free(orc_result* r) {
  if (!r) return;
  free(r->face_id);
  free(r->pos);
  free(r->mu);
  free(r->type);
  free(r->flags);
  free(r->label);
  memset(r, 0, sizeof(*r));
}

static int all_finite(const float* f, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!isfinite(f[i])) return 0;
  return 1;
}

/* dims = (nx, ny, [nz], nt).  kind 0 = scalar (length prod(dims)), 1 = vector (n components per vertex,
 * planar per time step). */
int orc_track(int n, const float* field, int kind, const int64_t* dims, int qshift, int nthreads,
              orc_result* out) {
  if (!field || !dims || !out || (kind != 0 && kind != 1) || qshift < 0 || qshift > 60) return ORC_ERR_ARG;
  if (n == 3 && kind != 0) return ORC_ERR_ARG;
  mesh_t m;
  int st = mesh_init(&m, n, dims, kind, qshift, field);
  if (st) return st;
  if (nthreads <= 0) nthreads = (int)sysconf(_SC_NPROCESSORS_ONLN);
  memset(out, 0, sizeof(*out));
  int64_t nvals = m.V * (kind == 1 ? n : 1);
  if (!all_finite(field, nvals)) return ORC_ERR_NONFINITE;

  job_t j;
  memset(&j, 0, sizeof(j));
  j.m = &m;
  j.nt = m.N[n];
  pthread_mutex_init(&j.lock, NULL);

  double t0 = now_s();
  j.q = (int64_t*)malloc((size_t)m.V * n * sizeof(int64_t));
  if (!j.q) return ORC_ERR_OOM;
  run_threads(nthreads, quantise_worker, &j);
  if (j.status) {
    free(j.q);
    return j.status;
  }
  double t1 = now_s();

  /* pass 1 */
  j.per_step = (vec64*)calloc((size_t)j.nt, sizeof(vec64));
  run_threads(nthreads, detect_worker, &j);
  if (j.status) {
    for (int64_t t = 0; t < j.nt; ++t) free(j.per_step[t].v);
    free(j.per_step);
    free(j.q);
    return j.status;
  }
  int64_t nh = 0;
  for (int64_t t = 0; t < j.nt; ++t) nh += j.per_step[t].n;
  out->n_hits = nh;
  out->face_id = (int64_t*)malloc((size_t)(nh ? nh : 1) * sizeof(int64_t));
  int64_t k = 0;
  for (int64_t t = 0; t < j.nt; ++t) {
    memcpy(out->face_id + k, j.per_step[t].v, (size_t)j.per_step[t].n * sizeof(int64_t));
    k += j.per_step[t].n;
    free(j.per_step[t].v);
    j.per_step[t].v = NULL;
    j.per_step[t].n = j.per_step[t].cap = 0;
  }
  double t2 = now_s();

  /* sublocation and classification of every punctured face */
  size_t w = (size_t)(nh ? nh : 1);
  out->pos = (double*)malloc(w * (n + 1) * sizeof(double));
  out->mu = (double*)malloc(w * (n + 1) * sizeof(double));
  out->type = (uint8_t*)malloc(w);
  out->flags = (uint8_t*)malloc(w);
  out->label = (int64_t*)malloc(w * sizeof(int64_t));
  j.res = out;
  run_threads(nthreads, subloc_worker, &j);
  double t3 = now_s();

  /* pass 2 */
  j.hits = out->face_id;
  j.n_hits = nh;
  j.viol = (int64_t*)calloc((size_t)j.nt, sizeof(int64_t));
  run_threads(nthreads, stitch_worker, &j);
  int64_t* parent = (int64_t*)malloc(w * sizeof(int64_t));
  for (int64_t i = 0; i < nh; ++i) parent[i] = i;
  int64_t viol = 0, pairs = 0;
  for (int64_t t = 0; t < j.nt; ++t) {
    for (int64_t e = 0; e + 1 < j.per_step[t].n; e += 2) uf_unite(parent, j.per_step[t].v[e], j.per_step[t].v[e + 1]);
    pairs += j.per_step[t].n / 2;
    viol += j.viol[t];
    free(j.per_step[t].v);
  }
  int64_t ntraj = 0;
  for (int64_t i = 0; i < nh; ++i) {
    int64_t r = uf_find(parent, i);
    out->label[i] = out->face_id[r];
    if (r == i) ntraj++;
  }
  out->n_traj = ntraj;
  out->cells_with_hits = pairs;
  out->invariant_violations = viol;
  double t4 = now_s();

  int64_t tested = 0;
  for (int ty = 0; ty < m.nface; ++ty) {
    int64_t c = 1;
    int used = 0;
    for (int i = 0; i < n; ++i) used |= m.face[ty][i];
    for (int a = 0; a < m.d; ++a) c *= m.N[a] - ((used >> a) & 1);
    tested += c;
  }
  out->simplices_tested = tested;
  out->t_quantise = t1 - t0;
  out->t_detect = t2 - t1;
  out->t_subloc = t3 - t2;
  out->t_stitch = t4 - t3;

  free(parent);
  free(j.viol);
  free(j.per_step);
  free(j.q);
  pthread_mutex_destroy(&j.lock);
  return viol ? ORC_ERR_INVARIANT : ORC_OK;
}

/* Detection only (pass 1) over time steps [t_begin, t_end) of the anchors: used for a bounded CPU baseline.
 * Returns the number of punctured faces; *tested receives the number of n-simplices tested. */
int64_t orc_detect_count(int n, const float* field, int kind, const int64_t* dims, int qshift, int nthreads,
                         int64_t t_begin, int64_t t_end, int64_t* tested) {
  mesh_t m;
  if (mesh_init(&m, n, dims, kind, qshift, field)) return -1;
  if (nthreads <= 0) nthreads = (int)sysconf(_SC_NPROCESSORS_ONLN);
  job_t j;
  memset(&j, 0, sizeof(j));
  j.m = &m;
  j.nt = m.N[n];
  pthread_mutex_init(&j.lock, NULL);
  j.q = (int64_t*)malloc((size_t)m.V * n * sizeof(int64_t));
  if (!j.q) return -1;
  run_threads(nthreads, quantise_worker, &j);
  j.per_step = (vec64*)calloc((size_t)j.nt, sizeof(vec64));
  /* restrict the anchors to [t_begin, t_end) by starting the work counter there */
  pthread_t th[256];
  int nth = nthreads > 256 ? 256 : nthreads;
  j.next = t_begin;
  j.nt = t_end;
  int started = 0;
  for (int i = 0; i < nth; ++i)
    if (pthread_create(&th[i], NULL, detect_worker, &j) == 0) started++;
  if (!started) detect_worker(&j);
  for (int i = 0; i < started; ++i) pthread_join(th[i], NULL);
  int64_t nh = 0;
  for (int64_t t = t_begin; t < t_end; ++t) {
    nh += j.per_step[t].n;
    free(j.per_step[t].v);
  }
  if (tested) {
    int64_t plane = m.V / m.N[n];
    int64_t cnt = 0;
    for (int64_t g = t_begin * plane; g < t_end * plane; ++g)
      for (int ty = 0; ty < m.nface; ++ty) {
        int64_t p[MAXD], v[MAXD + 1][MAXD];
        coords_of(&m, g, p);
        if (simplex_vertices(&m, p, m.face[ty], n, v)) cnt++;
      }
    *tested = cnt;
  }
  free(j.per_step);
  free(j.q);
  pthread_mutex_destroy(&j.lock);
  return nh;
}

/* ------------------------------------------------------------------------------------------------------------
 * Point queries for sampled checks at any grid size (no whole-field arrays are built).
 * ---------------------------------------------------------------------------------------------------------- */

/* For each face id: punct[i] = 1 punctured, 0 not, 255 not a valid face of this grid; mu/pos [nf][n+1];
 * type, flags.  Returns a status (NONFINITE/RANGE concern only the vertices these faces touch). */
int orc_eval_faces(int n, const float* field, int kind, const int64_t* dims, int qshift, int64_t nf,
                   const int64_t* fids, uint8_t* punct, double* mu, double* pos, uint8_t* type, uint8_t* flags) {
  mesh_t m;
  int st = mesh_init(&m, n, dims, kind, qshift, field);
  if (st) return st;
  int status = ORC_OK;
  for (int64_t i = 0; i < nf; ++i) {
    face_eval_t fe;
    if (fids[i] < 0 || fids[i] >= m.V * m.nface) {
      punct[i] = 255;
      continue;
    }
    eval_face(&m, fids[i], 1, &fe);
    if (fe.status) status = fe.status;
    punct[i] = fe.valid ? (uint8_t)fe.punctured : 255;
    for (int a = 0; a <= n; ++a) {
      if (mu) mu[i * (n + 1) + a] = fe.mu[a];
      if (pos) pos[i * (n + 1) + a] = fe.pos[a];
    }
    if (type) type[i] = (uint8_t)fe.type;
    if (flags) flags[i] = (uint8_t)fe.flags;
  }
  return status;
}

/* Sides of cells: out[i][0..d] face ids (-1 for an invalid cell id). */
int orc_cell_sides(int n, const int64_t* dims, int64_t nc, const int64_t* cids, int64_t* out) {
  mesh_t m;
  int st = mesh_init(&m, n, dims, 0, 20, NULL);
  if (st) return st;
  for (int64_t i = 0; i < nc; ++i) {
    if (cids[i] < 0 || cids[i] >= m.V * m.ncell || !cell_sides(&m, cids[i], out + i * (m.d + 1)))
      for (int k = 0; k <= m.d; ++k) out[i * (m.d + 1) + k] = -1;
  }
  return ORC_OK;
}

/* Cells containing a face (at most 2 for an n-simplex of the d-dimensional mesh). */
int orc_face_cofaces(int n, const int64_t* dims, int64_t fid, int64_t* cids /* [8] */) {
  mesh_t m;
  if (mesh_init(&m, n, dims, 0, 20, NULL)) return -1;
  return face_cofaces(&m, fid, cids);
}

/* Follow a trajectory from a punctured face through the cells (each cell with two punctured sides links them)
 * in both directions, up to max_steps faces.  Returns the number of faces visited (-1 on error);
 * *min_fid gets the smallest face id on the component; *closed = 1 for a cycle, 0 for a path whose two ends were
 * reached, -1 if max_steps ran out. */
int64_t orc_trace(int n, const float* field, int kind, const int64_t* dims, int qshift, int64_t fid,
                  int64_t max_steps, int64_t* min_fid, int* closed) {
  mesh_t m;
  if (mesh_init(&m, n, dims, kind, qshift, field)) return -1;
  face_eval_t fe;
  eval_face(&m, fid, 0, &fe);
  if (!fe.valid || !fe.punctured) return -1;
  int64_t best = fid, count = 1;
  int64_t start_cells[8];
  int ns = face_cofaces(&m, fid, start_cells);
  *closed = 0;
  for (int dir = 0; dir < ns; ++dir) {
    int64_t cur = fid, via = start_cells[dir];
    for (;;) {
      if (count >= max_steps) {
        *closed = -1;
        *min_fid = best;
        return count;
      }
      int64_t sides[MAXD + 1], other = -1;
      cell_sides(&m, via, sides);
      int cnt = 0;
      for (int i = 0; i <= m.d; ++i) {
        face_eval_t se;
        eval_face(&m, sides[i], 0, &se);
        if (se.punctured) {
          cnt++;
          if (sides[i] != cur) other = sides[i];
        }
      }
      if (cnt != 2 || other < 0) return -1; /* a cell holding a punctured side has exactly two */
      if (other == fid) { /* back at the start: a cycle */
        *closed = 1;
        *min_fid = best;
        return count;
      }
      count++;
      if (other < best) best = other;
      int64_t cells[8];
      int nc = face_cofaces(&m, other, cells);
      int64_t next = -1;
      for (int c = 0; c < nc; ++c)
        if (cells[c] != via) next = cells[c];
      cur = other;
      if (next < 0) break; /* other lies on the domain boundary: path end */
      via = next;
    }
  }
  *min_fid = best;
  return count;
}

/* Quantised vectors of all vertices (tests of the stencil and the quantisation). */
int orc_quantise_all(int n, const float* field, int kind, const int64_t* dims, int qshift, int64_t* q) {
  mesh_t m;
  int st = mesh_init(&m, n, dims, kind, qshift, field);
  if (st) return st;
  if (!all_finite(field, m.V * (kind == 1 ? n : 1))) return ORC_ERR_NONFINITE;
  for (int64_t g = 0; g < m.V; ++g) {
    int64_t p[MAXD];
    coords_of(&m, g, p);
    st = vertex_q(&m, p, &q[g * n]);
    if (st) return st;
  }
  return ORC_OK;
}

/* Binary32 Jacobians of all vertices, [V][n][n] (tests). */
int orc_jacobian_all(int n, const float* field, int kind, const int64_t* dims, float* J) {
  mesh_t m;
  int st = mesh_init(&m, n, dims, kind, 20, field);
  if (st) return st;
  for (int64_t g = 0; g < m.V; ++g) {
    int64_t p[MAXD];
    float Jv[3][3];
    coords_of(&m, g, p);
    jacobian_at(&m, p, Jv);
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) J[(g * n + a) * n + b] = Jv[a][b];
  }
  return ORC_OK;
}

/* Number of tested n-simplices: sum over types of prod_a (N_a - [axis a used by the type]). */
int64_t orc_simplex_count(int n, const int64_t* dims) {
  mesh_t m;
  if (mesh_init(&m, n, dims, 0, 20, NULL)) return -1;
  int64_t tested = 0;
  for (int ty = 0; ty < m.nface; ++ty) {
    int64_t c = 1;
    int used = 0;
    for (int i = 0; i < n; ++i) used |= m.face[ty][i];
    for (int a = 0; a < m.d; ++a) c *= m.N[a] - ((used >> a) & 1);
    tested += c;
  }
  return tested;
}

/* Classification on an explicit binary64 Jacobian (tests of the type rules). */
int orc_classify_matrix(int n, int kind, const double* J /* [n][n] */) {
  double Jc[3][3] = {{0}};
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) Jc[a][b] = J[a * n + b];
  if (n == 2) return kind == 0 ? classify2_gradient(Jc) : classify2_vector(Jc);
  return classify3_gradient(Jc);
}
