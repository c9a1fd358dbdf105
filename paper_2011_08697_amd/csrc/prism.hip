// prism.hip -- critical-point tracking of a 2D vector field on an unstructured triangle mesh extruded in time
// (Sec. 3.2, prismatic subdivision; Sec. 4.2 two passes).
//
// Every mesh triangle v0 < v1 < v2 becomes, between steps t and t + 1, the prism a0 a1 a2 - b0 b1 b2 split by the
// staircase into a0 a1 a2 b2, a0 a1 b1 b2 and a0 b0 b1 b2 (global vertex order g = t nv + v); the quadrilateral of
// a mesh edge a < b is split along its monotone diagonal a - b'.  Faces of step t are numbered t * S + local,
// S = nf + 2 ne + 2 nf: the mesh triangle T (local T), the edge faces (a, b, b') and (a, a', b') of edge E (nf + 2E,
// +1), and the interior faces (v0, v1, v2') and (v0, v1', v2') of T (nf + 2 ne + 2T, +1); interval faces exist for
// t < nt - 1.
//
//   pm_test  -- one lane per face, all steps (on a vertex-major copy of the field): the puncture test of the
//               quantised 2D vectors at its three vertices in global order (SoS signs of the three vertex-pair
//               determinants, as in the regular path).
//   pm_emit  -- face ids, points from the exact cofactors (Eq. 2) in (x, y, t), identity parents.
//   pm_unite_hits -- one lane per hit: the two punctured faces of each tetrahedron holding it are united (pm_unite,
//               one lane per (prism, step), for meshes with an edge of more than two triangles).
#include "common.h"
#include "offsets16.h"
#include "internal.h"
#include "uf_cached.h"

namespace ftk {

namespace {

struct PmMesh {
  const float* xy;      // [nv][2]
  const int* tri;       // [nf][3], ascending per row
  const int* edge;      // [ne][2], a < b, ascending
  const int* tri_edge;  // [nf][3]: edges (v0 v1), (v1 v2), (v0 v2)
  const float* field;   // [nt][2][nv]
  long long nv, nf, ne, S;
  int nt;
  float qscale;
};

// vertices (vertex, step offset) of local face f of a step, in global order
__device__ __forceinline__ void pm_face(const PmMesh& m, long long f, int* v, int* dt) {
  if (f < m.nf) {
    const int* a = m.tri + 3 * f;
    v[0] = a[0], v[1] = a[1], v[2] = a[2];
    dt[0] = dt[1] = dt[2] = 0;
  } else if (f < m.nf + 2 * m.ne) {
    const long long E = (f - m.nf) >> 1;
    const int up = (int)((f - m.nf) & 1);
    const int a = m.edge[2 * E], b = m.edge[2 * E + 1];
    v[0] = a, dt[0] = 0;
    v[1] = up ? a : b, dt[1] = up ? 1 : 0;
    v[2] = b, dt[2] = 1;
  } else {
    const long long T = (f - m.nf - 2 * m.ne) >> 1;
    const int up = (int)((f - m.nf - 2 * m.ne) & 1);
    const int* a = m.tri + 3 * T;
    v[0] = a[0], dt[0] = 0;
    v[1] = a[1], dt[1] = up;
    v[2] = a[2], dt[2] = 1;
  }
}

__device__ __forceinline__ void pm_q(const PmMesh& m, int v, int t, long long* q, unsigned& st) {
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const float x = m.field[((long long)t * 2 + c) * m.nv + v] * m.qscale;
    if (!isfinite(x)) {
      st |= ST_NONFINITE;
      q[c] = 0;
    } else if (!(fabsf(x) < 2147483648.0f)) {
      st |= ST_RANGE;
      q[c] = 0;
    } else {
      q[c] = (long long)rintf(x);
    }
  }
}

// SoS sign of det(a, b), columns in global vertex order: first nonzero of (a0 b1 - a1 b0, b1, -b0, -a1, -1)
__device__ __forceinline__ unsigned pm_sos2(const long long* a, const long long* b) {
  const long long d = a[0] * b[1] - a[1] * b[0];
  if (d != 0) return d > 0;
  if (b[1] != 0) return b[1] > 0;
  if (b[0] != 0) return b[0] < 0;
  if (a[1] != 0) return a[1] < 0;
  return 0u;
}

// quantised value of one field component (as pm_q)
__device__ __forceinline__ long long pm_q1(float v, float qscale, unsigned& st) {
  const float x = v * qscale;
  if (!isfinite(x)) {
    st |= ST_NONFINITE;
    return 0;
  }
  if (!(fabsf(x) < 2147483648.0f)) {
    st |= ST_RANGE;
    return 0;
  }
  return (long long)rintf(x);
}

// The field vertex-major, [nv][nt] pairs (u, v): a face's vertices are scattered over the mesh, so the test below
// reads each vertex's values for several steps from one or two cache lines instead of one line per step.  A
// workgroup moves a tile of 64 vertices x 16 steps through LDS: reads run along the vertices, writes along the steps
// of each vertex (128 contiguous bytes).
constexpr int kPmTV = 64, kPmTT = 16;
__global__ __launch_bounds__(256) void pm_vertex_major(const float* __restrict__ field, long long nv, int nt,
                                                       float2* __restrict__ ft) {
  __shared__ float tile[kPmTT][2][kPmTV + 1];
  const long long v0 = (long long)blockIdx.x * kPmTV;
  const int t0 = blockIdx.y * kPmTT;
  for (int e = threadIdx.x; e < kPmTT * 2 * kPmTV; e += 256) {
    const int dt = e / (2 * kPmTV), c = (e / kPmTV) & 1, dv = e % kPmTV;
    const long long v = v0 + dv;
    const int t = t0 + dt;
    tile[dt][c][dv] = (v < nv && t < nt) ? field[(long long)(2 * t + c) * nv + v] : 0.0f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kPmTV * kPmTT; e += 256) {
    const int dv = e / kPmTT, dt = e % kPmTT;
    const long long v = v0 + dv;
    const int t = t0 + dt;
    if (v < nv && t < nt) ft[v * nt + t] = make_float2(tile[dt][0][dv], tile[dt][1][dv]);
  }
}

// One lane per local face, all steps: the values of its vertices for a block of 8 steps (and the next step, for
// the interval faces) are loaded together, then each step's puncture test.
constexpr int kPmSteps = 8;
__global__ void pm_test(PmMesh m, const float2* __restrict__ ft, unsigned char* __restrict__ flag,
                        unsigned* __restrict__ status) {
  const long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= m.S) return;
  int v[3], dt[3];
  pm_face(m, f, v, dt);
  unsigned st = 0;
  for (int tb = 0; tb < m.nt; tb += kPmSteps) {
    float2 w[3][kPmSteps + 1];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k <= kPmSteps; ++k) w[i][k] = ft[(long long)v[i] * m.nt + min(tb + k, m.nt - 1)];
#pragma unroll
    for (int k = 0; k < kPmSteps; ++k) {
      const int t = tb + k;
      if (t >= m.nt) break;
      const long long id = (long long)t * m.S + f;
      if (f >= m.nf && t == m.nt - 1) {  // interval faces need step t + 1
        flag[id] = 0;
        continue;
      }
      long long q[3][2];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const float2 a = dt[i] ? w[i][k + 1] : w[i][k];
        q[i][0] = pm_q1(a.x, m.qscale, st);
        q[i][1] = pm_q1(a.y, m.qscale, st);
      }
      // cofactor signs +S(1,2), -S(0,2), +S(0,1) agree
      const unsigned s01 = pm_sos2(q[0], q[1]), s02 = pm_sos2(q[0], q[2]), s12 = pm_sos2(q[1], q[2]);
      flag[id] = (s12 == s01 && s02 != s01) ? 1 : 0;
    }
  }
  // every vertex value is checked by the ordinal faces of its triangles (each vertex belongs to one)
  if (st && f < m.nf) atomicOr(status, st);
}

__global__ void pm_emit(PmMesh m, const unsigned char* __restrict__ flag, const long long* __restrict__ base,
                        long long* __restrict__ face_id, float* __restrict__ pos, unsigned* __restrict__ parent) {
  const long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  if (f >= m.S) return;
  const long long id = (long long)t * m.S + f;
  if (!flag[id]) return;
  int v[3], dt[3];
  pm_face(m, f, v, dt);
  unsigned st = 0;
  long long q[3][2];
#pragma unroll
  for (int i = 0; i < 3; ++i) pm_q(m, v[i], t + dt[i], q[i], st);
  const long long C0 = q[1][0] * q[2][1] - q[1][1] * q[2][0];
  const long long C1 = -(q[0][0] * q[2][1] - q[0][1] * q[2][0]);
  const long long C2 = q[0][0] * q[1][1] - q[0][1] * q[1][0];
  double mu[3] = {1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0};
  if (C0 != 0 || C1 != 0 || C2 != 0) {
    const double D = ((double)C0 + (double)C1) + (double)C2;
    mu[0] = (double)C0 / D;
    mu[1] = (double)C1 / D;
    mu[2] = (double)C2 / D;
  }
  const long long o = off16(base, flag, id, false);
  face_id[o] = id;
  if (pos) {
    double p[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double c[3] = {(double)m.xy[2 * v[i]], (double)m.xy[2 * v[i] + 1], (double)(t + dt[i])};
#pragma unroll
      for (int k = 0; k < 3; ++k) p[k] = i == 0 ? mu[0] * c[k] : p[k] + mu[i] * c[k];
    }
    pos[o * 3 + 0] = (float)p[0];
    pos[o * 3 + 1] = (float)p[1];
    pos[o * 3 + 2] = (float)p[2];
  }
  parent[o] = (unsigned)o;
}

// Spacetime face ids of the sides of the three tetrahedra a0 a1 a2 b2, a0 a1 b1 b2, a0 b0 b1 b2 of the prism of
// triangle T between steps t and t + 1 (lower / upper edge and interior faces are +0 / +1).
__device__ __forceinline__ void pm_prism_tets(const PmMesh& m, long long T, int t, long long (&tet)[3][4]) {
  const long long base = (long long)t * m.S;
  const int* te = m.tri_edge + 3 * T;
  const long long e01 = base + m.nf + 2LL * te[0], e12 = base + m.nf + 2LL * te[1], e02 = base + m.nf + 2LL * te[2];
  const long long in = base + m.nf + 2 * m.ne + 2 * T;
  const long long ord0 = base + T, ord1 = base + m.S + T;
  const long long v[3][4] = {{ord0, in, e02, e12}, {e01, in, in + 1, e12 + 1}, {e01 + 1, e02 + 1, in + 1, ord1}};
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int j = 0; j < 4; ++j) tet[k][j] = v[k][j];
}

// One lane per hit (Alg. 1 pass 2 from the punctured faces' side): each tetrahedron of each prism holding the
// hit's face has exactly one other punctured side, united with it; any other count is an internal error.  Every
// tetrahedron with a punctured side is reached from its hits, so this is the all-prism pass below restricted to
// where it can act.  edge_tri: the (at most two) triangles of each mesh edge, -1 for none.
__global__ void pm_unite_hits(PmMesh m, const int* __restrict__ edge_tri, const unsigned char* __restrict__ flag,
                              const long long* __restrict__ gbase, const long long* __restrict__ face_id,
                              long long n_hits, unsigned* __restrict__ parent, unsigned* __restrict__ status) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_hits) return;
  const long long id = face_id[i];
  const int t = (int)(id / m.S);
  const long long f = id - (long long)t * m.S;
  long long pT[2] = {0, 0};
  int pt[2] = {0, 0}, np = 0;
  if (f < m.nf) {  // a mesh triangle: bottom of the prism above it, top of the one below
    if (t < m.nt - 1) {
      pT[np] = f;
      pt[np++] = t;
    }
    if (t >= 1) {
      pT[np] = f;
      pt[np++] = t - 1;
    }
  } else if (f < m.nf + 2 * m.ne) {  // an edge face: the prisms of the edge's triangles
    const long long E = (f - m.nf) >> 1;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int T = edge_tri[2 * E + k];
      if (T >= 0) {
        pT[np] = T;
        pt[np++] = t;
      }
    }
  } else {  // an interior face of one prism
    pT[np] = (f - m.nf - 2 * m.ne) >> 1;
    pt[np++] = t;
  }
  for (int p = 0; p < np; ++p) {
    long long tet[3][4];
    pm_prism_tets(m, pT[p], pt[p], tet);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (tet[k][0] != id && tet[k][1] != id && tet[k][2] != id && tet[k][3] != id) continue;
      int n = 0;
      long long other = -1;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (flag[tet[k][j]]) {
          ++n;
          if (tet[k][j] != id) other = tet[k][j];
        }
      if (n == 2)
        uf_unite_cached(parent, (unsigned)i, (unsigned)off16(gbase, flag, other, false));
      else
        atomicOr(status, ST_INVARIANT);
    }
  }
}

// One lane per (prism, step), for meshes with an edge of more than two triangles (no edge -> triangle table).
__global__ void pm_unite(PmMesh m, const unsigned char* __restrict__ flag, const long long* __restrict__ gbase,
                         unsigned* __restrict__ parent, unsigned* __restrict__ status) {
  const long long T = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  if (T >= m.nf || t >= m.nt - 1) return;
  long long tet[3][4];
  pm_prism_tets(m, T, t, tet);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    long long h[4];
    int n = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (flag[tet[k][j]]) h[n++] = off16(gbase, flag, tet[k][j], false);
    if (n == 2)
      uf_unite_cached(parent, (unsigned)h[0], (unsigned)h[1]);
    else if (n != 0)
      atomicOr(status, ST_INVARIANT);
  }
}

}  // namespace

hipError_t launch_pm_test(const float* xy, const int* tri, const int* edge, const int* tri_edge, const float* field,
                          long long nv, long long nf, long long ne, int nt, float qscale, float* ft_scratch,
                          unsigned char* flag, unsigned* status, hipStream_t s) {
  const PmMesh m{xy, tri, edge, tri_edge, field, nv, nf, ne, nf + 2 * ne + 2 * nf, nt, qscale};
  float2* ft = reinterpret_cast<float2*>(ft_scratch);
  pm_vertex_major<<<dim3((unsigned)((nv + kPmTV - 1) / kPmTV), (unsigned)((nt + kPmTT - 1) / kPmTT)), 256, 0, s>>>(
      field, nv, nt, ft);
  pm_test<<<(unsigned)((m.S + 255) / 256), 256, 0, s>>>(m, ft, flag, status);
  return hipGetLastError();
}

hipError_t launch_pm_emit(const float* xy, const int* tri, const int* edge, const int* tri_edge, const int* edge_tri,
                          const float* field, long long nv, long long nf, long long ne, int nt, float qscale,
                          const unsigned char* flag, const long long* base, long long n_hits, long long* face_id,
                          float* pos, unsigned* parent, unsigned* status, hipStream_t s) {
  const PmMesh m{xy, tri, edge, tri_edge, field, nv, nf, ne, nf + 2 * ne + 2 * nf, nt, qscale};
  pm_emit<<<dim3((unsigned)((m.S + 255) / 256), (unsigned)nt), 256, 0, s>>>(m, flag, base, face_id, pos, parent);
  if (edge_tri) {
    if (n_hits > 0)
      pm_unite_hits<<<(unsigned)((n_hits + 255) / 256), 256, 0, s>>>(m, edge_tri, flag, base, face_id, n_hits, parent,
                                                                    status);
  } else if (nt > 1) {
    pm_unite<<<dim3((unsigned)((nf + 255) / 256), (unsigned)(nt - 1)), 256, 0, s>>>(m, flag, base, parent, status);
  }
  return hipGetLastError();
}

}  // namespace ftk
