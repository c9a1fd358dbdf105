// vortex.hip -- quantum vortex surface tracking in 3D complex series (Sec. 6.1, two passes on the regular
// simplicial spacetime mesh; Alg. 1 middle column).
//
// The contour integral of the phase around a spacetime triangle, each edge's phase change wrapped into (-pi, pi],
// is 2 pi times the winding number of the image triangle (psi_0, psi_1, psi_2) around 0 (a straight segment that
// misses 0 turns by exactly the wrapped change).  So a triangle is positive when 0 lies inside its image: the
// puncture test of the 2-component field (Re psi, Im psi), decided exactly on quantised values with the symbolic
// perturbation (Sec. 4.3).  Its three cofactor signs are the SoS signs of the 2x2 determinants of the vertex pairs,
// i.e. of the triangle's edges, so one sign bit per spacetime edge is computed once and shared.
//
//   vx_edges -- one lane per vertex: SoS sign of det(q(p), q(p + e(M))) for the 15 edge masks M (bits x = 1, y = 2,
//               z = 4, t = 8), q = rint(psi * 2^s) below 2^31 so every 2x2 determinant is exact in 64 bits.
//   vx_tris  -- the 50 triangle types (M1, M2) anchored at each vertex (vertices p, p + e(a), p + e(b), a = M1,
//               b = M1 | M2): signs S01, S02 from the vertex's own edges, S12 from the edge (b ^ a) of p + e(a);
//               positive iff S12 == S01 and S02 != S01 (cofactor signs +S12, -S02, +S01 agree).
//   vx_emit  -- triangle ids g * 50 + type, the vortex point from the exact cofactors (Eq. 2), identity parents.
//   vx_unite -- per pentachoron: unite its positive triangle sides (3, 4 or 5 under the perturbation).
// Labels (smallest triangle id of each surface) come from the shared union-find label kernel.
#include "common.h"
#include "internal.h"
#include "kuhn.h"
#include "uf_cached.h"

namespace ftk {

namespace {

constexpr int kVxBX = 128;

struct VxGrid {
  const float* psi;  // [nt][2][nz][ny][nx]
  int nx, ny, nz, nt;
  float qscale;
};

__device__ __forceinline__ long long vx_vidx(const VxGrid& g, int x, int y, int z, int t) {
  return (((long long)t * g.nz + z) * g.ny + y) * g.nx + x;
}

// quantised (re, im) of a vertex; flags non-finite and out-of-range values
__device__ __forceinline__ void vx_q(const VxGrid& g, int x, int y, int z, int t, long long* q, unsigned& st) {
  const long long plane = (long long)g.nx * g.ny * g.nz;
  const long long off = ((long long)z * g.ny + y) * g.nx + x;
  const float* base = g.psi + (long long)t * 2 * plane;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const float v = base[c * plane + off] * g.qscale;
    if (!isfinite(v)) {
      st |= ST_NONFINITE;
      q[c] = 0;
    } else if (!(fabsf(v) < 2147483648.0f)) {
      st |= ST_RANGE;
      q[c] = 0;
    } else {
      q[c] = (long long)rintf(v);
    }
  }
}

// SoS sign of det(a, b) (columns in vertex order, entry (j, k) perturbed by eps^(2^(2k + j))): the first nonzero of
// (a0 b1 - a1 b0, b1, -b0, -a1, -1); 1 for positive
__device__ __forceinline__ unsigned vx_sos2(const long long* a, const long long* b) {
  const long long d = a[0] * b[1] - a[1] * b[0];
  if (d != 0) return d > 0;
  if (b[1] != 0) return b[1] > 0;
  if (b[0] != 0) return b[0] < 0;
  if (a[1] != 0) return a[1] < 0;
  return 0u;
}

__device__ __forceinline__ bool vx_corner_ok(const VxGrid& g, int x, int y, int z, int t, unsigned cm) {
  return x + (int)(cm & 1u) < g.nx && y + (int)((cm >> 1) & 1u) < g.ny && z + (int)((cm >> 2) & 1u) < g.nz &&
         t + (int)((cm >> 3) & 1u) < g.nt;
}

__global__ __launch_bounds__(kVxBX) void vx_edges(VxGrid g, unsigned short* __restrict__ emask,
                                                   unsigned* __restrict__ status) {
  const int x = blockIdx.x * kVxBX + threadIdx.x;
  const int y = blockIdx.y;
  const int z = blockIdx.z % g.nz, t = blockIdx.z / g.nz;
  if (x >= g.nx) return;
  unsigned st = 0;
  long long q0[2];
  vx_q(g, x, y, z, t, q0, st);
  unsigned m = 0;
  for (unsigned M = 1; M < 16; ++M) {
    if (!vx_corner_ok(g, x, y, z, t, M)) continue;
    long long q1[2];
    unsigned st1 = 0;  // each vertex reports its own values
    vx_q(g, x + (M & 1u), y + ((M >> 1) & 1u), z + ((M >> 2) & 1u), t + ((M >> 3) & 1u), q1, st1);
    m |= vx_sos2(q0, q1) << (M - 1);
  }
  emask[vx_vidx(g, x, y, z, t)] = (unsigned short)m;
  if (st) atomicOr(status, st);
}

__global__ __launch_bounds__(kVxBX) void vx_tris(VxGrid g, const unsigned short* __restrict__ emask,
                                                  unsigned long long* __restrict__ tmask, int* __restrict__ cnt) {
  const int x = blockIdx.x * kVxBX + threadIdx.x;
  const int y = blockIdx.y;
  const int z = blockIdx.z % g.nz, t = blockIdx.z / g.nz;
  if (x >= g.nx) return;
  const long long v = vx_vidx(g, x, y, z, t);
  const unsigned e0 = emask[v];
  unsigned ea[16];
#pragma unroll
  for (unsigned a = 1; a < 16; ++a)
    ea[a] = vx_corner_ok(g, x, y, z, t, a)
                ? emask[vx_vidx(g, x + (a & 1u), y + ((a >> 1) & 1u), z + ((a >> 2) & 1u), t + ((a >> 3) & 1u))]
                : 0u;
  ea[0] = e0;
  unsigned long long m = 0;
#pragma unroll
  for (int ty = 0; ty < 50; ++ty) {
    const unsigned a = kTri3.m[ty][0], b = a | kTri3.m[ty][1];
    if (!vx_corner_ok(g, x, y, z, t, b)) continue;
    const unsigned s01 = (e0 >> (a - 1)) & 1u, s02 = (e0 >> (b - 1)) & 1u, s12 = (ea[a] >> ((b ^ a) - 1)) & 1u;
    if (s12 == s01 && s02 != s01) m |= 1ull << ty;
  }
  tmask[v] = m;
  cnt[v] = __popcll(m);
}

__global__ __launch_bounds__(kVxBX) void vx_emit(VxGrid g, const unsigned long long* __restrict__ tmask,
                                                  const long long* __restrict__ hoff, long long* __restrict__ tri_id,
                                                  float* __restrict__ pos, unsigned* __restrict__ parent) {
  const int x = blockIdx.x * kVxBX + threadIdx.x;
  const int y = blockIdx.y;
  const int z = blockIdx.z % g.nz, t = blockIdx.z / g.nz;
  if (x >= g.nx) return;
  const long long v = vx_vidx(g, x, y, z, t);
  unsigned long long m = tmask[v];
  if (!m) return;
  long long o = hoff[v];
  unsigned st = 0;
  long long q0[2];
  vx_q(g, x, y, z, t, q0, st);
  while (m) {
    const int ty = __ffsll((long long)m) - 1;
    m &= m - 1;
    const unsigned a = kTri3.m[ty][0], b = a | kTri3.m[ty][1];
    long long q1[2], q2[2];
    vx_q(g, x + (a & 1u), y + ((a >> 1) & 1u), z + ((a >> 2) & 1u), t + ((a >> 3) & 1u), q1, st);
    vx_q(g, x + (b & 1u), y + ((b >> 1) & 1u), z + ((b >> 2) & 1u), t + ((b >> 3) & 1u), q2, st);
    // exact cofactors (each below 2^63); the nonzero ones share the puncture sign, so their sum has no
    // cancellation and binary64 weights carry one rounding each
    const long long C0 = q1[0] * q2[1] - q1[1] * q2[0];
    const long long C1 = -(q0[0] * q2[1] - q0[1] * q2[0]);
    const long long C2 = q0[0] * q1[1] - q0[1] * q1[0];
    double mu0 = 1.0 / 3.0, mu1 = 1.0 / 3.0, mu2 = 1.0 / 3.0;
    if (C0 != 0 || C1 != 0 || C2 != 0) {
      const double D = ((double)C0 + (double)C1) + (double)C2;
      mu0 = (double)C0 / D;
      mu1 = (double)C1 / D;
      mu2 = (double)C2 / D;
    }
    tri_id[o] = v * 50 + ty;
    if (pos) {
      const double c0[4] = {(double)x, (double)y, (double)z, (double)t};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double p1 = c0[k] + ((a >> k) & 1u), p2 = c0[k] + ((b >> k) & 1u);
        pos[o * 4 + k] = (float)((mu0 * c0[k] + mu1 * p1) + mu2 * p2);
      }
    }
    parent[o] = (unsigned)o;
    ++o;
  }
}

// chain corners of the 24 pentachoron types
struct VxPen {
  unsigned char c[24][5];
};
constexpr VxPen build_vx_pen() {
  VxPen r{};
  for (int ty = 0; ty < 24; ++ty) {
    int acc = 0;
    r.c[ty][0] = 0;
    for (int k = 0; k < 4; ++k) {
      acc |= kPen3.m[ty][k];
      r.c[ty][k + 1] = (unsigned char)acc;
    }
  }
  return r;
}
__constant__ VxPen kVxPen = build_vx_pen();

__global__ __launch_bounds__(kVxBX) void vx_unite(VxGrid g, const unsigned long long* __restrict__ tmask,
                                                   const long long* __restrict__ hoff, unsigned* __restrict__ parent) {
  const int x = blockIdx.x * kVxBX + threadIdx.x;
  const int y = blockIdx.y;
  const int z = blockIdx.z % g.nz, t = blockIdx.z / g.nz;
  if (x >= g.nx || x + 1 >= g.nx || y + 1 >= g.ny || z + 1 >= g.nz || t + 1 >= g.nt) return;
  // triangle sides of the cube's pentachora are anchored at chain corners with at most two axes
  unsigned long long tm[16];
  unsigned long long any = 0;
#pragma unroll
  for (unsigned a = 0; a < 16; ++a) {
    tm[a] = __popc(a) <= 2
                ? tmask[vx_vidx(g, x + (a & 1u), y + ((a >> 1) & 1u), z + ((a >> 2) & 1u), t + ((a >> 3) & 1u))]
                : 0ull;
    any |= tm[a];
  }
  if (!any) return;
  for (int pt = 0; pt < 24; ++pt) {
    long long first = -1;
    for (int i = 0; i < 3; ++i)
      for (int j = i + 1; j < 4; ++j)
        for (int k = j + 1; k < 5; ++k) {
          const unsigned ci = kVxPen.c[pt][i], cj = kVxPen.c[pt][j], ck = kVxPen.c[pt][k];
          const int ty = kTri3Index.idx[cj ^ ci][ck ^ cj];
          const unsigned long long mk = tm[ci];
          if (!((mk >> ty) & 1ull)) continue;
          const long long w = vx_vidx(g, x + (ci & 1u), y + ((ci >> 1) & 1u), z + ((ci >> 2) & 1u), t + ((ci >> 3) & 1u));
          const long long h = hoff[w] + __popcll(mk & ((1ull << ty) - 1ull));
          if (first < 0)
            first = h;
          else
            uf_unite_cached(parent, (unsigned)first, (unsigned)h);
        }
  }
}

dim3 vx_grid(const VxGrid& g) {
  return dim3((unsigned)((g.nx + kVxBX - 1) / kVxBX), (unsigned)g.ny, (unsigned)(g.nz * g.nt));
}

}  // namespace

hipError_t launch_vx_detect(const float* psi, int nx, int ny, int nz, int nt, float qscale, unsigned short* emask,
                            unsigned long long* tmask, int* cnt, unsigned* status, hipStream_t s) {
  const VxGrid g{psi, nx, ny, nz, nt, qscale};
  vx_edges<<<vx_grid(g), kVxBX, 0, s>>>(g, emask, status);
  vx_tris<<<vx_grid(g), kVxBX, 0, s>>>(g, emask, tmask, cnt);
  return hipGetLastError();
}

hipError_t launch_vx_emit(const float* psi, int nx, int ny, int nz, int nt, float qscale,
                          const unsigned long long* tmask, const long long* hoff, long long* tri_id, float* pos,
                          unsigned* parent, hipStream_t s) {
  const VxGrid g{psi, nx, ny, nz, nt, qscale};
  vx_emit<<<vx_grid(g), kVxBX, 0, s>>>(g, tmask, hoff, tri_id, pos, parent);
  vx_unite<<<vx_grid(g), kVxBX, 0, s>>>(g, tmask, hoff, parent);
  return hipGetLastError();
}

}  // namespace ftk
