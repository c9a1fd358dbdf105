// vortex.hip -- quantum vortex surface tracking in 3D complex series (Sec. 5.1, two passes on the regular
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
//   vx_unite -- per 4-cube: the positive sides of its pentachora (3, 4 or 5 per pentachoron under the
//               perturbation) united group by group.
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
  // the 15 corner vectors from clamped (in-grid) addresses, all loads in flight together; corners outside the grid
  // are dropped after
  long long q1[16][2];
#pragma unroll
  for (unsigned M = 1; M < 16; ++M) {
    unsigned st1 = 0;  // each vertex reports its own values
    vx_q(g, min(x + (int)(M & 1u), g.nx - 1), min(y + (int)((M >> 1) & 1u), g.ny - 1),
         min(z + (int)((M >> 2) & 1u), g.nz - 1), min(t + (int)((M >> 3) & 1u), g.nt - 1), q1[M], st1);
  }
#pragma unroll
  for (unsigned M = 1; M < 16; ++M)
    if (vx_corner_ok(g, x, y, z, t, M)) m |= vx_sos2(q0, q1[M]) << (M - 1);
  emask[vx_vidx(g, x, y, z, t)] = (unsigned short)m;
  if (st) atomicOr(status, st);
}

__global__ __launch_bounds__(kVxBX) void vx_tris(VxGrid g, const unsigned short* __restrict__ emask,
                                                  unsigned long long* __restrict__ tmask,
                                                  unsigned char* __restrict__ cnt) {
  const int x = blockIdx.x * kVxBX + threadIdx.x;
  const int y = blockIdx.y;
  const int z = blockIdx.z % g.nz, t = blockIdx.z / g.nz;
  if (x >= g.nx) return;
  const long long v = vx_vidx(g, x, y, z, t);
  const unsigned e0 = emask[v];
  // edge words of the 15 other corners from clamped (in-grid) addresses, all loads in flight together; a corner
  // outside the grid is never read below (a triangle is tested only when its corner b, a superset of a, is inside)
  unsigned ea[16];
#pragma unroll
  for (unsigned a = 1; a < 16; ++a)
    ea[a] = emask[vx_vidx(g, min(x + (int)(a & 1u), g.nx - 1), min(y + (int)((a >> 1) & 1u), g.ny - 1),
                          min(z + (int)((a >> 2) & 1u), g.nz - 1), min(t + (int)((a >> 3) & 1u), g.nt - 1))];
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
  cnt[v] = (unsigned char)__popcll(m);
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
    // cancellation, and binary64 weights from one reciprocal carry a few roundings each (relative error below
    // 2^-50, far inside the binary32 points written)
    const long long C0 = q1[0] * q2[1] - q1[1] * q2[0];
    const long long C1 = -(q0[0] * q2[1] - q0[1] * q2[0]);
    const long long C2 = q0[0] * q1[1] - q0[1] * q1[0];
    double mu0 = 1.0 / 3.0, mu1 = 1.0 / 3.0, mu2 = 1.0 / 3.0;
    if (C0 != 0 || C1 != 0 || C2 != 0) {
      const double rD = 1.0 / (((double)C0 + (double)C1) + (double)C2);
      mu0 = (double)C0 * rD;
      mu1 = (double)C1 * rD;
      mu2 = (double)C2 * rD;
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

// The triangles of a 4-cube's pentachora are its 110 corner chains ci < cj < ck (sets ordered by inclusion); local
// index k lists them in lexicographic order of (ci, cj, ck), with the anchor corner ci and the triangle type of
// masks (cj ^ ci, ck ^ cj); side[pt] is the 110-bit set (two words) of the 10 sides of pentachoron type pt.
constexpr int kCubeTriN = 110;
struct CubeTris {
  unsigned char ci[kCubeTriN], ty[kCubeTriN];
  unsigned long long side[24][2];
};
constexpr CubeTris build_cube_tris() {
  CubeTris r{};
  int cj_of[kCubeTriN] = {}, ck_of[kCubeTriN] = {};
  int n = 0;
  for (int ci = 0; ci < 16; ++ci)
    for (int cj = 0; cj < 16; ++cj)
      for (int ck = 0; ck < 16; ++ck) {
        const bool chain = cj != ci && (cj & ci) == ci && ck != cj && (ck & cj) == cj;
        if (!chain || n >= kCubeTriN) continue;
        r.ci[n] = (unsigned char)ci;
        r.ty[n] = (unsigned char)kTri3Index.idx[cj ^ ci][ck ^ cj];
        cj_of[n] = cj;
        ck_of[n] = ck;
        ++n;
      }
  for (int pt = 0; pt < 24; ++pt) {
    int c[5] = {0, 0, 0, 0, 0};
    for (int k = 0; k < 4; ++k) c[k + 1] = c[k] | kPen3.m[pt][k];
    for (int i = 0; i < 3; ++i)
      for (int j = i + 1; j < 4; ++j)
        for (int k = j + 1; k < 5; ++k)
          for (int l = 0; l < kCubeTriN; ++l)
            if (r.ci[l] == c[i] && cj_of[l] == c[j] && ck_of[l] == c[k]) r.side[pt][l >> 6] |= 1ull << (l & 63);
  }
  return r;
}
constexpr int count_chains() {
  int n = 0;
  for (int ci = 0; ci < 16; ++ci)
    for (int cj = 0; cj < 16; ++cj)
      for (int ck = 0; ck < 16; ++ck) n += cj != ci && (cj & ci) == ci && ck != cj && (ck & cj) == cj;
  return n;
}
static_assert(count_chains() == kCubeTriN, "110 corner chains (triangles) per 4-cube");
__constant__ CubeTris kCubeTris = build_cube_tris();

// Per 4-cube (anchor p with the whole cube in the grid): its positive triangles P (local set), grouped by "sides of a
// common pentachoron" (grow a group from its lowest member through the side sets until it is stable); each group
// member is united once with the group's first member.  Same connectivity as uniting the positive sides of every
// pentachoron, with |P| - groups unions instead of one star per pentachoron.
typedef unsigned __int128 u128;

__device__ __forceinline__ u128 side_set(int pt) {
  return ((u128)kCubeTris.side[pt][1] << 64) | (u128)kCubeTris.side[pt][0];
}

__device__ __forceinline__ int low_bit(u128 m) {
  const unsigned long long lo = (unsigned long long)m;
  return lo ? __ffsll((long long)lo) - 1 : 64 + __ffsll((long long)(unsigned long long)(m >> 64)) - 1;
}

// The pass is bound by the latency of the union finds: a register target of four waves per SIMD (128 VGPRs, a few
// spilled) hides more of it than the unconstrained three (14.6 -> 12.9 ms on 512 x 128 x 64 x 8).
__global__ __launch_bounds__(kVxBX) __attribute__((amdgpu_waves_per_eu(4))) void vx_unite(VxGrid g, const unsigned long long* __restrict__ tmask,
                                                   const long long* __restrict__ hoff, unsigned* __restrict__ parent) {
  // anchor corner and type of each local triangle, read per union with a lane-dependent index: an LDS copy keeps
  // a global table read out of the chain of dependent loads (table, hit offset, parents)
  __shared__ unsigned char s_ci[kCubeTriN], s_ty[kCubeTriN];
  if (threadIdx.x < kCubeTriN) {
    s_ci[threadIdx.x] = kCubeTris.ci[threadIdx.x];
    s_ty[threadIdx.x] = kCubeTris.ty[threadIdx.x];
  }
  __syncthreads();
  const int x = blockIdx.x * kVxBX + threadIdx.x;
  const int y = blockIdx.y;
  const int z = blockIdx.z % g.nz, t = blockIdx.z / g.nz;
  if (x >= g.nx || x + 1 >= g.nx || y + 1 >= g.ny || z + 1 >= g.nz || t + 1 >= g.nt) return;
  // triangle sides are anchored at chain corners with at most two axes
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
  u128 P = 0;
  for (int k = 0; k < kCubeTriN; ++k)
    if ((tm[kCubeTris.ci[k]] >> kCubeTris.ty[k]) & 1ull) P |= (u128)1 << k;
  auto hit = [&](int k) -> long long {
    const unsigned a = s_ci[k];
    const int ty = s_ty[k];
    const long long w = vx_vidx(g, x + (a & 1u), y + ((a >> 1) & 1u), z + ((a >> 2) & 1u), t + ((a >> 3) & 1u));
    return hoff[w] + __popcll(tm[a] & ((1ull << ty) - 1ull));
  };
  u128 R = P;
  while (R) {
    u128 C = (u128)1 << low_bit(R), prev;
    do {
      prev = C;
      for (int pt = 0; pt < 24; ++pt) {
        const u128 S = side_set(pt) & P;
        if (S & C) C |= S;
      }
    } while (C != prev);
    R &= ~C;
    const int k0 = low_bit(C);
    const long long h0 = hit(k0);
    C &= ~((u128)1 << k0);
    unsigned r = C ? uf_find_cached(parent, (unsigned)h0) : 0u;
    while (C) {
      const int k = low_bit(C);
      C &= ~((u128)1 << k);
      r = uf_unite_into(parent, r, (unsigned)hit(k));
    }
  }
}

dim3 vx_grid(const VxGrid& g) {
  return dim3((unsigned)((g.nx + kVxBX - 1) / kVxBX), (unsigned)g.ny, (unsigned)(g.nz * g.nt));
}

}  // namespace

hipError_t launch_vx_detect(const float* psi, int nx, int ny, int nz, int nt, float qscale, unsigned short* emask,
                            unsigned long long* tmask, unsigned char* cnt, unsigned* status, hipStream_t s) {
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
