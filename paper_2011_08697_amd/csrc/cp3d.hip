// cp3d.hip -- critical-point tracking in 3D space + time on gfx950.
//
// Mesh: the Kuhn subdivision of the (x, y, z, t) grid (Sec. 3.3): per vertex 15 edge, 50 triangle, 60 tetrahedron
// (the tested faces) and 24 pentachoron (cell) types.  A tetrahedron is punctured when the four signed cofactors of
// (v0 v1 v2 v3 ; 1 1 1 1) agree (Sec. 4.3, Eq. 2); each cofactor is, up to a fixed sign, the 3x3 determinant of the
// vectors of one of its triangles, so one SoS sign bit per triangle (50 per vertex, a 64-bit word) is computed and
// shared through LDS.
//
//   detect3d -- time-marching slab kernel over a 16 x 8 x 4 anchor tile: gradient stencils read from global memory
//               (L2-cached neighbours) and quantised into LDS, triangle sign words of the tile (+1 halo), 60
//               tetrahedron tests per anchor; writes a 60-bit puncture mask per vertex and the hit count of every
//               16-vertex row segment.  Without a staged field plane the block's LDS (38.5 KB) admits four blocks
//               per CU, and the register target of four waves per SIMD matches it.
//   emit3d   -- one lane per vertex (hits are sparse in 3D): output index from the segment prefix, exact cofactors,
//               sublocation, Hessian type, and the union-find links of the hit's two pentachora (Alg. 1 pass 2).
#include "common.h"
#include "internal.h"

namespace ftk {

namespace {

constexpr int TX3 = 16, TY3 = 8, TZ3 = 4;
constexpr int SEG3 = 16;  // row segment width (x)

constexpr unsigned long long kTetUseX = types_using_axis(kTet3, 1);
constexpr unsigned long long kTetUseY = types_using_axis(kTet3, 2);
constexpr unsigned long long kTetUseZ = types_using_axis(kTet3, 4);
constexpr unsigned long long kTetUseT = types_using_axis(kTet3, 8);

// triangle types without the time axis (ordinal) and with it (interval)
struct TriSplit {
  int n_ord, n_int;
  unsigned char ord[50], itv[50];
};
constexpr TriSplit build_tri_split() {
  TriSplit r{};
  for (int i = 0; i < kTri3.count; ++i) {
    if ((kTri3.m[i][0] | kTri3.m[i][1]) & 8)
      r.itv[r.n_int++] = (unsigned char)i;
    else
      r.ord[r.n_ord++] = (unsigned char)i;
  }
  return r;
}
constexpr TriSplit kTriSplit = build_tri_split();
static_assert(kTriSplit.n_ord == 12 && kTriSplit.n_int == 38, "12 ordinal + 38 interval triangle types");

template <bool WIDE>
struct Q3;
template <>
struct Q3<false> {
  typedef float T;  // integers below 2^20, exact in binary32
};
template <>
struct Q3<true> {
  typedef long long T;
};

__device__ __forceinline__ long long fpl3(const Grid3& g, int t) { return g.f_ring ? t % g.f_ring : t; }
__device__ __forceinline__ long long mpl3(const Grid3& g, int t) { return g.m_ring ? t % g.m_ring : t; }

template <bool WIDE>
__device__ __forceinline__ typename Q3<WIDE>::T to_q3(float r, unsigned& st) {
  if (!WIDE) {
    if (!(fabsf(r) < 1048576.0f)) {  // 2^20: every 3x3 determinant fits in 64 bits
      st |= ST_WIDE;
      return 0.0f;
    }
    return r;
  } else {
    if (!(fabsf(r) < 2199023255552.0f)) {  // 2^41: every 3x3 determinant fits in 128 bits
      st |= ST_RANGE;
      return 0;
    }
    return (long long)r;
  }
}

// Exact 3x3 determinant of columns a, b, c (rows = components): 64-bit when |entries| < 2^20, else 128-bit.
template <bool WIDE, typename Q>
__device__ __forceinline__ i128 det3x(const Q* a, const Q* b, const Q* c) {
  if (!WIDE) {
    long long m0 = (long long)b[1] * c[2] - (long long)b[2] * c[1];
    long long m1 = (long long)b[0] * c[2] - (long long)b[2] * c[0];
    long long m2 = (long long)b[0] * c[1] - (long long)b[1] * c[0];
    return (i128)((long long)a[0] * m0 - (long long)a[1] * m1 + (long long)a[2] * m2);
  }
  i128 m0 = (i128)b[1] * c[2] - (i128)b[2] * c[1];
  i128 m1 = (i128)b[0] * c[2] - (i128)b[2] * c[0];
  i128 m2 = (i128)b[0] * c[1] - (i128)b[1] * c[0];
  return (i128)a[0] * m0 - (i128)a[1] * m1 + (i128)a[2] * m2;
}

// SoS sign of the 3x3 determinant m[j][k] (row j = component, column k = vertex in index order), entry (j, k)
// perturbed by eps^(2^(3k+j)).  Expanding the perturbed determinant and ordering its terms by exponent, the sign
// is that of the first nonzero of
//   det, C00, C10, C20, C01, -m22, m12, C11, m22, -m02, C21, -m12, m02, C02, m21, -m11, -m20, -1
// with C_jk = (-1)^(j+k) times the 2x2 minor without row j and column k.  Returned as a bit: 1 for positive.
// (values passed by register: columns a = m[.][0], b = m[.][1], c = m[.][2])
__device__ __noinline__ unsigned sos3_tail(long long a0, long long a1, long long a2, long long b0, long long b1,
                                           long long b2, long long c0, long long c1, long long c2) {
  const i128 m00 = a0, m10 = a1, m20 = a2;
  const i128 m01 = b0, m11 = b1, m21 = b2;
  const i128 m02 = c0, m12 = c1, m22 = c2;
  i128 v;
  v = m11 * m22 - m12 * m21;          // C00
  if (v != 0) return v > 0;
  v = -(m01 * m22 - m02 * m21);       // C10
  if (v != 0) return v > 0;
  v = m01 * m12 - m02 * m11;          // C20
  if (v != 0) return v > 0;
  v = -(m10 * m22 - m12 * m20);       // C01
  if (v != 0) return v > 0;
  if (m22 != 0) return m22 < 0;       // -m22
  if (m12 != 0) return m12 > 0;       // m12
  v = m00 * m22 - m02 * m20;          // C11
  if (v != 0) return v > 0;
  // m22 == 0 here, so the next term (m22) vanishes
  if (m02 != 0) return m02 < 0;       // -m02
  v = -(m00 * m12 - m02 * m10);       // C21
  if (v != 0) return v > 0;
  // m12 == 0 and m02 == 0 here
  v = m10 * m21 - m11 * m20;          // C02
  if (v != 0) return v > 0;
  if (m21 != 0) return m21 > 0;       // m21
  if (m11 != 0) return m11 < 0;       // -m11
  if (m20 != 0) return m20 < 0;       // -m20
  return 0u;                          // -1
}

template <bool WIDE, typename Q>
__device__ __forceinline__ unsigned sos3_positive(const Q* a, const Q* b, const Q* c) {
  const i128 d = det3x<WIDE, Q>(a, b, c);
  if (d != 0) return d > 0;
  return sos3_tail(a[0], a[1], a[2], b[0], b[1], b[2], c[0], c[1], c[2]);
}

// The same sequence in binary64 for narrow entries (integers below 2^20): every term is an entry or a 2x2 minor,
// whose two products (below 2^40) and difference are exact in binary64.
__device__ __forceinline__ unsigned sos3_tail_f64(double m00, double m10, double m20, double m01, double m11,
                                                  double m21, double m02, double m12, double m22) {
  auto mn = [](double x, double y, double z, double w) { return __builtin_fma(x, y, -(z * w)); };  // exact
  double v;
  v = mn(m11, m22, m12, m21);         // C00
  if (v != 0.0) return v > 0.0;
  v = -mn(m01, m22, m02, m21);        // C10
  if (v != 0.0) return v > 0.0;
  v = mn(m01, m12, m02, m11);         // C20
  if (v != 0.0) return v > 0.0;
  v = -mn(m10, m22, m12, m20);        // C01
  if (v != 0.0) return v > 0.0;
  if (m22 != 0.0) return m22 < 0.0;   // -m22
  if (m12 != 0.0) return m12 > 0.0;   // m12
  v = mn(m00, m22, m02, m20);         // C11
  if (v != 0.0) return v > 0.0;
  if (m02 != 0.0) return m02 < 0.0;   // -m02 (m22 == 0 here)
  v = -mn(m00, m12, m02, m10);        // C21
  if (v != 0.0) return v > 0.0;
  v = mn(m10, m21, m11, m20);         // C02 (m12 == m02 == 0 here)
  if (v != 0.0) return v > 0.0;
  if (m21 != 0.0) return m21 > 0.0;   // m21
  if (m11 != 0.0) return m11 < 0.0;   // -m11
  if (m20 != 0.0) return m20 < 0.0;   // -m20
  return 0u;                          // -1
}

// Exact evaluation for narrow entries (below 2^20: minors below 2^41, terms below 2^61), then SoS.  A zero column
// makes the determinant vanish without evaluating it (frequent where gradients underflow the quantum); the
// sequence that follows runs in binary64, exactly.
__device__ __forceinline__ unsigned sos3_exact_narrow(float a0, float a1, float a2, float b0, float b1, float b2,
                                                      float c0, float c1, float c2) {
  const bool zero_col = (a0 == 0.0f && a1 == 0.0f && a2 == 0.0f) || (b0 == 0.0f && b1 == 0.0f && b2 == 0.0f) ||
                        (c0 == 0.0f && c1 == 0.0f && c2 == 0.0f);
  if (!zero_col) {
    const long long A0 = (long long)a0, A1 = (long long)a1, A2 = (long long)a2;
    const long long B0 = (long long)b0, B1 = (long long)b1, B2 = (long long)b2;
    const long long C0 = (long long)c0, C1 = (long long)c1, C2 = (long long)c2;
    const long long m0 = B1 * C2 - B2 * C1, m1 = B0 * C2 - B2 * C0, m2 = B0 * C1 - B1 * C0;
    const long long d = A0 * m0 - A1 * m1 + A2 * m2;
    if (d != 0) return d > 0;
  }
  return sos3_tail_f64(a0, a1, a2, b0, b1, b2, c0, c1, c2);
}

// Narrow sign of det(a, b, c): the 2x2 minors are exact in binary64 (integers below 2^41); the three products and
// two sums carry at most 3u (sum |p_i|) of rounding error (u = 2^-53), so |s| > 4e-16 sum |p_i| fixes the sign;
// otherwise (including every vanishing determinant) the exact integer evaluation and SoS decide.
__device__ __forceinline__ unsigned sos3_positive_narrow(float fa0, float fa1, float fa2, float fb0, float fb1,
                                                         float fb2, float fc0, float fc1, float fc2) {
  const double b0 = fb0, b1 = fb1, b2 = fb2, c0 = fc0, c1 = fc1, c2 = fc2;
  const double m0 = __builtin_fma(b1, c2, -(b2 * c1));
  const double m1 = __builtin_fma(b0, c2, -(b2 * c0));
  const double m2 = __builtin_fma(b0, c1, -(b1 * c0));
  const double p0 = (double)fa0 * m0, p1 = (double)fa1 * m1, p2 = (double)fa2 * m2;
  const double sdet = (p0 - p1) + p2;
  const double bound = ((fabs(p0) + fabs(p1)) + fabs(p2)) * 4e-16;
  if (fabs(sdet) > bound) return sdet > 0.0;
  return sos3_exact_narrow(fa0, fa1, fa2, fb0, fb1, fb2, fc0, fc1, fc2);
}

template <bool WIDE, typename Q>
__device__ __forceinline__ unsigned tri_sign(const Q* a, const Q* b, const Q* c) {
  if constexpr (!WIDE)
    return sos3_positive_narrow(a[0], a[1], a[2], b[0], b[1], b[2], c[0], c[1], c[2]);
  else
    return sos3_positive<true, Q>(a, b, c);
}

}  // namespace

// compile-time triangle lists of the two passes (ordinal types of a plane; interval types towards the next one)
struct OrdList {
  static constexpr int n = 12;
  static constexpr bool assign = true;
  static constexpr int ti(int k) { return kTriSplit.ord[k]; }
};
struct ItvList {
  static constexpr int n = 38;
  static constexpr bool assign = false;
  static constexpr int ti(int k) { return kTriSplit.itv[k]; }
};

// ---------------------------------------------------------------------------------------------------------------
// Pass 1: detection.  grid = (ceil(nx/16), ceil(ny/8) * ceil(nz/4), ceil(nt/TT)), block = 256.
// ---------------------------------------------------------------------------------------------------------------
template <bool WIDE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WIDE ? 2 : 4))) void detect3d(
    Grid3 g, int TT, int nyt, uint64_t* __restrict__ masks, int* __restrict__ seg_cnt, unsigned* __restrict__ status) {
  typedef typename Q3<WIDE>::T Q;
  constexpr int QX = TX3 + 2, QY = TY3 + 2, QZ = TZ3 + 2;  // quantised vectors: x0 .. x0+TX+1
  constexpr int WX = TX3 + 1, WY = TY3 + 1, WZ = TZ3 + 1;  // triangle words: x0 .. x0+TX
  constexpr int QN = QX * QY * QZ, WN = WX * WY * WZ;
  __shared__ Q qs[2][3][QN];
  __shared__ unsigned long long tw[2][WN];
  __shared__ unsigned s_tri[50];
  __shared__ int s_cdelta[16];
  __shared__ unsigned char s_tcor[50];  // triangle type -> corner a | corner b << 4

  const int tid = threadIdx.x;
  if (tid < 50) {
    const int k = tid;
    const int ti = k < 12 ? kTriSplit.ord[k] : kTriSplit.itv[k - 12];
    const int ca = kTri3.m[ti][0], cb = ca | kTri3.m[ti][1];
    s_tri[k] = (unsigned)ti | ((unsigned)ca << 8) | ((unsigned)cb << 12);
  }
  if (tid < 16) s_cdelta[tid] = (((tid >> 2) & 1) * QY + ((tid >> 1) & 1)) * QX + (tid & 1);
  if (tid < 50) s_tcor[tid] = (unsigned char)(kTri3.m[tid][0] | ((kTri3.m[tid][0] | kTri3.m[tid][1]) << 4));
  __syncthreads();
  const int nx = g.nx, ny = g.ny, nz = g.nz, nt = g.nt;
  // logical tile of this workgroup (XCD-contiguous ranges of tiles, x fastest, then y, z, slab; an x, z, y order
  // read 14% less but ran 9% slower)
  const unsigned nb = gridDim.x * gridDim.y * gridDim.z;
  const unsigned L = xcd_remap(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), nb);
  const int bxl = (int)(L % gridDim.x), byz = (int)((L / gridDim.x) % gridDim.y), bsl = (int)(L / (gridDim.x * gridDim.y));
  const int x0 = bxl * TX3;
  const int by = byz % nyt, bz = byz / nyt;
  const int y0 = by * TY3, z0 = bz * TZ3;
  const int t0 = g.t_begin + bsl * TT, t1 = min(t0 + TT, g.t_end);
  const long long plane = (long long)nx * ny * nz;
  unsigned st = 0;
  unsigned facts = 0x7Fu;  // sign facts of the gradients quantised by this thread since the last plane_facts()

  // Quantised gradients of plane tq into slot par.  fetch(): the thread's share of the plane's field block with a
  // one-cell halo, from clamped (in-grid) addresses into registers, all loads in flight together; halo cells
  // outside the grid hold copies of edge values, which diff3 never reads (one-sided differences at the first and
  // last index).  quantise(par): the block into the LDS of slot par (its previous plane is dead by then), the
  // stencils from LDS, then the quantised vectors into the slot.  Every thread reaches quantise() (it contains
  // barriers).
  constexpr int SX = QX + 2, SY = QY + 2, SZ = QZ + 2, SN = SX * SY * SZ;
  constexpr int NS = (SN + 255) / 256, NE = (QN + 255) / 256;
  static_assert(SN * sizeof(float) <= sizeof(qs[0]), "staged field block exceeds the plane slot");
  float fv[NS];
  auto fetch = [&](int tq) {
    const float* src = g.f + fpl3(g, tq) * plane;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      int e = tid + 256 * i;
      asm volatile("" : "+v"(e));  // opaque: the index math is redone per plane, not held in registers across steps
      const int lx = e % SX, r = e / SX, ly = r % SY, lz = r / SY;
      const int cx = min(max(x0 - 1 + lx, 0), nx - 1), cy = min(max(y0 - 1 + ly, 0), ny - 1);
      const int cz = min(max(z0 - 1 + lz, 0), nz - 1);
      fv[i] = src[((long long)cz * ny + cy) * nx + cx];
    }
  };
  auto quantise = [&](int par) {
    float* fb = reinterpret_cast<float*>(&qs[par][0][0]);
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int e = tid + 256 * i;
      if (e < SN) fb[e] = fv[i];
    }
    __syncthreads();
    Q q[NE][3];
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      int e = tid + 256 * i;
      asm volatile("" : "+v"(e));
      q[i][0] = q[i][1] = q[i][2] = 0;
      if (e < QN) {
        const int lx = e % QX, r = e / QX, ly = r % QY, lz = r / QY;
        const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
        if (gx < nx && gy < ny && gz < nz) {
          const float* c = fb + ((lz + 1) * SY + (ly + 1)) * SX + (lx + 1);
          const float c0 = c[0];
          if (!isfinite(c0)) st |= ST_NONFINITE;  // every vertex is the centre of some tile's element
          const float v0 = diff3(c[-1], c0, c[1], gx, nx);
          const float v1 = diff3(c[-SX], c0, c[SX], gy, ny);
          const float v2 = diff3(c[-SX * SY], c0, c[SX * SY], gz, nz);
          q[i][0] = to_q3<WIDE>(quant(v0, g.qscale), st);
          q[i][1] = to_q3<WIDE>(quant(v1, g.qscale), st);
          q[i][2] = to_q3<WIDE>(quant(v2, g.qscale), st);
          facts &= (q[i][0] > (Q)0 ? 1u : 0u) | (q[i][0] < (Q)0 ? 2u : 0u) | (q[i][1] > (Q)0 ? 4u : 0u) |
                   (q[i][1] < (Q)0 ? 8u : 0u) | (q[i][2] > (Q)0 ? 16u : 0u) | (q[i][2] < (Q)0 ? 32u : 0u) |
                   ((q[i][0] == (Q)0 && q[i][1] == (Q)0 && q[i][2] == (Q)0) ? 64u : 0u);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = tid + 256 * i;
      if (e < QN) {
        qs[par][0][e] = q[i][0];
        qs[par][1][e] = q[i][1];
        qs[par][2][e] = q[i][2];
      }
    }
  };
  // Triangle sign words.  Triangle type ti = (M1, M2) anchored at p has vertices at the unit 4-cube corners
  // 0, a = M1, b = M1|M2 (corner bit 0 x, 1 y, 2 z, 3 t; a corner with the t bit lies in the next plane).
  // s_tri[k] = ti | a << 8 | b << 12, ordinal types first (k < 12), then interval ones.
  auto tris = [&](int par, int kbeg, int kend, bool assign) {
    const Q* q0p = qs[par][0];
    for (int e = tid; e < WN; e += 256) {
      const int wx = e % WX, r = e / WX, wy = r % WY, wz = r / WY;
      const int base = (wz * QY + wy) * QX + wx;
      const Q a0 = qs[par][0][base], a1 = qs[par][1][base], a2 = qs[par][2][base];
      unsigned long long w = 0;
#pragma unroll 2
      for (int k = kbeg; k < kend; ++k) {
        const unsigned tk = s_tri[k];
        const int ti = tk & 63, ca = (tk >> 8) & 15, cb = (tk >> 12) & 15;
        const int ia = base + s_cdelta[ca], ib = base + s_cdelta[cb];
        const int pa = (ca >> 3) ? (par ^ 1) : par, pb = (cb >> 3) ? (par ^ 1) : par;
        const Q qa[3] = {qs[pa][0][ia], qs[pa][1][ia], qs[pa][2][ia]};
        const Q qb[3] = {qs[pb][0][ib], qs[pb][1][ib], qs[pb][2][ib]};
        const Q q0[3] = {a0, a1, a2};
        w |= (unsigned long long)tri_sign<WIDE, Q>(q0, qa, qb) << ti;
      }
      if (assign)
        tw[par][e] = w;
      else
        tw[par][e] |= w;
    }
    (void)q0p;
  };
  // Narrow variant: det(c0, ca, cb) = (c0 x ca) . cb.  The cross product of two quantised vectors (below 2^20)
  // is exact in binary64 (components below 2^41) and shared by every triangle with the same corner a; the dot
  // product carries at most 3u sum |p_i| of rounding error, so |s| > 4e-16 sum |p_i| fixes the sign, as in
  // sos3_positive_narrow.  Undecided triangles (every vanishing determinant among them) take the exact integer
  // evaluation and SoS afterwards.
  auto tris_narrow = [&](int ap, auto list) {
    constexpr int N = decltype(list)::n;
    const int op = ap ^ 1;
    for (int e0 = tid; e0 < WN; e0 += 256) {
      int e = e0;
      asm volatile("" : "+v"(e));  // opaque: positions are recomputed per pass, not held across steps
      const int wx = e % WX, r = e / WX, wy = r % WY, wz = r / WY;
      const int base = (wz * QY + wy) * QX + wx;
      auto ld = [&](int cm, int comp) -> double {
        return (double)qs[(cm >> 3) ? op : ap][comp][base + (((cm >> 2) & 1) * QY + ((cm >> 1) & 1)) * QX + (cm & 1)];
      };
      const double u0 = ld(0, 0), u1 = ld(0, 1), u2 = ld(0, 2);
      unsigned long long w = 0, slow = 0;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const int ti = decltype(list)::ti(k);
        const int a = kTri3.m[ti][0], b = a | kTri3.m[ti][1];
        const double a0 = ld(a, 0), a1 = ld(a, 1), a2 = ld(a, 2);
        const double X0 = __builtin_fma(u1, a2, -(u2 * a1));
        const double X1 = __builtin_fma(u2, a0, -(u0 * a2));
        const double X2 = __builtin_fma(u0, a1, -(u1 * a0));
        const double b0 = ld(b, 0), b1 = ld(b, 1), b2 = ld(b, 2);
        const double p0 = X0 * b0, p1 = X1 * b1, p2 = X2 * b2;
        const double sdet = (p0 + p1) + p2;
        const double bound = ((fabs(p0) + fabs(p1)) + fabs(p2)) * 4e-16;
        w |= (unsigned long long)(sdet > 0.0) << ti;
        slow |= (unsigned long long)!(fabs(sdet) > bound) << ti;
      }
      while (slow) {
        const int ti = __ffsll((long long)slow) - 1;
        slow &= slow - 1;
        const int cc = s_tcor[ti], a = cc & 15, b = cc >> 4;
        const unsigned bit = sos3_exact_narrow((float)u0, (float)u1, (float)u2, (float)ld(a, 0), (float)ld(a, 1),
                                               (float)ld(a, 2), (float)ld(b, 0), (float)ld(b, 1), (float)ld(b, 2));
        w = (w & ~(1ull << ti)) | ((unsigned long long)bit << ti);
      }
      if (decltype(list)::assign)
        tw[ap][e] = w;
      else
        tw[ap][e] |= w;
    }
  };
  auto ordinal_tris = [&](int par) {
    if constexpr (!WIDE)
      tris_narrow(par, OrdList{});
    else
      tris(par, 0, 12, true);
  };
  auto interval_tris = [&](int par) {
    if constexpr (!WIDE)
      tris_narrow(par, ItvList{});
    else
      tris(par, 12, 50, false);
  };

  // Sign facts of a plane's quantised gradients over the tile (anchors and their +1 neighbours, inside the grid):
  // bits 2c / 2c+1: component c > 0 / < 0 at every vertex; bit 6: every vector zero.  When a fact holds on both
  // planes of a step, no tetrahedron anchored in the tile at that step is punctured: a component of one strict
  // sign at all four vertices keeps its sign under the symbolic perturbation, so the origin is outside; with all
  // vectors zero every triangle determinant takes the perturbation's last term (-1), so the four cofactor signs
  // never agree.  The triangle and tetrahedron passes of such a step are skipped (masks and counts zero).
  __shared__ unsigned s_fact[2];
  __shared__ int s_ord_ok[2];  // the ordinal triangle words of the plane slot have been computed
  const int lane = tid & 63;
  auto plane_facts = [&](int p) {  // block reduction of the facts gathered while the plane was quantised
    const unsigned bits = facts;
    facts = 0x7Fu;
    unsigned wb = 0;
#pragma unroll
    for (int k = 0; k < 7; ++k)
      if (__ballot(!((bits >> k) & 1u)) == 0) wb |= 1u << k;
    if (lane == 0) atomicAnd(&s_fact[p], wb);
  };

  if (tid == 0) {
    s_fact[0] = s_fact[1] = 0x7Fu;
    s_ord_ok[0] = s_ord_ok[1] = 0;
  }
  __syncthreads();
  fetch(t0);
  quantise(t0 & 1);
  plane_facts(t0 & 1);

  for (int t = t0; t < t1; ++t) {
    const int par = t & 1, nxp = par ^ 1;
    const bool has_next = t + 1 < nt;
    __syncthreads();  // previous tetrahedron pass done; facts and flags of plane t visible
    if (has_next) {  // s_fact[nxp] was reset at the end of the previous step (or in the prologue)
      fetch(t + 1);
      quantise(nxp);
      plane_facts(nxp);
      __syncthreads();  // quantised plane and its facts visible
    }
    const bool certified = (s_fact[par] & (has_next ? s_fact[nxp] : 0x7Fu)) != 0u;  // uniform
    if (!certified) {
      if (s_ord_ok[par] == 0) ordinal_tris(par);  // each thread ORs into the words it assigned here
      if (has_next) {
        ordinal_tris(nxp);
        interval_tris(par);
      }
    }
    __syncthreads();
    if (tid == 0) {
      if (has_next) s_ord_ok[nxp] = certified ? 0 : 1;
      s_fact[par] = 0x7Fu;  // plane t's facts are not read again; the slot receives plane t + 2's
      g.cert[((mpl3(g, t) * ((nz + TZ3 - 1) / TZ3) + bz) * nyt + by) * gridDim.x + bxl] = certified ? 1 : 0;
    }

    // 60 tetrahedron tests for the TX x TY x TZ anchors, 2 per thread; lanes of a wave: 16 x 4 rows
    for (int a0 = tid; a0 < TX3 * TY3 * TZ3; a0 += 256) {
      int a = a0;
      asm volatile("" : "+v"(a));
      const int lx = a % TX3, r = a / TX3, ly = r % TY3, lz = r / TY3;
      const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
      unsigned long long m = 0;
      const bool in = gx < nx && gy < ny && gz < nz;
      if (in && !certified) {
        const int w0 = (lz * WY + ly) * WX + lx;
        unsigned long long W[16];
#pragma unroll
        for (int cm = 0; cm < 16; ++cm) {
          // neighbour p + e(cm); only masks with at most two axes are used as M1
          const int dz = (cm >> 2) & 1, dy = (cm >> 1) & 1, dx = cm & 1;
          const int p = (cm >> 3) ? nxp : par;
          W[cm] = (__popc((unsigned)cm) <= 2 && (!(cm >> 3) || has_next)) ? tw[p][w0 + (dz * WY + dy) * WX + dx] : 0ull;
        }
#pragma unroll
        for (int k = 0; k < 60; ++k) {
          const int m1 = kTet3.m[k][0], m2 = kTet3.m[k][1], m3 = kTet3.m[k][2];
          // sides opposite v0..v3: (p+e(M1); M2, M3), (p; M1|M2, M3), (p; M1, M2|M3), (p; M1, M2); cofactor signs
          // -S0, +S1, -S2, +S3: punctured iff S1 = S3 and S0, S2 differ from them
          const unsigned long long e0 = (W[m1] >> kTri3Index.idx[m2][m3]) & 1ull;
          const unsigned long long e1 = (W[0] >> kTri3Index.idx[m1 | m2][m3]) & 1ull;
          const unsigned long long e2 = (W[0] >> kTri3Index.idx[m1][m2 | m3]) & 1ull;
          const unsigned long long e3 = (W[0] >> kTri3Index.idx[m1][m2]) & 1ull;
          m |= (((e1 == e3) & (e0 != e1) & (e2 != e1)) ? 1ull : 0ull) << k;
        }
        unsigned long long valid = (1ull << 60) - 1ull;
        if (gx == nx - 1) valid &= ~kTetUseX;
        if (gy == ny - 1) valid &= ~kTetUseY;
        if (gz == nz - 1) valid &= ~kTetUseZ;
        if (t == nt - 1) valid &= ~kTetUseT;
        m &= valid;
      }
      if (in && !certified) masks[((mpl3(g, t) * nz + gz) * ny + gy) * nx + gx] = m;  // certified: read as zero
      // count per 16-lane row segment
      unsigned c = (unsigned)__popcll(m);
#pragma unroll
      for (int d = 8; d >= 1; d >>= 1) c += __shfl_xor(c, d, 16);
      if (lx == 0 && gy < ny && gz < nz)
        seg_cnt[((mpl3(g, t) * nz + gz) * ny + gy) * g.nxt + bxl] = (int)c;
    }
  }
  if (st) atomicOr(status, st);
}

// ---------------------------------------------------------------------------------------------------------------
// Emission + links (hits are sparse: one lane per vertex, 4 row segments per wavefront).
// ---------------------------------------------------------------------------------------------------------------
namespace {

struct Field3 {
  const float* f;
  int nx, ny, nz;
  long long plane;
  int ring;  // steps stored as a ring of `ring` slots (0: step t at t)
  // Binary32 gradient (c) and Jacobian stencil J (row-major 3x3, J[a][b] = d grad_a / d x_b) of vertex (x, y, z, t),
  // the same operations as the detection's stencils.  The 25 field values of the stencil are read from clamped
  // (in-grid) addresses, all independent loads; the clamped ones are never used (diff3 takes one-sided differences
  // at the first and last index).
  __device__ __forceinline__ void stencil(int x, int y, int z, int t, float c[3], float J[9]) const {
    const float* P = f + (long long)(ring ? t % ring : t) * plane;
    auto at = [&](int dx, int dy, int dz) {
      const int xx = min(max(x + dx, 0), nx - 1), yy = min(max(y + dy, 0), ny - 1), zz = min(max(z + dz, 0), nz - 1);
      return P[((long long)zz * ny + yy) * nx + xx];
    };
    const int N[3] = {nx, ny, nz}, I[3] = {x, y, z};
    float v[3][3][3];  // v[dz+1][dy+1][dx+1] on the unit neighbourhood (corners unused)
    float far[3][2];   // f(x -+ 2 e_a)
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx)
          v[dz + 1][dy + 1][dx + 1] = (dx != 0 && dy != 0 && dz != 0) ? 0.0f : at(dx, dy, dz);
    far[0][0] = at(-2, 0, 0);
    far[0][1] = at(2, 0, 0);
    far[1][0] = at(0, -2, 0);
    far[1][1] = at(0, 2, 0);
    far[2][0] = at(0, 0, -2);
    far[2][1] = at(0, 0, 2);
    // value at offset d (|d|_inf <= 1, at most two nonzero) and at -+2 e_a
    auto val = [&](int dx, int dy, int dz) { return v[dz + 1][dy + 1][dx + 1]; };
    // gradient component a at the vertex offset by o = s e_b (s in {-1, 0, 1})
    auto grad_at = [&](int a, int b, int sgn) -> float {
      int o[3] = {0, 0, 0};
      o[b] = sgn;
      int lo[3] = {o[0], o[1], o[2]}, hi[3] = {o[0], o[1], o[2]};
      lo[a] -= 1;
      hi[a] += 1;
      float fl, fh;
      if (a == b && sgn != 0) {  // neighbours at o -+ e_a: the centre and the far value
        fl = sgn < 0 ? far[a][0] : val(0, 0, 0);
        fh = sgn < 0 ? val(0, 0, 0) : far[a][1];
      } else {
        fl = val(lo[0], lo[1], lo[2]);
        fh = val(hi[0], hi[1], hi[2]);
      }
      return diff3(fl, val(o[0], o[1], o[2]), fh, I[a] + o[a], N[a]);
    };
#pragma unroll
    for (int a = 0; a < 3; ++a) c[a] = grad_at(a, 0, 0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
        J[a * 3 + b] = diff3(grad_at(a, b, -1), c[a], grad_at(a, b, 1), I[b], N[b]);
  }
};

// Binary64 classification of the gradient's Jacobian (the Hessian) in the reference order: H = (J + J^T) * 0.5,
// s1 = trace, s2 = sum of principal 2x2 minors, s3 = det (first-row expansion); Descartes' rule on (1, s1, s2, s3)
// counts negative eigenvalues (exact for the real-rooted characteristic polynomial of a symmetric matrix).
__device__ __noinline__ int classify3_fp64(double mu0, double mu1, double mu2, double mu3, const float* J0,
                                           const float* J1, const float* J2, const float* J3) {
  double Jc[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    double s = mu0 * (double)J0[e];
    s = s + mu1 * (double)J1[e];
    s = s + mu2 * (double)J2[e];
    s = s + mu3 * (double)J3[e];
    Jc[e] = s;
  }
  double H[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      double s = Jc[a * 3 + b] + Jc[b * 3 + a];
      H[a * 3 + b] = s * 0.5;
    }
  const double s1 = (H[0] + H[4]) + H[8];
  const double m01 = H[0] * H[4] - H[1] * H[3];
  const double m02 = H[0] * H[8] - H[2] * H[6];
  const double m12 = H[4] * H[8] - H[5] * H[7];
  const double s2 = (m01 + m02) + m12;
  const double c0 = H[4] * H[8] - H[5] * H[7];
  const double c1 = H[3] * H[8] - H[5] * H[6];
  const double c2 = H[3] * H[7] - H[4] * H[6];
  const double s3 = (H[0] * c0 - H[1] * c1) + H[2] * c2;
  if (s3 == 0) return T_DEG;
  int changes = 0;
  bool prev_neg = false;
  const double seq[3] = {s1, s2, s3};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if (seq[i] == 0) continue;
    const bool neg = seq[i] < 0;
    if (neg != prev_neg) ++changes;
    prev_neg = neg;
  }
  return changes == 0 ? T_MIN : (changes == 1 ? T_SADDLE1 : (changes == 2 ? T_SADDLE2 : T_MAX));
}

}  // namespace

// Row chunks of 64 vertices that hold hits (wavefronts of the emission kernel): a light pass over the per-segment
// hit counts (one lane per chunk, its four 16-vertex segments) lists them with one append per wavefront, so the
// heavy emission kernel (large register footprint, low occupancy) runs only where there is work.
__global__ __launch_bounds__(256) void emit3d_rows(Grid3 g, const int* __restrict__ seg_cnt, long long nvtx_rows,
                                                   long long* __restrict__ list,
                                                   unsigned long long* __restrict__ list_n) {
  const int ny = g.ny, nz = g.nz, nxt = g.nxt;
  const int xblocks = (g.nx + 63) / 64;
  const long long chunk = (long long)blockIdx.x * 256 + threadIdx.x;
  bool has = false;
  if (chunk < nvtx_rows * xblocks) {
    const long long r = chunk / xblocks;
    const int xb = (int)(chunk - r * xblocks);
    const int y = (int)(r % ny), z = (int)((r / ny) % nz), t = g.t_begin + (int)(r / ((long long)ny * nz));
    const long long sb = ((mpl3(g, t) * nz + z) * ny + y) * nxt;
#pragma unroll
    for (int k = 0; k < 64 / SEG3; ++k) {
      const int sx = xb * (64 / SEG3) + k;
      if (sx < nxt && seg_cnt[sb + sx] > 0) has = true;
    }
  }
  const unsigned long long bal = __ballot(has);
  if (bal == 0) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)bal) - 1;
  unsigned long long pos = 0;
  if (lane == leader) pos = atomicAdd(list_n, (unsigned long long)__popcll(bal));
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)pos, leader);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(pos >> 32), leader);
  pos = ((unsigned long long)hi << 32) | lo;
  if (has) list[pos + (unsigned long long)__popcll(bal & ((1ull << lane) - 1ull))] = chunk;
}

template <bool WIDE>
__global__ __launch_bounds__(256) void emit3d(Grid3 g, const uint64_t* __restrict__ masks,
                                              const long long* __restrict__ seg_off, long long nvtx_rows, Out3 o,
                                              unsigned* __restrict__ status, unsigned long long* __restrict__ cnt,
                                              const long long* __restrict__ list,
                                              const unsigned long long* __restrict__ list_n) {
  // thread -> vertex (x fastest, 16-wide segments); wavefront -> one listed 64-vertex row chunk
  const int nx = g.nx, ny = g.ny, nz = g.nz, nt = g.nt, nxt = g.nxt;
  const unsigned long long wi = (unsigned long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wi >= *list_n) return;
  const long long row = list[wi];
  const int lane = threadIdx.x & 63;
  const int xblocks = (nx + 63) / 64;
  if (row >= nvtx_rows * xblocks) return;
  const long long r = row / xblocks;
  const int xb = (int)(row - r * xblocks);
  const int x = xb * 64 + lane;
  const int y = (int)(r % ny), z = (int)((r / ny) % nz), t = g.t_begin + (int)(r / ((long long)ny * nz));
  const bool in = x < nx;
  const long long plane = (long long)nx * ny * nz;
  const long long vofs = ((long long)z * ny + y) * nx + x;
  const long long gidx = (long long)t * plane + vofs;  // global vertex index (face ids)
  // the puncture mask of vertex u: zero where its detection tile-step was certified (those masks are not written)
  const long long ntx = (nx + TX3 - 1) / TX3, nty = (ny + TY3 - 1) / TY3, ntz = (nz + TZ3 - 1) / TZ3;
  auto certified_at = [&](int ux, int uy, int uz, int ut) -> bool {
    return g.cert[((mpl3(g, ut) * ntz + uz / TZ3) * nty + uy / TY3) * ntx + ux / TX3] != 0;
  };
  const unsigned long long m = (in && !certified_at(x, y, z, t)) ? masks[mpl3(g, t) * plane + vofs] : 0ull;
  if (__ballot(m != 0) == 0) return;
  unsigned st = 0;
  unsigned long long n_deg = 0, n_linked = 0;

  // first-hit index of vertex u (global coordinates, inside the grid): segment offset + hits of the earlier
  // vertices of its 16-vertex segment
  auto first_hit = [&](int ux, int uy, int uz, int ut) -> unsigned {
    const long long seg = ((mpl3(g, ut) * nz + uz) * ny + uy) * nxt + ux / SEG3;
    unsigned off = (unsigned)seg_off[seg];
    const long long ub = mpl3(g, ut) * plane + ((long long)uz * ny + uy) * nx;
    const int x0s = (ux / SEG3) * SEG3;
#pragma unroll
    for (int k = 0; k < SEG3 - 1; ++k) {  // independent loads (clamped index), counted below ux only
      const int xx = x0s + k;
      const unsigned long long mk = masks[ub + min(xx, nx - 1)];
      off += xx < ux ? (unsigned)__popcll(mk) : 0u;
    }
    return off;
  };
  auto mask_at = [&](int ux, int uy, int uz, int ut) -> unsigned long long {
    if (certified_at(ux, uy, uz, ut)) return 0ull;
    return masks[mpl3(g, ut) * plane + ((long long)uz * ny + uy) * nx + ux];
  };

  Field3 F{g.f, nx, ny, nz, plane, g.f_ring};
  unsigned long long rem = m;
  if (rem) {
    unsigned k = 0;
    const unsigned base = first_hit(x, y, z, t);
    while (rem) {
      const int ty = __ffsll((long long)rem) - 1;
      rem &= rem - 1;
      const unsigned idx = base + k;
      ++k;
      const int m1 = kTet3.m[ty][0], m2 = kTet3.m[ty][1], m3 = kTet3.m[ty][2];
      int vx[4], vy[4], vz[4], vt[4];
      const int cm[4] = {0, m1, m1 | m2, m1 | m2 | m3};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        vx[i] = x + (cm[i] & 1);
        vy[i] = y + ((cm[i] >> 1) & 1);
        vz[i] = z + ((cm[i] >> 2) & 1);
        vt[i] = t + ((cm[i] >> 3) & 1);
      }
      long long q[4][3];
      float J[4][9];
      bool wide = false;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float gr[3];
        F.stencil(vx[i], vy[i], vz[i], vt[i], gr, J[i]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float rq = quant(gr[c], g.qscale);
          if (!(fabsf(rq) < 1048576.0f)) wide = true;
          q[i][c] = (long long)rq;
        }
      }
      // exact cofactors C_i = (-1)^(3+i) det(columns without i)
      i128 C[4];
      C[0] = -det3x<WIDE, long long>(q[1], q[2], q[3]);
      C[1] = det3x<WIDE, long long>(q[0], q[2], q[3]);
      C[2] = -det3x<WIDE, long long>(q[0], q[1], q[3]);
      C[3] = det3x<WIDE, long long>(q[0], q[1], q[2]);
      const i128 D = (C[0] + C[1]) + (C[2] + C[3]);
      unsigned fl = wide ? FL_WIDE : 0u;
      double mu64[4];
      if (D == 0) {
        fl |= FL_DEGENERATE;
        ++n_deg;
#pragma unroll
        for (int i = 0; i < 4; ++i) mu64[i] = 1.0 / 4.0;
      } else {
        const double dD = (double)D;
#pragma unroll
        for (int i = 0; i < 4; ++i) mu64[i] = (double)C[i] / dD;
      }
      const int type = classify3_fp64(mu64[0], mu64[1], mu64[2], mu64[3], J[0], J[1], J[2], J[3]);
      float pos[4], muo[4];
      if (g.precision == 0) {
        float mu32[4];
        if (D == 0) {
#pragma unroll
          for (int i = 0; i < 4; ++i) mu32[i] = 0.25f;
        } else {
          const float fD = (float)D;
#pragma unroll
          for (int i = 0; i < 4; ++i) mu32[i] = (float)C[i] / fD;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int* vc = c == 0 ? vx : (c == 1 ? vy : (c == 2 ? vz : vt));
          float s = mu32[0] * (float)vc[0];
          s = s + mu32[1] * (float)vc[1];
          s = s + mu32[2] * (float)vc[2];
          s = s + mu32[3] * (float)vc[3];
          pos[c] = s;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) muo[i] = mu32[i];
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int* vc = c == 0 ? vx : (c == 1 ? vy : (c == 2 ? vz : vt));
          double s = mu64[0] * (double)vc[0];
          s = s + mu64[1] * (double)vc[1];
          s = s + mu64[2] * (double)vc[2];
          s = s + mu64[3] * (double)vc[3];
          pos[c] = (float)s;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) muo[i] = (float)mu64[i];
      }
      o.face_id[idx] = gidx * 60 + ty;
      if (o.pos)
#pragma unroll
        for (int c = 0; c < 4; ++c) o.pos[(size_t)idx * 4 + c] = pos[c];
      if (o.mu)
#pragma unroll
        for (int c = 0; c < 4; ++c) o.mu[(size_t)idx * 4 + c] = muo[c];
      if (o.type) o.type[idx] = (uint8_t)type;
      if (o.flags) o.flags[idx] = (uint8_t)fl;

      // ---- links: the (at most two) pentachora holding this tetrahedron.  A pentachoron with chain
      // (c1, c2, c3, c4) anchored at c has sides: drop w0 -> (c + e_c1; c2, c3, c4), drop w1 -> (c; c1|c2, c3, c4),
      // drop w2 -> (c; c1, c2|c3, c4), drop w3 -> (c; c1, c2, c3|c4), drop w4 -> (c; c1, c2, c3).
      unsigned p0 = idx, p1 = idx;
      int np = 0;
      auto visit_cell = [&](int cx, int cy, int cz, int ct, int c1, int c2, int c3, int c4) {
        const int fx = cx + (c1 & 1), fy = cy + ((c1 >> 1) & 1), fz = cz + ((c1 >> 2) & 1), ft = ct + ((c1 >> 3) & 1);
        const unsigned long long bm = mask_at(cx, cy, cz, ct);
        const unsigned long long fm = mask_at(fx, fy, fz, ft);
        int found = 0;
        unsigned other = 0xFFFFFFFFu;
#pragma unroll
        for (int s = 0; s < 5; ++s) {
          int ti;
          if (s == 0)
            ti = kTet3Index.idx[c2][c3][c4];
          else if (s == 1)
            ti = kTet3Index.idx[c1 | c2][c3][c4];
          else if (s == 2)
            ti = kTet3Index.idx[c1][c2 | c3][c4];
          else if (s == 3)
            ti = kTet3Index.idx[c1][c2][c3 | c4];
          else
            ti = kTet3Index.idx[c1][c2][c3];
          const unsigned long long um = s == 0 ? fm : bm;
          if ((um >> ti) & 1ull) {
            ++found;
            const unsigned hi = (s == 0 ? first_hit(fx, fy, fz, ft) : first_hit(cx, cy, cz, ct)) +
                                (unsigned)__popcll(um & ((1ull << ti) - 1ull));
            if (hi != idx) other = hi;
          }
        }
        if (found != 2 || other == 0xFFFFFFFFu) {
          st |= ST_INVARIANT;
          return;
        }
        if (np == 0)
          p0 = other;
        else
          p1 = other;
        ++np;
        if (other > idx) ++n_linked;
      };
      const int b = m1 | m2 | m3;
      const int N[4] = {nx, ny, nz, nt};
      const int P[4] = {x, y, z, t};
      if (__popc((unsigned)m1) == 1 && __popc((unsigned)m2) == 1 && __popc((unsigned)m3) == 1) {
        const int a = 15 & ~b;  // missing axis
        const int ai = __ffs(a) - 1;
        if (P[ai] >= 1)
          visit_cell(x - (a & 1), y - ((a >> 1) & 1), z - ((a >> 2) & 1), t - ((a >> 3) & 1), a, m1, m2, m3);
        if (P[ai] + 1 <= N[ai] - 1) visit_cell(x, y, z, t, m1, m2, m3, a);
      } else if (__popc((unsigned)m1) == 2) {
        const int lo = m1 & -m1, hi = m1 - lo;
        visit_cell(x, y, z, t, lo, hi, m2, m3);
        visit_cell(x, y, z, t, hi, lo, m2, m3);
      } else if (__popc((unsigned)m2) == 2) {
        const int lo = m2 & -m2, hi = m2 - lo;
        visit_cell(x, y, z, t, m1, lo, hi, m3);
        visit_cell(x, y, z, t, m1, hi, lo, m3);
      } else {
        const int lo = m3 & -m3, hi = m3 - lo;
        visit_cell(x, y, z, t, m1, m2, lo, hi);
        visit_cell(x, y, z, t, m1, m2, hi, lo);
      }
      unsigned par0 = idx, smaller = 0, big_small = 0;
      if (np > 0 && p0 < idx) {
        ++smaller;
        par0 = p0;
        big_small = p0;
      }
      if (np > 1 && p1 < idx) {
        ++smaller;
        if (p1 < par0) par0 = p1;
        if (p1 > big_small) big_small = p1;
      }
      o.parent[idx] = par0;
      if (smaller == 2) {
        unsigned long long slot = atomicAdd(&cnt[CNT_WORK], 1ull);
        o.work[slot] = make_uint2(idx, big_small);
      }
    }
  }
  unsigned long long s2 = wave_sum64(n_deg), s3 = wave_sum64(n_linked);
  if (lane == 0) {
    if (s2) atomicAdd(&cnt[CNT_DEGEN], s2);
    if (s3) atomicAdd(&cnt[CNT_LINKED], s3);
  }
  if (st) atomicOr(status, st);
}

hipError_t launch_detect3d(const Grid3& g, int tt, bool wide, uint64_t* masks, int* seg_cnt, unsigned* status,
                           hipStream_t s) {
  if (!g.cert) return hipErrorInvalidValue;  // the kernel records its certified tile-steps there
  const int nyt = (g.ny + TY3 - 1) / TY3, nzt = (g.nz + TZ3 - 1) / TZ3;
  dim3 grid((unsigned)((g.nx + TX3 - 1) / TX3), (unsigned)(nyt * nzt),
            (unsigned)((g.t_end - g.t_begin + tt - 1) / tt));
  if (wide)
    detect3d<true><<<grid, 256, 0, s>>>(g, tt, nyt, masks, seg_cnt, status);
  else
    detect3d<false><<<grid, 256, 0, s>>>(g, tt, nyt, masks, seg_cnt, status);
  return hipGetLastError();
}

hipError_t launch_emit3d(const Grid3& g, bool wide, const uint64_t* masks, const int* seg_cnt,
                         const long long* seg_off, long long n_hits, const Out3& o, unsigned* status,
                         unsigned long long* cnt, long long* list, unsigned long long* list_n, hipStream_t s) {
  if (!g.cert) return hipErrorInvalidValue;  // the certified-tile flags are read with the masks
  const long long rows = (long long)(g.t_end - g.t_begin) * g.nz * g.ny;
  const long long waves = rows * ((g.nx + 63) / 64);
  emit3d_rows<<<(unsigned)((waves + 255) / 256), 256, 0, s>>>(g, seg_cnt, rows, list, list_n);
  // at most one listed wavefront per hit
  const long long lw = n_hits < waves ? n_hits : waves;
  const unsigned blocks = (unsigned)((lw + 3) / 4 > 0 ? (lw + 3) / 4 : 1);
  if (wide)
    emit3d<true><<<blocks, 256, 0, s>>>(g, masks, seg_off, rows, o, status, cnt, list, list_n);
  else
    emit3d<false><<<blocks, 256, 0, s>>>(g, masks, seg_off, rows, o, status, cnt, list, list_n);
  return hipGetLastError();
}

}  // namespace ftk
