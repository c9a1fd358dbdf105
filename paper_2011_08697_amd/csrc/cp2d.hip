// cp2d.hip -- critical-point tracking in 2D space + time on gfx950.
//
// Mesh: the Kuhn subdivision of the (x, y, t) grid (Sec. 3.3): per vertex 7 edge types, 12 triangle types (the
// tested faces) and 6 tetrahedra (the cells).  Pass 1 of Alg. 1 (left column) tests every triangle: it is
// punctured when the origin is interior to the triangle of its (quantised) vertex vectors, i.e. when the three
// signed cofactors of (v0 v1 v2 ; 1 1 1) agree (Sec. 4.3, Eq. 2).  Each cofactor is, up to a fixed sign, the 2x2
// determinant of the two vertex vectors of one edge, so a sign bit is computed once per edge (7 per vertex) and
// shared by the triangles through LDS.
//
// Kernels:
//   detect2d  -- time-marching slab kernel over a 64 x TY tile (TX = one wavefront): loads the field plane with a
//                2-cell halo into LDS, forms the gradient (scalar input), quantises, evaluates the 7 edge signs of
//                every vertex of the tile (+1 halo) and the 12 triangle tests of every anchor; writes a 12-bit
//                puncture mask per vertex and the hit count of every 64-vertex row segment.
//   emit2d    -- one wavefront per row segment: prefix sums give each hit its output index (face ids come out
//                sorted); computes the sublocation (Eq. 2) from the exact cofactors, the Jacobian type (FP32 with
//                certified FP64 fallback), and the union-find links of the hit's two tetrahedra (Alg. 1 pass 2).
#include "common.h"
#include "internal.h"

namespace ftk {

namespace {

constexpr int TX = 64;
constexpr int kEmitTT = 16;  // steps per emission workgroup

// triangle types using each axis (validity masks at the last index of an axis)
constexpr unsigned kUseX = (unsigned)types_using_axis(kTri2, 1);
constexpr unsigned kUseY = (unsigned)types_using_axis(kTri2, 2);
constexpr unsigned kUseT = (unsigned)types_using_axis(kTri2, 4);

// Quantised components: the narrow path keeps integers below 2^24 in binary32 (exact, and every determinant and
// cofactor of the path stays exact in binary64); the wide path keeps 64-bit integers below 2^62.
template <bool WIDE>
struct QType;
template <>
struct QType<false> {
  typedef float T;
};
template <>
struct QType<true> {
  typedef long long T;
};

constexpr float kNarrow2 = 16777216.0f;  // 2^24

// Bit-gather tables for the 12 triangle tests: t[0][w] bit k = edge-word bit (M1 - 1) (edge v0 v1), t[1][w] bit k =
// bit (M1|M2 - 1) (edge v0 v2), t[1 + n][w] bit k = bit (M2 - 1) for the types with M1 = n (edge v1 v2, read from
// the word of the neighbour p + e(n)).
struct Tri2Lut {
  unsigned short t[8][128];
};
constexpr Tri2Lut build_tri2_lut() {
  Tri2Lut r{};
  for (int w = 0; w < 128; ++w)
    for (int k = 0; k < 12; ++k) {
      const int m1 = kTri2.m[k][0], m2 = kTri2.m[k][1];
      if ((w >> (m1 - 1)) & 1) r.t[0][w] |= (unsigned short)(1u << k);
      if ((w >> ((m1 | m2) - 1)) & 1) r.t[1][w] |= (unsigned short)(1u << k);
      if ((w >> (m2 - 1)) & 1) r.t[1 + m1][w] |= (unsigned short)(1u << k);
    }
  return r;
}
constexpr Tri2Lut kTri2Lut = build_tri2_lut();

template <bool WIDE>
__device__ __forceinline__ typename QType<WIDE>::T to_q(float r, unsigned& st) {
  if (!WIDE) {
    if (!(fabsf(r) < kNarrow2)) {
      st |= ST_WIDE;
      return 0.0f;
    }
    return r;
  } else {
    if (!(fabsf(r) < 4611686018427387904.0f)) {
      st |= ST_RANGE;
      return 0;
    }
    return (long long)r;
  }
}

__device__ __forceinline__ int fpl(const Grid2& g, int t) { return g.f_ring ? t % g.f_ring : t; }
__device__ __forceinline__ int mpl(const Grid2& g, int t) { return g.m_ring ? t % g.m_ring : t; }

}  // namespace

// ---------------------------------------------------------------------------------------------------------------
// Pass 1: detection.
// grid = (ceil(nx / 64), ceil(ny / TY), ceil(nt / TT)), block = 256.
// ---------------------------------------------------------------------------------------------------------------
template <int TY, bool WIDE>
__device__ __forceinline__ void detect2d_tile(const Grid2& g, int TT, int bx, int by, int bz,
                                              uint16_t* __restrict__ masks, int* __restrict__ seg_cnt,
                                              unsigned* __restrict__ status) {
  typedef typename QType<WIDE>::T Q;
  constexpr int FW = TX + 4, FH = TY + 4;  // field plane + 2-cell halo (x0-1 .. x0+TX+2)
  constexpr int QW = TX + 2, QH = TY + 2;  // quantised vectors (x0 .. x0+TX+1)
  constexpr int EW = TX + 1, EH = TY + 1;  // edge words (x0 .. x0+TX)
  __shared__ float fs[FH * FW];     // scalar input: the field plane being loaded
  __shared__ Q qs[2][2][QH * QW];  // [plane parity][component]
  __shared__ uint8_t ew[2][EH * EW];

  const int tid = threadIdx.x;
  const int x0 = bx * TX, y0 = by * TY;
  const int t0 = g.t_begin + bz * TT;
  const int t1 = min(t0 + TT, g.t_end);
  const int nx = g.nx, ny = g.ny, nt = g.nt;
  const long long plane = (long long)nx * ny;
  unsigned st = 0;
  unsigned facts = 0x1Fu;  // sign facts of the vectors quantised by this thread since the last plane_facts()
  auto fact_bits = [](Q a, Q b) -> unsigned {
    return (a > (Q)0 ? 1u : 0u) | (a < (Q)0 ? 2u : 0u) | (b > (Q)0 ? 4u : 0u) | (b < (Q)0 ? 8u : 0u) |
           ((a == (Q)0 && b == (Q)0) ? 16u : 0u);
  };

  // Load plane t: scalar input into fs (FH x FW with halo); vector input straight into qs[par] (quantised).  The
  // loads use clamped (in-grid) addresses and are issued back to back; cells outside the grid are zeroed after.
  auto load_plane = [&](int t, int par) {
    if (g.kind == 0) {
      constexpr int NL = (FH * FW + 255) / 256;
      const float* src = g.f + (long long)fpl(g, t) * plane;
      float fv[NL];
      bool in[NL];
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        int e = tid + 256 * i;
        asm volatile("" : "+v"(e));  // opaque: the index math is redone per plane, not held across steps
        const int ly = e / FW, lx = e - ly * FW;
        const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
        in[i] = e < FH * FW && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        fv[i] = src[(long long)min(max(gy, 0), ny - 1) * nx + min(max(gx, 0), nx - 1)];
      }
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        const int e = tid + 256 * i;
        const float v = in[i] ? fv[i] : 0.0f;
        if (in[i] && !isfinite(v)) st |= ST_NONFINITE;
        if (e < FH * FW) fs[e] = v;
      }
    } else {
      constexpr int NL = (QH * QW + 255) / 256;
      const float* su = g.f + (long long)fpl(g, t) * 2 * plane;
      const float* sv = su + plane;
      float f0[NL], f1[NL];
      bool in[NL];
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        int e = tid + 256 * i;
        asm volatile("" : "+v"(e));
        const int ly = e / QW, lx = e - ly * QW;
        const int gx = x0 + lx, gy = y0 + ly;
        in[i] = e < QH * QW && gx < nx && gy < ny;
        const long long k = (long long)min(gy, ny - 1) * nx + min(gx, nx - 1);
        f0[i] = su[k];
        f1[i] = sv[k];
      }
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        const int e = tid + 256 * i;
        Q q0 = 0, q1 = 0;
        if (in[i]) {
          if (!isfinite(f0[i]) || !isfinite(f1[i])) st |= ST_NONFINITE;
          q0 = to_q<WIDE>(quant(f0[i], g.qscale), st);
          q1 = to_q<WIDE>(quant(f1[i], g.qscale), st);
          facts &= fact_bits(q0, q1);
        }
        if (e < QH * QW) {
          qs[par][0][e] = q0;
          qs[par][1][e] = q1;
        }
      }
    }
  };

  // Quantised gradient of plane (parity par) from fs (scalar input; vector input is quantised while loading).
  auto quantise_plane = [&](int par) {
    if (g.kind != 0) return;
    for (int e = tid; e < QH * QW; e += 256) {
      int ly = e / QW, lx = e - ly * QW;
      int gx = x0 + lx, gy = y0 + ly;
      Q q0 = 0, q1 = 0;
      if (gx < nx && gy < ny) {
        const float* r = &fs[(ly + 1) * FW + (lx + 1)];
        const float v0 = diff3(r[-1], r[0], r[1], gx, nx);
        const float v1 = diff3(r[-FW], r[0], r[FW], gy, ny);
        q0 = to_q<WIDE>(quant(v0, g.qscale), st);
        q1 = to_q<WIDE>(quant(v1, g.qscale), st);
        facts &= fact_bits(q0, q1);
      }
      qs[par][0][e] = q0;
      qs[par][1][e] = q1;
    }
  };

  // Ordinal edge bits (masks x=1, y=2, xy=3) of plane parity par for the EH x EW anchors.
  auto ordinal_edges = [&](int par) {
    for (int e = tid; e < EH * EW; e += 256) {
      int ly = e / EW, lx = e - ly * EW;
      int qa = ly * QW + lx;
      Q a0 = qs[par][0][qa], a1 = qs[par][1][qa];
      unsigned w = 0;
      w |= sos2_positive<Q>(a0, a1, qs[par][0][qa + 1], qs[par][1][qa + 1]) << 0;
      w |= sos2_positive<Q>(a0, a1, qs[par][0][qa + QW], qs[par][1][qa + QW]) << 1;
      w |= sos2_positive<Q>(a0, a1, qs[par][0][qa + QW + 1], qs[par][1][qa + QW + 1]) << 2;
      ew[par][e] = (uint8_t)w;
    }
  };

  // Interval edge bits (masks t=4, xt=5, yt=6, xyt=7) from plane parity par to par^1, OR-ed into ew[par].
  auto interval_edges = [&](int par) {
    const int nxp = par ^ 1;
    for (int e = tid; e < EH * EW; e += 256) {
      int ly = e / EW, lx = e - ly * EW;
      int qa = ly * QW + lx;
      Q a0 = qs[par][0][qa], a1 = qs[par][1][qa];
      unsigned w = 0;
      w |= sos2_positive<Q>(a0, a1, qs[nxp][0][qa], qs[nxp][1][qa]) << 3;
      w |= sos2_positive<Q>(a0, a1, qs[nxp][0][qa + 1], qs[nxp][1][qa + 1]) << 4;
      w |= sos2_positive<Q>(a0, a1, qs[nxp][0][qa + QW], qs[nxp][1][qa + QW]) << 5;
      w |= sos2_positive<Q>(a0, a1, qs[nxp][0][qa + QW + 1], qs[nxp][1][qa + QW + 1]) << 6;
      ew[par][e] |= (uint8_t)w;
    }
  };

  // Narrow variant: one pass per position computes the ordinal edges of step t+1 (masks x, y, xy) and the interval
  // edges t -> t+1 (masks t, xt, yt, xyt) from five vertex vectors converted to binary64 once.
  auto fused_edges = [&](int par) {
    const int nxp = par ^ 1;
    for (int e = tid; e < EH * EW; e += 256) {
      const int ly = e / EW, lx = e - ly * EW;
      const int qa = ly * QW + lx;
      const double a0 = (double)qs[par][0][qa], a1 = (double)qs[par][1][qa];
      const double b0 = (double)qs[nxp][0][qa], b1 = (double)qs[nxp][1][qa];
      const double c0 = (double)qs[nxp][0][qa + 1], c1 = (double)qs[nxp][1][qa + 1];
      const double d0 = (double)qs[nxp][0][qa + QW], d1 = (double)qs[nxp][1][qa + QW];
      const double f0 = (double)qs[nxp][0][qa + QW + 1], f1 = (double)qs[nxp][1][qa + QW + 1];
      // edges (b c), (b d), (b f) -> ordinal bits 0-2 of step t+1; (a b), (a c), (a d), (a f) -> interval bits 3-6
      const double P0[7] = {b0, b0, b0, a0, a0, a0, a0}, P1[7] = {b1, b1, b1, a1, a1, a1, a1};
      const double Q0[7] = {c0, d0, f0, b0, c0, d0, f0}, Q1[7] = {c1, d1, f1, b1, c1, d1, f1};
      unsigned bits = 0, zero = 0;
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        const double d = __builtin_fma(P0[k], Q1[k], -(P1[k] * Q0[k]));  // exact
        bits |= (unsigned)(d > 0.0) << k;
        zero |= (unsigned)(d == 0.0) << k;
      }
      if (zero) {  // the perturbation decides exact zeros only (rare on generic data)
#pragma unroll
        for (int k = 0; k < 7; ++k)
          if ((zero >> k) & 1u) bits |= sos2_positive_d(P0[k], P1[k], Q0[k], Q1[k]) << k;
      }
      ew[nxp][e] = (uint8_t)(bits & 7u);
      ew[par][e] |= (uint8_t)(bits & 0x78u);
    }
  };

  // triangle lookup tables (LDS copy of the compile-time tables)
  __shared__ unsigned short s_lut[8][128];
  for (int i = tid; i < 8 * 128; i += 256) s_lut[i >> 7][i & 127] = kTri2Lut.t[i >> 7][i & 127];

  // Sign facts of a plane's quantised vectors over the tile (anchors and their +1 neighbours, inside the grid):
  // bit 0 every x component > 0, bit 1 every x < 0, bit 2 every y > 0, bit 3 every y < 0, bit 4 every vector zero.
  // When a fact holds on both planes of a step, no triangle anchored in the tile at that step is punctured: a
  // component of one strict sign at all three vertices keeps that sign under the symbolic perturbation (its
  // entries move by infinitesimals only), so the origin is outside the triangle; and with all vectors zero every
  // edge determinant takes the perturbation's last, negative term, so the three cofactor signs never agree.  The
  // edge and triangle passes of such a step are skipped (its masks and counts are zero).
  __shared__ unsigned s_fact[2];
  __shared__ int s_ord_ok[2];  // the ordinal edge words of the plane slot have been computed
  const int wave = tid >> 6, lane = tid & 63;
  auto plane_facts = [&](int p) {  // block reduction of the facts gathered while the plane was quantised
    const unsigned bits = facts;
    facts = 0x1Fu;
    unsigned wb = 0;
#pragma unroll
    for (int k = 0; k < 5; ++k)
      if (__ballot(!((bits >> k) & 1u)) == 0) wb |= 1u << k;
    if (lane == 0) atomicAnd(&s_fact[p], wb);
  };

  // prologue: plane t0 (its ordinal edges are formed when a step first needs them)
  if (tid == 0) {
    s_fact[t0 & 1] = 0x1Fu;
    s_ord_ok[0] = s_ord_ok[1] = 0;
  }
  __syncthreads();
  load_plane(t0, t0 & 1);
  __syncthreads();
  quantise_plane(t0 & 1);
  plane_facts(t0 & 1);

  const int gx = x0 + lane;
  for (int t = t0; t < t1; ++t) {
    const int par = t & 1, nxp = par ^ 1;
    const bool has_next = (t + 1 < nt);
    __syncthreads();  // previous triangle pass done with ew / fs; facts and edge flags of plane t visible
    if (has_next) {
      if (tid == 0) s_fact[nxp] = 0x1Fu;  // ordered before the atomics by the barrier after the load
      load_plane(t + 1, nxp);
      __syncthreads();
      quantise_plane(nxp);
      plane_facts(nxp);
      __syncthreads();  // quantised plane and its facts visible
    }
    const bool certified = (s_fact[par] & (has_next ? s_fact[nxp] : 0x1Fu)) != 0u;  // uniform
    const bool ord_ok = s_ord_ok[par] != 0;
    if (!certified) {
      if (!ord_ok) ordinal_edges(par);  // each thread ORs into the words it assigned here
      if (has_next) {
        if constexpr (!WIDE) {
          fused_edges(par);
        } else {
          ordinal_edges(nxp);
          interval_edges(par);
        }
      }
    }
    __syncthreads();
    if (tid == 0 && has_next) s_ord_ok[nxp] = certified ? 0 : 1;

    // triangle tests: wave w handles rows w, w+4, ...
    for (int ly = wave; ly < TY; ly += 4) {
      const int gy = y0 + ly;
      unsigned m = 0;
      if (gx < nx && gy < ny && !certified) {
        const int a = ly * EW + lane;
        // word of the anchor and of its neighbours p + e(M1): plane t for M1 in {x, y, xy}, plane t+1 (ordinal
        // bits only) for M1 in {t, xt, yt}
        // sides opposite v0, v1, v2 of triangle (M1, M2): edges (v1 v2) = (p + e(M1), M2), (v0 v2) = (p, M1|M2),
        // (v0 v1) = (p, M1); cofactor signs +S(v1v2), -S(v0v2), +S(v0v1): punctured iff S(v1v2) = S(v0v1) != S(v0v2).
        // The 12 tests run bit-parallel: E0/E1/E2 gather, for every type, the sign bit of its edge opposite
        // v0/v1/v2 through 128-entry tables indexed by the 7-bit edge words.
        const unsigned W0 = ew[par][a];
        unsigned E0 = s_lut[2][ew[par][a + 1]] | s_lut[3][ew[par][a + EW]] | s_lut[4][ew[par][a + EW + 1]];
        if (has_next) E0 |= s_lut[5][ew[nxp][a]] | s_lut[6][ew[nxp][a + 1]] | s_lut[7][ew[nxp][a + EW]];
        const unsigned E1 = s_lut[1][W0], E2 = s_lut[0][W0];
        m = ~(E0 ^ E2) & (E1 ^ E0) & 0xFFFu;
        unsigned valid = 0xFFFu;
        if (gx == nx - 1) valid &= ~kUseX;
        if (gy == ny - 1) valid &= ~kUseY;
        if (t == nt - 1) valid &= ~kUseT;
        m &= valid;
      }
      if (gx < nx && gy < ny) masks[((long long)mpl(g, t) * ny + gy) * nx + gx] = (uint16_t)m;
      unsigned c = wave_sum(__popc(m));
      if (lane == 0 && gy < ny) seg_cnt[((long long)mpl(g, t) * ny + gy) * g.nxt + bx] = (int)c;
    }
  }
  if (st) atomicOr(status, st);
}

template <int TY, bool WIDE>
__global__ __launch_bounds__(256) void detect2d(Grid2 g, int TT, uint16_t* __restrict__ masks,
                                                int* __restrict__ seg_cnt, unsigned* __restrict__ status) {
  detect2d_tile<TY, WIDE>(g, TT, blockIdx.x, blockIdx.y, blockIdx.z, masks, seg_cnt, status);
}

// ---------------------------------------------------------------------------------------------------------------
// Pass 1b: emission + pass 2 links.
// Same tiling as detection (64 x TY anchors, marching over a slab of TT steps).  The vector field of planes t and
// t+1 (gradient of the scalar, or the input vector) is kept in LDS with a 1-cell halo; quantised vectors and
// Jacobians of a hit's vertices are formed from it on the fly, with the same binary32 stencils as pass 1.  Each
// wavefront takes one row segment at a time and processes its hits hit-parallel (hit j of the segment on lane
// j mod 64), so output writes are contiguous.
// ---------------------------------------------------------------------------------------------------------------
namespace {

// Side tables of the triangle types, built at compile time.
// kTri2Pack[ty] = M1 | M2 << 4.  kTri2Cof[ty][k] describes the k-th tetrahedron holding a triangle of type ty
// (Alg. 1 pass 2; the cells holding a triangle, the side-of query of Sec. 3.2): bits 0-1 existence rule (1 always,
// 2 when p_a >= 1, 3 when p_a + 1 <= N_a - 1), bits 2-3 the axis a, then its three other sides as (anchor slot,
// type) in 7-bit fields.
enum { NB_SELF = 0, NB_MX, NB_PX, NB_MY, NB_PY, NB_MT, NB_PT };

struct Tri2Tables {
  unsigned char pack[12];
  unsigned cof[12][2];
};

constexpr int slot_minus(int ab) { return ab == 1 ? NB_MX : (ab == 2 ? NB_MY : NB_MT); }
constexpr int slot_plus(int ab) { return ab == 1 ? NB_PX : (ab == 2 ? NB_PY : NB_PT); }
constexpr int axis_of(int ab) { return ab == 1 ? 0 : (ab == 2 ? 1 : 2); }

// A tetrahedron with chain (c1, c2, c3) anchored at c has sides: drop w0 -> (c + e_c1; c2, c3),
// drop w1 -> (c; c1|c2, c3), drop w2 -> (c; c1, c2|c3), drop w3 -> (c; c1, c2).  at_minus: c = p - e_c1.
constexpr unsigned cof_word(int ty, bool at_minus, int rule, int axis, int c1, int c2, int c3) {
  const int first = at_minus ? NB_SELF : slot_plus(c1);
  const int base = at_minus ? slot_minus(c1) : NB_SELF;
  const int st[4] = {first, base, base, base};
  const int tt[4] = {kTri2Index.idx[c2][c3], kTri2Index.idx[c1 | c2][c3], kTri2Index.idx[c1][c2 | c3],
                     kTri2Index.idx[c1][c2]};
  unsigned w = (unsigned)rule | ((unsigned)axis << 2);
  int k = 0;
  for (int s = 0; s < 4; ++s) {
    if (st[s] == NB_SELF && tt[s] == ty) continue;  // the triangle itself
    w |= (unsigned)(st[s] | (tt[s] << 3)) << (4 + 7 * k);
    ++k;
  }
  return w;
}

constexpr Tri2Tables build_tri2_tables() {
  Tri2Tables r{};
  for (int ty = 0; ty < 12; ++ty) {
    const int m1 = kTri2.m[ty][0], m2 = kTri2.m[ty][1];
    r.pack[ty] = (unsigned char)(m1 | (m2 << 4));
    if (popc_c(m1) == 1 && popc_c(m2) == 1) {
      const int a = 7 & ~(m1 | m2);
      r.cof[ty][0] = cof_word(ty, true, 2, axis_of(a), a, m1, m2);
      r.cof[ty][1] = cof_word(ty, false, 3, axis_of(a), m1, m2, a);
    } else if (popc_c(m1) == 2) {
      const int lo = m1 & -m1, hi = m1 - lo;
      r.cof[ty][0] = cof_word(ty, false, 1, 0, lo, hi, m2);
      r.cof[ty][1] = cof_word(ty, false, 1, 0, hi, lo, m2);
    } else {
      const int lo = m2 & -m2, hi = m2 - lo;
      r.cof[ty][0] = cof_word(ty, false, 1, 0, m1, lo, hi);
      r.cof[ty][1] = cof_word(ty, false, 1, 0, m1, hi, lo);
    }
  }
  return r;
}
constexpr Tri2Tables kTri2Tab = build_tri2_tables();

// The same tables as 24 words for an LDS copy: word 2 ty + k = cof[ty][k] (bits 0-24), and pack[ty] in bits 25-31
// of word 2 ty.  Per-hit reads from LDS leave the vector memory counter to the stores, which a global table read
// would have to wait for.
struct Tri2Words {
  unsigned w[24];
};
constexpr Tri2Words build_tri2_words() {
  Tri2Words r{};
  for (int ty = 0; ty < 12; ++ty) {
    r.w[2 * ty] = kTri2Tab.cof[ty][0] | ((unsigned)kTri2Tab.pack[ty] << 25);
    r.w[2 * ty + 1] = kTri2Tab.cof[ty][1];
  }
  return r;
}
static_assert(build_tri2_words().w[0] >> 25 == kTri2Tab.pack[0], "pack field");
__constant__ Tri2Words kTri2WordsDev = build_tri2_words();

// Neighbour anchor slots (SELF, MX, PX, MY, PY, MT, PT) in 2-bit fields: column + 1 and row + 1 of the anchor.
constexpr unsigned kSlotCol = 0x1561u, kSlotRow = 0x1615u;

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

}  // namespace

// Local union-find in LDS over the hits of one tile and a run of consecutive steps (a chunk); the smallest local id
// (= smallest hit index) is the root.
__device__ __forceinline__ unsigned lfind(unsigned* lp, unsigned x) {
  unsigned p = lp[x];
  while (p != x) {
    unsigned gp = lp[p];
    if (gp != p) lp[x] = gp;
    x = p;
    p = gp;
  }
  return x;
}

__device__ __forceinline__ void lunite(unsigned* lp, unsigned a, unsigned b) {
  unsigned ra = lfind(lp, a), rb = lfind(lp, b);
  while (ra != rb) {
    if (ra < rb) {
      unsigned t = ra;
      ra = rb;
      rb = t;
    }
    unsigned old = atomicCAS(&lp[ra], ra, rb);
    if (old == ra) return;
    ra = lfind(lp, old);
    rb = lfind(lp, rb);
  }
}

// Union-find on the global parent array restricted to the hits of one workgroup's tile and slab: during emission
// nothing outside the workgroup reads or writes these parents, so workgroup-scope atomics (served by the CU's own
// caches) are coherent for them.
__device__ __forceinline__ unsigned wg_load(const unsigned* p, unsigned i) {
  return __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ unsigned wg_find(unsigned* parent, unsigned x) {
  unsigned p = wg_load(parent, x);
  while (p != x) {
    const unsigned gp = wg_load(parent, p);
    if (gp != p) __hip_atomic_store(parent + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    x = p;
    p = gp;
  }
  return x;
}

__device__ __forceinline__ void wg_unite(unsigned* parent, unsigned a, unsigned b) {
  unsigned ra = wg_find(parent, a), rb = wg_find(parent, b);
  while (ra != rb) {
    if (ra < rb) {
      const unsigned t = ra;
      ra = rb;
      rb = t;
    }
    unsigned expected = ra;
    if (__hip_atomic_compare_exchange_strong(parent + ra, &expected, rb, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WORKGROUP))
      return;
    ra = wg_find(parent, expected);
    rb = wg_find(parent, rb);
  }
}

// Edge list staging: links that leave the tile/chunk are collected in LDS and appended to the global list in
// batches (one global atomic per batch; same-address atomics serialise at one L2 channel).
constexpr int kEdgeStage = 496;

// Wave-aggregated append of (idx, partner) for the active lanes with want == true: one LDS add reserves the
// wave's slots; slots past the stage capacity go straight to the global list (one global add for them).
__device__ __forceinline__ void append_edge(bool want, unsigned idx, unsigned partner, uint2* stage, int* stage_n,
                                            int scap, uint2* work, unsigned long long* counter) {
  const unsigned long long bal = __ballot(want);
  if (bal == 0) return;
  const int lane = lane_id();
  const int leader = __ffsll((long long)bal) - 1;
  const int k = __popcll(bal);
  int pos = 0;
  if (lane == leader) pos = atomicAdd(stage_n, k);
  pos = __builtin_amdgcn_readlane(pos, leader);
  const int first_over = pos > scap ? pos : scap;  // first slot number routed to the global list
  const int n_over = pos + k - first_over;
  unsigned long long gpos = 0;
  if (n_over > 0) {
    if (lane == leader) gpos = atomicAdd(counter, (unsigned long long)n_over);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)gpos, leader);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(gpos >> 32), leader);
    gpos = ((unsigned long long)hi << 32) | lo;
  }
  if (want) {
    const int slot = pos + __popcll(bal & ((1ull << lane) - 1ull));
    const uint2 e = make_uint2(idx, partner);
    if (slot < scap)
      stage[slot] = e;
    else
      work[gpos + (unsigned long long)(slot - first_over)] = e;
  }
}

// Block-wide sum of a per-thread value (256 threads), returned on thread 0.
__device__ __forceinline__ unsigned long long block_sum256(unsigned long long v, unsigned long long* red) {
  v = wave_sum64(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  unsigned long long s = 0;
  if (threadIdx.x == 0) s = red[0] + red[1] + red[2] + red[3];
  return s;
}

// Record of one hit (Eq. 2, Sec. 4.1): exact cofactors of (v0 v1 v2 ; 1 1 1) from the quantised vectors qf of the
// triangle's vertices, barycentric coordinates mu, position, and the Jacobian type (FP32 with a certified error
// bound, else FP64); written at output index idx - o.gbase.  J holds the binary32 Jacobian stencil of each vertex.
template <bool WIDE>
__device__ __forceinline__ void hit_record2(const Grid2& g, const Out2& o, const float (&qf)[3][2],
                                            const float (&J)[3][4], bool wide, bool vector, int ax, int y, int t,
                                            int ty, int dx1, int dy1, int dt1, int dx2, int dy2, int dt2,
                                            unsigned idx, unsigned long long& n_fp64, unsigned long long& n_deg) {
  const long long plane = (long long)g.nx * g.ny;
  // exact cofactors of (v0 v1 v2 ; 1 1 1): C_i = (-1)^i det(columns without i)
  double Cd[3], Dd;
  bool degenerate;
  if (!WIDE) {
    // |q| < 2^24: every cofactor is an integer below 2^49 and D below 2^51, exact in binary64
    auto det2d = [](float a0, float a1, float b0, float b1) {
      const double p = (double)a1 * (double)b0;
      return __builtin_fma((double)a0, (double)b1, -p);
    };
    Cd[0] = det2d(qf[1][0], qf[1][1], qf[2][0], qf[2][1]);
    Cd[1] = -det2d(qf[0][0], qf[0][1], qf[2][0], qf[2][1]);
    Cd[2] = det2d(qf[0][0], qf[0][1], qf[1][0], qf[1][1]);
    Dd = (Cd[0] + Cd[1]) + Cd[2];
    degenerate = (Dd == 0.0);
  } else {
    long long q[3][2];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      q[i][0] = (long long)qf[i][0];
      q[i][1] = (long long)qf[i][1];
    }
    i128 C[3];
    C[0] = (i128)q[1][0] * q[2][1] - (i128)q[1][1] * q[2][0];
    C[1] = -((i128)q[0][0] * q[2][1] - (i128)q[0][1] * q[2][0]);
    C[2] = (i128)q[0][0] * q[1][1] - (i128)q[0][1] * q[1][0];
    const i128 D = C[0] + C[1] + C[2];
    degenerate = (D == 0);
#pragma unroll
    for (int i = 0; i < 3; ++i) Cd[i] = (double)C[i];
    Dd = (double)D;
  }
  unsigned fl = wide ? FL_WIDE : 0u;
  if (degenerate) {
    fl |= FL_DEGENERATE;
    ++n_deg;
  }
  float mu32[3];
  double mu64[3];
  int type = -1;
  if (g.precision == 0) {
    if (degenerate) {
      mu32[0] = mu32[1] = mu32[2] = 1.0f / 3.0f;
    } else {
      // hardware reciprocal (1 ulp): mu carries at most five roundings, inside the classifier's bound
      const float rD = __builtin_amdgcn_rcpf((float)Dd);
#pragma unroll
      for (int i = 0; i < 3; ++i) mu32[i] = (float)Cd[i] * rD;
    }
    type = classify2_fp32(mu32, J, vector);
  }
  if (g.precision != 0 || type < 0) {
    if (degenerate) {
      mu64[0] = mu64[1] = mu64[2] = 1.0 / 3.0;
    } else {
#pragma unroll
      for (int i = 0; i < 3; ++i) mu64[i] = Cd[i] / Dd;
    }
    type = classify2_fp64(mu64, J, vector);
    if (g.precision == 0) {
      fl |= FL_FP64;
      ++n_fp64;
    }
  }
  float pos[3], muo[3];
  const float cx0 = (float)ax, cy0 = (float)y, ct0 = (float)t;
  if (g.precision == 0) {
    float sx = mu32[0] * cx0;
    sx = sx + mu32[1] * (cx0 + dx1);
    sx = sx + mu32[2] * (cx0 + dx2);
    float sy = mu32[0] * cy0;
    sy = sy + mu32[1] * (cy0 + dy1);
    sy = sy + mu32[2] * (cy0 + dy2);
    float stt = mu32[0] * ct0;
    stt = stt + mu32[1] * (ct0 + dt1);
    stt = stt + mu32[2] * (ct0 + dt2);
    pos[0] = sx;
    pos[1] = sy;
    pos[2] = stt;
#pragma unroll
    for (int i = 0; i < 3; ++i) muo[i] = mu32[i];
  } else {
    const double X = ax, Y = y, T = t;
    double sx = mu64[0] * X;
    sx = sx + mu64[1] * (X + dx1);
    sx = sx + mu64[2] * (X + dx2);
    double sy = mu64[0] * Y;
    sy = sy + mu64[1] * (Y + dy1);
    sy = sy + mu64[2] * (Y + dy2);
    double stt = mu64[0] * T;
    stt = stt + mu64[1] * (T + dt1);
    stt = stt + mu64[2] * (T + dt2);
    pos[0] = (float)sx;
    pos[1] = (float)sy;
    pos[2] = (float)stt;
#pragma unroll
    for (int i = 0; i < 3; ++i) muo[i] = (float)mu64[i];
  }
  const long long agid = (long long)t * plane + (long long)y * g.nx + ax;
  const size_t oi = idx - o.gbase;
  o.face_id[oi] = agid * 12 + ty;
  if (o.pos) {
    o.pos[oi * 3 + 0] = pos[0];
    o.pos[oi * 3 + 1] = pos[1];
    o.pos[oi * 3 + 2] = pos[2];
  }
  if (o.mu) {
    o.mu[oi * 3 + 0] = muo[0];
    o.mu[oi * 3 + 1] = muo[1];
    o.mu[oi * 3 + 2] = muo[2];
  }
  if (o.type) o.type[oi] = (uint8_t)type;
  if (o.flags) o.flags[oi] = (uint8_t)fl;
}

template <int TY, bool WIDE>
__device__ __forceinline__ void emit2d_tile(const Grid2& g, int TT, int bx, int by, int bz,
                                            const uint16_t* __restrict__ masks, const int* __restrict__ seg_cnt,
                                            const long long* __restrict__ seg_off, const Out2& o,
                                            unsigned* __restrict__ status,
                                            unsigned long long* __restrict__ cnt,
                                            unsigned long long* __restrict__ work_cnt) {
  constexpr int GW = TX + 3, GH = TY + 3;  // vector field: x0-1 .. x0+TX+1, y0-1 .. y0+TY+1
  constexpr int FW = TX + 5, FH = TY + 5;  // scalar field: x0-2 .. x0+TX+2
  constexpr int RW = TX + 2, RH = TY + 2;  // mask slices: x0-1 .. x0+TX, y0-1 .. y0+TY
  constexpr int CAP = 2048;                // local union-find capacity (hits)
  constexpr int MAXTT = kEmitTT;           // step tables (TT <= kEmitTT)
  __shared__ float2 gs[2][GH * GW];
  // Mask slices of steps t-1, t, t+1 (ring slot = step mod 3) over the tile's anchors with a one-anchor halo: hit
  // masks, first hit of each anchor relative to its row segment's first hit (left halo column: minus its hit
  // count, right halo column: the segment's total), and the segments' first hit indices.
  __shared__ unsigned short rm[3][RH * RW];
  __shared__ short rx[3][RH * RW];
  __shared__ unsigned rb[3][RH];
  __shared__ int s_slice[3];  // step held by each ring slot
  // hit j of the wave's current row -> anchor lane | type << 6; between hit phases the same LDS holds the scalar
  // field of a plane being loaded
  __shared__ __align__(16) unsigned short s_lane[4][12 * 64];
  static_assert(FH * FW * sizeof(float) <= sizeof(s_lane), "scalar plane staging exceeds the hit map");
  float* const fs = reinterpret_cast<float*>(&s_lane[0][0]);
  __shared__ unsigned lpar[CAP];
  // non-empty row segments of the current chunk in local-id order: first local id and first global hit index
  __shared__ unsigned s_segl[MAXTT * TY], s_segg[MAXTT * TY];
  __shared__ int s_nseg;
  __shared__ unsigned lbase[MAXTT][TY];  // local id of the first hit of (step t - t0, row)
  __shared__ unsigned s_rc[MAXTT][TY], s_ro[MAXTT][TY];  // hits and first hit index of (step t - t0, row)
  __shared__ int s_chunk_t0, s_chunk_n, s_flush, s_global, s_plane_lbase, s_plane_total;
  __shared__ int s_have[2];  // step held by each field buffer (-1: none)
  __shared__ uint2 s_stage[kEdgeStage];
  __shared__ int s_stage_n;
  __shared__ unsigned long long s_red[4];
  __shared__ unsigned s_cof[24];  // triangle side words (Tri2Words)

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int x0 = bx * TX, y0 = by * TY;
  const int t0 = g.t_begin + bz * TT;
  const int t1 = min(t0 + TT, g.t_end);
  const int nx = g.nx, ny = g.ny, nt = g.nt, nxt = g.nxt;
  const long long plane = (long long)nx * ny;
  const bool vector = g.kind != 0;
  // workgroup-local capacities: the LDS sizes, or tiny ones under the FTK_DEBUG_SMALL_LDS test hook
  const int cap = (g.debug & 1) ? 128 : CAP;
  const int scap = (g.debug & 1) ? 8 : kEdgeStage;
  unsigned st = 0;
  unsigned long long n_fp64 = 0, n_deg = 0, n_linked = 0;


  // vector field of plane t into gs[par] (field loads from clamped in-grid addresses, all in flight together;
  // cells outside the grid are zeroed after)
  auto load_plane = [&](int t, int par) {
    if (!vector) {
      constexpr int NL = (FH * FW + 255) / 256;
      const float* src = g.f + (long long)fpl(g, t) * plane;
      float fv[NL];
      bool in[NL];
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        int e = tid + 256 * i;
        asm volatile("" : "+v"(e));  // opaque: the index math is redone per plane, not held across steps
        const int ly = e / FW, lx = e - ly * FW;
        const int gx = x0 - 2 + lx, gy = y0 - 2 + ly;
        in[i] = e < FH * FW && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        fv[i] = src[(long long)min(max(gy, 0), ny - 1) * nx + min(max(gx, 0), nx - 1)];
      }
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        const int e = tid + 256 * i;
        if (e < FH * FW) fs[e] = in[i] ? fv[i] : 0.0f;
      }
      __syncthreads();
      for (int e = tid; e < GH * GW; e += 256) {
        int ly = e / GW, lx = e - ly * GW;
        int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
        float2 v = make_float2(0.0f, 0.0f);
        if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
          const float* r = &fs[(ly + 1) * FW + (lx + 1)];
          v.x = diff3(r[-1], r[0], r[1], gx, nx);
          v.y = diff3(r[-FW], r[0], r[FW], gy, ny);
        }
        gs[par][e] = v;
      }
    } else {
      constexpr int NL = (GH * GW + 255) / 256;
      const float* su = g.f + (long long)fpl(g, t) * 2 * plane;
      const float* sv = su + plane;
      float f0[NL], f1[NL];
      bool in[NL];
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        int e = tid + 256 * i;
        asm volatile("" : "+v"(e));
        const int ly = e / GW, lx = e - ly * GW;
        const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
        in[i] = e < GH * GW && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        const long long k = (long long)min(max(gy, 0), ny - 1) * nx + min(max(gx, 0), nx - 1);
        f0[i] = su[k];
        f1[i] = sv[k];
      }
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        const int e = tid + 256 * i;
        if (e < GH * GW) gs[par][e] = in[i] ? make_float2(f0[i], f1[i]) : make_float2(0.0f, 0.0f);
      }
    }
  };

  // mask slice of step s (zero outside [0, nt)) into ring slot (s + 3) % 3
  auto load_slice = [&](int s) {
    constexpr int NL = (RH * RW + 255) / 256;
    const int slot = (s + 3) % 3;
    const bool ok = s >= 0 && s < nt;
    const long long mp = ok ? (long long)mpl(g, s) : 0;
    unsigned short mv[NL];
    bool in[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {  // clamped addresses, loads in flight together
      int e = tid + 256 * i;
      asm volatile("" : "+v"(e));
      const int r = e / RW, c = e - r * RW;
      const int y = y0 - 1 + r, x = x0 - 1 + c;
      in[i] = ok && e < RH * RW && y >= 0 && y < ny && x >= 0 && x < nx;
      mv[i] = masks[(mp * ny + min(max(y, 0), ny - 1)) * nx + min(max(x, 0), nx - 1)];
    }
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int e = tid + 256 * i;
      if (e < RH * RW) rm[slot][e] = in[i] ? mv[i] : (unsigned short)0;
    }
    if (tid < RH) {
      const int y = y0 - 1 + tid;
      rb[slot][tid] = (ok && y >= 0 && y < ny) ? (unsigned)seg_off[(mp * ny + y) * nxt + bx] : 0u;
    }
  };
  // per-anchor offsets of a loaded slice: one wavefront per row
  auto scan_slice = [&](int slot) {
    for (int r = wave; r < RH; r += 4) {
      const unsigned c = __popc((unsigned)rm[slot][r * RW + 1 + lane]);
      const unsigned incl = wave_incl_scan(c);
      rx[slot][r * RW + 1 + lane] = (short)(incl - c);
      if (lane == 63) rx[slot][r * RW + RW - 1] = (short)incl;
      if (lane == 0) rx[slot][r * RW] = (short)(-(int)__popc((unsigned)rm[slot][r * RW]));
    }
  };

  // Local root of x in the flushing chunk: a local id, or CAP + i once the set has been attached to the set of an
  // earlier chunk of this tile whose global root sits in stage slot i.
  auto lroot = [&](unsigned x) -> unsigned {
    for (;;) {
      const unsigned p = lpar[x];
      if (p == x || p >= (unsigned)CAP) return p;
      x = p;
    }
  };
  // Before the parents are written, each remaining local root r of segment k holds kRootTag + k (above every local
  // id and stage marker), so that its hit index s_segg[k] + (r - s_segl[k]) needs no search.
  constexpr unsigned kRootTag = 0x8000u;
  static_assert(CAP + kEdgeStage <= (int)kRootTag, "root tags above local ids and stage markers");
  // local id of a hit of the current chunk from its global index (segments are in increasing global order)
  auto seg_search = [&](const unsigned* key, unsigned v) -> int {
    int lo = 0, hi = s_nseg;  // last segment with key <= v
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (key[mid] <= v)
        lo = mid;
      else
        hi = mid;
    }
    return lo;
  };
  // Write the parent of every hit of the chunk.  Links staged as (earlier partner, hit) go from the chunk's first
  // step to an earlier chunk of this tile, whose parents are final: the hit's local set is attached to the
  // partner's global root (two such roots met by one set are united in place), and each hit of the chunk gets its
  // set's global root, or the hit index of its local root.  Attached links stay in the stage as no-op (R, R).
  auto flush = [&]() {
    __syncthreads();  // parents written so far by this workgroup are visible to it
    const int n = s_chunk_n, nseg = s_nseg;
    {
      // The chunk's local links: the hit loop made each hit's first smaller partner its parent (a forest: parents
      // point to smaller local ids) and left a second one in the entry's high half.  Take those out, point every
      // entry at its root (path halving), then unite the second partners through the shallow trees.
      unsigned sec[CAP / 256];
#pragma unroll
      for (int k = 0; k < CAP / 256; ++k) {
        const int i = tid + 256 * k;
        sec[k] = 0u;
        if (i < n) {
          const unsigned e = lpar[i];
          sec[k] = e >> 16;
          if (sec[k]) lpar[i] = e & 0xFFFFu;
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < CAP / 256; ++k) {
        const int i = tid + 256 * k;
        if (i < n) lpar[i] = lfind(lpar, (unsigned)i);
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < CAP / 256; ++k)
        if (sec[k]) lunite(lpar, (unsigned)(tid + 256 * k), sec[k] - 1u);
      __syncthreads();
    }
    const int nst = s_stage_n < scap ? s_stage_n : scap;
    for (int i = tid; i < nst; i += 256) {
      const uint2 e = s_stage[i];
      if (e.x >= e.y) continue;  // (hit, smaller partner): for the global list
      // The partner's parent was written by an earlier flush of this workgroup: an ancestor of its set, which
      // serves as the attachment point (the load is in flight during the local search).
      const unsigned R = wg_load(o.parent, e.x);
      const int k = seg_search(s_segg, e.y);
      unsigned r = lroot(s_segl[k] + (e.y - s_segg[k]));
      s_stage[i] = make_uint2(R, R);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      for (;;) {
        if (r >= (unsigned)CAP) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
          wg_unite(o.parent, R, s_stage[r - CAP].x);
          break;
        }
        const unsigned old = atomicCAS(&lpar[r], r, (unsigned)(CAP + i));
        if (old == r) break;
        r = old >= (unsigned)CAP ? old : lroot(old);
      }
    }
    __syncthreads();
    for (int k = wave; k < nseg; k += 4) {
      const unsigned l0 = s_segl[k], l1 = k + 1 < nseg ? s_segl[k + 1] : (unsigned)n;
      for (unsigned li = l0 + lane; li < l1; li += 64)
        if (lpar[li] == li) lpar[li] = kRootTag + (unsigned)k;
    }
    __syncthreads();
    for (int k = wave; k < nseg; k += 4) {
      const unsigned l0 = s_segl[k], l1 = k + 1 < nseg ? s_segl[k + 1] : (unsigned)n, g0 = s_segg[k];
      for (unsigned li = l0 + lane; li < l1; li += 64) {
        unsigned x = li, p = lpar[li];
        while (p < (unsigned)CAP) {
          x = p;
          p = lpar[x];
        }
        unsigned target;
        if (p >= kRootTag) {
          const unsigned kr = p - kRootTag;
          target = s_segg[kr] + (x - s_segl[kr]);
        } else {
          target = s_stage[p - CAP].x;
        }
        o.parent[g0 + (li - l0)] = target;
      }
    }
  };
  // Move the staged links (hit, smaller partner) to the global list.  Links staged as (partner, hit) wait in the
  // stage for their chunk's flush (compacted to the front); attached ones, (R, R), are dropped.  One wavefront.
  auto drain = [&]() {
    __syncthreads();  // nobody reads the stage any more (a flush may just have)
    const int n = s_stage_n < scap ? s_stage_n : scap;  // slots past the capacity went to the list
    if (wave == 0) {
      unsigned n_out = 0;
      for (int b = 0; b < n; b += 64) {
        bool out = false;
        if (b + lane < n) {
          const uint2 e = s_stage[b + lane];
          out = e.x > e.y;
        }
        n_out += (unsigned)__popcll(__ballot(out));
      }
      unsigned long long gb = 0;
      if (lane == 0 && n_out) gb = atomicAdd(work_cnt, (unsigned long long)n_out);
      gb = ((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)(gb >> 32), 0) << 32) |
           (unsigned)__builtin_amdgcn_readlane((int)(unsigned)gb, 0);
      const unsigned long long below = (1ull << lane) - 1ull;
      unsigned wo = 0, wk = 0;
      for (int b = 0; b < n; b += 64) {
        uint2 e = make_uint2(0u, 0u);
        bool out = false, keep = false;
        if (b + lane < n) {
          e = s_stage[b + lane];
          out = e.x > e.y;
          keep = e.x < e.y;
        }
        const unsigned long long bo = __ballot(out), bk = __ballot(keep);
        if (out) o.work[gb + wo + (unsigned)__popcll(bo & below)] = e;
        if (keep) s_stage[wk + (unsigned)__popcll(bk & below)] = e;  // below b + 64: not read again
        wo += (unsigned)__popcll(bo);
        wk += (unsigned)__popcll(bk);
      }
      if (lane == 0) s_stage_n = (int)wk;
    }
    __syncthreads();
  };

  if (tid == 0) {
    s_chunk_t0 = t0;
    s_chunk_n = 0;
    s_nseg = 0;
    s_stage_n = 0;
    s_have[0] = s_have[1] = -1;
    s_slice[0] = s_slice[1] = s_slice[2] = -2;
  }
  if (tid < 24) s_cof[tid] = kTri2WordsDev.w[tid];
  // hit counts and offsets of this tile's row segments for all its steps, read once: empty steps are skipped
  // without touching their masks
  for (int i = tid; i < (t1 - t0) * TY; i += 256) {
    const int dt = i / TY, r = i - dt * TY, y = y0 + r;
    unsigned c = 0, b = 0;
    if (y < ny) {
      const long long k = ((long long)mpl(g, t0 + dt) * ny + y) * nxt + bx;
      c = (unsigned)seg_cnt[k];
      b = (unsigned)seg_off[k];
    }
    s_rc[dt][r] = c;
    s_ro[dt][r] = b;
  }
  __syncthreads();

  for (int t = t0; t < t1; ++t) {
    const int par = t & 1;
    {
      unsigned tot = 0;
#pragma unroll
      for (int r = 0; r < TY; ++r) tot += s_rc[t - t0][r];
      if (tot == 0) continue;  // uniform
    }
    __syncthreads();
    // ring slots still to be filled for steps t-1, t, t+1 (read before any slot is rewritten)
    const bool need_prev = s_slice[(t + 2) % 3] != t - 1;
    const bool need_cur = s_slice[t % 3] != t;
    const bool need_next = s_slice[(t + 1) % 3] != t + 1;
    if (tid == 0) {
      unsigned tot = 0;
      for (int r = 0; r < TY; ++r) tot += s_rc[t - t0][r];
      s_plane_total = (int)tot;
      s_flush = (s_chunk_n > 0 && (s_chunk_n + (int)tot > cap || t - s_chunk_t0 >= MAXTT)) ? 1 : 0;
    }
    __syncthreads();
    if (s_flush) {
      flush();
      __syncthreads();
      if (tid == 0) {
        s_chunk_n = 0;
        s_nseg = 0;
        s_chunk_t0 = t;
      }
      __syncthreads();
    }
    if (s_stage_n > scap / 2) drain();
    if (tid == 0) {
      const int tot = s_plane_total;
      if (tot > cap) {  // too many hits for the local structure: this step links through the global list only
        s_global = 1;
        s_chunk_t0 = t + 1;
        s_chunk_n = 0;
        s_nseg = 0;
      } else {
        s_global = 0;
        if (s_chunk_n == 0) s_chunk_t0 = t;
        s_plane_lbase = s_chunk_n;
        unsigned run = (unsigned)s_chunk_n;
        int ns = s_nseg;
        for (int r = 0; r < TY; ++r) {
          lbase[t - t0][r] = run;
          const unsigned c = s_rc[t - t0][r];
          if (c) {  // non-empty segments only: both keys strictly increase (rows past the grid have no base)
            s_segl[ns] = run;
            s_segg[ns] = s_ro[t - t0][r];
            ++ns;
          }
          run += c;
        }
        s_nseg = ns;
        s_chunk_n = (int)run;
      }
    }
    __syncthreads();
    const bool plane_global = s_global != 0;
    const int chunk_t0 = s_chunk_t0;
    if (s_plane_total == 0) continue;  // uniform: nothing anchored in this tile at this step
    if (!plane_global)
      for (int i = tid; i < s_plane_total; i += 256) lpar[s_plane_lbase + i] = (unsigned)(s_plane_lbase + i);
    // mask slices of steps t-1, t, t+1 (only those not held yet), then the vector field of steps t and t+1
    if (need_prev) load_slice(t - 1);
    if (need_cur) load_slice(t);
    if (need_next) load_slice(t + 1);
    __syncthreads();
    if (need_prev) scan_slice((t + 2) % 3);
    if (need_cur) scan_slice(t % 3);
    if (need_next) scan_slice((t + 1) % 3);
    if (tid == 0) {
      s_slice[(t + 2) % 3] = t - 1;
      s_slice[t % 3] = t;
      s_slice[(t + 1) % 3] = t + 1;
    }
    if (s_have[par] != t) {
      load_plane(t, par);
      __syncthreads();
      if (tid == 0) s_have[par] = t;
    }
    if (t + 1 < nt && s_have[par ^ 1] != t + 1) {
      load_plane(t + 1, par ^ 1);
      __syncthreads();
      if (tid == 0) s_have[par ^ 1] = t + 1;
    }
    __syncthreads();

    for (int ly = wave; ly < TY; ly += 4) {
      const int y = y0 + ly;
      if (y >= ny) break;
      const unsigned total = s_rc[t - t0][ly];
      if (total == 0) continue;
      const unsigned base = s_ro[t - t0][ly];
      const unsigned row_lbase = plane_global ? 0u : lbase[t - t0][ly];
      const int cur = t % 3;
      // ring slot of each neighbour anchor slot (2-bit fields, as kSlotCol)
      const unsigned rsw = (unsigned)cur * 0x155u | (unsigned)((t + 2) % 3) << 10 | (unsigned)((t + 1) % 3) << 12;
      // local id of a smaller partner = its hit index + (local base - first hit index) of its row segment: the
      // same anchor or x - 1 (this row), y - 1, or step t - 1 (read only when that segment is in this chunk)
      const unsigned d_self = row_lbase - base;
      const unsigned d_my = (!plane_global && ly > 0) ? lbase[t - t0][ly - 1] - s_ro[t - t0][ly - 1] : 0u;
      const unsigned d_mt = (!plane_global && t - 1 >= chunk_t0) ? lbase[t - 1 - t0][ly] - s_ro[t - 1 - t0][ly] : 0u;
      // link class per smaller-partner slot (2-bit fields): 0 united here, 1 global list, 2 staged for the flush
      const unsigned cls_mt = t - 1 >= chunk_t0 ? 0u : (t - 1 >= t0 ? 2u : 1u);
      const unsigned clw = (ly == 0 ? 1u << (2 * NB_MY) : 0u) | cls_mt << (2 * NB_MT);

      // hit -> (anchor lane, type) map of this row segment (wavefront-private)
      {
        const int a = (ly + 1) * RW + 1 + lane;
        unsigned m = rm[cur][a];
        unsigned k = (unsigned)rx[cur][a];
        while (m) {
          const unsigned ty = (unsigned)__ffs((int)m) - 1u;
          m &= m - 1u;
          s_lane[wave][k++] = (unsigned short)((unsigned)lane | (ty << 6));
        }
      }
      wave_lds_sync();

      for (unsigned j = lane; j < total; j += 64) {
        const unsigned ent = s_lane[wave][j];
        const int L = (int)(ent & 63u), ty = (int)(ent >> 6);
        const unsigned idx = base + j;
        const int ax = x0 + L;
        const unsigned w0 = s_cof[2 * ty], w1 = s_cof[2 * ty + 1];
        const unsigned pk = w0 >> 25;
        const int m1 = pk & 15, m2 = pk >> 4;
        // vertex offsets along x, y, t of v1 and v2
        const int dx1 = m1 & 1, dy1 = (m1 >> 1) & 1, dt1 = (m1 >> 2) & 1;
        const int dx2 = dx1 + (m2 & 1), dy2 = dy1 + ((m2 >> 1) & 1), dt2 = dt1 + ((m2 >> 2) & 1);
        const int lxs[3] = {L, L + dx1, L + dx2};
        const int lys[3] = {ly, ly + dy1, ly + dy2};
        const int dts[3] = {0, dt1, dt2};

        float qf[3][2];
        float J[3][4];
        bool wide = false;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const float2* G = gs[par ^ dts[i]];
          const int c = (lys[i] + 1) * GW + (lxs[i] + 1);
          const float2 v = G[c];
          qf[i][0] = quant(v.x, g.qscale);
          qf[i][1] = quant(v.y, g.qscale);
          if constexpr (WIDE)  // the narrow variant only runs when every |q| < 2^24
            if (!(fabsf(qf[i][0]) < 2147483648.0f) || !(fabsf(qf[i][1]) < 2147483648.0f)) wide = true;
          const int gxv = x0 + lxs[i], gyv = y0 + lys[i];
          const float2 xl = G[c - 1], xh = G[c + 1], yl = G[c - GW], yh = G[c + GW];
          J[i][0] = diff3(xl.x, v.x, xh.x, gxv, nx);
          J[i][1] = diff3(yl.x, v.x, yh.x, gyv, ny);
          J[i][2] = diff3(xl.y, v.y, xh.y, gxv, nx);
          J[i][3] = diff3(yl.y, v.y, yh.y, gyv, ny);
        }
        hit_record2<WIDE>(g, o, qf, J, wide, vector, ax, y, t, ty, dx1, dy1, dt1, dx2, dy2, dt2, idx, n_fp64,
                          n_deg);

        // ---- pass 2 links: each of the (at most two) tetrahedra holding this triangle has exactly one other
        // punctured side.  Each link is recorded by its larger endpoint: inside this tile and chunk it goes to the
        // LDS union-find, otherwise to the global edge list.
        // (branch-free: every neighbour lookup stays inside the ring slices)
        unsigned sm0 = 0, sm1 = 0;
        int sl0 = 0, sl1 = 0;
        int ns = 0;
        bool bad = false;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const unsigned w = k == 0 ? w0 : w1;
          const int rule = w & 3, axis = (w >> 2) & 3;
          const int pa = axis == 0 ? ax : (axis == 1 ? y : t);
          const int Na = axis == 0 ? nx : (axis == 1 ? ny : nt);
          const bool exists = !((rule == 2 && pa < 1) || (rule == 3 && pa + 1 > Na - 1));  // the cell is in the grid
          int found = 0, oslot = 0;
          unsigned other = 0;
#pragma unroll
          for (int sdx = 0; sdx < 3; ++sdx) {
            const unsigned f = (w >> (4 + 7 * sdx)) & 127u;
            const int slot = f & 7, tt = f >> 3;
            // ring slot, slice row and column of the neighbour anchor (bit fields: no branch on the slot)
            const unsigned s2 = (unsigned)slot * 2u;
            const int rs = (int)((rsw >> s2) & 3u);
            const int rr = ly + (int)((kSlotRow >> s2) & 3u);
            const int rc = L + (int)((kSlotCol >> s2) & 3u);
            const unsigned um = rm[rs][rr * RW + rc];
            const unsigned hit = (um >> tt) & 1u;
            const unsigned cand = rb[rs][rr] + (unsigned)(int)rx[rs][rr * RW + rc] + __popc(um & ((1u << tt) - 1u));
            found += (int)hit;
            other = hit ? cand : other;
            oslot = hit ? slot : oslot;
          }
          bad = bad || (exists && found != 1);
          const bool take = exists && found == 1 && other < idx;
          sm1 = (take && ns == 1) ? other : sm1;
          sl1 = (take && ns == 1) ? oslot : sl1;
          sm0 = (take && ns == 0) ? other : sm0;
          sl0 = (take && ns == 0) ? oslot : sl0;
          ns += take ? 1 : 0;
        }
        if (bad || t == g.debug_step) st |= ST_INVARIANT;
        n_linked += ns;
        // link class of each smaller partner: 0 united here (anchor in this tile and chunk), 1 global list,
        // 2 partner in an earlier chunk of this tile (staged as (partner, hit), attached at this chunk's flush);
        // -1 none
        int c0 = -1, c1 = -1;
        if (plane_global) {
          o.parent[idx] = idx;
          c0 = ns > 0 ? 1 : -1;
          c1 = ns > 1 ? 1 : -1;
        } else {
          const unsigned li = row_lbase + j;
          const unsigned clw_l = clw | (L == 0 ? 1u << (2 * NB_MX) : 0u);
          auto link_class = [&](int sl) -> int { return (int)((clw_l >> (2 * sl)) & 3u); };
          auto local_id = [&](unsigned other, int sl) -> unsigned {
            return other + (sl == NB_MY ? d_my : (sl == NB_MT ? d_mt : d_self));
          };
          c0 = ns > 0 ? link_class(sl0) : -1;
          c1 = ns > 1 ? link_class(sl1) : -1;
          // The first smaller partner of this chunk becomes the parent (parents point to smaller local ids: a
          // forest); a second one waits in the high half of the entry for the chunk's flush.  Only this lane writes
          // the entry, and nothing reads the chunk's entries before the flush.
          const unsigned l0 = local_id(sm0, sl0), l1 = local_id(sm1, sl1);
          lpar[li] = (c0 == 0 ? l0 : li) | (c1 == 0 ? (l1 + 1u) << 16 : 0u);
        }
        append_edge(c0 > 0, c0 == 2 ? sm0 : idx, c0 == 2 ? idx : sm0, s_stage, &s_stage_n, scap, o.work, work_cnt);
        append_edge(c1 > 0, c1 == 2 ? sm1 : idx, c1 == 2 ? idx : sm1, s_stage, &s_stage_n, scap, o.work, work_cnt);
      }
      wave_lds_sync();
    }
  }
  __syncthreads();
  flush();
  drain();
  unsigned long long s1 = block_sum256(n_fp64, s_red);
  unsigned long long s2 = block_sum256(n_deg, s_red);
  unsigned long long s3 = block_sum256(n_linked, s_red);
  if (tid == 0) {
    if (s1) atomicAdd(&cnt[CNT_FP64], s1);
    if (s2) atomicAdd(&cnt[CNT_DEGEN], s2);
    if (s3) atomicAdd(&cnt[CNT_LINKED], s3);
  }
  if (st) atomicOr(status, st);
}

// The narrow variant is held to 128 VGPRs so that four workgroups share a CU (its LDS allows four).
template <int TY, bool WIDE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WIDE ? 2 : 4))) void emit2d(Grid2 g, int TT, const uint16_t* __restrict__ masks,
                                              const int* __restrict__ seg_cnt, const long long* __restrict__ seg_off,
                                              Out2 o, unsigned* __restrict__ status,
                                              unsigned long long* __restrict__ cnt) {
  emit2d_tile<TY, WIDE>(g, TT, blockIdx.x, blockIdx.y, blockIdx.z, masks, seg_cnt, seg_off, o, status, cnt,
                        &cnt[CNT_WORK]);
}

// ---------------------------------------------------------------------------------------------------------------
// Sparse emission: one wavefront per non-empty row segment, with no workgroup barriers.  When hits are rare (a few
// per thousand vertices) the tile-marching emission above pays a fixed cost per tile and step (ring loads, scans
// and barriers for a handful of hits).  Here a wavefront reads only what its segment's hits need: the hit masks of
// the five rows that hold the other sides of their cells (steps t-1..t+1 along y = const, rows y-1..y+1 at step
// t), the first-hit offsets of the three rows that can hold smaller partners (a partner with a smaller face id has
// an anchor at t-1, y-1, x-1 or at the same anchor), and the field values of each hit vertex's stencils, gathered
// through the caches.  No counter is shared: every link joins a hit to a smaller partner, so a hit with one or two
// smaller partners takes the first as its union-find parent (the parents then point to smaller indices and form a
// forest whose trees are connected parts of a trajectory; a tree's root is a hit with no smaller partner), and a
// hit with two writes the second to its own slot of the link array ((i, i) when absent), united afterwards by
// uf_hook_slots.  A trajectory is a path or a loop of hits (each lies in at most two cells), so the slot links
// (one per local maximum of the index along it) join all its trees.  To keep the trees shallow, a hit takes its
// partner's parent instead of the partner when that one is already written (parents start as 0xFFFFFFFF).  The
// records are the same operations as in the tiled form (hit_record2), so both forms give identical outputs.
// ---------------------------------------------------------------------------------------------------------------
namespace {

constexpr int kSpW = TX + 2;  // anchors x0-1 .. x0+64

// Per-wavefront LDS of the sparse emission.
struct SparseWave {
  unsigned short m[5][kSpW];       // hit masks: rows (t, y), (t, y-1), (t, y+1), (t-1, y), (t+1, y)
  short x[3][kSpW];                // first hit of each anchor relative to its segment: rows (t,y), (t,y-1), (t-1,y)
  unsigned b[3];                   // first hit index of the segments of those rows
  unsigned short map[12 * TX];     // hit j of the segment -> anchor lane | type << 6
  unsigned cof[24];                // triangle side words (Tri2Words), read per hit with a lane-dependent type
};

// mask row of each neighbour slot, and its offset row (-1: the row only holds larger partners)
__device__ __forceinline__ int sp_row(int slot) {
  return slot <= NB_PX ? 0 : (slot == NB_MY ? 1 : (slot == NB_PY ? 2 : (slot == NB_MT ? 3 : 4)));
}

// Binary32 vector of vertex (x, y) of field plane P (gradient of a scalar by the stencil of pass 1, or the vector
// itself) and its Jacobian stencil J: the same operations as the staged form.  Coordinates outside the grid are
// clamped; diff3 never uses those values (one-sided differences at the first and last index).
__device__ __forceinline__ void vertex_stencil2(const Grid2& g, int x, int y, int t, float2& v, float (&J)[4]) {
  const int nx = g.nx, ny = g.ny;
  const long long plane = (long long)nx * ny;
  auto cx = [&](int i) { return i < 0 ? 0 : (i >= nx ? nx - 1 : i); };
  auto cy = [&](int i) { return i < 0 ? 0 : (i >= ny ? ny - 1 : i); };
  float2 xl, xh, yl, yh;
  if (g.kind == 0) {
    const float* P = g.f + (long long)fpl(g, t) * plane;
    auto F = [&](int dx, int dy) { return P[(long long)cy(y + dy) * nx + cx(x + dx)]; };
    const float f00 = F(0, 0), fm0 = F(-1, 0), fp0 = F(1, 0), f0m = F(0, -1), f0p = F(0, 1);
    const float fmm0 = F(-2, 0), fpp0 = F(2, 0), f0mm = F(0, -2), f0pp = F(0, 2);
    const float fmm = F(-1, -1), fpm = F(1, -1), fmp = F(-1, 1), fpp = F(1, 1);
    const int xm = x - 1, xp = x + 1, ym = y - 1, yp = y + 1;
    v.x = diff3(fm0, f00, fp0, x, nx);
    v.y = diff3(f0m, f00, f0p, y, ny);
    xl = make_float2(diff3(fmm0, fm0, f00, xm, nx), diff3(fmm, fm0, fmp, y, ny));
    xh = make_float2(diff3(f00, fp0, fpp0, xp, nx), diff3(fpm, fp0, fpp, y, ny));
    yl = make_float2(diff3(fmm, f0m, fpm, x, nx), diff3(f0mm, f0m, f00, ym, ny));
    yh = make_float2(diff3(fmp, f0p, fpp, x, nx), diff3(f00, f0p, f0pp, yp, ny));
  } else {
    const float* U = g.f + (long long)fpl(g, t) * 2 * plane;
    const float* W = U + plane;
    auto V = [&](int dx, int dy) {
      const long long k = (long long)cy(y + dy) * nx + cx(x + dx);
      return make_float2(U[k], W[k]);
    };
    v = V(0, 0);
    xl = V(-1, 0);
    xh = V(1, 0);
    yl = V(0, -1);
    yh = V(0, 1);
  }
  J[0] = diff3(xl.x, v.x, xh.x, x, nx);
  J[1] = diff3(yl.x, v.x, yh.x, y, ny);
  J[2] = diff3(xl.y, v.y, xh.y, x, nx);
  J[3] = diff3(yl.y, v.y, yh.y, y, ny);
}

// One row segment (anchors x0 .. x0+63 of row y, step t) with `total` hits from global index `base`.
template <bool WIDE>
__device__ __forceinline__ void emit2d_segment(const Grid2& g, int t, int y, int bx, const uint16_t* __restrict__ masks,
                                               const long long* __restrict__ seg_off, const Out2& o, SparseWave& W,
                                               unsigned& st,
                                               unsigned long long& n_fp64, unsigned long long& n_deg,
                                               unsigned long long& n_linked) {
  const int lane = lane_id();
  const int nx = g.nx, ny = g.ny, nt = g.nt, nxt = g.nxt;
  const int x0 = bx * TX;
  const bool vector = g.kind != 0;
  // the five mask rows (clamped addresses: all loads in flight together; cells outside the grid zeroed after)
  constexpr int NR = (5 * kSpW + 63) / 64;
  unsigned short mv[NR];
  bool in[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const int e = lane + 64 * i;
    const int r = e / kSpW, c = e - r * kSpW;
    const int tt = t + (r == 3 ? -1 : (r == 4 ? 1 : 0));
    const int yy = y + (r == 1 ? -1 : (r == 2 ? 1 : 0));
    const int xx = x0 - 1 + c;
    in[i] = e < 5 * kSpW && tt >= 0 && tt < nt && yy >= 0 && yy < ny && xx >= 0 && xx < nx;
    const int tc = min(max(tt, 0), nt - 1), yc = min(max(yy, 0), ny - 1), xc = min(max(xx, 0), nx - 1);
    mv[i] = masks[((long long)mpl(g, tc) * ny + yc) * nx + xc];
  }
  unsigned bv = 0;
  if (lane < 3) {
    const int tt = lane == 2 ? t - 1 : t, yy = lane == 1 ? y - 1 : y;
    bv = (unsigned)seg_off[((long long)mpl(g, max(tt, 0)) * ny + max(yy, 0)) * nxt + bx];
    if (tt < 0 || yy < 0) bv = 0u;
  }
  wave_lds_sync();  // the previous segment's reads of W are done
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const int e = lane + 64 * i;
    if (e < 5 * kSpW) (&W.m[0][0])[e] = in[i] ? mv[i] : (unsigned short)0;
  }
  if (lane < 3) W.b[lane] = bv;
  wave_lds_sync();
  unsigned total = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int r = i == 2 ? 3 : i;
    const unsigned c = __popc((unsigned)W.m[r][1 + lane]);
    const unsigned incl = wave_incl_scan(c);
    W.x[i][1 + lane] = (short)(incl - c);
    if (lane == 63) W.x[i][kSpW - 1] = (short)incl;
    if (lane == 0) W.x[i][0] = (short)(-(int)__popc((unsigned)W.m[r][0]));
    if (i == 0) total = (unsigned)__builtin_amdgcn_readlane((int)incl, 63);
  }
  {
    unsigned m = W.m[0][1 + lane];
    unsigned k = (unsigned)(W.x[0][1 + lane]);
    while (m) {
      const unsigned ty = (unsigned)__ffs((int)m) - 1u;
      m &= m - 1u;
      W.map[k++] = (unsigned short)((unsigned)lane | (ty << 6));
    }
  }
  wave_lds_sync();
  const unsigned base = W.b[0];
  for (unsigned j = lane; j < total; j += 64) {
    const unsigned ent = W.map[j];
    const int L = (int)(ent & 63u), ty = (int)(ent >> 6);
    const unsigned idx = base + j;
    const int ax = x0 + L;
    const unsigned w0 = W.cof[2 * ty], w1 = W.cof[2 * ty + 1];
    const unsigned pk = w0 >> 25;
    const int m1 = pk & 15, m2 = pk >> 4;
    const int dx1 = m1 & 1, dy1 = (m1 >> 1) & 1, dt1 = (m1 >> 2) & 1;
    const int dx2 = dx1 + (m2 & 1), dy2 = dy1 + ((m2 >> 1) & 1), dt2 = dt1 + ((m2 >> 2) & 1);
    const int dxs[3] = {0, dx1, dx2}, dys[3] = {0, dy1, dy2}, dts[3] = {0, dt1, dt2};
    float qf[3][2];
    float J[3][4];
    bool wide = false;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      float2 v;
      vertex_stencil2(g, ax + dxs[i], y + dys[i], t + dts[i], v, J[i]);
      qf[i][0] = quant(v.x, g.qscale);
      qf[i][1] = quant(v.y, g.qscale);
      if constexpr (WIDE)
        if (!(fabsf(qf[i][0]) < 2147483648.0f) || !(fabsf(qf[i][1]) < 2147483648.0f)) wide = true;
    }
    hit_record2<WIDE>(g, o, qf, J, wide, vector, ax, y, t, ty, dx1, dy1, dt1, dx2, dy2, dt2, idx, n_fp64, n_deg);

    // links (Alg. 1 pass 2): the other punctured side of each tetrahedron holding the triangle; the larger end of
    // each link records it
    unsigned sm0 = 0, sm1 = 0;
    int ns = 0;
    bool bad = false;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const unsigned w = k == 0 ? w0 : w1;
      const int rule = w & 3, axis = (w >> 2) & 3;
      const int pa = axis == 0 ? ax : (axis == 1 ? y : t);
      const int Na = axis == 0 ? nx : (axis == 1 ? ny : nt);
      const bool exists = !((rule == 2 && pa < 1) || (rule == 3 && pa + 1 > Na - 1));
      int found = 0;
      unsigned other = 0;
#pragma unroll
      for (int sdx = 0; sdx < 3; ++sdx) {
        const unsigned f = (w >> (4 + 7 * sdx)) & 127u;
        const int slot = f & 7, tt = f >> 3;
        const int row = sp_row(slot);
        const int col = L + 1 + (slot == NB_MX ? -1 : (slot == NB_PX ? 1 : 0));
        const unsigned um = W.m[row][col];
        const unsigned hit = (um >> tt) & 1u;
        const int xr = row == 0 ? 0 : (row == 1 ? 1 : (row == 3 ? 2 : -1));
        const unsigned cand = xr < 0 ? 0xFFFFFFFFu
                                     : W.b[xr] + (unsigned)(int)W.x[xr][col] + __popc(um & ((1u << tt) - 1u));
        found += (int)hit;
        other = hit ? cand : other;
      }
      bad = bad || (exists && found != 1);
      const bool take = exists && found == 1 && other < idx;
      sm1 = (take && ns == 1) ? other : sm1;
      sm0 = (take && ns == 0) ? other : sm0;
      ns += take ? 1 : 0;
    }
    if (bad || t == g.debug_step) st |= ST_INVARIANT;
    n_linked += ns;
    unsigned par = idx;
    if (ns > 0) {  // an ancestor of the partner if already written (a stale read only gives a deeper tree)
      const unsigned q = __hip_atomic_load(o.parent + sm0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      par = q == 0xFFFFFFFFu ? sm0 : q;
    }
    __hip_atomic_store(o.parent + idx, par, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    o.work[idx] = make_uint2(idx, ns > 1 ? sm1 : idx);
  }
}

// Per-wavefront counters into the call's (or series') counters.
__device__ __forceinline__ void sparse_flush_counts(unsigned long long* cnt, unsigned long long& n_fp64,
                                                    unsigned long long& n_deg, unsigned long long& n_linked) {
  const unsigned long long a = wave_sum64(n_fp64), b = wave_sum64(n_deg), c = wave_sum64(n_linked);
  if (lane_id() == 0) {
    if (a) atomicAdd(&cnt[CNT_FP64], a);
    if (b) atomicAdd(&cnt[CNT_DEGEN], b);
    if (c) atomicAdd(&cnt[CNT_LINKED], c);
  }
  n_fp64 = n_deg = n_linked = 0;
}

// Segments [64 blk, 64 blk + 64) of the steps [t_begin, t_end): each lane reads one segment's count, the wavefront
// walks the non-empty ones.
template <bool WIDE>
__device__ __forceinline__ void emit2d_sparse_block(const Grid2& g, long long blk, const uint16_t* __restrict__ masks,
                                                    const int* __restrict__ seg_cnt,
                                                    const long long* __restrict__ seg_off, const Out2& o,
                                                    SparseWave& W, unsigned& st, unsigned long long& n_fp64,
                                                    unsigned long long& n_deg, unsigned long long& n_linked) {
  const unsigned per_step = (unsigned)g.ny * (unsigned)g.nxt;  // segments per step
  const long long nseg = (long long)(g.t_end - g.t_begin) * per_step;
  const long long s0 = blk * 64;
  // step and in-step segment of the block's first segment; the block's 64 segments span at most a few steps
  const int tb = (int)(s0 / per_step);
  const unsigned rb0 = (unsigned)(s0 - (long long)tb * per_step);
  auto locate = [&](int b, int& t, unsigned& r) {
    t = tb;
    r = rb0 + (unsigned)b;
    while (r >= per_step) {
      r -= per_step;
      ++t;
    }
    t += g.t_begin;
  };
  int c = 0;
  if (s0 + lane_id() < nseg) {
    int t;
    unsigned r;
    locate(lane_id(), t, r);
    c = seg_cnt[(long long)mpl(g, t) * per_step + r];
  }
  unsigned long long bal = __ballot(c > 0);
  while (bal) {
    const int b = __ffsll((long long)bal) - 1;
    bal &= bal - 1ull;
    int t;
    unsigned r;
    locate(b, t, r);
    const int y = (int)(r / (unsigned)g.nxt), bx = (int)(r - (unsigned)y * (unsigned)g.nxt);
    emit2d_segment<WIDE>(g, t, y, bx, masks, seg_off, o, W, st, n_fp64, n_deg, n_linked);
  }
}

// Wavefronts of the sparse emission: enough for four per SIMD.  A wavefront takes one 64-segment block per turn, so
// the blocks in flight span about 4096 x 64 segments (a few steps at most): the partners at step t-1 of a hit are
// then mostly written already, which keeps the parent trees shallow.
constexpr int kSparseWaves = 4096;

}  // namespace

template <bool WIDE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void emit2d_sparse(Grid2 g, const uint16_t* __restrict__ masks,
                                                     const int* __restrict__ seg_cnt,
                                                     const long long* __restrict__ seg_off, Out2 o,
                                                     unsigned* __restrict__ status,
                                                     unsigned long long* __restrict__ cnt) {
  __shared__ SparseWave sw[4];
  __shared__ unsigned long long red[3][4];
  SparseWave& W = sw[threadIdx.x >> 6];
  if ((threadIdx.x & 63) < 24) W.cof[threadIdx.x & 63] = kTri2WordsDev.w[threadIdx.x & 63];
  wave_lds_sync();
  const long long nblk = ((long long)(g.t_end - g.t_begin) * g.ny * g.nxt + 63) / 64;
  const long long nw = (long long)gridDim.x * 4;
  unsigned st = 0;
  unsigned long long n_fp64 = 0, n_deg = 0, n_linked = 0;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // wave-uniform: scalar loop state
  for (long long blk = (long long)blockIdx.x * 4 + wv; blk < nblk; blk += nw)
    emit2d_sparse_block<WIDE>(g, blk, masks, seg_cnt, seg_off, o, W, st, n_fp64, n_deg, n_linked);
  // one counter update per workgroup (same-address atomics serialise)
  const int w = threadIdx.x >> 6;
  const unsigned long long a = wave_sum64(n_fp64), b = wave_sum64(n_deg), c = wave_sum64(n_linked);
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = a;
    red[1][w] = b;
    red[2][w] = c;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int k = threadIdx.x;
    const unsigned long long v = red[k][0] + red[k][1] + red[k][2] + red[k][3];
    if (v) atomicAdd(&cnt[k == 0 ? CNT_FP64 : (k == 1 ? CNT_DEGEN : CNT_LINKED)], v);
  }
  if (st) atomicOr(status, st);
}

// ---------------------------------------------------------------------------------------------------------------
// Batched form: one persistent launch per stage for many independent series.  Workgroups pull (series, tile) items
// from a device counter; the item -> series map is a binary search over the per-series item prefix.
// ---------------------------------------------------------------------------------------------------------------
__device__ __forceinline__ int take_item(int* counter, int total, int* s_item) {
  __syncthreads();
  if (threadIdx.x == 0) *s_item = atomicAdd(counter, 1);
  __syncthreads();
  const int it = *s_item;
  return it < total ? it : -1;
}

__device__ __forceinline__ int series_of(const int* prefix, int nser, int item) {
  int lo = 0, hi = nser;  // prefix[lo] <= item < prefix[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= item)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

template <int TY, bool WIDE>
__global__ __launch_bounds__(256) void detect2d_batched(const Series2* __restrict__ S, const int* __restrict__ prefix,
                                                        int nser, int TT, int* counter, unsigned* status) {
  __shared__ int s_item;
  const int total = prefix[nser];
  for (;;) {
    const int it = take_item(counter, total, &s_item);
    if (it < 0) break;
    const int s = series_of(prefix, nser, it);
    const Grid2 g = S[s].g;
    const int local = it - prefix[s];
    const int tx = g.nxt, tyn = (g.ny + TY - 1) / TY;
    const int bx = local % tx, by = (local / tx) % tyn, bz = local / (tx * tyn);
    detect2d_tile<TY, WIDE>(g, TT, bx, by, bz, S[s].masks, S[s].seg_cnt, status);
  }
}

template <int TY, bool WIDE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WIDE ? 2 : 3))) void emit2d_batched(const Series2* __restrict__ S, const int* __restrict__ prefix,
                                                      int nser, int TT, int* counter, unsigned* status,
                                                      unsigned long long* work_cnt) {
  __shared__ int s_item;
  const int total = prefix[nser];
  for (;;) {
    const int it = take_item(counter, total, &s_item);
    if (it < 0) break;
    const int s = series_of(prefix, nser, it);
    const Grid2 g = S[s].g;
    const Out2 o = S[s].o;
    const int local = it - prefix[s];
    const int tx = g.nxt, tyn = (g.ny + TY - 1) / TY;
    const int bx = local % tx, by = (local / tx) % tyn, bz = local / (tx * tyn);
    emit2d_tile<TY, WIDE>(g, TT, bx, by, bz, S[s].masks, S[s].seg_cnt, S[s].seg_off, o, status, S[s].cnt,
                          work_cnt);
  }
}

// Batched sparse emission: the 64-segment blocks of the series that take the sparse form, concatenated (bprefix:
// per-series block prefix, zero blocks for the others); a wavefront's block -> series by binary search.
template <bool WIDE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void emit2d_sparse_batched(const Series2* __restrict__ S,
                                                             const long long* __restrict__ bprefix, int nser,
                                                             unsigned* status) {
  __shared__ SparseWave sw[4];
  SparseWave& W = sw[threadIdx.x >> 6];
  if ((threadIdx.x & 63) < 24) W.cof[threadIdx.x & 63] = kTri2WordsDev.w[threadIdx.x & 63];
  wave_lds_sync();
  const long long nblk = bprefix[nser];
  const long long nw = (long long)gridDim.x * 4;
  unsigned st = 0;
  unsigned long long n_fp64 = 0, n_deg = 0, n_linked = 0;
  int cur = -1;  // series whose counts are being gathered (flushed when the wavefront moves to another)
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // wave-uniform: scalar loop state
  for (long long B = (long long)blockIdx.x * 4 + wv; B < nblk; B += nw) {
    int lo = 0, hi = nser;  // bprefix[lo] <= B < bprefix[lo + 1]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (bprefix[mid] <= B)
        lo = mid;
      else
        hi = mid;
    }
    if (lo != cur) {
      if (cur >= 0) sparse_flush_counts(S[cur].cnt, n_fp64, n_deg, n_linked);
      cur = lo;
    }
    const Grid2 g = S[lo].g;
    const Out2 o = S[lo].o;
    emit2d_sparse_block<WIDE>(g, B - bprefix[lo], S[lo].masks, S[lo].seg_cnt, S[lo].seg_off, o, W, st, n_fp64, n_deg,
                              n_linked);
  }
  if (cur >= 0) sparse_flush_counts(S[cur].cnt, n_fp64, n_deg, n_linked);
  if (st) atomicOr(status, st);
}

// Emission of single steps (streaming): one step per launch, local union-find per step.
hipError_t launch_emit2d_steps(const Grid2& g, bool wide, const uint16_t* masks, const int* seg_cnt,
                               const long long* seg_off, const Out2& o, unsigned* status, unsigned long long* cnt,
                               hipStream_t s) {
  constexpr int TYE = 8;
  dim3 grid((unsigned)g.nxt, (unsigned)((g.ny + TYE - 1) / TYE), (unsigned)(g.t_end - g.t_begin));
  if (wide)
    emit2d<TYE, true><<<grid, 256, 0, s>>>(g, 1, masks, seg_cnt, seg_off, o, status, cnt);
  else
    emit2d<TYE, false><<<grid, 256, 0, s>>>(g, 1, masks, seg_cnt, seg_off, o, status, cnt);
  return hipGetLastError();
}

hipError_t launch_detect2d_batched(const Series2* S, const int* prefix, int nser, int total_items, int tt, bool wide,
                                   int* counter, unsigned* status, hipStream_t s) {
  int blocks = total_items < 2048 ? total_items : 2048;
  if (blocks < 1) blocks = 1;
  if (wide)
    detect2d_batched<16, true><<<blocks, 256, 0, s>>>(S, prefix, nser, tt, counter, status);
  else
    detect2d_batched<16, false><<<blocks, 256, 0, s>>>(S, prefix, nser, tt, counter, status);
  return hipGetLastError();
}

hipError_t launch_emit2d_batched(const Series2* S, const int* prefix, int nser, int total_items, bool wide,
                                 int* counter, unsigned* status, unsigned long long* work_cnt, hipStream_t s) {
  int blocks = total_items < 1536 ? total_items : 1536;
  if (blocks < 1) blocks = 1;
  if (wide)
    emit2d_batched<8, true><<<blocks, 256, 0, s>>>(S, prefix, nser, kEmitTT, counter, status, work_cnt);
  else
    emit2d_batched<8, false><<<blocks, 256, 0, s>>>(S, prefix, nser, kEmitTT, counter, status, work_cnt);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------------------------------------------
hipError_t launch_detect2d(const Grid2& g, int ty, int tt, bool wide, uint16_t* masks, int* seg_cnt,
                           unsigned* status, hipStream_t s) {
  dim3 grid((unsigned)g.nxt, (unsigned)((g.ny + ty - 1) / ty), (unsigned)((g.t_end - g.t_begin + tt - 1) / tt));
  if (ty == 8) {
    if (wide)
      detect2d<8, true><<<grid, 256, 0, s>>>(g, tt, masks, seg_cnt, status);
    else
      detect2d<8, false><<<grid, 256, 0, s>>>(g, tt, masks, seg_cnt, status);
  } else if (ty == 16) {
    if (wide)
      detect2d<16, true><<<grid, 256, 0, s>>>(g, tt, masks, seg_cnt, status);
    else
      detect2d<16, false><<<grid, 256, 0, s>>>(g, tt, masks, seg_cnt, status);
  } else {
    if (wide)
      detect2d<32, true><<<grid, 256, 0, s>>>(g, tt, masks, seg_cnt, status);
    else
      detect2d<32, false><<<grid, 256, 0, s>>>(g, tt, masks, seg_cnt, status);
  }
  return hipGetLastError();
}

hipError_t launch_emit2d(const Grid2& g, bool wide, const uint16_t* masks, const int* seg_cnt,
                         const long long* seg_off, const Out2& o, unsigned* status, unsigned long long* cnt,
                         hipStream_t s) {
  constexpr int TYE = 8, TTE = kEmitTT;
  static_assert(TTE <= 32, "steps per emission tile exceed the tile's step tables");
  dim3 grid((unsigned)g.nxt, (unsigned)((g.ny + TYE - 1) / TYE), (unsigned)((g.t_end - g.t_begin + TTE - 1) / TTE));
  if (wide)
    emit2d<TYE, true><<<grid, 256, 0, s>>>(g, TTE, masks, seg_cnt, seg_off, o, status, cnt);
  else
    emit2d<TYE, false><<<grid, 256, 0, s>>>(g, TTE, masks, seg_cnt, seg_off, o, status, cnt);
  return hipGetLastError();
}

hipError_t launch_emit2d_sparse(const Grid2& g, bool wide, const uint16_t* masks, const int* seg_cnt,
                                const long long* seg_off, const Out2& o, unsigned* status, unsigned long long* cnt,
                                hipStream_t s) {
  const long long nblk = ((long long)(g.t_end - g.t_begin) * g.ny * g.nxt + 63) / 64;
  long long blocks = (nblk + 3) / 4;
  if (blocks > kSparseWaves / 4) blocks = kSparseWaves / 4;
  if (blocks < 1) blocks = 1;
  if (wide)
    emit2d_sparse<true><<<(unsigned)blocks, 256, 0, s>>>(g, masks, seg_cnt, seg_off, o, status, cnt);
  else
    emit2d_sparse<false><<<(unsigned)blocks, 256, 0, s>>>(g, masks, seg_cnt, seg_off, o, status, cnt);
  return hipGetLastError();
}

hipError_t launch_emit2d_sparse_batched(const Series2* S, const long long* bprefix, int nser, long long total_blocks,
                                        bool wide, unsigned* status, hipStream_t s) {
  long long blocks = (total_blocks + 3) / 4;
  if (blocks > kSparseWaves / 4) blocks = kSparseWaves / 4;
  if (blocks < 1) blocks = 1;
  if (wide)
    emit2d_sparse_batched<true><<<(unsigned)blocks, 256, 0, s>>>(S, bprefix, nser, status);
  else
    emit2d_sparse_batched<false><<<(unsigned)blocks, 256, 0, s>>>(S, bprefix, nser, status);
  return hipGetLastError();
}

}  // namespace ftk
