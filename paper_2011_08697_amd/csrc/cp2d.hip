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

// triangle types using each axis (validity masks at the last index of an axis)
constexpr unsigned kUseX = (unsigned)types_using_axis(kTri2, 1);
constexpr unsigned kUseY = (unsigned)types_using_axis(kTri2, 2);
constexpr unsigned kUseT = (unsigned)types_using_axis(kTri2, 4);

template <bool WIDE>
struct QType;
template <>
struct QType<false> {
  typedef int T;
};
template <>
struct QType<true> {
  typedef long long T;
};

// Round-to-integer with range classification.  Narrow: |q| < 2^31.  Wide: |q| < 2^62.
template <bool WIDE>
__device__ __forceinline__ typename QType<WIDE>::T to_q(float r, unsigned& st) {
  if (!WIDE) {
    if (!(fabsf(r) < 2147483648.0f)) {
      st |= ST_WIDE;
      return 0;
    }
    return (int)r;
  } else {
    if (!(fabsf(r) < 4611686018427387904.0f)) {
      st |= ST_RANGE;
      return 0;
    }
    return (long long)r;
  }
}

}  // namespace

// ---------------------------------------------------------------------------------------------------------------
// Pass 1: detection.
// grid = (ceil(nx / 64), ceil(ny / TY), ceil(nt / TT)), block = 256.
// ---------------------------------------------------------------------------------------------------------------
template <int TY, bool WIDE>
__global__ __launch_bounds__(256) void detect2d(Grid2 g, int TT, uint16_t* __restrict__ masks,
                                                int* __restrict__ seg_cnt, unsigned* __restrict__ status) {
  typedef typename QType<WIDE>::T Q;
  constexpr int FW = TX + 4, FH = TY + 4;  // field plane + 2-cell halo (x0-1 .. x0+TX+2)
  constexpr int QW = TX + 2, QH = TY + 2;  // quantised vectors (x0 .. x0+TX+1)
  constexpr int EW = TX + 1, EH = TY + 1;  // edge words (x0 .. x0+TX)
  __shared__ float fs[2][FH * FW];
  __shared__ Q qs[2][2][QH * QW];  // [plane parity][component]
  __shared__ uint8_t ew[2][EH * EW];

  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  const int t0 = blockIdx.z * TT;
  const int t1 = min(t0 + TT, g.nt);
  const int nx = g.nx, ny = g.ny, nt = g.nt;
  const long long plane = (long long)nx * ny;
  unsigned st = 0;

  // Load plane t into fs (scalar: FH x FW with halo; vector: both components over the QH x QW region).
  auto load_plane = [&](int t) {
    if (g.kind == 0) {
      const float* src = g.f + (long long)t * plane;
      for (int e = tid; e < FH * FW; e += 256) {
        int ly = e / FW, lx = e - ly * FW;
        int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
        float v = 0.0f;
        if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
          v = src[(long long)gy * nx + gx];
          if (!isfinite(v)) st |= ST_NONFINITE;
        }
        fs[0][e] = v;
      }
    } else {
      for (int c = 0; c < 2; ++c) {
        const float* src = g.f + ((long long)t * 2 + c) * plane;
        for (int e = tid; e < QH * QW; e += 256) {
          int ly = e / QW, lx = e - ly * QW;
          int gx = x0 + lx, gy = y0 + ly;
          float v = 0.0f;
          if (gx < nx && gy < ny) {
            v = src[(long long)gy * nx + gx];
            if (!isfinite(v)) st |= ST_NONFINITE;
          }
          fs[c][e] = v;
        }
      }
    }
  };

  // Quantised vectors of plane (parity par) from fs.
  auto quantise_plane = [&](int par) {
    for (int e = tid; e < QH * QW; e += 256) {
      int ly = e / QW, lx = e - ly * QW;
      int gx = x0 + lx, gy = y0 + ly;
      Q q0 = 0, q1 = 0;
      if (gx < nx && gy < ny) {
        float v0, v1;
        if (g.kind == 0) {
          const float* r = &fs[0][(ly + 1) * FW + (lx + 1)];
          v0 = diff3(r[-1], r[0], r[1], gx, nx);
          v1 = diff3(r[-FW], r[0], r[FW], gy, ny);
        } else {
          v0 = fs[0][e];
          v1 = fs[1][e];
        }
        q0 = to_q<WIDE>(quant(v0, g.qscale), st);
        q1 = to_q<WIDE>(quant(v1, g.qscale), st);
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

  // prologue: plane t0
  load_plane(t0);
  __syncthreads();
  quantise_plane(t0 & 1);
  __syncthreads();
  ordinal_edges(t0 & 1);

  const int wave = tid >> 6, lane = tid & 63;
  const int gx = x0 + lane;
  for (int t = t0; t < t1; ++t) {
    const int par = t & 1, nxp = par ^ 1;
    const bool has_next = (t + 1 < nt);
    __syncthreads();  // previous triangle pass done with ew / fs
    if (has_next) {
      load_plane(t + 1);
      __syncthreads();
      quantise_plane(nxp);
      __syncthreads();
      ordinal_edges(nxp);
      interval_edges(par);
    }
    __syncthreads();

    // triangle tests: wave w handles rows w, w+4, ...
    for (int ly = wave; ly < TY; ly += 4) {
      const int gy = y0 + ly;
      unsigned m = 0;
      if (gx < nx && gy < ny) {
        const int a = ly * EW + lane;
        // word of the anchor and of its neighbours p + e(M1): plane t for M1 in {x, y, xy}, plane t+1 (ordinal
        // bits only) for M1 in {t, xt, yt}
        unsigned W[7];
        W[0] = ew[par][a];
        W[1] = ew[par][a + 1];
        W[2] = ew[par][a + EW];
        W[3] = ew[par][a + EW + 1];
        W[4] = has_next ? ew[nxp][a] : 0u;
        W[5] = has_next ? ew[nxp][a + 1] : 0u;
        W[6] = has_next ? ew[nxp][a + EW] : 0u;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          const int m1 = kTri2.m[k][0], m2 = kTri2.m[k][1];
          // sides opposite v0, v1, v2: edges (v1 v2) = (p + e(M1), M2), (v0 v2) = (p, M1|M2), (v0 v1) = (p, M1);
          // cofactor signs are +S(v1v2), -S(v0v2), +S(v0v1): punctured iff S(v1v2) = S(v0v1) != S(v0v2)
          const unsigned e0 = (W[m1] >> (m2 - 1)) & 1u;
          const unsigned e1 = (W[0] >> ((m1 | m2) - 1)) & 1u;
          const unsigned e2 = (W[0] >> (m1 - 1)) & 1u;
          m |= ((e0 == e2) & (e1 != e0)) << k;
        }
        unsigned valid = 0xFFFu;
        if (gx == nx - 1) valid &= ~kUseX;
        if (gy == ny - 1) valid &= ~kUseY;
        if (t == nt - 1) valid &= ~kUseT;
        m &= valid;
        masks[((long long)t * ny + gy) * nx + gx] = (uint16_t)m;
      }
      unsigned c = wave_sum(__popc(m));
      if (lane == 0 && gy < ny) seg_cnt[((long long)t * ny + gy) * gridDim.x + blockIdx.x] = (int)c;
    }
  }
  if (st) atomicOr(status, st);
}

// ---------------------------------------------------------------------------------------------------------------
// Pass 1b: emission + pass 2 links.  One wavefront per row segment (t, y, x-block); block = 256 (4 segments).
// ---------------------------------------------------------------------------------------------------------------
namespace {

// Field samples for the stencils.
struct Field2 {
  const float* f;
  int kind, nx, ny;
  long long plane;
  __device__ __forceinline__ float s(int x, int y, int t) const { return f[(long long)t * plane + (long long)y * nx + x]; }
  __device__ __forceinline__ float u(int c, int x, int y, int t) const {
    return f[((long long)t * 2 + c) * plane + (long long)y * nx + x];
  }
  // vector component c at (x, y, t): the gradient (scalar input) or the input vector
  __device__ __forceinline__ float vec(int c, int x, int y, int t) const {
    if (kind != 0) return u(c, x, y, t);
    if (c == 0) {
      float lo = x > 0 ? s(x - 1, y, t) : 0.0f, hi = x < nx - 1 ? s(x + 1, y, t) : 0.0f;
      return diff3(lo, s(x, y, t), hi, x, nx);
    }
    float lo = y > 0 ? s(x, y - 1, t) : 0.0f, hi = y < ny - 1 ? s(x, y + 1, t) : 0.0f;
    return diff3(lo, s(x, y, t), hi, y, ny);
  }
  // Jacobian J[a][b] = d v_a / d x_b (the same stencil applied to the binary32 components); J as [J00 J01 J10 J11]
  __device__ __forceinline__ void jac(int x, int y, int t, float J[4]) const {
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      float c = vec(a, x, y, t);
      float lo = x > 0 ? vec(a, x - 1, y, t) : 0.0f, hi = x < nx - 1 ? vec(a, x + 1, y, t) : 0.0f;
      J[a * 2 + 0] = diff3(lo, c, hi, x, nx);
      lo = y > 0 ? vec(a, x, y - 1, t) : 0.0f;
      hi = y < ny - 1 ? vec(a, x, y + 1, t) : 0.0f;
      J[a * 2 + 1] = diff3(lo, c, hi, y, ny);
    }
  }
};

// Exact 2x2 determinant of integer columns (a, b); 128-bit for the wide path.
template <bool WIDE>
__device__ __forceinline__ i128 det2x(long long a0, long long a1, long long b0, long long b1) {
  if (!WIDE) return (i128)(a0 * b1 - a1 * b0);  // |q| < 2^31: both products and the difference fit in 64 bits
  return (i128)a0 * b1 - (i128)a1 * b0;
}

struct Nb {
  unsigned m;    // puncture mask of the vertex
  unsigned off;  // hit index of its first hit
};

}  // namespace

template <bool WIDE>
__global__ __launch_bounds__(256) void emit2d(Grid2 g, const uint16_t* __restrict__ masks,
                                              const long long* __restrict__ seg_off, long long nseg, Out2 o,
                                              unsigned* __restrict__ status, unsigned long long* __restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  const long long seg = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (seg >= nseg) return;
  const int nxt = g.nxt, nx = g.nx, ny = g.ny, nt = g.nt;
  const long long row = seg / nxt;
  const int xb = (int)(seg - row * nxt);
  const int t = (int)(row / ny), y = (int)(row - (long long)t * ny);
  const int x = xb * TX + lane;
  const bool in = x < nx;
  const long long plane = (long long)nx * ny;
  const long long gidx = (long long)t * plane + (long long)y * nx + x;

  const unsigned m = in ? masks[gidx] : 0u;
  if (__ballot(m != 0) == 0) return;

  // own offsets
  const unsigned cnt_self = __popc(m);
  const unsigned incl = wave_incl_scan(cnt_self);
  const unsigned base_seg = (unsigned)seg_off[seg];
  Nb self{m, base_seg + incl - cnt_self};
  const unsigned seg_total = __shfl(incl, 63, 64);

  // neighbours along x: lanes of this segment, or the adjacent segments' edge vertices
  Nb mx{0, 0}, px{0, 0};
  {
    unsigned lm = __shfl_up(m, 1, 64), lo = __shfl_up(self.off, 1, 64);
    unsigned rm = __shfl_down(m, 1, 64), ro = __shfl_down(self.off, 1, 64);
    if (lane > 0) {
      mx = Nb{lm, lo};
    } else if (x > 0) {
      unsigned pm = masks[gidx - 1];
      mx = Nb{pm, base_seg - __popc(pm)};
    }
    if (lane < 63 && x + 1 < nx) {
      px = Nb{rm, ro};
    } else if (lane == 63 && x + 1 < nx) {
      px = Nb{masks[gidx + 1], base_seg + seg_total};
    }
  }
  // neighbours along y and t: whole neighbouring segments, same lanes
  auto seg_nb = [&](long long dseg, long long dg, bool ok) -> Nb {
    unsigned mm = 0;
    bool valid = ok && in;
    if (valid) mm = masks[gidx + dg];
    unsigned inc = wave_incl_scan(mm ? __popc(mm) : 0u);
    unsigned b = ok ? (unsigned)seg_off[seg + dseg] : 0u;
    return Nb{mm, b + inc - __popc(mm)};
  };
  const long long segs_per_row = nxt;
  Nb my = seg_nb(-segs_per_row, -(long long)nx, y > 0);
  Nb py = seg_nb(segs_per_row, (long long)nx, y + 1 < ny);
  Nb mt = seg_nb(-segs_per_row * ny, -plane, t > 0);
  Nb pt = seg_nb(segs_per_row * ny, plane, t + 1 < nt);

  // neighbour selector: u = p + delta for a single-axis delta (axis bit ab, sign)
  auto nb_plus = [&](int ab) -> Nb { return ab == 1 ? px : (ab == 2 ? py : pt); };
  auto nb_minus = [&](int ab) -> Nb { return ab == 1 ? mx : (ab == 2 ? my : mt); };
  auto hit_index = [&](const Nb& u, int ty) -> unsigned { return u.off + __popc(u.m & ((1u << ty) - 1u)); };
  auto is_hit = [&](const Nb& u, int ty) -> bool { return (u.m >> ty) & 1u; };

  Field2 F{g.f, g.kind, nx, ny, plane};
  unsigned st = 0;
  unsigned long long n_fp64 = 0, n_deg = 0, n_linked = 0;

  unsigned rem = m;
  unsigned k = 0;
  while (rem) {
    const int ty = __ffs(rem) - 1;
    rem &= rem - 1;
    const unsigned idx = self.off + k;
    ++k;
    const int m1 = kTri2.m[ty][0], m2 = kTri2.m[ty][1];
    // vertices in chain order
    int vx[3], vy[3], vt[3];
    vx[0] = x;
    vy[0] = y;
    vt[0] = t;
    vx[1] = x + (m1 & 1);
    vy[1] = y + ((m1 >> 1) & 1);
    vt[1] = t + ((m1 >> 2) & 1);
    vx[2] = vx[1] + (m2 & 1);
    vy[2] = vy[1] + ((m2 >> 1) & 1);
    vt[2] = vt[1] + ((m2 >> 2) & 1);

    // quantised vectors (same stencil and rounding as pass 1)
    long long q[3][2];
    bool wide = false;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        float r = quant(F.vec(c, vx[i], vy[i], vt[i]), g.qscale);
        q[i][c] = (long long)r;
        if (!(fabsf(r) < 2147483648.0f)) wide = true;
      }
    }
    // exact cofactors of (v0 v1 v2 ; 1 1 1): C_i = (-1)^i det(columns without i)
    i128 C[3];
    C[0] = det2x<WIDE>(q[1][0], q[1][1], q[2][0], q[2][1]);
    C[1] = -det2x<WIDE>(q[0][0], q[0][1], q[2][0], q[2][1]);
    C[2] = det2x<WIDE>(q[0][0], q[0][1], q[1][0], q[1][1]);
    const i128 D = C[0] + C[1] + C[2];
    unsigned fl = wide ? FL_WIDE : 0u;

    float J[3][4];
#pragma unroll
    for (int i = 0; i < 3; ++i) F.jac(vx[i], vy[i], vt[i], J[i]);

    float mu32[3];
    double mu64[3];
    const bool degenerate = (D == 0);
    if (degenerate) {
      fl |= FL_DEGENERATE;
      ++n_deg;
    }
    int type = -1;
    if (g.precision == 0) {
      if (degenerate) {
        mu32[0] = mu32[1] = mu32[2] = 1.0f / 3.0f;
      } else {
        float fD = (float)D;
#pragma unroll
        for (int i = 0; i < 3; ++i) mu32[i] = (float)C[i] / fD;
      }
      type = classify2_fp32(mu32, J, g.kind != 0);
    }
    if (g.precision != 0 || type < 0) {
      if (degenerate) {
        mu64[0] = mu64[1] = mu64[2] = 1.0 / 3.0;
      } else {
        double dD = (double)D;
#pragma unroll
        for (int i = 0; i < 3; ++i) mu64[i] = (double)C[i] / dD;
      }
      type = classify2_fp64(mu64, J, g.kind != 0);
      if (g.precision == 0) {
        fl |= FL_FP64;
        ++n_fp64;
      }
    }
    // sublocation: x = sum mu_i p_i, in the requested precision
    float pos[3], muo[3];
    if (g.precision == 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int* vc = c == 0 ? vx : (c == 1 ? vy : vt);
        float s = mu32[0] * (float)vc[0];
        s = s + mu32[1] * (float)vc[1];
        s = s + mu32[2] * (float)vc[2];
        pos[c] = s;
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) muo[i] = mu32[i];
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int* vc = c == 0 ? vx : (c == 1 ? vy : vt);
        double s = mu64[0] * (double)vc[0];
        s = s + mu64[1] * (double)vc[1];
        s = s + mu64[2] * (double)vc[2];
        pos[c] = (float)s;
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) muo[i] = (float)mu64[i];
    }

    o.face_id[idx] = gidx * 12 + ty;
    if (o.pos) {
      o.pos[(size_t)idx * 3 + 0] = pos[0];
      o.pos[(size_t)idx * 3 + 1] = pos[1];
      o.pos[(size_t)idx * 3 + 2] = pos[2];
    }
    if (o.mu) {
      o.mu[(size_t)idx * 3 + 0] = muo[0];
      o.mu[(size_t)idx * 3 + 1] = muo[1];
      o.mu[(size_t)idx * 3 + 2] = muo[2];
    }
    if (o.type) o.type[idx] = (uint8_t)type;
    if (o.flags) o.flags[idx] = (uint8_t)fl;

    // ---- pass 2 links: the (at most two) tetrahedra containing this triangle.  A tetrahedron with chain
    // (c1, c2, c3) anchored at c has sides: drop w0 -> (c + e_c1; c2, c3), drop w1 -> (c; c1|c2, c3),
    // drop w2 -> (c; c1, c2|c3), drop w3 -> (c; c1, c2).
    unsigned partner[2];
    int np = 0;
    const int b = m1 | m2;
    auto visit_cell = [&](bool at_minus, int ma, int c1, int c2, int c3) {
      // at_minus: cell anchored at p - e_ma (then c1 == ma), else at p
      const Nb base = at_minus ? nb_minus(ma) : self;
      const Nb first = at_minus ? self : nb_plus(c1);
      int found = 0;
      unsigned other = 0xFFFFFFFFu;
      const int ts[4] = {kTri2Index.idx[c2][c3], kTri2Index.idx[c1 | c2][c3], kTri2Index.idx[c1][c2 | c3],
                         kTri2Index.idx[c1][c2]};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const Nb& u = (s == 0) ? first : base;
        if (is_hit(u, ts[s])) {
          unsigned hi = hit_index(u, ts[s]);
          ++found;
          if (hi != idx) other = hi;
        }
      }
      if (found != 2 || other == 0xFFFFFFFFu) {
        st |= ST_INVARIANT;
        return;
      }
      partner[np++] = other;
      if (other > idx) ++n_linked;
    };
    if (__popc((unsigned)m1) == 1 && __popc((unsigned)m2) == 1) {
      const int a = 7 & ~b;  // missing axis
      const int pa = a == 1 ? x : (a == 2 ? y : t);
      const int Na = a == 1 ? nx : (a == 2 ? ny : nt);
      if (pa >= 1) visit_cell(true, a, a, m1, m2);
      if (pa + 1 <= Na - 1) visit_cell(false, 0, m1, m2, a);
    } else if (__popc((unsigned)m1) == 2) {
      const int lo = m1 & -m1, hi = m1 - lo;
      visit_cell(false, 0, lo, hi, m2);
      visit_cell(false, 0, hi, lo, m2);
    } else {
      const int lo = m2 & -m2, hi = m2 - lo;
      visit_cell(false, 0, m1, lo, hi);
      visit_cell(false, 0, m1, hi, lo);
    }
    unsigned par0 = idx, smaller = 0, big_small = 0;
    for (int i = 0; i < np; ++i) {
      if (partner[i] < par0) par0 = partner[i];
      if (partner[i] < idx) {
        ++smaller;
        big_small = big_small > partner[i] ? big_small : partner[i];
      }
    }
    o.parent[idx] = par0;
    if (smaller == 2) {
      unsigned long long slot = atomicAdd(&cnt[CNT_WORK], 1ull);
      o.work[slot] = make_uint2(idx, big_small);
    }
  }
  unsigned long long s1 = wave_sum64(n_fp64), s2 = wave_sum64(n_deg), s3 = wave_sum64(n_linked);
  if (lane == 0) {
    if (s1) atomicAdd(&cnt[CNT_FP64], s1);
    if (s2) atomicAdd(&cnt[CNT_DEGEN], s2);
    if (s3) atomicAdd(&cnt[CNT_LINKED], s3);
  }
  if (st) atomicOr(status, st);
}

// ---------------------------------------------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------------------------------------------
hipError_t launch_detect2d(const Grid2& g, int ty, int tt, bool wide, uint16_t* masks, int* seg_cnt,
                           unsigned* status, hipStream_t s) {
  dim3 grid((unsigned)g.nxt, (unsigned)((g.ny + ty - 1) / ty), (unsigned)((g.nt + tt - 1) / tt));
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

hipError_t launch_emit2d(const Grid2& g, bool wide, const uint16_t* masks, const long long* seg_off, long long nseg,
                         const Out2& o, unsigned* status, unsigned long long* cnt, hipStream_t s) {
  unsigned blocks = (unsigned)((nseg + 3) / 4);
  if (wide)
    emit2d<true><<<blocks, 256, 0, s>>>(g, masks, seg_off, nseg, o, status, cnt);
  else
    emit2d<false><<<blocks, 256, 0, s>>>(g, masks, seg_off, nseg, o, status, cnt);
  return hipGetLastError();
}

}  // namespace ftk
