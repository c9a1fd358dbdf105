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
// Pass 1b: emission + pass 2 links.
// Same tiling as detection (64 x TY anchors, marching over a slab of TT steps).  The vector field of planes t and
// t+1 (gradient of the scalar, or the input vector) is kept in LDS with a 1-cell halo; quantised vectors and
// Jacobians of a hit's vertices are formed from it on the fly, with the same binary32 stencils as pass 1.  Each
// wavefront takes one row segment at a time and processes its hits hit-parallel (hit j of the segment on lane
// j mod 64), so output writes are contiguous.
// ---------------------------------------------------------------------------------------------------------------
namespace {

// Exact 2x2 determinant of integer columns (a, b); 128-bit for the wide path.
template <bool WIDE>
__device__ __forceinline__ i128 det2x(long long a0, long long a1, long long b0, long long b1) {
  if (!WIDE) return (i128)(a0 * b1 - a1 * b0);  // |q| < 2^31: both products and the difference fit in 64 bits
  return (i128)a0 * b1 - (i128)a1 * b0;
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// neighbour slots of an anchor: self, -x, +x, -y, +y, -t, +t
enum { NB_SELF = 0, NB_MX, NB_PX, NB_MY, NB_PY, NB_MT, NB_PT };

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

// Edge list staging: links that leave the tile/chunk are collected in LDS and appended to the global list in
// batches (one global atomic per batch; same-address atomics serialise at one L2 channel).
constexpr int kEdgeStage = 768;

// Wave-aggregated append of (idx, partner) for the active lanes with want == true: into the LDS stage if it has
// room, otherwise straight to the global list.
__device__ __forceinline__ void append_edge(bool want, unsigned idx, unsigned partner, uint2* stage, int* stage_n,
                                            uint2* work, unsigned long long* counter) {
  const unsigned long long bal = __ballot(want);
  if (bal == 0) return;
  const int lane = lane_id();
  const int leader = __ffsll((long long)bal) - 1;
  const int k = __popcll(bal);
  int pos = -1;
  unsigned long long gpos = 0;
  if (lane == leader) {
    int old = *(volatile int*)stage_n;
    while (old + k <= kEdgeStage) {
      int prev = atomicCAS(stage_n, old, old + k);
      if (prev == old) {
        pos = old;
        break;
      }
      old = prev;
    }
    if (pos < 0) gpos = atomicAdd(counter, (unsigned long long)k);
  }
  pos = __shfl(pos, leader, 64);
  gpos = __shfl(gpos, leader, 64);
  if (want) {
    const int rank = __popcll(bal & ((1ull << lane) - 1ull));
    const uint2 e = make_uint2(idx, partner);
    if (pos >= 0)
      stage[pos + rank] = e;
    else
      work[gpos + rank] = e;
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

template <int TY, bool WIDE>
__global__ __launch_bounds__(256) void emit2d(Grid2 g, int TT, const uint16_t* __restrict__ masks,
                                              const long long* __restrict__ seg_off, Out2 o,
                                              unsigned* __restrict__ status, unsigned long long* __restrict__ cnt) {
  constexpr int GW = TX + 3, GH = TY + 3;  // vector field: x0-1 .. x0+TX+1, y0-1 .. y0+TY+1
  constexpr int FW = TX + 5, FH = TY + 5;  // scalar field: x0-2 .. x0+TX+2
  constexpr int CAP = 2048;                // local union-find capacity (hits)
  constexpr int MAXTT = 32;
  __shared__ float fs[FH * FW];
  __shared__ float2 gs[2][GH * GW];
  __shared__ unsigned short s_ex[TY][64];
  __shared__ unsigned short s_m[TY][64];
  __shared__ unsigned s_rowtot[TY], s_rowbase[TY];
  __shared__ unsigned short nbm[4][7][64];
  __shared__ unsigned nbo[4][7][64];
  __shared__ unsigned lpar[CAP];
  __shared__ unsigned lglob[CAP];
  __shared__ unsigned lbase[MAXTT][TY];  // local id of the first hit of (chunk step, row)
  __shared__ unsigned segb[MAXTT][TY];   // global hit index of the first hit of (chunk step, row)
  __shared__ int s_chunk_t0, s_chunk_n, s_flush, s_global, s_plane_lbase, s_plane_total;
  __shared__ uint2 s_stage[kEdgeStage];
  __shared__ int s_stage_n;
  __shared__ unsigned long long s_stage_base;
  __shared__ unsigned long long s_red[4];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  const int t0 = blockIdx.z * TT;
  const int t1 = min(t0 + TT, g.nt);
  const int nx = g.nx, ny = g.ny, nt = g.nt, nxt = g.nxt;
  const long long plane = (long long)nx * ny;
  const bool vector = g.kind != 0;
  unsigned st = 0;
  unsigned long long n_fp64 = 0, n_deg = 0, n_linked = 0;

  // vector field of plane t into gs[par]
  auto load_plane = [&](int t, int par) {
    if (!vector) {
      const float* src = g.f + (long long)t * plane;
      for (int e = tid; e < FH * FW; e += 256) {
        int ly = e / FW, lx = e - ly * FW;
        int gx = x0 - 2 + lx, gy = y0 - 2 + ly;
        fs[e] = (gx >= 0 && gx < nx && gy >= 0 && gy < ny) ? src[(long long)gy * nx + gx] : 0.0f;
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
      const float* su = g.f + (long long)t * 2 * plane;
      const float* sv = su + plane;
      for (int e = tid; e < GH * GW; e += 256) {
        int ly = e / GW, lx = e - ly * GW;
        int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
        float2 v = make_float2(0.0f, 0.0f);
        if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
          long long k = (long long)gy * nx + gx;
          v = make_float2(su[k], sv[k]);
        }
        gs[par][e] = v;
      }
    }
  };

  // write the parent of every hit of the chunk: the hit index of its local root
  auto flush = [&]() {
    const int n = s_chunk_n;
    for (int li = tid; li < n; li += 256) {
      unsigned r = lfind(lpar, (unsigned)li);
      o.parent[lglob[li]] = lglob[r];
    }
  };

  // move the staged edges to the global list
  auto drain = [&]() {
    if (tid == 0) s_stage_base = s_stage_n ? atomicAdd(&cnt[CNT_WORK], (unsigned long long)s_stage_n) : 0ull;
    __syncthreads();
    const int n = s_stage_n;
    for (int i = tid; i < n; i += 256) o.work[s_stage_base + i] = s_stage[i];
    __syncthreads();
    if (tid == 0) s_stage_n = 0;
  };

  if (tid == 0) {
    s_chunk_t0 = t0;
    s_chunk_n = 0;
    s_stage_n = 0;
  }
  load_plane(t0, t0 & 1);
  for (int t = t0; t < t1; ++t) {
    const int par = t & 1;
    __syncthreads();
    if (s_stage_n > kEdgeStage / 2) drain();
    if (t + 1 < nt) load_plane(t + 1, par ^ 1);

    // row masks, prefixes and totals of this step
    for (int ly = wave; ly < TY; ly += 4) {
      const int y = y0 + ly, x = x0 + lane;
      unsigned m = 0;
      if (y < ny && x < nx) m = masks[(long long)t * plane + (long long)y * nx + x];
      const unsigned c = __popc(m);
      const unsigned incl = wave_incl_scan(c);
      s_m[ly][lane] = (unsigned short)m;
      s_ex[ly][lane] = (unsigned short)(incl - c);
      if (lane == 63) {
        s_rowtot[ly] = incl;
        s_rowbase[ly] = y < ny ? (unsigned)seg_off[((long long)t * ny + y) * nxt + blockIdx.x] : 0u;
      }
    }
    __syncthreads();
    if (tid == 0) {
      unsigned tot = 0;
      for (int r = 0; r < TY; ++r) tot += s_rowtot[r];
      s_plane_total = (int)tot;
      s_flush = (s_chunk_n > 0 && (s_chunk_n + (int)tot > CAP || t - s_chunk_t0 >= MAXTT)) ? 1 : 0;
    }
    __syncthreads();
    if (s_flush) {
      flush();
      __syncthreads();
      if (tid == 0) {
        s_chunk_n = 0;
        s_chunk_t0 = t;
      }
      __syncthreads();
    }
    if (tid == 0) {
      const int tot = s_plane_total;
      if (tot > CAP) {  // too many hits for the local structure: this step links through the global list only
        s_global = 1;
        s_chunk_t0 = t + 1;
        s_chunk_n = 0;
      } else {
        s_global = 0;
        if (s_chunk_n == 0) s_chunk_t0 = t;
        s_plane_lbase = s_chunk_n;
        unsigned run = (unsigned)s_chunk_n;
        for (int r = 0; r < TY; ++r) {
          lbase[t - s_chunk_t0][r] = run;
          segb[t - s_chunk_t0][r] = s_rowbase[r];
          run += s_rowtot[r];
        }
        s_chunk_n = (int)run;
      }
    }
    __syncthreads();
    const bool plane_global = s_global != 0;
    const int chunk_t0 = s_chunk_t0;
    if (!plane_global)
      for (int i = tid; i < s_plane_total; i += 256) lpar[s_plane_lbase + i] = (unsigned)(s_plane_lbase + i);
    __syncthreads();

    for (int ly = wave; ly < TY; ly += 4) {
      const int y = y0 + ly;
      if (y >= ny) break;
      const unsigned total = s_rowtot[ly];
      if (total == 0) continue;
      const int x = x0 + lane;
      const bool in = x < nx;
      const long long seg = ((long long)t * ny + y) * nxt + blockIdx.x;
      const long long gidx = (long long)t * plane + (long long)y * nx + x;
      const unsigned m = s_m[ly][lane];
      const unsigned ex = s_ex[ly][lane];
      const unsigned base = s_rowbase[ly];
      const unsigned row_lbase = plane_global ? 0u : lbase[t - chunk_t0][ly];

      // neighbour masks and first-hit indices (wavefront-private LDS slots)
      {
        unsigned mxm = 0, mxo = 0, pxm = 0, pxo = 0;
        if (lane > 0) {
          mxm = s_m[ly][lane - 1];
          mxo = base + s_ex[ly][lane - 1];
        } else if (x > 0) {
          mxm = masks[gidx - 1];
          mxo = base - __popc(mxm);
        }
        if (x + 1 < nx) {
          if (lane < 63) {
            pxm = s_m[ly][lane + 1];
            pxo = base + s_ex[ly][lane + 1];
          } else {
            pxm = masks[gidx + 1];
            pxo = base + total;
          }
        }
        nbm[wave][NB_SELF][lane] = (unsigned short)m;
        nbo[wave][NB_SELF][lane] = base + ex;
        nbm[wave][NB_MX][lane] = (unsigned short)mxm;
        nbo[wave][NB_MX][lane] = mxo;
        nbm[wave][NB_PX][lane] = (unsigned short)pxm;
        nbo[wave][NB_PX][lane] = pxo;
        auto seg_nb = [&](int slot, long long dseg, long long dg, bool ok) {
          unsigned mm = (ok && in) ? masks[gidx + dg] : 0u;
          unsigned inc = wave_incl_scan(__popc(mm));
          unsigned b = ok ? (unsigned)seg_off[seg + dseg] : 0u;
          nbm[wave][slot][lane] = (unsigned short)mm;
          nbo[wave][slot][lane] = b + inc - __popc(mm);
        };
        seg_nb(NB_MY, -(long long)nxt, -(long long)nx, y > 0);
        seg_nb(NB_PY, (long long)nxt, (long long)nx, y + 1 < ny);
        seg_nb(NB_MT, -(long long)nxt * ny, -plane, t > 0);
        seg_nb(NB_PT, (long long)nxt * ny, plane, t + 1 < nt);
      }
      wave_lds_sync();

      for (unsigned j = lane; j < total; j += 64) {
        // anchor lane: the largest L with ex[L] <= j
        int L = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1)
          if (s_ex[ly][L + step] <= j) L += step;
        unsigned mm = s_m[ly][L];
        for (unsigned k = j - s_ex[ly][L]; k > 0; --k) mm &= mm - 1;
        const int ty = __ffs(mm) - 1;
        const unsigned idx = base + j;
        const int ax = x0 + L;
        const int m1 = kTri2.m[ty][0], m2 = kTri2.m[ty][1];

        // vertices (local coordinates in the LDS tile, plane offset 0/1)
        int lx[3], lyv[3], dt[3];
        lx[0] = L;
        lyv[0] = ly;
        dt[0] = 0;
        lx[1] = L + (m1 & 1);
        lyv[1] = ly + ((m1 >> 1) & 1);
        dt[1] = (m1 >> 2) & 1;
        lx[2] = lx[1] + (m2 & 1);
        lyv[2] = lyv[1] + ((m2 >> 1) & 1);
        dt[2] = dt[1] + ((m2 >> 2) & 1);

        long long q[3][2];
        float J[3][4];
        bool wide = false;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const float2* G = gs[par ^ dt[i]];
          const int c = (lyv[i] + 1) * GW + (lx[i] + 1);
          const float2 v = G[c];
          const float r0 = quant(v.x, g.qscale), r1 = quant(v.y, g.qscale);
          if (!(fabsf(r0) < 2147483648.0f) || !(fabsf(r1) < 2147483648.0f)) wide = true;
          q[i][0] = (long long)r0;
          q[i][1] = (long long)r1;
          const int gxv = x0 + lx[i], gyv = y0 + lyv[i];
          const float2 xl = G[c - 1], xh = G[c + 1], yl = G[c - GW], yh = G[c + GW];
          J[i][0] = diff3(xl.x, v.x, xh.x, gxv, nx);
          J[i][1] = diff3(yl.x, v.x, yh.x, gyv, ny);
          J[i][2] = diff3(xl.y, v.y, xh.y, gxv, nx);
          J[i][3] = diff3(yl.y, v.y, yh.y, gyv, ny);
        }
        // exact cofactors of (v0 v1 v2 ; 1 1 1): C_i = (-1)^i det(columns without i)
        i128 C[3];
        C[0] = det2x<WIDE>(q[1][0], q[1][1], q[2][0], q[2][1]);
        C[1] = -det2x<WIDE>(q[0][0], q[0][1], q[2][0], q[2][1]);
        C[2] = det2x<WIDE>(q[0][0], q[0][1], q[1][0], q[1][1]);
        const i128 D = C[0] + C[1] + C[2];
        unsigned fl = wide ? FL_WIDE : 0u;
        const bool degenerate = (D == 0);
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
            const float fD = (float)D;
#pragma unroll
            for (int i = 0; i < 3; ++i) mu32[i] = (float)C[i] / fD;
          }
          type = classify2_fp32(mu32, J, vector);
        }
        if (g.precision != 0 || type < 0) {
          if (degenerate) {
            mu64[0] = mu64[1] = mu64[2] = 1.0 / 3.0;
          } else {
            const double dD = (double)D;
#pragma unroll
            for (int i = 0; i < 3; ++i) mu64[i] = (double)C[i] / dD;
          }
          type = classify2_fp64(mu64, J, vector);
          if (g.precision == 0) {
            fl |= FL_FP64;
            ++n_fp64;
          }
        }
        float pos[3], muo[3];
        // vertex coordinates per component: x, y, t of v0, v1, v2
        const int cx0 = ax, cx1 = ax + (m1 & 1), cx2 = cx1 + (m2 & 1);
        const int cy0 = y, cy1 = y + ((m1 >> 1) & 1), cy2 = cy1 + ((m2 >> 1) & 1);
        const int ct0 = t, ct1 = t + dt[1], ct2 = t + dt[2];
        if (g.precision == 0) {
          float sx = mu32[0] * (float)cx0;
          sx = sx + mu32[1] * (float)cx1;
          sx = sx + mu32[2] * (float)cx2;
          float sy = mu32[0] * (float)cy0;
          sy = sy + mu32[1] * (float)cy1;
          sy = sy + mu32[2] * (float)cy2;
          float stt = mu32[0] * (float)ct0;
          stt = stt + mu32[1] * (float)ct1;
          stt = stt + mu32[2] * (float)ct2;
          pos[0] = sx;
          pos[1] = sy;
          pos[2] = stt;
#pragma unroll
          for (int i = 0; i < 3; ++i) muo[i] = mu32[i];
        } else {
          double sx = mu64[0] * (double)cx0;
          sx = sx + mu64[1] * (double)cx1;
          sx = sx + mu64[2] * (double)cx2;
          double sy = mu64[0] * (double)cy0;
          sy = sy + mu64[1] * (double)cy1;
          sy = sy + mu64[2] * (double)cy2;
          double stt = mu64[0] * (double)ct0;
          stt = stt + mu64[1] * (double)ct1;
          stt = stt + mu64[2] * (double)ct2;
          pos[0] = (float)sx;
          pos[1] = (float)sy;
          pos[2] = (float)stt;
#pragma unroll
          for (int i = 0; i < 3; ++i) muo[i] = (float)mu64[i];
        }
        const long long agid = (long long)t * plane + (long long)y * nx + ax;
        o.face_id[idx] = agid * 12 + ty;
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

        // ---- pass 2 links: the (at most two) tetrahedra holding this triangle.  A tetrahedron with chain
        // (c1, c2, c3) anchored at c has sides: drop w0 -> (c + e_c1; c2, c3), drop w1 -> (c; c1|c2, c3),
        // drop w2 -> (c; c1, c2|c3), drop w3 -> (c; c1, c2).  Each link is recorded by its larger endpoint:
        // inside this tile and chunk it goes to the LDS union-find, otherwise to the global edge list.
        unsigned sm0 = 0, sm1 = 0;
        int sl0 = -1, sl1 = -1;
        int ns = 0;
        auto visit_cell = [&](bool at_minus, int c1, int c2, int c3) {
          const int bslot = at_minus ? (c1 == 1 ? NB_MX : (c1 == 2 ? NB_MY : NB_MT)) : NB_SELF;
          const int fslot = at_minus ? NB_SELF : (c1 == 1 ? NB_PX : (c1 == 2 ? NB_PY : NB_PT));
          const int bm = nbm[wave][bslot][L], fm = nbm[wave][fslot][L];
          const unsigned bo = nbo[wave][bslot][L], fo = nbo[wave][fslot][L];
          int found = 0, oslot = -1;
          unsigned other = 0xFFFFFFFFu;
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int tsv = s == 0 ? kTri2Index.idx[c2][c3]
                                   : (s == 1 ? kTri2Index.idx[c1 | c2][c3]
                                             : (s == 2 ? kTri2Index.idx[c1][c2 | c3] : kTri2Index.idx[c1][c2]));
            const int um = s == 0 ? fm : bm;
            const unsigned uo = s == 0 ? fo : bo;
            if ((um >> tsv) & 1) {
              const unsigned hi = uo + __popc((unsigned)um & ((1u << tsv) - 1u));
              ++found;
              if (hi != idx) {
                other = hi;
                oslot = s == 0 ? fslot : bslot;
              }
            }
          }
          if (found != 2 || other == 0xFFFFFFFFu) {
            st |= ST_INVARIANT;
            return;
          }
          if (other < idx) {
            if (ns == 0) {
              sm0 = other;
              sl0 = oslot;
            } else {
              sm1 = other;
              sl1 = oslot;
            }
            ++ns;
          }
        };
        const int b = m1 | m2;
        if (__popc((unsigned)m1) == 1 && __popc((unsigned)m2) == 1) {
          const int a = 7 & ~b;  // missing axis
          const int pa = a == 1 ? ax : (a == 2 ? y : t);
          const int Na = a == 1 ? nx : (a == 2 ? ny : nt);
          if (pa >= 1) visit_cell(true, a, m1, m2);
          if (pa + 1 <= Na - 1) visit_cell(false, m1, m2, a);
        } else if (__popc((unsigned)m1) == 2) {
          const int lo = m1 & -m1, hi = m1 - lo;
          visit_cell(false, lo, hi, m2);
          visit_cell(false, hi, lo, m2);
        } else {
          const int lo = m2 & -m2, hi = m2 - lo;
          visit_cell(false, m1, lo, hi);
          visit_cell(false, m1, hi, lo);
        }
        n_linked += ns;
        bool g0 = false, g1 = false;
        if (plane_global) {
          o.parent[idx] = idx;
          g0 = ns > 0;
          g1 = ns > 1;
        } else {
          const unsigned li = row_lbase + j;
          lglob[li] = idx;
          // smaller partners are anchored at p (same row), p - x, p - y or p - t; the link stays local when that
          // anchor lies in this tile and this chunk
          auto link = [&](unsigned other, int sl) -> bool {
            int prow = ly, pstep = t - chunk_t0;
            bool local = true;
            if (sl == NB_MX) {
              local = L > 0;
            } else if (sl == NB_MY) {
              local = ly > 0;
              prow = ly - 1;
            } else if (sl == NB_MT) {
              local = t - 1 >= chunk_t0;
              pstep = t - 1 - chunk_t0;
            }
            if (!local) return true;
            lunite(lpar, li, lbase[pstep][prow] + (other - segb[pstep][prow]));
            return false;
          };
          if (ns > 0) g0 = link(sm0, sl0);
          if (ns > 1) g1 = link(sm1, sl1);
        }
        append_edge(g0, idx, sm0, s_stage, &s_stage_n, o.work, &cnt[CNT_WORK]);
        append_edge(g1, idx, sm1, s_stage, &s_stage_n, o.work, &cnt[CNT_WORK]);
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
  (void)nseg;
  constexpr int TYE = 8, TTE = 16;
  dim3 grid((unsigned)g.nxt, (unsigned)((g.ny + TYE - 1) / TYE), (unsigned)((g.nt + TTE - 1) / TTE));
  if (wide)
    emit2d<TYE, true><<<grid, 256, 0, s>>>(g, TTE, masks, seg_off, o, status, cnt);
  else
    emit2d<TYE, false><<<grid, 256, 0, s>>>(g, TTE, masks, seg_off, o, status, cnt);
  return hipGetLastError();
}

}  // namespace ftk
