// iso.hip -- isovolume tracking in 3D space + time (Sec. 6.1, two passes on the regular simplicial spacetime mesh;
// Alg. 1 right column).
//
// Mesh (Sec. 3.3): an edge anchored at vertex p with axis mask M (1..15; x = 1, y = 2, z = 4, t = 8) joins p and
// p + e(M); its id is g(p) * 15 + (M - 1) with the t-major vertex index g.  A pentachoron anchored at p with axis
// order (s1, s2, s3, s4) has the chain vertices p, p + e(s1), p + e(s1|s2), p + e(s1|s2|s3), p + e(1111).
//
//   iso_bits  -- the side of the level set of every vertex as one bit, 64 per word (a value equal to the isovalue
//                lies above it: the symbolic perturbation of a single entry is positive, Sec. 6.2).
//   iso_count -- one lane per vertex: the sides at the 16 corners of its unit 4-cube (from the bit words),
//                the crossing mask of its 15 edges, and the tetrahedra of its 24 pentachora (case I: one vertex on
//                its side, 1 tetrahedron; case II: two, 3 tetrahedra).
//   iso_emit  -- edge ids and intersection points p + mu e(M), mu = (c - f(p)) / (f(q) - f(p)), from the scanned
//                counts; union-find parents start as the identity.
//   iso_unite -- per 4-cube with crossings (compacted list): unite its crossed edges group by group (CAS hooking,
//                larger root under the smaller), and per pentachoron write its tetrahedra (indices of crossed
//                edges): case I the four edges of the lone vertex in chain order; case II the prism pair x triple
//                split along the three monotone paths (staircase), which matches on the quadrilateral shared with
//                the neighbouring pentachoron.
// Labels (smallest edge id of each isovolume) come from the shared union-find label kernel.
#include <utility>

#include "common.h"
#include "offsets16.h"
#include "internal.h"
#include "kuhn.h"
#include "uf_cached.h"

namespace ftk {

namespace {

constexpr int kIsoBX = 128;  // lanes per block along x

// chain corners of the 24 pentachoron types: corner k = s1 | ... | sk
struct PenCorners {
  unsigned char c[24][5];
};
constexpr PenCorners build_pen_corners() {
  PenCorners r{};
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

// The edges of a 4-cube's pentachora are its 65 corner pairs a < a | M (a & M == 0, M != 0).  idx[a][M] is the local
// index (255 for no edge), ea / eM its anchor corner and mask, side[pt] the 65-bit set (two words) of the 10 edges of
// pentachoron type pt.
constexpr int kCubeEdgeN = 65;
struct CubeEdges {
  unsigned char idx[16][16];
  unsigned char ea[kCubeEdgeN], eM[kCubeEdgeN];
  unsigned long long side[24][2];
};
constexpr CubeEdges build_cube_edges() {
  CubeEdges r{};
  int k = 0;
  for (int a = 0; a < 16; ++a)
    for (int M = 0; M < 16; ++M) r.idx[a][M] = 255;
  for (int a = 0; a < 16; ++a)
    for (int M = 1; M < 16; ++M)
      if (!(a & M) && k < kCubeEdgeN) {
        r.idx[a][M] = (unsigned char)k;
        r.ea[k] = (unsigned char)a;
        r.eM[k] = (unsigned char)M;
        ++k;
      }
  for (int pt = 0; pt < 24; ++pt) {
    int c[5] = {0, 0, 0, 0, 0};
    for (int i = 0; i < 4; ++i) c[i + 1] = c[i] | kPen3.m[pt][i];
    for (int i = 0; i < 5; ++i)
      for (int j = i + 1; j < 5; ++j) {
        const int l = r.idx[c[i]][c[j] ^ c[i]];
        r.side[pt][l >> 6] |= 1ull << (l & 63);
      }
  }
  return r;
}
constexpr int count_cube_edges() {
  int k = 0;
  for (int a = 0; a < 16; ++a)
    for (int M = 1; M < 16; ++M) k += !(a & M);
  return k;
}
static_assert(count_cube_edges() == kCubeEdgeN, "65 corner pairs (edges) per 4-cube");
__constant__ CubeEdges kCubeEdges = build_cube_edges();

typedef unsigned __int128 u128;

__device__ __forceinline__ u128 edge_side_set(int pt) {
  return ((u128)kCubeEdges.side[pt][1] << 64) | (u128)kCubeEdges.side[pt][0];
}

__device__ __forceinline__ int low_bit128(u128 m) {
  const unsigned long long lo = (unsigned long long)m;
  return lo ? __ffsll((long long)lo) - 1 : 64 + __ffsll((long long)(unsigned long long)(m >> 64)) - 1;
}

struct IsoGrid {
  const float* f;
  int nx, ny, nz, nt;
  float c;
  const unsigned long long* bits;  // side of every vertex, one bit per vertex: row-major 64-vertex words
  int nwx;                         // words per row, ceil(nx / 64)
};

__device__ __forceinline__ long long vidx(const IsoGrid& g, int x, int y, int z, int t) {
  return (((long long)t * g.nz + z) * g.ny + y) * g.nx + x;
}

// Side of every vertex as one bit (a value equal to the isovalue counts as above), packed per 64 vertices of a row
// by a wave ballot: the passes that need the 16 corners of a 4-cube read these words (L2-resident, shared by
// neighbouring lanes) instead of 16 field values.  Non-finite values are reported here.
// Word k of the packed sides covers vertices 64 (k mod nwx) .. + 63 of grid row k / nwx (rows in (t, z, y) order).
// A wavefront packs kBitsWords consecutive words, their loads in flight together.
constexpr int kBitsWords = 4;
__global__ __launch_bounds__(256) void iso_bits(IsoGrid g, long long n_words, unsigned long long* __restrict__ bits,
                                                unsigned* __restrict__ status) {
  const int lane = threadIdx.x & 63;
  const long long k0 = ((long long)blockIdx.x * 4 + (threadIdx.x >> 6)) * kBitsWords;
  float v[kBitsWords];
  bool in[kBitsWords];
#pragma unroll
  for (int j = 0; j < kBitsWords; ++j) {
    const long long k = min(k0 + j, n_words - 1);
    const long long row = k / g.nwx;
    const int x = (int)(k - row * g.nwx) * 64 + lane;
    in[j] = k0 + j < n_words && x < g.nx;
    v[j] = g.f[row * g.nx + min(x, g.nx - 1)];
  }
  unsigned bad = 0;
#pragma unroll
  for (int j = 0; j < kBitsWords; ++j) {
    if (in[j] && !isfinite(v[j])) bad = ST_NONFINITE;
    const unsigned long long w = __ballot(in[j] && v[j] >= g.c);
    if (lane == 0 && k0 + j < n_words) bits[k0 + j] = w;
  }
  if (bad) atomicOr(status, bad);
}

// above bits of the 16 cube corners (bit cm) and their validity (bit cm: corner in the grid)
__device__ __forceinline__ void corner_bits(const IsoGrid& g, int x, int y, int z, int t, unsigned& above,
                                            unsigned& valid) {
  above = 0;
  valid = 0;
  unsigned long long w[16];
#pragma unroll
  for (int cm = 0; cm < 16; ++cm) {  // clamped (in-grid) word addresses: the 16 loads are independent
    const int cx = min(x + (cm & 1), g.nx - 1), cy = min(y + ((cm >> 1) & 1), g.ny - 1);
    const int cz = min(z + ((cm >> 2) & 1), g.nz - 1), ct = min(t + ((cm >> 3) & 1), g.nt - 1);
    w[cm] = g.bits[(((long long)ct * g.nz + cz) * g.ny + cy) * g.nwx + (cx >> 6)];
  }
#pragma unroll
  for (int cm = 0; cm < 16; ++cm) {
    const int cx = x + (cm & 1), cy = y + ((cm >> 1) & 1), cz = z + ((cm >> 2) & 1), ct = t + ((cm >> 3) & 1);
    if (cx < g.nx && cy < g.ny && cz < g.nz && ct < g.nt) {
      valid |= 1u << cm;
      above |= (unsigned)((w[cm] >> (cx & 63)) & 1ull) << cm;
    }
  }
}

// Tetrahedra of the isovolume in the pentachoron of type TY (Sec. 6.1): with k of its five chain vertices above the
// level, 1 for case I (k = 1 or 4), 3 for case II (k = 2 or 3), 0 otherwise; the chain corners are a compile-time
// mask, and the count per k is a nibble of 0x13310.
template <int TY>
__device__ __forceinline__ int pen_tets(unsigned above) {
  constexpr PenCorners kP = build_pen_corners();
  constexpr unsigned chain = 1u << kP.c[TY][0] | 1u << kP.c[TY][1] | 1u << kP.c[TY][2] | 1u << kP.c[TY][3] |
                             1u << kP.c[TY][4];
  return (int)((0x13310u >> (4u * (unsigned)__popc(above & chain))) & 15u);
}

template <int... TY>
__device__ __forceinline__ int pen_tets_all(std::integer_sequence<int, TY...>, unsigned above) {
  return (pen_tets<TY>(above) + ...);
}

__global__ __launch_bounds__(kIsoBX) void iso_count(IsoGrid g, unsigned short* __restrict__ emask,
                                                     unsigned char* __restrict__ hcnt, unsigned char* __restrict__ tcnt,
                                                     unsigned* __restrict__ status) {
  const int x = blockIdx.x * kIsoBX + threadIdx.x;
  const int y = blockIdx.y;
  const int z = blockIdx.z % g.nz, t = blockIdx.z / g.nz;
  if (x >= g.nx) return;
  const long long v = vidx(g, x, y, z, t);
  unsigned above, valid;
  corner_bits(g, x, y, z, t, above, valid);
  unsigned m = 0;
#pragma unroll
  for (int M = 1; M < 16; ++M)
    if (((valid >> M) & 1u) && (((above >> M) ^ above) & 1u)) m |= 1u << (M - 1);
  int tets = 0;
  if (valid == 0xffffu && above != 0u && above != 0xffffu)
    tets = pen_tets_all(std::make_integer_sequence<int, 24>{}, above);
  emask[v] = (unsigned short)m;
  hcnt[v] = (unsigned char)__popc(m);
  tcnt[v] = (unsigned char)tets;
}

// list of the vertices whose cube has crossed pentachora (about one in sixteen on smooth fields), in vertex order,
// so that the pentachoron pass runs on busy lanes only
__global__ void iso_active_list(const unsigned char* __restrict__ tcnt, const long long* __restrict__ abase,
                                long long V, long long* __restrict__ list) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < V && tcnt[v]) list[off16(abase, tcnt, v, true)] = v;
}

__global__ __launch_bounds__(kIsoBX) void iso_emit(IsoGrid g, const unsigned short* __restrict__ emask,
                                                    const long long* __restrict__ hbase,
                                                    const unsigned char* __restrict__ hcnt, long long* __restrict__ edge_id,
                                                    float* __restrict__ pos, unsigned* __restrict__ parent) {
  const int x = blockIdx.x * kIsoBX + threadIdx.x;
  const int y = blockIdx.y;
  const int z = blockIdx.z % g.nz, t = blockIdx.z / g.nz;
  if (x >= g.nx) return;
  const long long v = vidx(g, x, y, z, t);
  const unsigned m = emask[v];
  if (!m) return;
  const float f0 = g.f[v];
  // the far ends of the 15 edges from clamped (in-grid) addresses, all loads in flight before any store (a load
  // issued after a store waits for it); crossed edges only reach corners inside the grid
  float f1[16];
#pragma unroll
  for (int M = 1; M < 16; ++M)
    f1[M] = g.f[vidx(g, min(x + (M & 1), g.nx - 1), min(y + ((M >> 1) & 1), g.ny - 1),
                     min(z + ((M >> 2) & 1), g.nz - 1), min(t + ((M >> 3) & 1), g.nt - 1))];
  const long long o0 = off16(hbase, hcnt, v, false);
#pragma unroll
  for (int M = 1; M < 16; ++M) {
    if (!((m >> (M - 1)) & 1u)) continue;
    const long long o = o0 + __popc(m & ((1u << (M - 1)) - 1u));
    const int dx = M & 1, dy = (M >> 1) & 1, dz = (M >> 2) & 1, dt = (M >> 3) & 1;
    const float mu = (g.c - f0) / (f1[M] - f0);
    edge_id[o] = v * 15 + (M - 1);
    if (pos)
      reinterpret_cast<float4*>(pos)[o] = make_float4((float)x + mu * (float)dx, (float)y + mu * (float)dy,
                                                      (float)z + mu * (float)dz, (float)t + mu * (float)dt);
    parent[o] = (unsigned)o;
  }
}

// Tessellation of the cube's pentachoron of type TY (Sec. 6.1): with k of its five chain vertices above the level,
// case I (one vertex on the smaller side) gives the tetrahedron of its four crossed edges, case II (two) the three
// tetrahedra of the prism between their crossed edges.  The chain corners are compile-time constants, so the
// corners' first hit indices and crossing masks are read from registers by constant index; the lane-dependent
// chain positions are bit fields, and every tetrahedron is one 16-byte store.  Returns false after flagging an
// internal error (a crossed edge the count pass did not record, or more tetrahedra than it counted).
// Hit index of the crossed edge between chain positions i and j of a pentachoron (chain corners in 4-bit fields of
// chw; lower end at position min(i, j) <= 3, whose corner's first hit index and crossing mask are b_k and m_k).
// The values come by value: selecting between references would become a load through a selected address, which
// keeps them in scratch memory.
__device__ __forceinline__ int iso_edge(unsigned i, unsigned j, unsigned chw, long long b0, long long b1, long long b2,
                                        long long b3, unsigned m0, unsigned m1, unsigned m2, unsigned m3, bool& bad) {
  const unsigned lo = min(i, j), hi = max(i, j);
  const unsigned a = (chw >> (4u * lo)) & 15u, M = ((chw >> (4u * hi)) & 15u) ^ a;
  const long long b = lo == 0 ? b0 : (lo == 1 ? b1 : (lo == 2 ? b2 : b3));
  const unsigned mk = lo == 0 ? m0 : (lo == 1 ? m1 : (lo == 2 ? m2 : m3));
  bad = bad || !((mk >> (M - 1u)) & 1u);
  return (int)(b + __popc(mk & ((1u << (M - 1u)) - 1u)));
}

template <int TY>
__device__ __forceinline__ bool iso_tess(unsigned above, const long long (&cb)[16], const unsigned (&cm_mask)[15],
                                         long long& o, long long o_end, int* __restrict__ tets, unsigned* status) {
  constexpr PenCorners kP = build_pen_corners();
  constexpr unsigned c0 = kP.c[TY][0], c1 = kP.c[TY][1], c2 = kP.c[TY][2], c3 = kP.c[TY][3], c4 = kP.c[TY][4];
  constexpr unsigned chw = c0 | c1 << 4 | c2 << 8 | c3 << 12 | c4 << 16;
  const unsigned lm = ((above >> c0) & 1u) | ((above >> c1) & 1u) << 1 | ((above >> c2) & 1u) << 2 |
                      ((above >> c3) & 1u) << 3 | ((above >> c4) & 1u) << 4;
  const int k = __popc(lm);
  if (k == 0 || k == 5) return true;
  // chain positions on the smaller side (minority: one or two) and the others, each in increasing order
  const unsigned mino = k <= 2 ? lm : (~lm & 31u);
  const int nm = __popc(mino);
  const unsigned mi0 = (unsigned)__ffs((int)mino) - 1u, mi1 = (unsigned)__ffs((int)(mino & (mino - 1u))) - 1u;
  unsigned majo = ~mino & 31u;
  unsigned ma[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    ma[q] = (unsigned)__ffs((int)majo) - 1u;
    majo &= majo - 1u;
  }
  // hit index of the crossed edge between chain positions i and j (lower end at position min(i, j) <= 3)
  const long long cb0 = cb[c0], cb1 = cb[c1], cb2 = cb[c2], cb3 = cb[c3];
  const unsigned mk0 = cm_mask[c0], mk1 = cm_mask[c1], mk2 = cm_mask[c2], mk3 = cm_mask[c3];
  bool bad = false;
  auto edge = [&](unsigned i, unsigned j) -> int {
    return iso_edge(i, j, chw, cb0, cb1, cb2, cb3, mk0, mk1, mk2, mk3, bad);
  };
  const bool two = nm == 2;
  // case I: (m, a0..a3); case II: (p1, a0..a2), (p2, a0..a2)
  const int e0 = edge(mi0, ma[0]), e1 = edge(mi0, ma[1]), e2 = edge(mi0, ma[2]);
  const int e3 = two ? edge(mi1, ma[0]) : edge(mi0, ma[3]);
  int e4 = 0, e5 = 0;
  if (two) {
    e4 = edge(mi1, ma[1]);
    e5 = edge(mi1, ma[2]);
  }
  const int nt_here = two ? 3 : 1;
  if (bad || o + nt_here > o_end) {
    atomicOr(status, ST_INVARIANT);
    return false;
  }
  int4* T = reinterpret_cast<int4*>(tets) + o;
  if (!two) {
    T[0] = make_int4(e0, e1, e2, e3);
  } else {
    T[0] = make_int4(e0, e1, e2, e5);
    T[1] = make_int4(e0, e1, e4, e5);
    T[2] = make_int4(e0, e3, e4, e5);
  }
  o += nt_here;
  return true;
}

template <int... TY>
__device__ __forceinline__ void iso_tess_all(std::integer_sequence<int, TY...>, unsigned above,
                                             const long long (&cb)[16], const unsigned (&cm_mask)[15], long long& o,
                                             long long o_end, int* __restrict__ tets, unsigned* status) {
  (void)(iso_tess<TY>(above, cb, cm_mask, o, o_end, tets, status) && ...);  // stops at the first error
}

__global__ __launch_bounds__(kIsoBX) void iso_unite(IsoGrid g, const long long* __restrict__ active,
                                                     long long n_active, const unsigned short* __restrict__ emask,
                                                     const long long* __restrict__ hbase,
                                                     const unsigned char* __restrict__ hcnt,
                                                     const unsigned char* __restrict__ tcnt,
                                                     const long long* __restrict__ tbase, unsigned* __restrict__ parent,
                                                     int* __restrict__ tets, unsigned* __restrict__ status) {
  const long long a_i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (a_i >= n_active) return;
  const long long v = active[a_i];
  const int x = (int)(v % g.nx);
  const int y = (int)((v / g.nx) % g.ny);
  const int z = (int)((v / ((long long)g.nx * g.ny)) % g.nz);
  const int t = (int)(v / ((long long)g.nx * g.ny * g.nz));
  if (tcnt[v] == 0) return;
  unsigned above, valid;
  corner_bits(g, x, y, z, t, above, valid);
  // first hit index and crossing mask of every corner that anchors an edge of a pentachoron (all but 1111)
  long long cb[16];
  unsigned cm_mask[15];
  // corners in x pairs (w, w + 1): one group load gives both offsets unless w ends its group of 16
#pragma unroll
  for (int cm = 0; cm < 15; cm += 2) {
    const long long w = vidx(g, x, y + ((cm >> 1) & 1), z + ((cm >> 2) & 1), t + ((cm >> 3) & 1));
    const long long g0 = w & ~15ll;
    const int k = (int)(w - g0);
    const uint4 q = *reinterpret_cast<const uint4*>(hcnt + g0);
    cb[cm] = hbase[w >> 4] + sum_first(q, k, false);
    const unsigned wk = k < 4 ? q.x : (k < 8 ? q.y : (k < 12 ? q.z : q.w));
    cb[cm + 1] = k < 15 ? cb[cm] + ((wk >> (8 * (k & 3))) & 0xFFu) : hbase[(w + 1) >> 4];
    cm_mask[cm] = emask[w];
    if (cm + 1 < 15) cm_mask[cm + 1] = emask[w + 1];
  }
  long long o = off16(tbase, tcnt, v, false);
  const long long o_end = o + tcnt[v];
  // Unions: the cube's crossed edges P (local set) grouped by "edges of a common pentachoron" (a group grows from
  // its lowest member through the side sets until it is stable); each member is united once with the group's first.
  // Same connectivity as uniting the crossed edges of every pentachoron, with |P| - groups unions.
  {
    u128 P = 0;
    for (int k = 0; k < kCubeEdgeN; ++k) {
      const unsigned a = kCubeEdges.ea[k], b = a | kCubeEdges.eM[k];
      if (((above >> a) ^ (above >> b)) & 1u) {
        if (!((cm_mask[a] >> (kCubeEdges.eM[k] - 1)) & 1u)) {  // the count pass took the same decisions
          atomicOr(status, ST_INVARIANT);
          return;
        }
        P |= (u128)1 << k;
      }
    }
    auto hit = [&](int k) -> long long {
      const unsigned a = kCubeEdges.ea[k], M = kCubeEdges.eM[k];
      return cb[a] + __popc(cm_mask[a] & ((1u << (M - 1)) - 1u));
    };
    u128 R = P;
    while (R) {
      u128 C = (u128)1 << low_bit128(R), prev;
      do {
        prev = C;
        for (int pt = 0; pt < 24; ++pt) {
          const u128 S = edge_side_set(pt) & P;
          if (S & C) C |= S;
        }
      } while (C != prev);
      R &= ~C;
      const int k0 = low_bit128(C);
      const long long h0 = hit(k0);
      C &= ~((u128)1 << k0);
      unsigned r = C ? uf_find_cached(parent, (unsigned)h0) : 0u;
      while (C) {
        const int k = low_bit128(C);
        C &= ~((u128)1 << k);
        r = uf_unite_into(parent, r, (unsigned)hit(k));
      }
    }
  }
  iso_tess_all(std::make_integer_sequence<int, 24>{}, above, cb, cm_mask, o, o_end, tets, status);
}

dim3 iso_grid(const IsoGrid& g) { return dim3((unsigned)((g.nx + kIsoBX - 1) / kIsoBX), (unsigned)g.ny, (unsigned)(g.nz * g.nt)); }

}  // namespace

hipError_t launch_iso_count(const float* f, int nx, int ny, int nz, int nt, float c, unsigned long long* bits,
                            unsigned short* emask, unsigned char* hcnt, unsigned char* tcnt, unsigned* status,
                            hipStream_t s) {
  const IsoGrid g{f, nx, ny, nz, nt, c, bits, (nx + 63) / 64};
  const long long n_words = (long long)nt * nz * ny * g.nwx;
  iso_bits<<<(unsigned)((n_words + 4 * kBitsWords - 1) / (4 * kBitsWords)), 256, 0, s>>>(g, n_words, bits, status);
  iso_count<<<iso_grid(g), kIsoBX, 0, s>>>(g, emask, hcnt, tcnt, status);
  return hipGetLastError();
}

hipError_t launch_iso_emit(const float* f, int nx, int ny, int nz, int nt, float c, const unsigned short* emask,
                           const long long* hbase, const unsigned char* hcnt, long long* edge_id, float* pos,
                           unsigned* parent, hipStream_t s) {
  const IsoGrid g{f, nx, ny, nz, nt, c, nullptr, (nx + 63) / 64};
  iso_emit<<<iso_grid(g), kIsoBX, 0, s>>>(g, emask, hbase, hcnt, edge_id, pos, parent);
  return hipGetLastError();
}

hipError_t launch_iso_active(const unsigned char* tcnt, const long long* abase, long long V, long long* list,
                             hipStream_t s) {
  iso_active_list<<<(unsigned)((V + 255) / 256), 256, 0, s>>>(tcnt, abase, V, list);
  return hipGetLastError();
}

hipError_t launch_iso_unite(const float* f, int nx, int ny, int nz, int nt, float c,
                            const unsigned long long* bits, const long long* active, long long n_active,
                            const unsigned short* emask, const long long* hbase, const unsigned char* hcnt,
                            const unsigned char* tcnt, const long long* tbase, unsigned* parent, int* tets,
                            unsigned* status, hipStream_t s) {
  if (n_active == 0) return hipSuccess;
  const IsoGrid g{f, nx, ny, nz, nt, c, bits, (nx + 63) / 64};
  iso_unite<<<(unsigned)((n_active + kIsoBX - 1) / kIsoBX), kIsoBX, 0, s>>>(g, active, n_active, emask, hbase, hcnt,
                                                                            tcnt, tbase, parent, tets, status);
  return hipGetLastError();
}

}  // namespace ftk
