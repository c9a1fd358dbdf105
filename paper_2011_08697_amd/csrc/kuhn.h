// kuhn.h -- compile-time tables of the regular simplicial spacetime mesh (Sec. 3.3).
//
// Every d-cube of the spacetime grid is split into the d! simplices whose vertex lists are monotone paths from
// corner 0..0 to 1..1.  A k-simplex is indexed by its lowest vertex (the anchor) and a type: the ordered tuple
// (M_1..M_k) of nonempty, pairwise disjoint axis masks between consecutive vertices.  Types are numbered in
// lexicographic order of the tuple.  Axis bits: x = 1, y = 2, [z = 4], t = last.
#pragma once

namespace ftk {

template <int D, int K, int N>
struct TypeTable {
  int count;
  unsigned char m[N][K > 0 ? K : 1];
};

// Ordered K-tuples of nonempty disjoint subsets of D axes, lexicographic.
template <int D, int K, int N>
constexpr TypeTable<D, K, N> build_types() {
  TypeTable<D, K, N> r{};
  r.count = 0;
  int cur[4] = {0, 0, 0, 0};
  int used[5] = {0, 0, 0, 0, 0};
  int depth = 0;
  cur[0] = 0;
  // iterative depth-first enumeration (constexpr-friendly)
  while (depth >= 0) {
    cur[depth]++;
    if (cur[depth] >= (1 << D)) {
      cur[depth] = 0;
      depth--;
      continue;
    }
    if (cur[depth] & used[depth]) continue;
    if (depth == K - 1) {
      for (int i = 0; i < K; ++i) r.m[r.count][i] = (unsigned char)cur[i];
      r.count++;
    } else {
      used[depth + 1] = used[depth] | cur[depth];
      depth++;
      cur[depth] = 0;
    }
  }
  return r;
}

constexpr int popc_c(int x) { return x ? (x & 1) + popc_c(x >> 1) : 0; }

// 2D space + time: triangles (tested faces), tetrahedra (cells).
constexpr auto kTri2 = build_types<3, 2, 12>();
constexpr auto kTet2 = build_types<3, 3, 6>();
static_assert(kTri2.count == 12, "12 triangle types per vertex in 3D spacetime");
static_assert(kTet2.count == 6, "6 tetrahedra per 3-cube");

// 3D space + time: triangles (sub-faces), tetrahedra (tested faces), pentachora (cells).
constexpr auto kTri3 = build_types<4, 2, 50>();
constexpr auto kTet3 = build_types<4, 3, 60>();
constexpr auto kPen3 = build_types<4, 4, 24>();
static_assert(kTri3.count == 50, "50 triangle types per vertex in 4D spacetime");
static_assert(kTet3.count == 60, "60 tetrahedron types per vertex in 4D spacetime");
static_assert(kPen3.count == 24, "24 pentachora per 4-cube");

// Inverse lookup: type index of the tuple (a, b) among 2-tuples over D axes, -1 if not a type.
template <int D, int N>
struct PairIndex {
  signed char idx[16][16];
};
template <int D, int N>
constexpr PairIndex<D, N> build_pair_index(const TypeTable<D, 2, N>& t) {
  PairIndex<D, N> r{};
  for (int a = 0; a < 16; ++a)
    for (int b = 0; b < 16; ++b) r.idx[a][b] = -1;
  for (int i = 0; i < t.count; ++i) r.idx[t.m[i][0]][t.m[i][1]] = (signed char)i;
  return r;
}
constexpr auto kTri2Index = build_pair_index<3, 12>(kTri2);
constexpr auto kTri3Index = build_pair_index<4, 50>(kTri3);

// Inverse lookup for 3-tuples over 4 axes (tetrahedra of 4D spacetime).
struct TripleIndex {
  signed char idx[16][16][16];
};
constexpr TripleIndex build_triple_index() {
  TripleIndex r{};
  for (int a = 0; a < 16; ++a)
    for (int b = 0; b < 16; ++b)
      for (int c = 0; c < 16; ++c) r.idx[a][b][c] = -1;
  for (int i = 0; i < kTet3.count; ++i) r.idx[kTet3.m[i][0]][kTet3.m[i][1]][kTet3.m[i][2]] = (signed char)i;
  return r;
}
constexpr auto kTet3Index = build_triple_index();

// Bit set of the types of a table whose masks use axis bit `axis`.
template <int D, int K, int N>
constexpr unsigned long long types_using_axis(const TypeTable<D, K, N>& t, int axis) {
  unsigned long long s = 0;
  for (int i = 0; i < t.count; ++i) {
    int u = 0;
    for (int k = 0; k < K; ++k) u |= t.m[i][k];
    if (u & axis) s |= 1ull << i;
  }
  return s;
}

}  // namespace ftk
