// post.hip -- trajectory post-processing on the device, after the tracking passes.
//
//   * Slicing at a time step (Sec. 3.2, "Ordinal and interval mesh elements"): the critical points of step t0 are
//     the punctured ordinal faces anchored at t0 (faces whose axis masks do not use the time axis).  Hits are
//     sorted by face id and face ids are t-major, so they form one contiguous range of the hit arrays.
//   * Per-trajectory attributes for filtering (Sec. 4.4, "Filtering"): number of points, time extent of their
//     spacetime positions, and the number of ends.  Under the symbolic perturbation every punctured face lies in
//     exactly two cells with one more punctured side each, unless it lies in a boundary hyperplane of the grid
//     (a coordinate equal to 0 with the axis unused, or equal to N - 1), where only one cell exists; so a
//     trajectory is a path with two boundary ends or a closed loop with none.
//   * Loop filtering: drop closed loops (a transient birth-death pair) whose time extent is below a threshold.
//   * Order of the points along each trajectory (cell neighbours, list ranking over a sparse ruling set), and the type
//     smoothing and run simplification that walk it (Sec. 4.4, "Simplification" and "Smoothing").
#include <climits>

#include "common.h"
#include "internal.h"
#include "kuhn.h"

namespace ftk {

namespace {

// Axes used by a face type and its anchor coordinates (x, y, [z], t) from the face id.
struct FaceSpace {
  int n;              // spatial dimension
  long long N[4];     // x, y, [z], t extents
  long long T;        // face types per vertex
};

__device__ __forceinline__ unsigned face_used_axes(int n, int ty) {
  if (n == 2) return (unsigned)(kTri2.m[ty][0] | kTri2.m[ty][1]);
  return (unsigned)(kTet3.m[ty][0] | kTet3.m[ty][1] | kTet3.m[ty][2]);
}

// anchor coordinates c[0..n] (time last) and type of a face id
__device__ __forceinline__ int face_decode(const FaceSpace& fs, long long fid, long long* c) {
  const int ty = (int)(fid % fs.T);
  long long g = fid / fs.T;
  for (int a = 0; a < fs.n; ++a) {
    c[a] = g % fs.N[a];
    g /= fs.N[a];
  }
  c[fs.n] = g;
  return ty;
}

// the face lies in a boundary hyperplane of the grid (one cell holds it)
__device__ __forceinline__ bool face_on_boundary(const FaceSpace& fs, long long fid) {
  long long c[4];
  const int ty = face_decode(fs, fid, c);
  const unsigned used = face_used_axes(fs.n, ty);
  for (int a = 0; a <= fs.n; ++a) {
    if (c[a] == fs.N[a] - 1) return true;
    if (c[a] == 0 && !((used >> a) & 1u)) return true;
  }
  return false;
}

// first index in [0, n) with keys[i] >= v (keys ascending)
__device__ __forceinline__ long long lower_bound64(const long long* keys, long long n, long long v) {
  long long lo = 0, hi = n;
  while (lo < hi) {
    const long long mid = (lo + hi) >> 1;
    if (keys[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Sorted face ids (hits, or trajectory labels) bucketed by vertex row: bucket b holds the ids in [b B, (b + 1) B)
// with B = T nx, and bstart[b] is its first index, so a lookup searches one row instead of the whole array.
__global__ void k_buckets(const long long* __restrict__ face_id, long long n_hits, long long B, long long n_buckets,
                          long long* __restrict__ bstart) {
  const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (b <= n_buckets) bstart[b] = lower_bound64(face_id, n_hits, b * B);
}

// The same table built from the sorted ids themselves: id i fills the buckets after the previous id's bucket up to
// its own (thread n_hits closes the table), O(ids + buckets) work.  Used with one bucket per vertex when ids are
// dense, where a binary search per bucket would cost more than the lookups it saves.
__global__ void k_gapfill(const long long* __restrict__ face_id, long long n_ids, long long B, long long n_buckets,
                          long long* __restrict__ bstart) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n_ids) return;
  long long hi = i < n_ids ? face_id[i] / B : n_buckets;
  long long lo = i > 0 ? face_id[i - 1] / B + 1 : 0;
  if (lo < 0) lo = 0;
  if (hi > n_buckets) hi = n_buckets;
  for (long long b = lo; b <= hi; ++b) bstart[b] = i;
}

// index of face id v in the sorted array, -1 if absent
__device__ __forceinline__ long long find_sorted(const long long* face_id, const long long* bstart, long long B,
                                                 long long n_buckets, long long v) {
  const long long b = v / B;
  if (v < 0 || b >= n_buckets) return -1;
  const long long lo = bstart[b], hi = bstart[b + 1];
  const long long k = lo + lower_bound64(face_id + lo, hi - lo, v);
  return (k < hi && face_id[k] == v) ? k : -1;
}

// Per-trajectory (or per-run) accumulation.  Consecutive hits often belong to the same trajectory, so the lanes of
// a wave first combine over runs of equal keys (segmented reduction by shuffles) and only the first lane of each
// run issues the atomics.  Lanes without a key pass a negative one of their own.
struct RunAcc {
  unsigned long long cnt;
  int mn, mx, ends;
};

__device__ __forceinline__ bool wave_run_reduce(long long key, RunAcc& a) {
  const int lane = threadIdx.x & 63;
  const long long prev = __shfl_up(key, 1);
  const bool head = lane == 0 || prev != key;
  const unsigned long long hb = __ballot(head);
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const int rid = __popcll(hb & upto);
  for (int o = 1; o < 64; o <<= 1) {
    const int r2 = __shfl_down(rid, o);
    const unsigned long long c2 = __shfl_down(a.cnt, o);
    const int mn2 = __shfl_down(a.mn, o), mx2 = __shfl_down(a.mx, o), e2 = __shfl_down(a.ends, o);
    if (lane + o < 64 && r2 == rid) {
      a.cnt += c2;
      a.mn = min(a.mn, mn2);
      a.mx = max(a.mx, mx2);
      a.ends += e2;
    }
  }
  return head;
}

__global__ void k_root_flags(const long long* __restrict__ face_id, const long long* __restrict__ label, long long n,
                             int* __restrict__ flag) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = label[i] == face_id[i] ? 1 : 0;
}

__global__ void k_root_scatter(const long long* __restrict__ face_id, const int* __restrict__ flag,
                               const long long* __restrict__ off, long long n, long long n_traj,
                               long long* __restrict__ roots, unsigned* __restrict__ status) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flag[i]) return;
  const long long j = off[i];
  if (j < n_traj)
    roots[j] = face_id[i];
  else
    atomicOr(status, ST_INVARIANT);
}

__global__ void k_traj_init(long long n_traj, unsigned long long* __restrict__ n_hits, int* __restrict__ t_min,
                            int* __restrict__ t_max, int* __restrict__ n_ends) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_traj) return;
  n_hits[j] = 0;
  t_min[j] = 0x7f800000;  // +inf
  t_max[j] = 0;           // 0.0f: spacetime times are >= 0, so their bit patterns order like the values
  n_ends[j] = 0;
}

__global__ void k_traj_accum(FaceSpace fs, const long long* __restrict__ face_id, const long long* __restrict__ label,
                             const float* __restrict__ pos, long long n, const long long* __restrict__ roots,
                             const long long* __restrict__ rb, long long B, long long nbk,
                             unsigned long long* __restrict__ n_hits, int* __restrict__ t_min,
                             int* __restrict__ t_max, int* __restrict__ n_ends, unsigned* __restrict__ status) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long key = -1 - (long long)(threadIdx.x & 63);
  RunAcc a = {0ull, 0x7f800000, 0, 0};
  if (i < n) {
    const long long j = find_sorted(roots, rb, B, nbk, label[i]);
    if (j < 0) {
      atomicOr(status, ST_INVARIANT);
    } else {
      key = j;
      const int tb = __float_as_int(pos[i * (fs.n + 1) + fs.n]);
      a.cnt = 1;
      a.mn = tb;
      a.mx = tb;
      a.ends = face_on_boundary(fs, face_id[i]) ? 1 : 0;
    }
  }
  if (wave_run_reduce(key, a) && key >= 0) {
    atomicAdd(&n_hits[key], a.cnt);
    atomicMin(&t_min[key], a.mn);
    atomicMax(&t_max[key], a.mx);
    if (a.ends) atomicAdd(&n_ends[key], a.ends);
  }
}

__global__ void k_slice_flags(FaceSpace fs, const long long* __restrict__ face_id, long long lo, long long hi,
                              int* __restrict__ flag) {
  const long long i = lo + (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= hi) return;
  const int ty = (int)(face_id[i] % fs.T);
  const unsigned tbit = 1u << fs.n;
  flag[i - lo] = (face_used_axes(fs.n, ty) & tbit) ? 0 : 1;
}

__global__ void k_slice_scatter(const int* __restrict__ flag, const long long* __restrict__ off, long long lo,
                                long long cnt, long long* __restrict__ idx) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < cnt && flag[k]) idx[off[k]] = lo + k;
}

__global__ void k_filter_loops(const long long* __restrict__ label, long long n, const long long* __restrict__ roots,
                               long long n_traj, const int* __restrict__ t_min, const int* __restrict__ t_max,
                               const int* __restrict__ n_ends, float min_duration, uint8_t* __restrict__ keep) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long j = lower_bound64(roots, n_traj, label[i]);
  bool k = true;
  if (j < n_traj && roots[j] == label[i] && n_ends[j] == 0)
    k = !(__int_as_float(t_max[j]) - __int_as_float(t_min[j]) < min_duration);
  keep[i] = k ? 1 : 0;
}

__global__ void k_range(FaceSpace fs, const long long* __restrict__ face_id, long long n, long long t0,
                        long long* __restrict__ out) {
  if (threadIdx.x != 0) return;
  long long plane_faces = fs.T;
  for (int a = 0; a < fs.n; ++a) plane_faces *= fs.N[a];
  out[0] = lower_bound64(face_id, n, t0 * plane_faces);
  out[1] = lower_bound64(face_id, n, (t0 + 1) * plane_faces);
}

// ---------------------------------------------------------------------------------------------------------------
// Order of the points along each trajectory.  The curve's piece in a cell is the segment between the cell's two
// punctured sides, so the neighbours of a hit are the other punctured side of each cell that holds it (at most
// two cells).  A face with axis masks (M_1..M_n) and unused axes R lies in the cells (R, M_1..M_n) anchored one
// step back along R and (M_1..M_n, R) at its own anchor when R is one axis; when R is empty, exactly one mask
// holds two axes {a, b} and the cells split it as (.., a, b, ..) or (.., b, a, ..) at the same anchor.  A cell
// (s_0..s_n) anchored at c drops vertex k to give a side: k = 0 moves the anchor to c + e(s_0) with masks
// (s_1..s_n); k = n + 1 keeps (s_0..s_{n-1}); an inner k merges s_{k-1} | s_k.
// ---------------------------------------------------------------------------------------------------------------

__device__ __forceinline__ int face_masks(int n, int ty, unsigned* m) {
  if (n == 2) {
    m[0] = kTri2.m[ty][0];
    m[1] = kTri2.m[ty][1];
  } else {
    m[0] = kTet3.m[ty][0];
    m[1] = kTet3.m[ty][1];
    m[2] = kTet3.m[ty][2];
  }
  return n;
}

__device__ __forceinline__ int type_of_masks(int n, const unsigned* m) {
  return n == 2 ? (int)kTri2Index.idx[m[0]][m[1]] : (int)kTet3Index.idx[m[0]][m[1]][m[2]];
}

__device__ __forceinline__ long long vertex_index(const FaceSpace& fs, const long long* c) {
  long long g = c[fs.n];
  for (int a = fs.n - 1; a >= 0; --a) g = g * fs.N[a] + c[a];
  return g;
}

__global__ void k_neighbours(FaceSpace fs, const long long* __restrict__ face_id, long long n_hits,
                             const long long* __restrict__ bstart, long long B, long long n_buckets,
                             int2* __restrict__ nb, unsigned* __restrict__ status) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_hits) return;
  const int n = fs.n, d = fs.n + 1;
  const long long fid = face_id[i];
  long long p[4];
  const int ty = face_decode(fs, fid, p);
  unsigned M[3];
  face_masks(n, ty, M);
  unsigned used = 0;
  for (int k = 0; k < n; ++k) used |= M[k];
  const unsigned R = ((1u << d) - 1u) ^ used;
  int found[2] = {-1, -1};
  int nf = 0;
  bool bad = false;
  for (int cell = 0; cell < 2; ++cell) {
    unsigned s[4];
    long long c[4];
    for (int a = 0; a < d; ++a) c[a] = p[a];
    if (R) {
      if (cell == 0) {
        s[0] = R;
        for (int k = 0; k < n; ++k) s[k + 1] = M[k];
        for (int a = 0; a < d; ++a)
          if ((R >> a) & 1u) c[a] -= 1;
      } else {
        for (int k = 0; k < n; ++k) s[k] = M[k];
        s[n] = R;
      }
    } else {
      int o = 0;
      for (int k = 0; k < n; ++k) {
        if (__popc(M[k]) == 2) {
          const unsigned lo = M[k] & (0u - M[k]), hi = M[k] ^ lo;
          s[o++] = cell == 0 ? lo : hi;
          s[o++] = cell == 0 ? hi : lo;
        } else {
          s[o++] = M[k];
        }
      }
    }
    bool inside = true;
    for (int a = 0; a < d; ++a) inside &= c[a] >= 0 && c[a] <= fs.N[a] - 2;
    if (!inside) continue;
    int hits_here = 0;
    long long other = -1;
    for (int k = 0; k <= d; ++k) {
      long long a0[4];
      unsigned m[3];
      for (int a = 0; a < d; ++a) a0[a] = c[a];
      if (k == 0) {
        for (int a = 0; a < d; ++a)
          if ((s[0] >> a) & 1u) a0[a] += 1;
        for (int q = 0; q < n; ++q) m[q] = s[q + 1];
      } else if (k == d) {
        for (int q = 0; q < n; ++q) m[q] = s[q];
      } else {
        int o = 0;
        for (int q = 0; q < d; ++q) {
          if (q == k - 1) {
            m[o++] = s[q] | s[q + 1];
            ++q;
          } else {
            m[o++] = s[q];
          }
        }
      }
      const long long side = vertex_index(fs, a0) * fs.T + type_of_masks(n, m);
      if (side == fid) continue;
      const long long h = find_sorted(face_id, bstart, B, n_buckets, side);
      if (h >= 0) {
        ++hits_here;
        other = h;
      }
    }
    if (hits_here != 1) {
      bad = true;
      continue;
    }
    found[nf++] = (int)other;
  }
  if (bad || nf == 0) atomicOr(status, ST_INVARIANT);
  if (nf == 2 && found[1] < found[0]) {
    const int x = found[0];
    found[0] = found[1];
    found[1] = x;
  }
  nb[i] = make_int2(found[0], found[1]);
}

// A closed loop is cut between its label face (the root: smallest face id, so smallest index) and its neighbour
// with the larger face id; the walk then runs root, smaller neighbour, ..., larger neighbour.
__global__ void k_cut_loops(const long long* __restrict__ face_id, const long long* __restrict__ label,
                            long long n_hits, const long long* __restrict__ roots, const long long* __restrict__ rb,
                            long long B, long long nbk, const int* __restrict__ n_ends, int2* __restrict__ nb) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_hits || label[i] != face_id[i]) return;
  const long long j = find_sorted(roots, rb, B, nbk, label[i]);
  if (j < 0 || n_ends[j] != 0) return;
  int2 q = nb[i];
  const int b = q.y;
  if (b < 0 || b >= n_hits) return;
  q.y = -1;
  nb[i] = q;
  int2 r = nb[b];
  if (r.x == (int)i) r.x = -1;
  if (r.y == (int)i) r.y = -1;
  nb[b] = r;
}

// List ranking by a sparse ruling set.  Rulers are the path ends and about one hit in kRulerEvery chosen by an
// integer hash of the index (the "lowbias32" mixer of C. Wellons).  Each ruler walks both ways to the next ruler,
// recording in every node it passes, for the side facing the ruler, (ruler, distance, the ruler's arm).  Pointer
// jumping then runs on the rulers only: arm k of ruler R holds (far ruler F, F's arm facing R, distance, done),
// done once F has no neighbour on its far side, i.e. F is a path end.
constexpr unsigned kRulerEvery = 32;

__device__ __forceinline__ unsigned mix32(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

// wave-aggregated append of flagged lanes to a list; returns the lane's slot (valid where flagged)
__device__ __forceinline__ long long wave_append(bool flag, unsigned long long* count) {
  const unsigned long long bal = __ballot(flag);
  if (!bal) return -1;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)bal) - 1;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(count, (unsigned long long)__popcll(bal));
  base = __shfl(base, leader);
  return (long long)(base + __popcll(bal & ((1ull << lane) - 1ull)));
}

__global__ void k_ruler_flags(const int2* __restrict__ nb, long long n_hits, unsigned char* __restrict__ is_ruler,
                              int* __restrict__ flag) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_hits) return;
  const int2 q = nb[i];
  const bool r = q.x < 0 || q.y < 0 || (mix32((unsigned)i) & (kRulerEvery - 1u)) == 0u;
  is_ruler[i] = r ? 1 : 0;
  flag[i] = r ? 1 : 0;
}

__global__ void k_ruler_list(const int* __restrict__ flag, const long long* __restrict__ off, long long n_hits,
                             int* __restrict__ rid, int* __restrict__ list) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_hits || !flag[i]) return;
  rid[i] = (int)off[i];
  list[off[i]] = (int)i;
}

// one thread per (ruler, direction): walk to the next ruler
__global__ void k_walk(const int2* __restrict__ nb, const int* __restrict__ list, long long n_rulers, long long n_hits, uint2* __restrict__ seg,
                       unsigned* __restrict__ status) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * n_rulers) return;
  const int R = list[t >> 1];
  const unsigned k = (unsigned)(t & 1);
  const int2 q = nb[R];
  const int first = k ? q.y : q.x;
  if (first < 0) {  // no neighbour this way: the ruler is a path end, its own far end at distance 0
    seg[2 * (long long)R + k] = make_uint2((unsigned)R, k);
    return;
  }
  int prev = R, v = first;
  unsigned dist = 1;
  for (;;) {
    const int2 w = nb[v];
    unsigned s;
    if (w.x == prev)
      s = 0;
    else if (w.y == prev)
      s = 1;
    else {
      atomicOr(status, ST_INVARIANT);
      return;
    }
    seg[2 * (long long)v + s] = make_uint2((unsigned)R, (dist << 1) | k);
    const int nxt = s ? w.x : w.y;
    if (nxt < 0 || (mix32((unsigned)v) & (kRulerEvery - 1u)) == 0u) return;  // v is a ruler (as in k_ruler_flags)
    if ((long long)dist >= n_hits) {  // a walk cannot pass n_hits steps
      atomicOr(status, ST_INVARIANT);
      return;
    }
    prev = v;
    v = nxt;
    ++dist;
  }
}

__global__ void k_rinit(const int2* __restrict__ nb, const int* __restrict__ list, long long n_rulers,
                        long long n_hits, const uint2* __restrict__ seg, int4* __restrict__ st,
                        unsigned* __restrict__ status) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * n_rulers) return;
  const int R = list[t >> 1];
  const int k = (int)(t & 1);
  const int2 q = nb[R];
  const int nbk = k ? q.y : q.x;
  int4 v = make_int4(R, k, 0, 1);
  if (nbk >= 0) {
    const uint2 sg = seg[2 * (long long)R + k];
    if ((long long)sg.x >= n_hits) {
      atomicOr(status, ST_INVARIANT);
    } else {
      v = make_int4((int)sg.x, (int)(sg.y & 1u), (int)(sg.y >> 1), 0);
    }
  }
  st[t] = v;
}

// One jumping round over the listed rulers (all of them when act is null): every open arm takes the state of the
// far ruler's arm that leads on.  A ruler open at the start of the round stays listed for one more round, so that
// its final state reaches both buffers.
__global__ void k_rjump(const int2* __restrict__ nb, const int* __restrict__ rid, const int* __restrict__ act,
                        long long n_act, long long n_hits, const int4* __restrict__ in, int4* __restrict__ out,
                        int* __restrict__ next, unsigned long long* __restrict__ next_n,
                        unsigned* __restrict__ status) {
  const long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  bool keep = false;
  int slot = 0;
  if (a < n_act) {
    slot = act ? act[a] : (int)a;
    for (int k = 0; k < 2; ++k) {
      int4 s = in[2 * (long long)slot + k];
      if (!s.w) {
        keep = true;
        const int F = s.x, side = 1 - s.y;
        const int2 q = nb[F];
        if ((side ? q.y : q.x) < 0) {
          s.w = 1;
        } else {
          const int4 s2 = in[2 * (long long)rid[F] + side];
          const long long D = (long long)s.z + s2.z;
          if (D > n_hits) {  // longer than the hit count: a cycle the loop cut did not open
            atomicOr(status, ST_INVARIANT);
            s.w = 1;
          } else {
            s = make_int4(s2.x, s2.y, (int)D, s2.w);
          }
        }
      }
      out[2 * (long long)slot + k] = s;
    }
  }
  const long long pos = wave_append(keep, next_n);
  if (keep) next[pos] = slot;
}

__global__ void k_count_to_int(const unsigned long long* __restrict__ n_points, long long n_traj,
                               int* __restrict__ out) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n_traj) out[j] = (int)n_points[j];
}

// Position of each hit: trajectory start + distance to its start end (the end with the smaller index, i.e. the
// smaller face id); the path length through the hit must equal the trajectory's point count.
__global__ void k_place(const long long* __restrict__ label, long long n_hits, const long long* __restrict__ roots,
                        const long long* __restrict__ rb, long long B, long long nbk,
                        const long long* __restrict__ offsets,
                        const unsigned char* __restrict__ is_ruler, const int* __restrict__ rid,
                        const uint2* __restrict__ seg, const int4* __restrict__ st, long long* __restrict__ order,
                        unsigned* __restrict__ status) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_hits) return;
  long long E[2], D[2];
  if (is_ruler[v]) {
    for (int k = 0; k < 2; ++k) {
      const int4 s = st[2 * (long long)rid[v] + k];
      E[k] = s.x;
      D[k] = s.z;
    }
  } else {
    for (int k = 0; k < 2; ++k) {
      const uint2 sg = seg[2 * v + k];
      if ((long long)sg.x >= n_hits || !is_ruler[sg.x]) {
        atomicOr(status, ST_INVARIANT);
        return;
      }
      const int4 s = st[2 * (long long)rid[sg.x] + (1 - (int)(sg.y & 1u))];
      E[k] = s.x;
      D[k] = (long long)(sg.y >> 1) + s.z;
    }
  }
  const long long j = find_sorted(roots, rb, B, nbk, label[v]);
  if (j < 0) {
    atomicOr(status, ST_INVARIANT);
    return;
  }
  const long long len = D[0] + D[1] + 1;
  const long long rank = E[0] < E[1] ? D[0] : D[1];
  const long long lo = offsets[j], hi = offsets[j + 1];
  if (len != hi - lo || rank < 0 || rank >= len) {
    atomicOr(status, ST_INVARIANT);
    return;
  }
  order[lo + rank] = v;
}

// ---------------------------------------------------------------------------------------------------------------
// Type smoothing and run simplification along the order (Sec. 4.4).  Position k of order[] belongs to trajectory
// j with offsets[j] <= k < offsets[j + 1]; a trajectory without ends is a closed loop.
// ---------------------------------------------------------------------------------------------------------------

struct Walk {
  const long long* order;
  const long long* offsets;
  const int* n_ends;
  const int* head;         // [n_hits] 1 where a trajectory starts in order[]
  const long long* heads;  // [n_hits] exclusive prefix sum of head
  long long n_traj, n_hits;
};

// trajectory starts in order[] (head flags, cleared beforehand); their prefix sum gives each position's trajectory
__global__ void k_traj_heads(const long long* __restrict__ offsets, long long n_traj, long long n_hits,
                             int* __restrict__ head) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_traj) return;
  const long long o = offsets[j];
  if (o >= 0 && o < n_hits) head[o] = 1;
}

// trajectory of position k, its start and length; false for inconsistent offsets
__device__ __forceinline__ bool locate(const Walk& w, long long k, long long* j, long long* lo, long long* m) {
  const long long a = w.heads[k] + w.head[k] - 1;
  if (a < 0 || a >= w.n_traj) return false;
  *j = a;
  *lo = w.offsets[a];
  *m = w.offsets[a + 1] - *lo;
  return *lo >= 0 && *m > 0 && *lo + *m <= w.n_hits && k >= *lo && k < *lo + *m;
}

__device__ __forceinline__ long long hit_at(const Walk& w, long long q, unsigned* status) {
  const long long h = w.order[q];
  if (h < 0 || h >= w.n_hits) {
    atomicOr(status, ST_INVARIANT);
    return -1;
  }
  return h;
}

__global__ void k_smooth(Walk w, const uint8_t* __restrict__ type_in, int half, uint8_t* __restrict__ type_out,
                         unsigned* __restrict__ status) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= w.n_hits) return;
  long long j, lo, m;
  if (!locate(w, k, &j, &lo, &m)) {
    atomicOr(status, ST_INVARIANT);
    return;
  }
  const long long h = hit_at(w, k, status);
  if (h < 0) return;
  const uint8_t own = type_in[h];
  uint8_t res = own;
  const long long r = k - lo;
  const bool loop = w.n_ends[j] == 0;
  const bool fits = loop ? m >= 2LL * half + 1 : (r - half >= 0 && r + half <= m - 1);
  if (fits && half > 0) {
    int common = -1;
    bool same = true;
    for (int dlt = -half; dlt <= half && same; ++dlt) {
      if (dlt == 0) continue;
      long long q = r + dlt;
      if (loop) q = ((q % m) + m) % m;
      const long long hq = hit_at(w, lo + q, status);
      if (hq < 0) return;
      const int tq = type_in[hq];
      if (common < 0) common = tq;
      same = tq == common;
    }
    if (same && common >= 0 && common != own) res = (uint8_t)common;
  }
  type_out[h] = res;
}

// Loops are walked from their first type change (rotation), so that no run wraps around; rot[j] = the smallest
// position r with a type different from position r - 1 (cyclically), m when the whole loop has one type.
__global__ void k_rot_init(Walk w, long long* __restrict__ rot) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < w.n_traj) rot[j] = LLONG_MAX;
}

__global__ void k_rot_find(Walk w, const uint8_t* __restrict__ type_in, long long* __restrict__ rot,
                           unsigned* __restrict__ status) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= w.n_hits) return;
  long long j, lo, m;
  if (!locate(w, k, &j, &lo, &m)) {
    atomicOr(status, ST_INVARIANT);
    return;
  }
  if (w.n_ends[j] != 0) return;
  const long long r = k - lo;
  const long long h = hit_at(w, k, status), hp = hit_at(w, lo + (r + m - 1) % m, status);
  if (h < 0 || hp < 0) return;
  if (type_in[h] != type_in[hp]) atomicMin(&rot[j], r);
}

// position in order[] of rotated position q of trajectory j
__device__ __forceinline__ long long rotated(const Walk& w, const long long* rot, long long j, long long lo,
                                             long long m, long long q) {
  long long s = 0;
  if (w.n_ends[j] == 0) {
    s = rot[j];
    if (s < 0 || s >= m) s = 0;
  }
  return lo + (q - lo + s) % m;
}

__global__ void k_run_flags(Walk w, const uint8_t* __restrict__ type_in, const long long* __restrict__ rot,
                            int* __restrict__ flag, unsigned* __restrict__ status) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= w.n_hits) return;
  long long j, lo, m;
  if (!locate(w, q, &j, &lo, &m)) {
    atomicOr(status, ST_INVARIANT);
    flag[q] = 0;
    return;
  }
  int f = 1;
  if (q > lo) {
    const long long h = hit_at(w, rotated(w, rot, j, lo, m, q), status);
    const long long hp = hit_at(w, rotated(w, rot, j, lo, m, q - 1), status);
    f = (h >= 0 && hp >= 0 && type_in[h] == type_in[hp]) ? 0 : 1;
  }
  flag[q] = f;
}

__global__ void k_run_init(long long n, int* __restrict__ t_min, int* __restrict__ t_max) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  t_min[i] = 0x7f800000;
  t_max[i] = 0;
}

__global__ void k_run_stats(Walk w, int n, const float* __restrict__ pos, const uint8_t* __restrict__ type_in,
                            const long long* __restrict__ rot, const int* __restrict__ flag,
                            const long long* __restrict__ run_off, int* __restrict__ t_min, int* __restrict__ t_max,
                            uint8_t* __restrict__ run_type, unsigned* __restrict__ status) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long key = -1 - (long long)(threadIdx.x & 63);
  RunAcc a = {0ull, 0x7f800000, 0, 0};
  long long j, lo, m;
  if (q < w.n_hits && locate(w, q, &j, &lo, &m)) {
    const long long h = hit_at(w, rotated(w, rot, j, lo, m, q), status);
    const long long run = run_off[q] + flag[q] - 1;
    if (run < 0 || run >= w.n_hits) {
      atomicOr(status, ST_INVARIANT);
    } else if (h >= 0) {
      key = run;
      a.mn = a.mx = __float_as_int(pos[h * (n + 1) + n]);
      if (flag[q]) run_type[run] = type_in[h];
    }
  }
  if (wave_run_reduce(key, a) && key >= 0) {
    atomicMin(&t_min[key], a.mn);
    atomicMax(&t_max[key], a.mx);
  }
}

// New type of each run (decided at the run's first position), from the neighbouring runs of its trajectory.
__global__ void k_run_decide(Walk w, const int* __restrict__ flag, const long long* __restrict__ run_off,
                             const int* __restrict__ t_min, const int* __restrict__ t_max,
                             const uint8_t* __restrict__ run_type, float theta, uint8_t* __restrict__ new_type) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= w.n_hits || !flag[q]) return;
  long long j, lo, m;
  if (!locate(w, q, &j, &lo, &m)) return;
  const long long run = run_off[q];
  const long long first = run_off[lo];                       // flag[lo] == 1
  const long long last = run_off[lo + m - 1] + flag[lo + m - 1] - 1;
  if (first < 0 || last >= w.n_hits || run < first || run > last) return;
  const bool loop = w.n_ends[j] == 0;
  uint8_t res = run_type[run];
  long long pr = -1, nx = -1;
  if (last > first) {
    if (loop) {
      pr = run > first ? run - 1 : last;
      nx = run < last ? run + 1 : first;
    } else if (run > first && run < last) {
      pr = run - 1;
      nx = run + 1;
    }
  }
  if (pr >= 0) {
    const float ext = __int_as_float(t_max[run]) - __int_as_float(t_min[run]);
    const float ep = __int_as_float(t_max[pr]) - __int_as_float(t_min[pr]);
    const float en = __int_as_float(t_max[nx]) - __int_as_float(t_min[nx]);
    if (ext < theta && run_type[pr] == run_type[nx] && ep >= theta && en >= theta) res = run_type[pr];
  }
  new_type[run] = res;
}

__global__ void k_run_apply(Walk w, const long long* __restrict__ rot, const int* __restrict__ flag,
                            const long long* __restrict__ run_off, const uint8_t* __restrict__ new_type,
                            uint8_t* __restrict__ type_out, unsigned* __restrict__ status) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= w.n_hits) return;
  long long j, lo, m;
  if (!locate(w, q, &j, &lo, &m)) return;
  const long long h = hit_at(w, rotated(w, rot, j, lo, m, q), status);
  const long long run = run_off[q] + flag[q] - 1;
  if (h < 0 || run < 0 || run >= w.n_hits) return;
  type_out[h] = new_type[run];
}

unsigned blocks_for(long long n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

FaceSpace make_space(int n, const int64_t* dims_with_t) {
  FaceSpace fs;
  fs.n = n;
  for (int a = 0; a < 4; ++a) fs.N[a] = 1;
  for (int a = 0; a <= n; ++a) fs.N[a] = dims_with_t[a];
  fs.T = n == 2 ? 12 : 60;
  return fs;
}

}  // namespace

long long row_buckets(int n, const int64_t* dims_with_t) {
  long long nb = 1;
  for (int a = 1; a <= n; ++a) nb *= dims_with_t[a];
  return nb;
}

long long hit_buckets(int n, const int64_t* dims_with_t, long long n_hits, long long* B) {
  long long V = 1;
  for (int a = 0; a <= n; ++a) V *= dims_with_t[a];
  const long long T = n == 2 ? 12 : 60;
  if (V <= 16 * n_hits) {  // dense: one bucket per vertex
    *B = T;
    return V;
  }
  *B = T * dims_with_t[0];
  return row_buckets(n, dims_with_t);
}

hipError_t launch_traj_table(int n, const int64_t* dims_with_t, const long long* face_id, const long long* label,
                             const float* pos, long long n_hits, long long n_traj, int* flag, long long* off,
                             long long* scan_total, long long* scan_tmp, long long* roots, long long* rb,
                             unsigned long long* hits, int* t_min, int* t_max, int* n_ends, unsigned* status,
                             hipStream_t s) {
  const FaceSpace fs = make_space(n, dims_with_t);
  k_traj_init<<<blocks_for(n_traj), 256, 0, s>>>(n_traj, hits, t_min, t_max, n_ends);
  if (n_hits == 0) return hipGetLastError();
  k_root_flags<<<blocks_for(n_hits), 256, 0, s>>>(face_id, label, n_hits, flag);
  hipError_t e = launch_scan(flag, off, n_hits, scan_total, scan_tmp, s);
  if (e != hipSuccess) return e;
  k_root_scatter<<<blocks_for(n_hits), 256, 0, s>>>(face_id, flag, off, n_hits, n_traj, roots, status);
  const long long nbk = row_buckets(n, dims_with_t), B = fs.T * fs.N[0];
  k_buckets<<<blocks_for(nbk + 1), 256, 0, s>>>(roots, n_traj, B, nbk, rb);
  k_traj_accum<<<blocks_for(n_hits), 256, 0, s>>>(fs, face_id, label, pos, n_hits, roots, rb, B, nbk, hits, t_min,
                                                   t_max, n_ends, status);
  return hipGetLastError();
}

hipError_t launch_slice_range(int n, const int64_t* dims_with_t, const long long* face_id, long long n_hits,
                              long long t0, long long* range, hipStream_t s) {
  k_range<<<1, 64, 0, s>>>(make_space(n, dims_with_t), face_id, n_hits, t0, range);
  return hipGetLastError();
}

hipError_t launch_slice_compact(int n, const int64_t* dims_with_t, const long long* face_id, long long lo,
                                long long cnt, int* flag, long long* off, long long* total, long long* tmp,
                                long long* idx_out, bool scatter, hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  if (!scatter) {
    k_slice_flags<<<blocks_for(cnt), 256, 0, s>>>(make_space(n, dims_with_t), face_id, lo, lo + cnt, flag);
    return launch_scan(flag, off, cnt, total, tmp, s);
  }
  k_slice_scatter<<<blocks_for(cnt), 256, 0, s>>>(flag, off, lo, cnt, idx_out);
  return hipGetLastError();
}

hipError_t launch_filter_loops(const long long* label, long long n_hits, const long long* roots, long long n_traj,
                               const int* t_min, const int* t_max, const int* n_ends, float min_duration,
                               uint8_t* keep, hipStream_t s) {
  if (n_hits == 0) return hipSuccess;
  k_filter_loops<<<blocks_for(n_hits), 256, 0, s>>>(label, n_hits, roots, n_traj, t_min, t_max, n_ends, min_duration,
                                                    keep);
  return hipGetLastError();
}

namespace {

Walk make_walk(const long long* order, const long long* offsets, const int* n_ends, long long n_traj,
               long long n_hits, const int* head, const long long* heads) {
  Walk w;
  w.order = order;
  w.offsets = offsets;
  w.n_ends = n_ends;
  w.head = head;
  w.heads = heads;
  w.n_traj = n_traj;
  w.n_hits = n_hits;
  return w;
}

hipError_t walk_heads(const long long* offsets, long long n_traj, long long n_hits, int* head, long long* heads,
                      long long* total, long long* scan_tmp, hipStream_t s) {
  hipError_t e = hipMemsetAsync(head, 0, sizeof(int) * (size_t)n_hits, s);
  if (e != hipSuccess) return e;
  k_traj_heads<<<blocks_for(n_traj), 256, 0, s>>>(offsets, n_traj, n_hits, head);
  return launch_scan(head, heads, n_hits, total, scan_tmp, s);
}

}  // namespace

hipError_t launch_order_setup(int n, const int64_t* dims_with_t, const long long* face_id, const long long* label,
                              long long n_hits, const long long* roots, const unsigned long long* n_points,
                              const int* n_ends, long long n_traj, int* nb, unsigned* seg, unsigned char* is_ruler,
                              int* rid, int* list, long long* bstart, long long* rb, int* flag, long long* off,
                              long long* n_rulers, int* cnt, long long* offsets, long long* scan_tmp, unsigned* status,
                              hipStream_t s) {
  const FaceSpace fs = make_space(n, dims_with_t);
  k_count_to_int<<<blocks_for(n_traj), 256, 0, s>>>(n_points, n_traj, cnt);
  hipError_t e = launch_scan(cnt, offsets, n_traj, offsets + n_traj, scan_tmp, s);
  if (e != hipSuccess || n_hits == 0) return e;
  e = hipMemsetAsync(seg, 0xff, sizeof(uint2) * 2 * (size_t)n_hits, s);
  if (e != hipSuccess) return e;
  const long long nbk = row_buckets(n, dims_with_t), B = fs.T * fs.N[0];
  long long hB;
  const long long hbk = hit_buckets(n, dims_with_t, n_hits, &hB);
  k_gapfill<<<blocks_for(n_hits + 1), 256, 0, s>>>(face_id, n_hits, hB, hbk, bstart);
  k_buckets<<<blocks_for(nbk + 1), 256, 0, s>>>(roots, n_traj, B, nbk, rb);
  k_neighbours<<<blocks_for(n_hits), 256, 0, s>>>(fs, face_id, n_hits, bstart, hB, hbk, (int2*)nb, status);
  k_cut_loops<<<blocks_for(n_hits), 256, 0, s>>>(face_id, label, n_hits, roots, rb, B, nbk, n_ends, (int2*)nb);
  k_ruler_flags<<<blocks_for(n_hits), 256, 0, s>>>((const int2*)nb, n_hits, is_ruler, flag);
  e = launch_scan(flag, off, n_hits, n_rulers, scan_tmp, s);
  if (e != hipSuccess) return e;
  k_ruler_list<<<blocks_for(n_hits), 256, 0, s>>>(flag, off, n_hits, rid, list);
  return hipGetLastError();
}

hipError_t launch_order_walk(const int* nb, const unsigned char* is_ruler, const int* list, long long n_rulers,
                             long long n_hits, unsigned* seg, int* st, unsigned* status, hipStream_t s) {
  if (n_rulers == 0) return hipSuccess;
  k_walk<<<blocks_for(2 * n_rulers), 256, 0, s>>>((const int2*)nb, list, n_rulers, n_hits, (uint2*)seg, status);
  k_rinit<<<blocks_for(2 * n_rulers), 256, 0, s>>>((const int2*)nb, list, n_rulers, n_hits, (const uint2*)seg,
                                                   (int4*)st, status);
  return hipGetLastError();
}

hipError_t launch_order_jump(const int* nb, const int* rid, const int* act, long long n_act, long long n_hits,
                             const int* in, int* out, int* next, unsigned long long* next_n, unsigned* status,
                             hipStream_t s) {
  if (n_act == 0) return hipSuccess;
  k_rjump<<<blocks_for(n_act), 256, 0, s>>>((const int2*)nb, rid, act, n_act, n_hits, (const int4*)in, (int4*)out,
                                            next, next_n, status);
  return hipGetLastError();
}

hipError_t launch_order_place(int n, const int64_t* dims_with_t, const long long* label, long long n_hits,
                              const long long* roots, const long long* rb, const long long* offsets,
                              const unsigned char* is_ruler, const int* rid, const unsigned* seg, const int* st,
                              long long* order, unsigned* status, hipStream_t s) {
  if (n_hits == 0) return hipSuccess;
  const FaceSpace fs = make_space(n, dims_with_t);
  k_place<<<blocks_for(n_hits), 256, 0, s>>>(label, n_hits, roots, rb, fs.T * fs.N[0], row_buckets(n, dims_with_t),
                                             offsets, is_ruler, rid, (const uint2*)seg, (const int4*)st, order,
                                             status);
  return hipGetLastError();
}

hipError_t launch_smooth(const long long* order, const long long* offsets, const int* n_ends, long long n_traj,
                         long long n_hits, const uint8_t* type_in, int half, int* head, long long* heads,
                         long long* total, long long* scan_tmp, uint8_t* type_out, unsigned* status, hipStream_t s) {
  if (n_hits == 0) return hipSuccess;
  hipError_t e = walk_heads(offsets, n_traj, n_hits, head, heads, total, scan_tmp, s);
  if (e != hipSuccess) return e;
  k_smooth<<<blocks_for(n_hits), 256, 0, s>>>(make_walk(order, offsets, n_ends, n_traj, n_hits, head, heads), type_in,
                                              half, type_out, status);
  return hipGetLastError();
}

hipError_t launch_simplify(int n, const float* pos, const long long* order, const long long* offsets,
                           const int* n_ends, long long n_traj, long long n_hits, const uint8_t* type_in, float theta,
                           long long* rot, int* flag, long long* run_off, int* head, long long* heads,
                           long long* total, long long* scan_tmp, int* t_min, int* t_max, uint8_t* run_type,
                           uint8_t* new_type, uint8_t* type_out, unsigned* status, hipStream_t s) {
  if (n_hits == 0) return hipSuccess;
  hipError_t e = walk_heads(offsets, n_traj, n_hits, head, heads, total, scan_tmp, s);
  if (e != hipSuccess) return e;
  const Walk w = make_walk(order, offsets, n_ends, n_traj, n_hits, head, heads);
  const unsigned b = blocks_for(n_hits);
  k_rot_init<<<blocks_for(n_traj), 256, 0, s>>>(w, rot);
  k_rot_find<<<b, 256, 0, s>>>(w, type_in, rot, status);
  k_run_flags<<<b, 256, 0, s>>>(w, type_in, rot, flag, status);
  e = launch_scan(flag, run_off, n_hits, total, scan_tmp, s);
  if (e != hipSuccess) return e;
  k_run_init<<<b, 256, 0, s>>>(n_hits, t_min, t_max);
  k_run_stats<<<b, 256, 0, s>>>(w, n, pos, type_in, rot, flag, run_off, t_min, t_max, run_type, status);
  k_run_decide<<<b, 256, 0, s>>>(w, flag, run_off, t_min, t_max, run_type, theta, new_type);
  k_run_apply<<<b, 256, 0, s>>>(w, rot, flag, run_off, new_type, type_out, status);
  return hipGetLastError();
}

}  // namespace ftk
