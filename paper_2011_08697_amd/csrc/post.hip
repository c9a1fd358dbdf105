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
//   * Order of the points along each trajectory (cell neighbours, list ranking by pointer jumping), and the type
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
                             long long n_traj, unsigned long long* __restrict__ n_hits, int* __restrict__ t_min,
                             int* __restrict__ t_max, int* __restrict__ n_ends, unsigned* __restrict__ status) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long j = lower_bound64(roots, n_traj, label[i]);
  if (j >= n_traj || roots[j] != label[i]) {
    atomicOr(status, ST_INVARIANT);
    return;
  }
  const float t = pos[i * (fs.n + 1) + fs.n];
  atomicAdd(&n_hits[j], 1ull);
  atomicMin(&t_min[j], __float_as_int(t));
  atomicMax(&t_max[j], __float_as_int(t));
  if (face_on_boundary(fs, face_id[i])) atomicAdd(&n_ends[j], 1);
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

// index of face id v among the sorted hits, -1 if not punctured
__device__ __forceinline__ long long find_hit(const long long* face_id, long long n_hits, long long v) {
  const long long k = lower_bound64(face_id, n_hits, v);
  return (k < n_hits && face_id[k] == v) ? k : -1;
}

__global__ void k_neighbours(FaceSpace fs, const long long* __restrict__ face_id, long long n_hits,
                             long long* __restrict__ nb0, long long* __restrict__ nb1, unsigned* __restrict__ status) {
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
  long long found[2] = {-1, -1};
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
      const long long h = find_hit(face_id, n_hits, side);
      if (h >= 0) {
        ++hits_here;
        other = h;
      }
    }
    if (hits_here != 1) {
      bad = true;
      continue;
    }
    found[nf++] = other;
  }
  if (bad || nf == 0) atomicOr(status, ST_INVARIANT);
  if (nf == 2 && found[1] < found[0]) {
    const long long x = found[0];
    found[0] = found[1];
    found[1] = x;
  }
  nb0[i] = found[0];
  nb1[i] = found[1];
}

// A closed loop is cut between its label face (the root: smallest face id, so smallest index) and its neighbour
// with the larger face id; the walk then runs root, smaller neighbour, ..., larger neighbour.
__global__ void k_cut_loops(const long long* __restrict__ face_id, const long long* __restrict__ label,
                            long long n_hits, const long long* __restrict__ roots, long long n_traj,
                            const int* __restrict__ n_ends, long long* __restrict__ nb0, long long* __restrict__ nb1) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_hits || label[i] != face_id[i]) return;
  const long long j = lower_bound64(roots, n_traj, label[i]);
  if (j >= n_traj || roots[j] != label[i] || n_ends[j] != 0) return;
  const long long b = nb1[i];
  if (b < 0 || b >= n_hits) return;
  nb1[i] = -1;
  if (nb0[b] == i) nb0[b] = -1;
  if (nb1[b] == i) nb1[b] = -1;
}

// Pointer jumping over the (now open) paths.  Arm k of hit i walks away from i through nb_k: far = the node it
// has reached, prv = the node before far, dist = the steps taken, done once far has no neighbour further on.
struct Arms {
  long long* far[2];
  long long* prv[2];
  long long* dist[2];
  unsigned char* done[2];
};

__global__ void k_arms_init(const long long* __restrict__ nb0, const long long* __restrict__ nb1, long long n_hits,
                            Arms a) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_hits) return;
  for (int k = 0; k < 2; ++k) {
    const long long w = k == 0 ? nb0[i] : nb1[i];
    a.far[k][i] = w < 0 ? i : w;
    a.prv[k][i] = w < 0 ? -1 : i;
    a.dist[k][i] = w < 0 ? 0 : 1;
    a.done[k][i] = w < 0 ? 1 : 0;
  }
}

__global__ void k_arms_jump(const long long* __restrict__ nb0, const long long* __restrict__ nb1, long long n_hits,
                            Arms in, Arms out, unsigned long long* __restrict__ active,
                            unsigned* __restrict__ status) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_hits) return;
  int open = 0;
  for (int k = 0; k < 2; ++k) {
    long long f = in.far[k][i], p = in.prv[k][i], dd = in.dist[k][i];
    unsigned char dn = in.done[k][i];
    if (!dn) {
      // the arm of f that leads away from i starts at f's neighbour other than p
      const int kk = nb0[f] == p ? 1 : 0;
      const long long nxt = kk == 0 ? nb0[f] : nb1[f];
      if ((kk == 0 ? nb1[f] : nb0[f]) != p) {
        atomicOr(status, ST_INVARIANT);
        dn = 1;
      } else if (nxt < 0) {
        dn = 1;
      } else {
        const long long f2 = in.far[kk][f], p2 = in.prv[kk][f], d2 = in.dist[kk][f];
        const unsigned char dn2 = in.done[kk][f];
        f = f2;
        p = p2;
        dd += d2;
        dn = dn2;
        if (dd > n_hits) {  // a walk longer than the hit count can only be a cycle the cut did not open
          atomicOr(status, ST_INVARIANT);
          dn = 1;
        }
      }
      open |= dn ? 0 : 1;
    }
    out.far[k][i] = f;
    out.prv[k][i] = p;
    out.dist[k][i] = dd;
    out.done[k][i] = dn;
  }
  const unsigned long long bal = __ballot(open);
  if (bal && (threadIdx.x & 63) == __ffsll((long long)bal) - 1) atomicAdd(active, (unsigned long long)__popcll(bal));
}

__global__ void k_count_to_int(const unsigned long long* __restrict__ n_points, long long n_traj,
                               int* __restrict__ out) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n_traj) out[j] = (int)n_points[j];
}

// Position of each hit: trajectory start + distance to its start end (the end with the smaller index, i.e. the
// smaller face id); the path length through i must equal the trajectory's point count.
__global__ void k_place(const long long* __restrict__ label, long long n_hits, const long long* __restrict__ roots,
                        long long n_traj, const long long* __restrict__ offsets, Arms a, long long* __restrict__ order,
                        unsigned* __restrict__ status) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_hits) return;
  const long long j = lower_bound64(roots, n_traj, label[i]);
  if (j >= n_traj || roots[j] != label[i]) {
    atomicOr(status, ST_INVARIANT);
    return;
  }
  const long long e0 = a.far[0][i], e1 = a.far[1][i];
  const long long len = a.dist[0][i] + a.dist[1][i] + 1;
  const long long rank = e0 < e1 ? a.dist[0][i] : a.dist[1][i];
  const long long lo = offsets[j], hi = offsets[j + 1];
  if (len != hi - lo || rank < 0 || rank >= len) {
    atomicOr(status, ST_INVARIANT);
    return;
  }
  order[lo + rank] = i;
}

// ---------------------------------------------------------------------------------------------------------------
// Type smoothing and run simplification along the order (Sec. 4.4).  Position k of order[] belongs to trajectory
// j with offsets[j] <= k < offsets[j + 1]; a trajectory without ends is a closed loop.
// ---------------------------------------------------------------------------------------------------------------

struct Walk {
  const long long* order;
  const long long* offsets;
  const int* n_ends;
  long long n_traj, n_hits;
};

// trajectory of position k, its start and length; false (and the invariant flag) for inconsistent offsets
__device__ __forceinline__ bool locate(const Walk& w, long long k, long long* j, long long* lo, long long* m) {
  // last j with offsets[j] <= k
  long long a = 0, b = w.n_traj;
  while (a < b) {
    const long long mid = (a + b + 1) >> 1;
    if (w.offsets[mid] <= k)
      a = mid;
    else
      b = mid - 1;
  }
  *j = a;
  *lo = w.offsets[a];
  *m = (a < w.n_traj ? w.offsets[a + 1] : w.n_hits) - *lo;
  return a < w.n_traj && *lo >= 0 && *m > 0 && *lo + *m <= w.n_hits && k >= *lo && k < *lo + *m;
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
  if (q >= w.n_hits) return;
  long long j, lo, m;
  if (!locate(w, q, &j, &lo, &m)) return;
  const long long h = hit_at(w, rotated(w, rot, j, lo, m, q), status);
  if (h < 0) return;
  const long long run = run_off[q] + flag[q] - 1;
  if (run < 0 || run >= w.n_hits) {
    atomicOr(status, ST_INVARIANT);
    return;
  }
  const int tb = __float_as_int(pos[h * (n + 1) + n]);
  atomicMin(&t_min[run], tb);
  atomicMax(&t_max[run], tb);
  if (flag[q]) run_type[run] = type_in[h];
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

hipError_t launch_traj_table(int n, const int64_t* dims_with_t, const long long* face_id, const long long* label,
                             const float* pos, long long n_hits, long long n_traj, int* flag, long long* off,
                             long long* scan_total, long long* scan_tmp, long long* roots,
                             unsigned long long* hits, int* t_min, int* t_max, int* n_ends, unsigned* status,
                             hipStream_t s) {
  const FaceSpace fs = make_space(n, dims_with_t);
  k_traj_init<<<blocks_for(n_traj), 256, 0, s>>>(n_traj, hits, t_min, t_max, n_ends);
  if (n_hits == 0) return hipGetLastError();
  k_root_flags<<<blocks_for(n_hits), 256, 0, s>>>(face_id, label, n_hits, flag);
  hipError_t e = launch_scan(flag, off, n_hits, scan_total, scan_tmp, s);
  if (e != hipSuccess) return e;
  k_root_scatter<<<blocks_for(n_hits), 256, 0, s>>>(face_id, flag, off, n_hits, n_traj, roots, status);
  k_traj_accum<<<blocks_for(n_hits), 256, 0, s>>>(fs, face_id, label, pos, n_hits, roots, n_traj, hits, t_min, t_max,
                                                   n_ends, status);
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

// The pointer-jumping state lives in two buffers (double buffering across rounds) of 2 arms x (far, prv, dist)
// int64 arrays plus 2 done-byte arrays each.
Arms arms_view(long long* ws, unsigned char* dws, long long n, int buf) {
  Arms a;
  for (int k = 0; k < 2; ++k) {
    long long* base = ws + (long long)((buf * 2 + k) * 3) * n;
    a.far[k] = base;
    a.prv[k] = base + n;
    a.dist[k] = base + 2 * n;
    a.done[k] = dws + (long long)(buf * 2 + k) * n;
  }
  return a;
}

Walk make_walk(const long long* order, const long long* offsets, const int* n_ends, long long n_traj,
               long long n_hits) {
  Walk w;
  w.order = order;
  w.offsets = offsets;
  w.n_ends = n_ends;
  w.n_traj = n_traj;
  w.n_hits = n_hits;
  return w;
}

}  // namespace

hipError_t launch_order_setup(int n, const int64_t* dims_with_t, const long long* face_id, const long long* label,
                              long long n_hits, const long long* roots, const unsigned long long* n_points,
                              const int* n_ends, long long n_traj, long long* nb0, long long* nb1, long long* ws,
                              unsigned char* dws, int* cnt, long long* offsets, long long* scan_tmp,
                              unsigned* status, hipStream_t s) {
  const FaceSpace fs = make_space(n, dims_with_t);
  k_count_to_int<<<blocks_for(n_traj), 256, 0, s>>>(n_points, n_traj, cnt);
  hipError_t e = launch_scan(cnt, offsets, n_traj, offsets + n_traj, scan_tmp, s);
  if (e != hipSuccess || n_hits == 0) return e;
  k_neighbours<<<blocks_for(n_hits), 256, 0, s>>>(fs, face_id, n_hits, nb0, nb1, status);
  k_cut_loops<<<blocks_for(n_hits), 256, 0, s>>>(face_id, label, n_hits, roots, n_traj, n_ends, nb0, nb1);
  k_arms_init<<<blocks_for(n_hits), 256, 0, s>>>(nb0, nb1, n_hits, arms_view(ws, dws, n_hits, 0));
  return hipGetLastError();
}

hipError_t launch_order_jump(const long long* nb0, const long long* nb1, long long n_hits, long long* ws,
                             unsigned char* dws, int from, unsigned long long* active, unsigned* status,
                             hipStream_t s) {
  k_arms_jump<<<blocks_for(n_hits), 256, 0, s>>>(nb0, nb1, n_hits, arms_view(ws, dws, n_hits, from),
                                                 arms_view(ws, dws, n_hits, 1 - from), active, status);
  return hipGetLastError();
}

hipError_t launch_order_place(const long long* label, long long n_hits, const long long* roots, long long n_traj,
                              const long long* offsets, long long* ws, unsigned char* dws, int buf,
                              long long* order, unsigned* status, hipStream_t s) {
  k_place<<<blocks_for(n_hits), 256, 0, s>>>(label, n_hits, roots, n_traj, offsets,
                                             arms_view(ws, dws, n_hits, buf), order, status);
  return hipGetLastError();
}

hipError_t launch_smooth(const long long* order, const long long* offsets, const int* n_ends, long long n_traj,
                         long long n_hits, const uint8_t* type_in, int half, uint8_t* type_out, unsigned* status,
                         hipStream_t s) {
  if (n_hits == 0) return hipSuccess;
  k_smooth<<<blocks_for(n_hits), 256, 0, s>>>(make_walk(order, offsets, n_ends, n_traj, n_hits), type_in, half,
                                              type_out, status);
  return hipGetLastError();
}

hipError_t launch_simplify(int n, const float* pos, const long long* order, const long long* offsets,
                           const int* n_ends, long long n_traj, long long n_hits, const uint8_t* type_in, float theta,
                           long long* rot, int* flag, long long* run_off, long long* total, long long* scan_tmp,
                           int* t_min, int* t_max, uint8_t* run_type, uint8_t* new_type, uint8_t* type_out,
                           unsigned* status, hipStream_t s) {
  if (n_hits == 0) return hipSuccess;
  const Walk w = make_walk(order, offsets, n_ends, n_traj, n_hits);
  const unsigned b = blocks_for(n_hits);
  k_rot_init<<<blocks_for(n_traj), 256, 0, s>>>(w, rot);
  k_rot_find<<<b, 256, 0, s>>>(w, type_in, rot, status);
  k_run_flags<<<b, 256, 0, s>>>(w, type_in, rot, flag, status);
  hipError_t e = launch_scan(flag, run_off, n_hits, total, scan_tmp, s);
  if (e != hipSuccess) return e;
  k_run_init<<<b, 256, 0, s>>>(n_hits, t_min, t_max);
  k_run_stats<<<b, 256, 0, s>>>(w, n, pos, type_in, rot, flag, run_off, t_min, t_max, run_type, status);
  k_run_decide<<<b, 256, 0, s>>>(w, flag, run_off, t_min, t_max, run_type, theta, new_type);
  k_run_apply<<<b, 256, 0, s>>>(w, rot, flag, run_off, new_type, type_out, status);
  return hipGetLastError();
}

}  // namespace ftk
