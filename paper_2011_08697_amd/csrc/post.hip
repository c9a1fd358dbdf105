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

}  // namespace ftk
