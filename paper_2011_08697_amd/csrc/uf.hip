// uf.hip -- GPU union-find for trajectory stitching (Alg. 1 pass 2: unite the punctured sides of every cell).
//
// The emission kernels unite the links inside each tile (and, through the parents of earlier chunks, along time
// within the tile's slab) and leave every hit's parent pointing at a smaller hit of its set; links that cross
// tiles or slabs are queued, and are united here with compare-and-swap hooking (larger root under smaller root).
// Labels are the face id of each set's root, i.e. the smallest face id of the trajectory.
#include "common.h"
#include "internal.h"

namespace ftk {

namespace {

__global__ __launch_bounds__(256) void uf_hook(unsigned* __restrict__ parent, const uint2* __restrict__ work,
                                               const unsigned long long* __restrict__ work_count) {
  const unsigned long long n = *work_count;
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * blockDim.x) {
    uint2 e = work[i];
    uf_unite(parent, e.x, e.y);
  }
}

// grid-stride; one trajectory-count atomic per block
__global__ __launch_bounds__(256) void uf_label(unsigned* __restrict__ parent, const long long* __restrict__ face_id,
                                                long long* __restrict__ label, long long n,
                                                unsigned long long* __restrict__ cnt) {
  __shared__ unsigned long long red[4];
  unsigned long long roots = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    unsigned r = uf_find_plain(parent, (unsigned)i);
    if (label) label[i] = face_id[r];
    roots += (r == (unsigned)i);
  }
  roots = wave_sum64(roots);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = roots;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = red[0] + red[1] + red[2] + red[3];
    if (s) atomicAdd(&cnt[CNT_TRAJ], s);
  }
}

// Batched labels: the series of hit i by binary search over the series' first global indices (in LDS).
__global__ __launch_bounds__(256) void uf_label_batched(unsigned* __restrict__ parent, const Series2* __restrict__ S,
                                                        const unsigned* __restrict__ gbase, int nser, long long n) {
  extern __shared__ unsigned s_base[];
  for (int i = threadIdx.x; i <= nser; i += blockDim.x) s_base[i] = gbase[i];
  __syncthreads();
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    int lo = 0, hi = nser;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_base[mid] <= (unsigned)i)
        lo = mid;
      else
        hi = mid;
    }
    const unsigned b = s_base[lo];
    const unsigned r = uf_find_plain(parent, (unsigned)i);
    const Out2& o = S[lo].o;
    if (o.label) o.label[i - b] = o.face_id[r - b];
    if (r == (unsigned)i) atomicAdd(&S[lo].cnt[CNT_TRAJ], 1ull);
  }
}

}  // namespace

hipError_t launch_uf_label_batched(unsigned* parent, const Series2* S, const unsigned* gbase, int nser, long long n,
                                   hipStream_t s) {
  if (n <= 0) return hipSuccess;
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  uf_label_batched<<<(unsigned)blocks, 256, (nser + 1) * sizeof(unsigned), s>>>(parent, S, gbase, nser, n);
  return hipGetLastError();
}

hipError_t launch_uf_hook(unsigned* parent, const uint2* work, const unsigned long long* work_count,
                          long long max_work, hipStream_t s) {
  long long blocks = (max_work + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  uf_hook<<<(unsigned)blocks, 256, 0, s>>>(parent, work, work_count);
  return hipGetLastError();
}

hipError_t launch_uf_label(unsigned* parent, const long long* face_id, long long* label, long long n,
                           unsigned long long* cnt, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  long long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  uf_label<<<(unsigned)blocks, 256, 0, s>>>(parent, face_id, label, n, cnt);
  return hipGetLastError();
}

}  // namespace ftk
