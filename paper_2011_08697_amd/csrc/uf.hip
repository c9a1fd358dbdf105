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

// Fixed-slot links (the sparse emission's): (a, a) marks an empty slot.
__global__ __launch_bounds__(256) void uf_hook_slots(unsigned* __restrict__ parent, const uint2* __restrict__ slots,
                                                     long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const uint2 e = slots[i];
    if (e.x != e.y) uf_unite(parent, e.x, e.y);
  }
}

// Compression of a forest whose parents point to smaller indices (parent[i] <= i), in one pass: workgroup b takes
// hits [256 b, 256 b + 256).  A hit whose parent lies in an earlier range takes that parent's root (a short walk:
// workgroups are dispatched in increasing order, so the earlier range is mostly compressed already; the walk is
// capped, any ancestor being a valid parent), then pointer jumping inside the range in LDS points every hit at a
// root or at such an earlier ancestor.  Agent-scope accesses make the earlier ranges' writes visible across XCDs.
__global__ __launch_bounds__(256) void uf_compress(unsigned* __restrict__ parent, long long n) {
  __shared__ unsigned lp[2][256];
  const long long bs = (long long)blockIdx.x * 256;
  const long long i = bs + threadIdx.x;
  unsigned p = (unsigned)i;
  if (i < n) {
    p = uf_load(parent, (unsigned)i);
    if ((long long)p < bs) {
      for (int k = 0; k < 8; ++k) {
        const unsigned q = uf_load(parent, p);
        if (q == p) break;
        p = q;
      }
    }
  }
  lp[0][threadIdx.x] = p;
  __syncthreads();
  int cur = 0;
#pragma unroll
  for (int r = 0; r < 8; ++r) {  // 2^8 = 256: every in-range chain is resolved
    const unsigned v = lp[cur][threadIdx.x];
    const unsigned w = ((long long)v >= bs && (long long)v < bs + 256) ? lp[cur][v - bs] : v;
    lp[cur ^ 1][threadIdx.x] = w;
    cur ^= 1;
    __syncthreads();
  }
  if (i < n) __hip_atomic_store(parent + i, lp[cur][threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

hipError_t launch_uf_compress(unsigned* parent, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long blocks = (n + 255) / 256;
  if (blocks > 0x7FFFFFFFLL) return hipErrorInvalidValue;
  uf_compress<<<(unsigned)blocks, 256, 0, s>>>(parent, n);
  return hipGetLastError();
}

hipError_t launch_uf_hook_slots(unsigned* parent, const uint2* slots, long long n_slots, hipStream_t s) {
  if (n_slots <= 0) return hipSuccess;
  long long blocks = (n_slots + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  uf_hook_slots<<<(unsigned)blocks, 256, 0, s>>>(parent, slots, n_slots);
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
