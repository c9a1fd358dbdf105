// scan.hip -- exclusive prefix sum of per-segment hit counts (int32 or byte counts -> int64 offsets), the compaction
// step that gives every punctured simplex its position in the face-id-sorted output.
#include "common.h"
#include "internal.h"

namespace ftk {

namespace {
constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;

__device__ __forceinline__ long long block_excl_scan(long long v, long long* total) {
  __shared__ long long wsum[kThreads / kWave];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  long long x = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    long long o = __shfl_up(x, d, kWave);
    if (lane >= d) x += o;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  long long before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < kThreads / kWave; ++i) {
    if (i < w) before += wsum[i];
    all += wsum[i];
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void scan_reduce(const T* __restrict__ in, long long n,
                                                        long long* __restrict__ tmp) {
  const long long base = (long long)blockIdx.x * kTile + threadIdx.x * kItems;
  long long s = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i)
    if (base + i < n) s += in[base + i];
  long long tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) tmp[blockIdx.x] = tot;
}

// single block: tmp[0..nb) block sums -> exclusive offsets, total
__global__ __launch_bounds__(kThreads) void scan_blocks(long long* __restrict__ tmp, long long nb,
                                                        long long* __restrict__ total) {
  long long carry = 0;
  for (long long b0 = 0; b0 < nb; b0 += kThreads) {
    long long i = b0 + threadIdx.x;
    long long v = i < nb ? tmp[i] : 0;
    long long tot;
    long long ex = block_excl_scan(v, &tot);
    if (i < nb) tmp[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void scan_down(const T* __restrict__ in, long long* __restrict__ out,
                                                      long long n, const long long* __restrict__ tmp) {
  const long long base = (long long)blockIdx.x * kTile + threadIdx.x * kItems;
  int v[kItems];
  long long s = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0;
    s += v[i];
  }
  long long tot;
  long long run = tmp[blockIdx.x] + block_excl_scan(s, &tot);
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
}
}  // namespace

size_t scan_tmp_elems(long long n) { return (size_t)((n + kTile - 1) / kTile) + 1; }

namespace {
template <typename T>
hipError_t scan_any(const T* in, long long* out, long long n, long long* total, long long* tmp, hipStream_t s) {
  long long nb = (n + kTile - 1) / kTile;
  if (nb == 0) nb = 1;
  scan_reduce<T><<<(unsigned)nb, kThreads, 0, s>>>(in, n, tmp);
  scan_blocks<<<1, kThreads, 0, s>>>(tmp, nb, total);
  scan_down<T><<<(unsigned)nb, kThreads, 0, s>>>(in, out, n, tmp);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_scan(const int* in, long long* out, long long n, long long* total, long long* tmp, hipStream_t s) {
  return scan_any<int>(in, out, n, total, tmp, s);
}

hipError_t launch_scan_u8(const unsigned char* in, long long* out, long long n, long long* total, long long* tmp,
                          hipStream_t s) {
  return scan_any<unsigned char>(in, out, n, total, tmp, s);
}

}  // namespace ftk
