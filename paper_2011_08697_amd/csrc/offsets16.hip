// offsets16.hip -- group sums and bases of per-element byte counts (see offsets16.h).
#include "internal.h"
#include "offsets16.h"

namespace ftk {

namespace {

__global__ void group16_sums(const unsigned char* __restrict__ cnt, long long n, int* __restrict__ gsum,
                             bool nonzero) {
  const long long gi = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long g0 = gi * 16;
  if (g0 >= n) return;
  const long long rest = n - g0;
  gsum[gi] = (int)sum_first(*reinterpret_cast<const uint4*>(cnt + g0), rest < 16 ? (int)rest : 16, nonzero);
}

}  // namespace

hipError_t launch_group16_bases(const unsigned char* cnt, long long n, bool nonzero, int* gsum, long long* base,
                                long long* total, long long* scan_tmp, hipStream_t s) {
  const long long groups = (n + 15) / 16;
  if (groups > 0) group16_sums<<<(unsigned)((groups + 255) / 256), 256, 0, s>>>(cnt, n, gsum, nonzero);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_scan(gsum, base, groups, total, scan_tmp, s);
}

}  // namespace ftk
