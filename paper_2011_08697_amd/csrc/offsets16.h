// offsets16.h -- offsets of per-element byte counts without a full-length int64 scan (isovolume and extruded-mesh
// passes, whose counts are sparse bytes): one int64 base per group of 16 elements (the exclusive scan of the groups'
// byte sums, n / 16 entries) and, at lookup, the counts of the element's earlier group members summed from one
// 16-byte load.  Count arrays are allocated to a multiple of 16 bytes; bytes at or past n are never summed.
#pragma once
#include <hip/hip_runtime.h>

namespace ftk {

// Sum of the first k (0..16) bytes of a group; nonzero: the number of nonzero bytes among them.
__device__ __forceinline__ unsigned sum_first(const uint4 q, int k, bool nonzero) {
  const unsigned w[4] = {q.x, q.y, q.z, q.w};
  unsigned s = 0;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const int nb = k - 4 * d;  // bytes of word d that are counted
    unsigned x = nb >= 4 ? w[d] : (nb <= 0 ? 0u : (w[d] & ((1u << (8 * nb)) - 1u)));
    if (nonzero) x = ((((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x) & 0x80808080u) >> 7;  // 1 per nonzero byte
    s = __builtin_amdgcn_sad_u8(x, 0u, s);  // + sum of the four bytes
  }
  return s;
}

// Offset of element v: base of its group + counts of its earlier group members.
__device__ __forceinline__ long long off16(const long long* __restrict__ base, const unsigned char* __restrict__ cnt,
                                           long long v, bool nonzero) {
  const long long g0 = v & ~15ll;
  return base[v >> 4] + sum_first(*reinterpret_cast<const uint4*>(cnt + g0), (int)(v - g0), nonzero);
}

// base[g] for the n byte counts cnt (nonzero: of the nonzero counts); gsum, base: ceil(n / 16) entries; *total: the
// sum of all; scan_tmp: scan_tmp_elems(ceil(n / 16)).
hipError_t launch_group16_bases(const unsigned char* cnt, long long n, bool nonzero, int* gsum, long long* base,
                                long long* total, long long* scan_tmp, hipStream_t s);

}  // namespace ftk
