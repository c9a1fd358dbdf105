// common.h -- device building blocks shared by the 2D and 3D kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kuhn.h"

namespace ftk {

typedef __int128 i128;

// Device status bits (one word per call).
enum : unsigned {
  ST_NONFINITE = 1u,  // NaN/Inf in the input
  ST_WIDE = 2u,       // a quantised component outside the narrow (32-bit or 21-bit) range: rerun the wide path
  ST_RANGE = 4u,      // a quantised component beyond the exact-arithmetic bound
  ST_INVARIANT = 8u,  // a cell with a punctured-side count other than 0 or 2
};

// Device counters (int64 each).
enum { CNT_FP64 = 0, CNT_DEGEN = 1, CNT_LINKED = 2, CNT_WORK = 3, CNT_TRAJ = 4, CNT_LIST = 5, CNT_N = 8 };

// Hit flags.
enum : unsigned { FL_DEGENERATE = 1u, FL_FP64 = 2u, FL_WIDE = 4u };

// Critical-point types.
enum : int { T_DEG = 0, T_MIN, T_MAX, T_SADDLE, T_SADDLE1, T_SADDLE2, T_SOURCE, T_SINK, T_RFOCUS, T_AFOCUS,
             T_CENTER };

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Workgroups go to the 8 XCDs round-robin by linear id.  This maps a linear id to a logical tile index so that each
// XCD takes a contiguous range of tiles: neighbouring tiles then share that XCD's L2 and fetch their common halo
// once.  A bijection on [0, nb) (ids past the last multiple of 8 map to themselves).  Used by the 3D detection,
// whose field halos triple its reads otherwise; the 2D kernels keep the interleaved order, under which they ran
// faster (their concurrent tiles then spread over more memory channels).
__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned nb) {
  const unsigned per = nb / 8u;
  return b < per * 8u ? (b % 8u) * per + b / 8u : b;
}

// Inclusive prefix sum over the 64 lanes with DPP moves (all lanes active): shifts by 1, 2, 4, 8 inside each row
// of 16 lanes (lanes without a source add 0), then lane 15 of each row added to the next row and lane 31 to
// rows 2 and 3.
__device__ __forceinline__ unsigned wave_incl_scan(unsigned v) {
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

// Sum over the 64 lanes (all lanes active), returned on every lane.
__device__ __forceinline__ unsigned wave_sum(unsigned v) {
  return (unsigned)__builtin_amdgcn_readlane((int)wave_incl_scan(v), 63);
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// ---------------------------------------------------------------------------------------------------------------
// Stencils (Sec. 4.3 central differences; one-sided at the first and last index).  Binary32, fixed order; the
// library is compiled without floating-point contraction, so these are bit-reproducible.
// ---------------------------------------------------------------------------------------------------------------
// Branch-free: at the first index (hi - mid), at the last (mid - lo), inside (hi - lo) * 0.5 -- the same binary32
// operations as the three-way definition, so every kernel computes bit-identical values.
__device__ __forceinline__ float diff3(float lo, float mid, float hi, int i, int N) {
  const bool first = (i == 0), last = (i == N - 1);
  const float a = first ? mid : lo;
  const float b = last ? mid : hi;
  const float d = b - a;
  return (first || last) ? d : d * 0.5f;
}

// Quantisation to the integer lattice: round half to even of v * 2^s (exact scaling).  Returns the rounded value
// as float; the caller range-checks it before conversion.
__device__ __forceinline__ float quant(float v, float scale) { return rintf(v * scale); }

// ---------------------------------------------------------------------------------------------------------------
// Simulation of Simplicity for the 2x2 determinant of columns A (lower vertex index) and B.  Each entry (j, k)
// carries eps^(2^(2k+j)); the perturbed determinant is
//   (A0 B1 - A1 B0) + B1 e^1 - B0 e^2 - A1 e^4 - e^6 + A0 e^8 + e^9,
// so its sign is that of the first nonzero of (det, B1, -B0, -A1, -1).  Returned as a bit: 1 for positive.
// ---------------------------------------------------------------------------------------------------------------
template <typename Q>
__device__ __forceinline__ unsigned sos2_positive(Q a0, Q a1, Q b0, Q b1);

// Narrow path: components are integers below 2^24 carried in binary32 (exactly).  Both products are integers below
// 2^48 and their difference is below 2^49, so the binary64 evaluation below is the exact integer determinant.
template <>
__device__ __forceinline__ unsigned sos2_positive<float>(float a0, float a1, float b0, float b1) {
  const double p = (double)a1 * (double)b0;
  const double d = __builtin_fma((double)a0, (double)b1, -p);
  const unsigned r = d > 0.0;
  const unsigned seq = (b1 != 0.0f) ? (b1 > 0.0f) : ((b0 != 0.0f) ? (b0 < 0.0f) : ((a1 != 0.0f) ? (a1 < 0.0f) : 0u));
  return d != 0.0 ? r : seq;
}

// The same on values already converted to binary64 (exact integers below 2^24).
__device__ __forceinline__ unsigned sos2_positive_d(double a0, double a1, double b0, double b1) {
  const double d = __builtin_fma(a0, b1, -(a1 * b0));
  const unsigned seq = (b1 != 0.0) ? (b1 > 0.0) : ((b0 != 0.0) ? (b0 < 0.0) : ((a1 != 0.0) ? (a1 < 0.0) : 0u));
  return d != 0.0 ? (unsigned)(d > 0.0) : seq;
}

// Wide path: 64-bit components below 2^62, 128-bit products.
template <>
__device__ __forceinline__ unsigned sos2_positive<long long>(long long a0, long long a1, long long b0, long long b1) {
  i128 d = (i128)a0 * b1 - (i128)a1 * b0;
  if (d != 0) return d > 0;
  if (b1 != 0) return b1 > 0;
  if (b0 != 0) return b0 < 0;
  if (a1 != 0) return a1 < 0;
  return 0u;
}

// ---------------------------------------------------------------------------------------------------------------
// Classification (Sec. 4.1): types from the spatial Jacobian interpolated at the zero, J_c = sum mu_i J(v_i).
// Reference semantics are binary64 in a fixed order; the FP32 evaluation is accepted only when every sign it
// decides is certified: |value32| > E32 + E64, where E32 and E64 bound the distance of the binary32 and binary64
// evaluations from the exact value.  mu32 carries at most 5u of relative error (conversions of C_i and D, a 1-ulp
// hardware reciprocal, one product), the interpolation three more roundings: the entry bound 10u * sum mu |J_i|
// covers both with margin (u = 2^-24; the binary64 side uses u = 2^-53).
// ---------------------------------------------------------------------------------------------------------------
constexpr float kU32 = 5.9604645e-08f;  // 2^-24
constexpr float kU64 = 1.1102230e-16f;  // 2^-53

// Exact-arithmetic reference rules on a binary64 matrix (row a = component, column b = derivative axis).
__device__ __forceinline__ int classify2_rule_grad(double det, double tr) {
  if (det < 0) return T_SADDLE;
  if (det > 0 && tr < 0) return T_MAX;
  if (det > 0 && tr > 0) return T_MIN;
  return T_DEG;
}

__device__ __forceinline__ int classify2_rule_vec(double det, double tr, double disc) {
  if (det < 0) return T_SADDLE;
  if (det == 0) return T_DEG;
  if (tr == 0) return T_CENTER;
  if (tr < 0) return (disc >= 0) ? T_SINK : T_AFOCUS;
  return (disc >= 0) ? T_SOURCE : T_RFOCUS;
}

// Binary64 evaluation in the reference order: J_c entries as ((mu0 J0 + mu1 J1) + mu2 J2), det = J00 J11 - J01 J10,
// tr = J00 + J11, disc = tr tr - 4 det.
__device__ __forceinline__ int classify2_fp64(const double mu[3], const float J[3][4], bool vector) {
  double Jc[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    double s = mu[0] * (double)J[0][e];
    s = s + mu[1] * (double)J[1][e];
    s = s + mu[2] * (double)J[2][e];
    Jc[e] = s;
  }
  double p1 = Jc[0] * Jc[3];
  double p2 = Jc[1] * Jc[2];
  double det = p1 - p2;
  double tr = Jc[0] + Jc[3];
  if (!vector) return classify2_rule_grad(det, tr);
  double t2 = tr * tr;
  double d4 = 4.0 * det;
  return classify2_rule_vec(det, tr, t2 - d4);
}

// Bound on |fl(fl(a d) - fl(b c)) - (a d - b c)_exact| given magnitude bounds A..D (valid for evaluated and exact
// entries) and entry error bounds ea..ed, unit roundoff u.
__device__ __forceinline__ float bound_det2(float A, float B, float C, float D, float ea, float eb, float ec,
                                            float ed, float u) {
  return (A * ed + D * ea + B * ec + C * eb + u * 2.01f * (A * D + B * C)) * 1.01f;
}

// FP32 evaluation with certification.  Returns the type, or -1 when the FP32 decision is not certified.
__device__ __forceinline__ int classify2_fp32(const float mu[3], const float J[3][4], bool vector) {
  float Jc[4], S[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    float s = mu[0] * J[0][e];
    s = s + mu[1] * J[1][e];
    s = s + mu[2] * J[2][e];
    Jc[e] = s;
    float a = mu[0] * fabsf(J[0][e]);
    a = a + mu[1] * fabsf(J[1][e]);
    a = a + mu[2] * fabsf(J[2][e]);
    S[e] = a;
  }
  float smax = fmaxf(fmaxf(S[0], S[1]), fmaxf(S[2], S[3]));
  if (!(smax > 1e-15f) || !(smax < 1e15f)) return -1;  // keep the bounds away from under/overflow
  // One bound covers both evaluations: with e >= e32 + e64, M = |Jc| + e (>= the magnitudes of the binary32,
  // binary64 and exact entries) and u >= u32 + u64, bound_det2 dominates the sum of the two separate bounds term
  // by term.  (u32 (1 + 1e-4) exceeds u32 + u64 = u32 (1 + 2^-29) with room for the rounding of the constants.)
  constexpr float kU = kU32 * 1.0001f, kE = 10.0f * kU;
  float e[4], M[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    e[q] = kE * S[q];
    M[q] = fabsf(Jc[q]) + e[q];
  }
  float p1 = Jc[0] * Jc[3];
  float p2 = Jc[1] * Jc[2];
  float det = p1 - p2;
  float Edet = bound_det2(M[0], M[1], M[2], M[3], e[0], e[1], e[2], e[3], kU);
  float tr = Jc[0] + Jc[3];
  float Etr = (e[0] + e[3] + kU * (M[0] + M[3])) * 1.01f;
  bool det_ok = fabsf(det) > Edet;
  bool tr_ok = fabsf(tr) > Etr;
  if (!det_ok) return -1;
  if (det < 0) return T_SADDLE;
  if (!tr_ok) return -1;
  if (!vector) return tr < 0 ? T_MAX : T_MIN;
  float T = fabsf(tr) + Etr, Dm = fabsf(det) + Edet;
  float t2 = tr * tr;
  float d4 = 4.0f * det;
  float disc = t2 - d4;
  // the discriminant's bound for the two evaluations, summed (Etr and Edet already cover both)
  float Edisc = (2.0f * (2.0f * T * Etr + 4.0f * Edet) + kU * (2.02f * T * T + 4.02f * Dm)) * 1.01f;
  if (!(fabsf(disc) > Edisc)) return -1;
  if (tr < 0) return disc >= 0 ? T_SINK : T_AFOCUS;
  return disc >= 0 ? T_SOURCE : T_RFOCUS;
}

// ---------------------------------------------------------------------------------------------------------------
// Union-find on hit indices (parent[i] <= i; the root of a set is its smallest index).
// ---------------------------------------------------------------------------------------------------------------
__device__ __forceinline__ unsigned uf_load(const unsigned* p, unsigned i) {
  return __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Find with path halving: every write replaces a parent by an ancestor, so concurrent finds stay correct.
__device__ __forceinline__ unsigned uf_find(unsigned* parent, unsigned x) {
  unsigned p = uf_load(parent, x);
  while (p != x) {
    unsigned gp = uf_load(parent, p);
    if (gp != p) __hip_atomic_store(parent + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = p;
    p = gp;
  }
  return x;
}

// Find without coherence traffic, for passes in which nothing else changes the forest: every stored parent is an
// ancestor, so plain (L2-cached) loads reach the root.
__device__ __forceinline__ unsigned uf_find_plain(const unsigned* __restrict__ parent, unsigned x) {
  unsigned p = parent[x];
  while (p != x) {
    x = p;
    p = parent[x];
  }
  return x;
}

__device__ __forceinline__ void uf_unite(unsigned* parent, unsigned a, unsigned b) {
  unsigned ra = uf_find(parent, a), rb = uf_find(parent, b);
  while (ra != rb) {
    if (ra < rb) {
      unsigned t = ra;
      ra = rb;
      rb = t;
    }
    // hook the larger root under the smaller one
    unsigned expected = ra;
    if (__hip_atomic_compare_exchange_strong(parent + ra, &expected, rb, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return;
    ra = uf_find(parent, expected);
    rb = uf_find(parent, rb);
  }
}

}  // namespace ftk
