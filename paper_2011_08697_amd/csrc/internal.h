// internal.h -- host/device interface between the C ABI layer and the kernels (not installed).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ftk {

// 2D problem description passed by value to the kernels.
struct Grid2 {
  const float* f;
  int kind;       // 0 scalar, 1 vector (planar [t][2][y][x])
  int nx, ny, nt;
  int nxt;        // row segments per row: ceil(nx / 64)
  float qscale;   // 2^quant_log2
  int precision;  // 0 FP32 + certified FP64 fallback, 1 FP64
};

// 2D outputs (device pointers; pos/mu/type/flags may be null).
struct Out2 {
  long long* face_id;
  float* pos;
  float* mu;
  uint8_t* type;
  uint8_t* flags;
  unsigned* parent;  // union-find forest over hit indices
  uint2* work;       // extra union edges (hit, smaller partner)
};

// 3D problem description.
struct Grid3 {
  const float* f;
  int nx, ny, nz, nt;
  int nxt;
  float qscale;
  int precision;
};

struct Out3 {
  long long* face_id;
  float* pos;
  float* mu;
  uint8_t* type;
  uint8_t* flags;
  unsigned* parent;
  uint2* work;
};

hipError_t launch_detect2d(const Grid2& g, int ty, int tt, bool wide, uint16_t* masks, int* seg_cnt,
                           unsigned* status, hipStream_t s);
hipError_t launch_emit2d(const Grid2& g, bool wide, const uint16_t* masks, const long long* seg_off, long long nseg,
                         const Out2& o, unsigned* status, unsigned long long* cnt, hipStream_t s);

hipError_t launch_detect3d(const Grid3& g, int tt, bool wide, uint64_t* masks, int* seg_cnt, unsigned* status,
                           hipStream_t s);
hipError_t launch_emit3d(const Grid3& g, bool wide, const uint64_t* masks, const long long* seg_off, long long nseg,
                         const Out3& o, unsigned* status, unsigned long long* cnt, hipStream_t s);

// Exclusive scan of n int32 counts into int64 offsets; total written to *total (device).  tmp must hold
// scan_tmp_elems(n) int64 values.
size_t scan_tmp_elems(long long n);
hipError_t launch_scan(const int* in, long long* out, long long n, long long* total, long long* tmp, hipStream_t s);

// Union-find passes over n hits: extra unions from the work list, then labels = face_id of the root.
hipError_t launch_uf_hook(unsigned* parent, const uint2* work, const unsigned long long* work_count,
                          long long max_work, hipStream_t s);
hipError_t launch_uf_label(unsigned* parent, const long long* face_id, long long* label, long long n,
                           unsigned long long* cnt, hipStream_t s);

}  // namespace ftk
