// internal.h -- host/device interface between the C ABI layer and the kernels (not installed).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ftk {

// 2D problem description passed by value to the kernels.
struct Grid2 {
  const float* f;
  int kind;       // 0 scalar, 1 vector (planar [t][2][y][x])
  int nx, ny, nt; // nt: number of steps of the series (a large value while a stream is still open)
  int nxt;        // row segments per row: ceil(nx / 64)
  float qscale;   // 2^quant_log2
  int precision;  // 0 FP32 + certified FP64 fallback, 1 FP64
  int t_begin, t_end;  // anchors processed by a launch: steps [t_begin, t_end)
  int f_ring;     // field planes stored as a ring of f_ring steps (step t at slot t % f_ring); 0: plane t at t
  int m_ring;     // same for the puncture masks and the per-segment counts/offsets
  int debug;      // FTK_DEBUG_* test hooks (0 in normal use)
  int debug_step; // step at which FTK_DEBUG_INVARIANT reports a bad cell (-1: none)
};

// 2D outputs (device pointers; pos/mu/type/flags may be null).
struct Out2 {
  unsigned gbase;    // global hit index of this series' first hit (outputs are indexed by global - gbase)
  long long* face_id;
  float* pos;
  float* mu;
  uint8_t* type;
  uint8_t* flags;
  unsigned* parent;  // union-find forest over global hit indices
  uint2* work;       // union edges that leave a tile/chunk (global hit, smaller partner)
  long long* label;  // labels (read by the batched label pass)
};

// One series of a batched call (device copy read by the persistent kernels).
struct Series2 {
  Grid2 g;
  Out2 o;
  uint16_t* masks;
  int* seg_cnt;
  long long* seg_off;
  unsigned long long* cnt;  // per-series counters (CNT_*)
  int wide;
  int pad;
};

// 3D problem description.
struct Grid3 {
  const float* f;
  int nx, ny, nz, nt;  // nt: number of steps of the series (a large value while a stream is still open)
  int nxt;
  float qscale;
  int precision;
  int t_begin = 0, t_end = 0;  // anchors processed by a launch: steps [t_begin, t_end)
  int f_ring = 0;  // field steps stored as a ring of f_ring steps (step t at slot t % f_ring); 0: step t at t
  int m_ring = 0;  // same for the puncture masks and the per-segment counts/offsets
  // One byte per detection tile-step (16 x 8 x 4 anchors at one step; stored like the masks, ring slots included):
  // 1 when the sign certificate proved the tile-step empty, whose masks are then not written (read them as zero).
  unsigned char* cert = nullptr;
};
// Number of detection tiles per step (cert entries per plane).
inline long long cert3_plane(const Grid3& g) {
  return (long long)((g.nx + 15) / 16) * ((g.ny + 7) / 8) * ((g.nz + 3) / 4);
}

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
hipError_t launch_emit2d(const Grid2& g, bool wide, const uint16_t* masks, const int* seg_cnt,
                         const long long* seg_off, const Out2& o, unsigned* status, unsigned long long* cnt,
                         hipStream_t s);

// Sparse emission (one wavefront per non-empty row segment): same outputs as launch_emit2d, for fields with few hits
// per vertex.  The parents must hold 0xFFFFFFFF on entry; each hit writes its parent (its first smaller partner or
// an ancestor of it, or itself) and its link slot o.work[i] ((i, i) when absent), united by launch_uf_hook_slots.
hipError_t launch_emit2d_sparse(const Grid2& g, bool wide, const uint16_t* masks, const int* seg_cnt,
                                const long long* seg_off, const Out2& o, unsigned* status, unsigned long long* cnt,
                                hipStream_t s);
hipError_t launch_emit2d_sparse_batched(const Series2* S, const long long* bprefix, int nser, long long total_blocks,
                                        bool wide, unsigned* status, hipStream_t s);

hipError_t launch_emit2d_steps(const Grid2& g, bool wide, const uint16_t* masks, const int* seg_cnt,
                               const long long* seg_off, const Out2& o, unsigned* status, unsigned long long* cnt,
                               hipStream_t s);
hipError_t launch_detect2d_batched(const Series2* S, const int* prefix, int nser, int total_items, int tt, bool wide,
                                   int* counter, unsigned* status, hipStream_t s);
hipError_t launch_emit2d_batched(const Series2* S, const int* prefix, int nser, int total_items, bool wide,
                                 int* counter, unsigned* status, unsigned long long* work_cnt, hipStream_t s);
// Labels for concatenated series: hit i belongs to the series s with gbase[s] <= i < gbase[s+1].
hipError_t launch_uf_label_batched(unsigned* parent, const Series2* S, const unsigned* gbase, int nser, long long n,
                                   hipStream_t s);

hipError_t launch_detect3d(const Grid3& g, int tt, bool wide, uint64_t* masks, int* seg_cnt, unsigned* status,
                           hipStream_t s);
hipError_t launch_emit3d(const Grid3& g, bool wide, const uint64_t* masks, const int* seg_cnt,
                         const long long* seg_off, long long n_hits, const Out3& o, unsigned* status,
                         unsigned long long* cnt, long long* list, unsigned long long* list_n, hipStream_t s);

// Exclusive scan of n int32 counts into int64 offsets; total written to *total (device).  tmp must hold
// scan_tmp_elems(n) int64 values.
size_t scan_tmp_elems(long long n);
hipError_t launch_scan(const int* in, long long* out, long long n, long long* total, long long* tmp, hipStream_t s);
// the same over byte counts (per-vertex or per-face counts below 256)
hipError_t launch_scan_u8(const unsigned char* in, long long* out, long long n, long long* total, long long* tmp,
                          hipStream_t s);

// Trajectory post-processing (post.hip).
hipError_t launch_traj_table(int n, const int64_t* dims_with_t, const long long* face_id, const long long* label,
                             const float* pos, long long n_hits, long long n_traj, int* flag, long long* off,
                             long long* scan_total, long long* scan_tmp, long long* roots, long long* rb,
                             unsigned long long* hits, int* t_min, int* t_max, int* n_ends, unsigned* status,
                             hipStream_t s);
hipError_t launch_slice_range(int n, const int64_t* dims_with_t, const long long* face_id, long long n_hits,
                              long long t0, long long* range, hipStream_t s);
hipError_t launch_slice_compact(int n, const int64_t* dims_with_t, const long long* face_id, long long lo,
                                long long cnt, int* flag, long long* off, long long* total, long long* tmp,
                                long long* idx_out, bool scatter, hipStream_t s);
hipError_t launch_filter_loops(const long long* label, long long n_hits, const long long* roots, long long n_traj,
                               const int* t_min, const int* t_max, const int* n_ends, float min_duration,
                               uint8_t* keep, hipStream_t s);

// Order of the points along each trajectory.  setup: per-trajectory offsets (offsets[n_traj] = n_hits), cell
// neighbours nb ([n_hits][2] int32), loop cuts, rulers (is_ruler, rid = slot in list, *n_rulers = count); seg
// ([n_hits][2] x 2 uint32) is cleared.  walk: ruler-to-ruler walks filling seg, ruler states st ([n_rulers][2] x 4
// int32).  jump: one pointer-jumping round over the listed rulers (act = null: all), still-open ones appended to
// next.  place: order[] from the rulers' final states.
hipError_t launch_order_setup(int n, const int64_t* dims_with_t, const long long* face_id, const long long* label,
                              long long n_hits, const long long* roots, const unsigned long long* n_points,
                              const int* n_ends, long long n_traj, int* nb, unsigned* seg, unsigned char* is_ruler,
                              int* rid, int* list, long long* bstart, long long* rb, int* flag, long long* off,
                              long long* n_rulers, int* cnt, long long* offsets, long long* scan_tmp, unsigned* status,
                              hipStream_t s);
// Number of vertex rows of the grid: the sorted hit and label lookups of the post-processing bucket their face ids
// by row, so their bucket tables (bstart, rb) need row_buckets() + 1 entries.
long long row_buckets(int n, const int64_t* dims_with_t);
// Buckets of the hit lookup of the ordering: one per vertex when the hits are dense (at least one per 16 vertices),
// else one per row; *B = face ids per bucket.  bstart needs the returned count + 1 entries.
long long hit_buckets(int n, const int64_t* dims_with_t, long long n_hits, long long* B);
hipError_t launch_order_walk(const int* nb, const unsigned char* is_ruler, const int* list, long long n_rulers,
                             long long n_hits, unsigned* seg, int* st, unsigned* status, hipStream_t s);
hipError_t launch_order_jump(const int* nb, const int* rid, const int* act, long long n_act, long long n_hits,
                             const int* in, int* out, int* next, unsigned long long* next_n, unsigned* status,
                             hipStream_t s);
hipError_t launch_order_place(int n, const int64_t* dims_with_t, const long long* label, long long n_hits,
                              const long long* roots, const long long* rb, const long long* offsets,
                              const unsigned char* is_ruler, const int* rid, const unsigned* seg, const int* st,
                              long long* order, unsigned* status, hipStream_t s);
// Isovolume tracking (iso.hip): per-vertex crossing masks and hit / tetrahedron counts; emission of edge ids,
// positions and identity parents from the scanned counts; pentachoron unions and tetrahedra over the active
// vertices.  Per-vertex grids launch as (ceil(nx / 128), ny, nz * nt) blocks (ny, nz * nt <= 65535).
// bits: ceil(nx / 64) * ny * nz * nt words of vertex sides, written by the count launch, read by the unite launch
hipError_t launch_iso_count(const float* f, int nx, int ny, int nz, int nt, float c, unsigned long long* bits,
                            unsigned short* emask, unsigned char* hcnt, unsigned char* tcnt, unsigned* status,
                            hipStream_t s);
hipError_t launch_iso_emit(const float* f, int nx, int ny, int nz, int nt, float c, const unsigned short* emask,
                           const long long* hbase, const unsigned char* hcnt, long long* edge_id, float* pos,
                           unsigned* parent, hipStream_t s);
// ascending list of the vertices with tetrahedra (tcnt > 0), at their offsets from abase (nonzero counts)
hipError_t launch_iso_active(const unsigned char* tcnt, const long long* abase, long long V, long long* list,
                             hipStream_t s);
hipError_t launch_iso_unite(const float* f, int nx, int ny, int nz, int nt, float c,
                            const unsigned long long* bits, const long long* active, long long n_active,
                            const unsigned short* emask, const long long* hbase, const unsigned char* hcnt,
                            const unsigned char* tcnt, const long long* tbase, unsigned* parent, int* tets,
                            unsigned* status, hipStream_t s);

// Quantum vortex surfaces (vortex.hip): edge signs and positive-triangle masks (tmask, 50 bits) with per-vertex
// counts; then emission of triangle ids, points and identity parents, and the pentachoron unions.  Grids as iso.
hipError_t launch_vx_detect(const float* psi, int nx, int ny, int nz, int nt, float qscale, unsigned short* emask,
                            unsigned long long* tmask, unsigned char* cnt, unsigned* status, hipStream_t s);
hipError_t launch_vx_emit(const float* psi, int nx, int ny, int nz, int nt, float qscale,
                          const unsigned long long* tmask, const long long* hoff, long long* tri_id, float* pos,
                          unsigned* parent, hipStream_t s);
// Critical points on an extruded triangle mesh (prism.hip): face tests over nt * S faces (flag, allocated to a
// multiple of 16 bytes), then emission and the tetrahedron unions, with the hit offsets from the group bases of the
// flags (offsets16.h).
// ft_scratch: 2 nv nt floats (the field copied vertex-major for the test).
hipError_t launch_pm_test(const float* xy, const int* tri, const int* edge, const int* tri_edge, const float* field,
                          long long nv, long long nf, long long ne, int nt, float qscale, float* ft_scratch,
                          unsigned char* flag, unsigned* status, hipStream_t s);
// edge_tri: [ne][2] triangles of each edge (-1: none), or null for a mesh with an edge of more than two triangles
// (the unions then visit every prism).
hipError_t launch_pm_emit(const float* xy, const int* tri, const int* edge, const int* tri_edge, const int* edge_tri,
                          const float* field, long long nv, long long nf, long long ne, int nt, float qscale,
                          const unsigned char* flag, const long long* base, long long n_hits, long long* face_id,
                          float* pos, unsigned* parent, unsigned* status, hipStream_t s);
// Type smoothing and run simplification along an order (head/heads: [n_hits] int / int64 scratch).
hipError_t launch_smooth(const long long* order, const long long* offsets, const int* n_ends, long long n_traj,
                         long long n_hits, const uint8_t* type_in, int half, int* head, long long* heads,
                         long long* total, long long* scan_tmp, uint8_t* type_out, unsigned* status, hipStream_t s);
hipError_t launch_simplify(int n, const float* pos, const long long* order, const long long* offsets,
                           const int* n_ends, long long n_traj, long long n_hits, const uint8_t* type_in, float theta,
                           long long* rot, int* flag, long long* run_off, int* head, long long* heads,
                           long long* total, long long* scan_tmp, int* t_min, int* t_max, uint8_t* run_type,
                           uint8_t* new_type, uint8_t* type_out, unsigned* status, hipStream_t s);

// Union-find passes over n hits: extra unions from the work list, then labels = face_id of the root.
hipError_t launch_uf_hook(unsigned* parent, const uint2* work, const unsigned long long* work_count,
                          long long max_work, hipStream_t s);
// Compression of a forest whose parents all point to smaller indices (the sparse emission's), in one pass.
hipError_t launch_uf_compress(unsigned* parent, long long n, hipStream_t s);
// Unions of a link array with one slot per entry: entries (a, a) are empty.
hipError_t launch_uf_hook_slots(unsigned* parent, const uint2* slots, long long n_slots, hipStream_t s);
hipError_t launch_uf_label(unsigned* parent, const long long* face_id, long long* label, long long n,
                           unsigned long long* cnt, hipStream_t s);

}  // namespace ftk
