/*
 * ftk.h -- C ABI of libftk_mi355x.so: robust critical-point tracking on the simplicial spacetime mesh of a
 * regular grid, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Guo et al., "FTK: A Simplicial Spacetime Meshing Framework for Robust and Scalable Feature Tracking"
 * (IEEE TVCG).  The spacetime grid (space x time) is split into Kuhn/Freudenthal simplices (Sec. 3.3); every
 * n-simplex is tested for a zero of the piecewise-linear vector field (Sec. 4.1, Eq. 2) with exact integer
 * determinants under Simulation of Simplicity (Sec. 4.3, Sec. 2.4); punctured simplices receive a barycentric
 * sublocation (Eq. 2) and a critical-point type from the spatial Jacobian (Sec. 4.1); the punctured sides of every
 * (n+1)-simplex are united into trajectories (Alg. 1, left column).
 *
 * Conventions shared by every entry point
 *   - Pointers named `field`/`step` and every array inside ftk_cp_result are HIP DEVICE pointers unless stated.
 *   - Layouts are C order with x fastest:  scalar 2D  f[nt][ny][nx];  vector 2D  u[nt][2][ny][nx] (planar u, v
 *     per step);  scalar 3D  f[nt][nz][ny][nx].  float32, contiguous.
 *   - Spacetime vertex p = (x, y, [z], t) has global index g = ((t*nz + z)*ny + y)*nx + x (nz = 1 in 2D).  This
 *     order is the vertex order of the symbolic perturbation, so it fixes which simplex receives a degenerate zero
 *     (Sec. 4.3, Sec. 10.1).
 *   - A punctured n-simplex is identified by face_id = g(anchor) * T + type, T = 12 (2D) or 60 (3D), where the
 *     anchor is its lowest vertex and `type` indexes the ordered tuples (M_1..M_n) of nonempty disjoint axis masks
 *     (bit 0 = x, then y, [z], t) in lexicographic order; its vertices are anchor, anchor+e(M_1),
 *     anchor+e(M_1|M_2), ...  (the paper's (corner, unique type) indexing, Sec. 3.3).
 *   - Every call is ordered on `stream`.  Calls that return results synchronise `stream` once to learn the hit
 *     count (and once more at the end for the trajectory count).  Handles are not thread-safe; distinct handles
 *     and distinct calls on distinct streams are independent.
 *   - Errors: an ftk_status is returned, nothing is thrown across the ABI.  On error the result is left zeroed
 *     (except n_hits for FTK_ERR_CAPACITY); ftk_last_error() gives a thread-local message.
 */
#ifndef FTK_MI355X_H
#define FTK_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* ftk_stream_t; /* a hipStream_t; NULL = the null stream */

typedef enum {
  FTK_OK = 0,
  FTK_ERR_ARG = 1,        /* bad dimensions, null pointer, unsupported kind/option */
  FTK_ERR_NONFINITE = 2,  /* NaN or Inf in the input */
  FTK_ERR_RANGE = 3,      /* a quantised vector component beyond the exact-arithmetic bound */
  FTK_ERR_CAPACITY = 4,   /* more hits than the 32-bit index types hold (each entry point states its limit) */
  FTK_ERR_OOM = 5,        /* an allocation failed (device memory or the caller's allocator) */
  FTK_ERR_HIP = 6,        /* a HIP runtime call failed */
  FTK_ERR_INVARIANT = 7,  /* a cell with 1 or >= 3 punctured sides: impossible under SoS; internal error */
  FTK_ERR_STATE = 8       /* streaming call out of order */
} ftk_status;

typedef enum { FTK_SCALAR = 0, FTK_VECTOR = 1 } ftk_field_kind; /* scalar: the gradient is tracked */

typedef enum {
  FTK_CP_DEGENERATE = 0, FTK_CP_MIN = 1, FTK_CP_MAX = 2, FTK_CP_SADDLE = 3, FTK_CP_SADDLE1 = 4,
  FTK_CP_SADDLE2 = 5, FTK_CP_SOURCE = 6, FTK_CP_SINK = 7, FTK_CP_REPELLING_FOCUS = 8,
  FTK_CP_ATTRACTING_FOCUS = 9, FTK_CP_CENTER = 10
} ftk_cp_type;

/* Per-hit flag bits. */
#define FTK_FLAG_DEGENERATE_SUBLOC 1u /* all exact cofactors zero: punctured only by the perturbation; centroid used */
#define FTK_FLAG_FP64_FALLBACK 2u     /* the FP32 type decision was not certified and was redone in FP64 */
#define FTK_FLAG_WIDE 4u              /* a vertex vector beyond the narrow range (2D 2^31, 3D 2^20): 128-bit path */

/* Output selection bits (ftk_options.outputs). face_id is always produced. */
#define FTK_OUT_POS 1u
#define FTK_OUT_MU 2u
#define FTK_OUT_TYPE 4u
#define FTK_OUT_LABEL 8u
#define FTK_OUT_FLAGS 16u
#define FTK_OUT_ALL 31u
#define FTK_OUT_DEFAULT 29u /* POS | TYPE | LABEL | FLAGS: the 30-byte record per hit (face_id, pos, type, flags, label) */

/* Device allocator hooks (e.g. a framework's caching allocator).  Both must be stream-ordered on `stream`; alloc
 * must return memory aligned to at least 16 bytes (hipMalloc and torch's caching allocator align to 256): kernels
 * write some outputs with 16-byte stores, and a call that receives a misaligned output array fails with
 * FTK_ERR_ARG rather than writing it. */
typedef void* (*ftk_alloc_fn)(size_t bytes, ftk_stream_t stream, void* ctx);
typedef void (*ftk_free_fn)(void* ptr, ftk_stream_t stream, void* ctx);

typedef struct {
  int32_t quant_log2;  /* fixed-point scale 2^quant_log2 for the vectors; default 20; range [0, 40] */
  int32_t precision;   /* 0: FP32 sublocation/classification with certified FP64 fallback; 1: FP64 throughout */
  uint32_t outputs;    /* FTK_OUT_* bits; 0 means FTK_OUT_DEFAULT */
  int32_t tile_y;      /* rows per detection tile (0 = tuned default) */
  int32_t slab_depth;  /* time steps per detection workgroup (0 = tuned default) */
  ftk_alloc_fn alloc;  /* NULL: hipMallocAsync on the stream */
  ftk_free_fn free;    /* NULL: hipFreeAsync on the stream */
  void* alloc_ctx;
  int32_t profile;     /* 1: record HIP events around each kernel group on `stream`; times land in stats */
  int32_t debug;       /* 0 in normal use; FTK_DEBUG_* test hooks of the 2D tracker (below) */
} ftk_options;

/* Test hooks (ftk_options.debug), for tests of paths that realistic inputs rarely reach.  FTK_DEBUG_SMALL_LDS runs
 * the 2D emission with tiny workgroup-local capacities (union-find chunk and link stage), so that tile steps overflow
 * them and take the global-list paths; results are unchanged.  FTK_DEBUG_INVARIANT makes the 2D emission report a
 * cell with a wrong punctured-side count at time step (debug >> 8), so that tests can check how the error reaches
 * the caller (every form returns FTK_ERR_INVARIANT).  FTK_DEBUG_TILED_EMIT and FTK_DEBUG_SPARSE_EMIT force the 2D
 * emission form of the one-shot and batched calls (tiles marching through time, or one wavefront per non-empty row
 * segment; by default the sparse form runs below one hit per 128 vertices, FTK_DEBUG_SMALL_LDS implies the tiled
 * form); results are identical. */
#define FTK_DEBUG_SMALL_LDS 1
#define FTK_DEBUG_INVARIANT 2
#define FTK_DEBUG_TILED_EMIT 4
#define FTK_DEBUG_SPARSE_EMIT 8

typedef struct {
  int64_t simplices_tested; /* n-simplices tested (the throughput numerator) */
  int64_t cells_linked;     /* (n+1)-simplices holding two punctured sides */
  int64_t fp64_fallbacks;   /* hits whose type needed the FP64 re-evaluation */
  int64_t degenerate_sublocations;
  int32_t wide_path;        /* 1 if the 128-bit determinant path ran */
  int32_t reserved;
  float t_detect_ms;        /* with ftk_options.profile: detection kernel (pass 1) */
  float t_scan_ms;          /* prefix sum of the per-segment hit counts */
  float t_emit_ms;          /* emission: sublocation, classification, union-find links */
  float t_link_ms;          /* union-find hooking and labelling (pass 2) */
} ftk_stats;

typedef struct {
  int32_t n;                /* spatial dimension (2 or 3) */
  int32_t reserved;
  int64_t n_hits;           /* punctured n-simplices */
  int64_t n_trajectories;   /* connected components */
  int64_t* face_id;         /* [n_hits], strictly ascending */
  float* pos;               /* [n_hits][n+1] spacetime position (x, y, [z], t) in grid/step units, or NULL */
  float* mu;                /* [n_hits][n+1] barycentric coordinates of the zero (Eq. 2), or NULL */
  uint8_t* type;            /* [n_hits] ftk_cp_type, or NULL */
  uint8_t* flags;           /* [n_hits] FTK_FLAG_* bits, or NULL */
  int64_t* label;           /* [n_hits] smallest face_id of the trajectory holding the hit, or NULL */
  ftk_stats stats;
} ftk_cp_result;

typedef struct ftk_tracker ftk_tracker;

/* Default options (quant_log2 = 20, precision 0, FTK_OUT_DEFAULT outputs, tuned tiles, HIP stream-ordered
 * allocator). */
void ftk_default_options(ftk_options* opt);

/*
 * Track critical points of a 2D time-varying field (Sec. 4.1-4.3, Eq. 2, Alg. 1 left column).
 *   field : device pointer, scalar f[nt][ny][nx] or vector u[nt][2][ny][nx] (kind), float32.
 *   nx, ny, nt >= 2.  opt may be NULL (defaults).  out receives device arrays allocated through opt->alloc (or
 *   hipMallocAsync); release them with ftk_result_free using the same options.
 * Scalar input: the gradient (central differences inside, one-sided at the first/last index, float32) is
 * quantised to integers q = rint(g * 2^quant_log2); vector input is quantised directly.  Errors:
 * FTK_ERR_NONFINITE, FTK_ERR_RANGE (|q| >= 2^62), FTK_ERR_ARG, FTK_ERR_OOM, FTK_ERR_HIP, FTK_ERR_CAPACITY (more
 * than 2^32 - 2 punctured simplices).
 */
ftk_status ftk_track_cp2d(const float* field, ftk_field_kind kind, int64_t nx, int64_t ny, int64_t nt,
                          const ftk_options* opt, ftk_stream_t stream, ftk_cp_result* out);

/*
 * For callers that cannot allocate device memory (serving loops that must not call hipMalloc, harnesses that
 * forbid allocation): ftk_track_cp2d with the outputs in caller-owned arrays and the scratch (puncture masks,
 * per-segment hit counts and offsets, union-find parents and link list) in one fixed region inside the library,
 * FTK_STATIC_SCRATCH_BYTES per device, held from the first call on a device until the process ends.  No device
 * memory is allocated or freed by the call.
 *   io (host pointer): on entry, face_id and, for each FTK_OUT_* bit set in opt->outputs, the matching array among
 *     pos ([capacity][3] floats), mu ([capacity][3]), type, flags ([capacity] bytes), label ([capacity] int64) are
 *     device arrays owned by the caller with room for `capacity` hits; on FTK_OK the call fills n_hits,
 *     n_trajectories and stats and sets the pointers of outputs not asked for to NULL.
 *   opt->alloc/free/alloc_ctx and opt->profile are ignored.  Results are identical to ftk_track_cp2d's.
 *   The scratch need is 2 bytes per vertex plus 12 bytes per 64-vertex row segment (detection) and 20 bytes per
 *     hit (union-find), each rounded up to 256 bytes, plus a few KiB; when it exceeds the region the call returns
 *     FTK_ERR_CAPACITY (n_hits set once the hits are counted), as it does for more than `capacity` hits.
 *   Calls that overlap in time on one device (several host threads, or streams not ordered with each other)
 *     share the region and race: serialise them.  Errors otherwise as ftk_track_cp2d; on error *io is left as
 *     given except n_hits for FTK_ERR_CAPACITY.
 */
#define FTK_STATIC_SCRATCH_BYTES (256ull << 20)
ftk_status ftk_track_cp2d_into(const float* field, ftk_field_kind kind, int64_t nx, int64_t ny, int64_t nt,
                               const ftk_options* opt, ftk_stream_t stream, int64_t capacity, ftk_cp_result* io);

/*
 * Track critical points of a 3D time-varying scalar field f[nt][nz][ny][nx] through its gradient (Sec. 4.1-4.3,
 * Alg. 1 left column with tetrahedral sides of pentachora).  kind must be FTK_SCALAR.  FTK_ERR_RANGE when a
 * quantised component reaches 2^41.  Otherwise as ftk_track_cp2d.
 */
ftk_status ftk_track_cp3d(const float* field, ftk_field_kind kind, int64_t nx, int64_t ny, int64_t nz,
                          int64_t nt, const ftk_options* opt, ftk_stream_t stream, ftk_cp_result* out);

/*
 * Streaming form, after the paper's push_field_data() and its two-step sliding window of ordinal and interval
 * elements (Sec. 3.2 "Ordinal and interval mesh elements", Sec. 8 "C++ programming interface").
 *   ftk_cp_create: n = 2 or 3, dims = (nx, ny[, nz]); the tracker holds a window of the last three steps on the
 *                  device (field, puncture masks, per-segment counts and offsets), independent of the series length;
 *                  only the outputs grow with the hits found.
 *   ftk_cp_push:   step = device pointer to one time step in the layout above (for vector input [2][ny][nx]); the
 *                  caller may overwrite it once the call returns.  Pushing step s tests the simplices anchored at
 *                  step s - 1 (its ordinal simplices and the interval ones towards s) and emits the hits anchored at
 *                  step s - 2 (whose cells reach steps s - 3 .. s - 1).
 *   ftk_cp_finish: stitches, labels and returns the whole trajectory set, identical to the one-shot call on the
 *                  concatenated steps.  The tracker may not be pushed to afterwards (FTK_ERR_STATE).
 */
ftk_status ftk_cp_create(int32_t n, const int64_t* dims, ftk_field_kind kind, const ftk_options* opt,
                         ftk_stream_t stream, ftk_tracker** h);
ftk_status ftk_cp_push(ftk_tracker* h, const float* step);
ftk_status ftk_cp_finish(ftk_tracker* h, ftk_cp_result* out);
void ftk_cp_destroy(ftk_tracker* h);

/*
 * Batched form: many independent 2D series of uneven sizes in one call.  fields[i] is a device pointer to
 * series i (layout as ftk_track_cp2d, shared kind); nx/ny/nt are HOST arrays of n_series entries; outs is a HOST
 * array of n_series results, each as from ftk_track_cp2d.  Detection of all series runs as one persistent launch
 * over a device work queue of (series, row block, time slab) items.
 */
ftk_status ftk_track_cp2d_batched(int32_t n_series, const float* const* fields, const int64_t* nx,
                                  const int64_t* ny, const int64_t* nt, ftk_field_kind kind,
                                  const ftk_options* opt, ftk_stream_t stream, ftk_cp_result* outs);

/*
 * Trajectory post-processing (after a tracking call; n = 2 or 3, dims_with_t = (nx, ny, [nz,] nt) as tracked).
 *
 * Trajectory table (Sec. 4.4 "Filtering": per-trajectory attributes).  Device arrays of n entries, allocated through
 * opt->alloc (or hipMallocAsync) in ascending label order; release with ftk_traj_table_free.  Needs the result's
 * pos and label arrays (FTK_ERR_ARG otherwise).  Under the symbolic perturbation a punctured face lies in two cells
 * with one more punctured side each, except on a boundary hyperplane of the grid (a coordinate equal to 0 along an
 * axis the face does not use, or equal to N - 1), where only one cell holds it: every trajectory is a path with
 * two such ends or a closed loop with none.
 */
typedef struct {
  int64_t n;          /* trajectories (the result's n_trajectories) */
  int64_t* label;     /* [n] smallest face id of the trajectory (its label), ascending */
  uint64_t* n_points; /* [n] punctured faces in the trajectory */
  float* t_min;       /* [n] smallest time coordinate of its points (pos[.][n]) */
  float* t_max;       /* [n] largest time coordinate of its points */
  int32_t* n_ends;    /* [n] points on a boundary hyperplane: 2 for a path, 0 for a closed loop */
} ftk_traj_table;

ftk_status ftk_traj_table_build(const ftk_cp_result* r, int32_t n, const int64_t* dims_with_t,
                                const ftk_options* opt, ftk_stream_t stream, ftk_traj_table* out);
void ftk_traj_table_free(ftk_traj_table* tt, const ftk_options* opt, ftk_stream_t stream);

/*
 * Critical points at time step t0 (Sec. 3.2, slicing through the ordinal faces): *idx receives a device array
 * (allocated through opt->alloc; release with ftk_buffer_free) of the ascending indices, into the result's
 * arrays, of the punctured faces anchored at step t0 that do not use the time axis; *count their number (host).
 * 0 <= t0 < nt, else FTK_ERR_ARG.
 */
ftk_status ftk_cp_slice(const ftk_cp_result* r, int32_t n, const int64_t* dims_with_t, int64_t t0,
                        const ftk_options* opt, ftk_stream_t stream, int64_t** idx, int64_t* count);

/*
 * Loop filter (Sec. 4.4 "Filtering"): keep[i] (device array of the result's n_hits bytes, owned by the caller)
 * becomes 0 for the points of closed loops (n_ends == 0) whose time extent t_max - t_min is below min_duration,
 * 1 for every other point.  tt must come from ftk_traj_table_build on the same result.
 */
ftk_status ftk_cp_filter_loops(const ftk_cp_result* r, const ftk_traj_table* tt, float min_duration,
                               ftk_stream_t stream, uint8_t* keep);

/*
 * Order of the points along each trajectory (Sec. 3.1: a trajectory is a PL curve whose piece in each cell is the
 * segment between the cell's two punctured sides; Alg. 1 pass 2).  tt must come from ftk_traj_table_build on the
 * same result, which must carry its label array.
 *   order   (device, caller-owned, n_hits entries): hit indices grouped by trajectory in the table's (ascending
 *           label) order, each in curve order.  A path runs from its end with the smaller face id to the other
 *           end; a closed loop starts at its label face and steps first to its neighbour with the smaller face id.
 *   offsets (device, caller-owned, n_trajectories + 1 entries): start of each trajectory in order[], n_hits last.
 * Synchronises the stream once per list-ranking round (about log2 of the longest trajectory).  FTK_ERR_CAPACITY
 * beyond 2^31 - 1 points; FTK_ERR_INVARIANT if a cell holding a punctured face has no or several other punctured
 * sides, or a trajectory is not one curve.
 */
ftk_status ftk_traj_order(const ftk_cp_result* r, int32_t n, const int64_t* dims_with_t, const ftk_traj_table* tt,
                          const ftk_options* opt, ftk_stream_t stream, int64_t* order, int64_t* offsets);

/*
 * Type smoothing along the order (Sec. 4.4 "Smoothing", window shifting): type_out[i] becomes the type shared by
 * the half_window points before and the half_window points after hit i on its trajectory when those points all
 * have one type that differs from type_in[i]; otherwise type_in[i].  Every decision reads type_in (marks first,
 * changes after the pass).  Loops wrap around; a loop of fewer than 2 * half_window + 1 points and the points of a
 * path closer than half_window to an end keep their types.  order/offsets as from ftk_traj_order; type_in and
 * type_out are device arrays of n_hits bytes (for instance the result's type array) that must not overlap.
 */
ftk_status ftk_traj_smooth_types(const ftk_cp_result* r, const ftk_traj_table* tt, const int64_t* order,
                                 const int64_t* offsets, const uint8_t* type_in, int32_t half_window,
                                 const ftk_options* opt, ftk_stream_t stream, uint8_t* type_out);

/*
 * Type simplification along the order (Sec. 4.4 "Simplification", persistence in time): a run is a maximal
 * stretch of consecutive points of one type on a trajectory (on a loop, runs wrap around), its time extent the
 * largest minus the smallest time coordinate (pos[.][n], FP32) of its points.  A run whose extent is below
 * min_persistence, lying between two runs of one common type whose extents are both at least min_persistence,
 * takes that type.  Runs at the ends of a path have one neighbour and keep their type; on a loop of two runs both
 * neighbours are the other run.  Decisions read type_in only.  Arrays as ftk_traj_smooth_types; needs pos.
 */
ftk_status ftk_traj_simplify_types(const ftk_cp_result* r, const ftk_traj_table* tt, const int64_t* order,
                                   const int64_t* offsets, const uint8_t* type_in, float min_persistence,
                                   const ftk_options* opt, ftk_stream_t stream, uint8_t* type_out);

/* Release a device array returned by the library (with the allocator given in opt, which may be NULL). */
void ftk_buffer_free(void* p, const ftk_options* opt, ftk_stream_t stream);

/*
 * Autotuning of the 2D detection tiling (an implementation choice; the paper prescribes none): times the detection
 * kernel on the caller's field (device pointer, layout as ftk_track_cp2d) for tile rows {8, 16, 32} x slab depths
 * {8, 16, 32} and returns opt with the fastest tile_y / slab_depth in *tuned (host struct).  The choice is also
 * remembered for (kind, nx, ny) in this process and used by later calls that leave tile_y / slab_depth at 0
 * (the batched form takes the slab depth of its largest series).  Errors as ftk_track_cp2d.
 */
ftk_status ftk_autotune_cp2d(const float* field, ftk_field_kind kind, int64_t nx, int64_t ny, int64_t nt,
                             const ftk_options* opt, ftk_stream_t stream, ftk_options* tuned);

/*
 * Isovolume tracking in a 3D scalar series (Sec. 6.1, two passes on the spacetime mesh; Sec. 6.2 robustness).
 * field: device pointer, contiguous binary32 [nt][nz][ny][nx]; isovalue c (finite).  An edge anchored at vertex p
 * (t-major index g) with axis mask M (1..15; x = 1, y = 2, z = 4, t = 8) joins p and p + e(M) and has the id
 * g * 15 + (M - 1).  It crosses the level set when its two vertices lie on different sides, a value equal to c
 * counting as above (the symbolic perturbation of a single value is positive).  The crossed edges of every
 * pentachoron are united into isovolumes; every pentachoron with crossings contributes one tetrahedron (one vertex
 * on its side) or three (two vertices: the prism of crossed edges split along monotone paths in vertex order).
 * Outputs are allocated through opt->alloc (or hipMallocAsync on stream); release with ftk_iso_result_free.
 * Synchronises the stream twice (hit and tetrahedron counts, component count).  Every dimension >= 2; ny and
 * nz * nt at most 65535.  FTK_ERR_NONFINITE for NaN/Inf in the field; FTK_ERR_CAPACITY beyond 2^31 - 1 crossings
 * (tetrahedra hold 32-bit indices).
 */
typedef struct {
  int64_t n_hits;       /* crossed edges */
  int64_t n_components; /* isovolumes (connected components) */
  int64_t n_tets;       /* tetrahedra of the tessellation */
  int64_t* edge_id;     /* [n_hits] ascending */
  float* pos;           /* [n_hits][4] intersection point (x, y, z, t): p + mu e(M), mu = (c - f(p)) / (f(q) - f(p)) */
  int64_t* label;       /* [n_hits] smallest edge id of the isovolume */
  int32_t* tets;        /* [n_tets][4] indices into the hit arrays, by pentachoron (g * 24 + type) */
} ftk_iso_result;

ftk_status ftk_track_iso3d(const float* field, int64_t nx, int64_t ny, int64_t nz, int64_t nt, float isovalue,
                           const ftk_options* opt, ftk_stream_t stream, ftk_iso_result* out);
void ftk_iso_result_free(ftk_iso_result* r, const ftk_options* opt, ftk_stream_t stream);

/* Number of spacetime edges tested for a 3D grid: sum over the 15 axis masks M of prod_a (N_a - [a in M]),
 * dims_with_t = (nx, ny, nz, nt).  Returns -1 for bad arguments. */
int64_t ftk_edge_count(const int64_t* dims_with_t);

/*
 * Quantum vortex surface tracking in a 3D complex series (Sec. 5.1, two passes on the spacetime mesh).
 * psi: device pointer, contiguous binary32 [nt][2][nz][ny][nx] (real and imaginary planes per step).  A spacetime
 * triangle anchored at vertex p (t-major index g) with axis masks (M1, M2) (x = 1, y = 2, z = 4, t = 8; 50 types in
 * lexicographic order) has the vertices p, p + e(M1), p + e(M1|M2) and the id g * 50 + type.  It is positive when
 * the phase changes along its edges, each wrapped into (-pi, pi], sum to +-2 pi: exactly when 0 lies inside the
 * triangle (psi_0, psi_1, psi_2) of the complex plane, decided on q = rint(psi * 2^opt->quant_log2) with the symbolic
 * perturbation.  The positive triangles of every pentachoron are united into vortex surfaces.  Outputs through
 * opt->alloc (or hipMallocAsync on stream); release with ftk_vortex_result_free.  Synchronises the stream twice.
 * Every dimension >= 2; ny and nz * nt at most 65535.  FTK_ERR_NONFINITE for NaN/Inf; FTK_ERR_RANGE when a
 * quantised value reaches 2^31; FTK_ERR_CAPACITY beyond 2^32 - 2 positive triangles.
 */
typedef struct {
  int64_t n_hits;       /* positive triangles */
  int64_t n_components; /* vortex surfaces */
  int64_t* tri_id;      /* [n_hits] ascending */
  float* pos;           /* [n_hits][4] vortex point (x, y, z, t) from the exact barycentric weights (Eq. 2) */
  int64_t* label;       /* [n_hits] smallest triangle id of the surface */
} ftk_vortex_result;

ftk_status ftk_track_vortex3d(const float* psi, int64_t nx, int64_t ny, int64_t nz, int64_t nt,
                              const ftk_options* opt, ftk_stream_t stream, ftk_vortex_result* out);
void ftk_vortex_result_free(ftk_vortex_result* r, const ftk_options* opt, ftk_stream_t stream);

/* Number of triangles tested for a 3D grid: sum over the 50 triangle types of prod_a (N_a - [a used]),
 * dims_with_t = (nx, ny, nz, nt).  Returns -1 for bad arguments. */
int64_t ftk_triangle_count(const int64_t* dims_with_t);

/*
 * Critical-point tracking of a 2D vector field on an unstructured triangle mesh extruded in time (Sec. 3.2,
 * prismatic subdivision).  xy: device [nv][2] vertex positions; tri: device [nf][3] vertex indices (any order per
 * row); field: device [nt][2][nv] binary32 vector components per step.  Each triangle v0 < v1 < v2 and step interval
 * becomes a prism split by the staircase into the tetrahedra a0 a1 a2 b2, a0 a1 b1 b2, a0 b0 b1 b2 (global vertex
 * order g = t nv + v); the quadrilateral of a mesh edge a < b is split along a - b'.  With the mesh edges sorted
 * (a < b, ascending) and S = 3 nf + 2 ne faces per step, face ids are t * S + local: the triangle T (local T); the
 * edge faces (a, b, b') and (a, a', b') of edge E (nf + 2E, +1); the interior faces (v0, v1, v2') and (v0, v1', v2')
 * of T (nf + 2 ne + 2T, +1).  Faces are tested like the regular path (quantised with opt->quant_log2, SoS); points
 * are (x, y, t) from the exact barycentric weights; the two punctured faces of every tetrahedron are united, labels
 * = smallest face id.  No critical-point types (the field's Jacobian on a mesh is out of scope here).
 * Synchronises the stream.  nv >= 3, nf >= 1, 2 <= nt <= 65535;
 * FTK_ERR_ARG for indices out of range or repeated within a triangle; errors otherwise as ftk_track_cp2d.
 */
typedef struct {
  int64_t n_hits;          /* punctured faces */
  int64_t n_trajectories;  /* connected components */
  int64_t faces_per_step;  /* S */
  int64_t n_edges;         /* ne */
  int64_t* face_id;        /* [n_hits] ascending */
  float* pos;              /* [n_hits][3] (x, y, t) */
  int64_t* label;          /* [n_hits] smallest face id of the trajectory */
} ftk_mesh_result;

/* Mesh handle: the topology (sorted triangles, unique edges, triangle edges) built once on the host from tri
 * (copied back) and kept on the device; xy is referenced, so it must outlive the handle.  Errors as above. */
typedef struct ftk_mesh ftk_mesh;
ftk_status ftk_mesh_create(const float* xy, int64_t nv, const int32_t* tri, int64_t nf, ftk_stream_t stream,
                           ftk_mesh** m);
void ftk_mesh_destroy(ftk_mesh* m);
/* Tracking on a mesh handle (no host work besides the two count read-backs).  Scratch includes a vertex-major copy
 * of the field (8 nv nt bytes) besides one flag byte per spacetime face. */
ftk_status ftk_track_cp_mesh(const ftk_mesh* m, const float* field, int64_t nt, const ftk_options* opt,
                             ftk_stream_t stream, ftk_mesh_result* out);
/* One-shot form: create, track, destroy. */
ftk_status ftk_track_cp_mesh2d(const float* xy, int64_t nv, const int32_t* tri, int64_t nf, const float* field,
                               int64_t nt, const ftk_options* opt, ftk_stream_t stream, ftk_mesh_result* out);
void ftk_mesh_result_free(ftk_mesh_result* r, const ftk_options* opt, ftk_stream_t stream);

/* Release the device arrays of a result (with the allocator given in opt, which may be NULL). */
void ftk_result_free(ftk_cp_result* r, const ftk_options* opt, ftk_stream_t stream);

/* Number of n-simplices tested for a grid: sum over simplex types of prod_a (N_a - [axis a used]).
 * dims_with_t = (nx, ny, [nz,] nt).  Returns -1 for bad arguments. */
int64_t ftk_simplex_count(int32_t n, const int64_t* dims_with_t);

/* Thread-local text of the last error of this thread ("" if none). */
const char* ftk_last_error(void);

/* Library version string. */
const char* ftk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FTK_MI355X_H */
