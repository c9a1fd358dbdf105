// api.hip -- the C ABI (include/ftk.h): argument checks, device memory, launch sequence, status decoding.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/ftk.h"
#include "common.h"
#include "internal.h"

namespace {

thread_local std::string g_err;

ftk_status fail(ftk_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
ftk_status fail(ftk_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

// Allocation through the caller's hooks or the stream-ordered HIP allocator.
struct Alloc {
  ftk_alloc_fn a = nullptr;
  ftk_free_fn f = nullptr;
  void* ctx = nullptr;
  hipStream_t s = nullptr;
  void* get(size_t bytes) const {
    if (bytes == 0) bytes = 16;
    bytes = (bytes + 255) & ~size_t(255);
    if (a) return a(bytes, (ftk_stream_t)s, ctx);
    void* p = nullptr;
    if (hipMallocAsync(&p, bytes, s) != hipSuccess) return nullptr;
    return p;
  }
  void put(void* p) const {
    if (!p) return;
    if (f)
      f(p, (ftk_stream_t)s, ctx);
    else
      (void)hipFreeAsync(p, s);
  }
};

// Scratch list released on scope exit.
struct Scratch {
  const Alloc& al;
  void* p[16];
  int n = 0;
  explicit Scratch(const Alloc& a) : al(a) {}
  template <typename T>
  T* get(size_t count) {
    void* q = al.get(count * sizeof(T));
    if (q) p[n++] = q;
    return (T*)q;
  }
  ~Scratch() {
    for (int i = n - 1; i >= 0; --i) al.put(p[i]);
  }
};

// Optional phase timing with HIP events on the call's stream.
struct Phases {
  bool on = false;
  hipEvent_t ev[8] = {};
  int n = 0;
  hipStream_t s = nullptr;
  void init(bool enable, hipStream_t st) {
    on = enable;
    s = st;
    if (!on) return;
    for (int i = 0; i < 8; ++i)
      if (hipEventCreate(&ev[i]) != hipSuccess) on = false;
  }
  void mark(int i) {
    if (on) (void)hipEventRecord(ev[i], s);
  }
  float ms(int a, int b) const {
    float t = 0.0f;
    if (on && hipEventElapsedTime(&t, ev[a], ev[b]) != hipSuccess) t = 0.0f;
    return t;
  }
  ~Phases() {
    if (on)
      for (int i = 0; i < 8; ++i) (void)hipEventDestroy(ev[i]);
  }
};

// Control block read back by the host.
struct Ctl {
  unsigned status;
  unsigned pad;
  long long total;
  unsigned long long cnt[ftk::CNT_N];
};

void resolve(const ftk_options* in, ftk_options* o) {
  ftk_default_options(o);
  if (in) {
    *o = *in;
    if (o->outputs == 0) o->outputs = FTK_OUT_DEFAULT;
  }
}

// Keep freed stream-ordered memory in the device's default pool between calls (a release threshold of 0 would hand
// it back to the driver at every synchronisation and re-map it on the next call).
void keep_pool_memory() {
  static thread_local int done_mask = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev >= 31 || (done_mask >> dev) & 1) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = ~0ull;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  done_mask |= 1 << dev;
}

Alloc make_alloc(const ftk_options& o, hipStream_t s) {
  if (!o.alloc) keep_pool_memory();
  Alloc a;
  a.a = o.alloc;
  a.f = o.free;
  a.ctx = o.alloc_ctx;
  a.s = s;
  return a;
}

#define HIP_TRY(expr)                                                                                 \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess) return fail(FTK_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));           \
  } while (0)

ftk_status read_ctl(Ctl* h, const Ctl* d, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(h, d, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return FTK_OK;
}

ftk_status decode_status(unsigned st) {
  if (st & ftk::ST_NONFINITE) return fail(FTK_ERR_NONFINITE, "non-finite value in the input field");
  if (st & ftk::ST_RANGE) return fail(FTK_ERR_RANGE, "quantised vector component beyond the exact-arithmetic bound");
  if (st & ftk::ST_INVARIANT)
    return fail(FTK_ERR_INVARIANT, "a cell has a punctured-side count other than 0 or 2 (internal error)");
  return FTK_OK;
}

int64_t count_tested(int n, const int64_t* dims) {
  // sum over n-simplex types of prod_a (N_a - [axis a used])
  int64_t tot = 0;
  if (n == 2) {
    for (int k = 0; k < ftk::kTri2.count; ++k) {
      int u = ftk::kTri2.m[k][0] | ftk::kTri2.m[k][1];
      int64_t c = 1;
      for (int a = 0; a < 3; ++a) c *= dims[a] - ((u >> a) & 1);
      tot += c;
    }
  } else {
    for (int k = 0; k < ftk::kTet3.count; ++k) {
      int u = ftk::kTet3.m[k][0] | ftk::kTet3.m[k][1] | ftk::kTet3.m[k][2];
      int64_t c = 1;
      for (int a = 0; a < 4; ++a) c *= dims[a] - ((u >> a) & 1);
      tot += c;
    }
  }
  return tot;
}

}  // namespace

extern "C" {

void ftk_default_options(ftk_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->quant_log2 = 20;
  opt->precision = 0;
  opt->outputs = FTK_OUT_DEFAULT;
}

const char* ftk_last_error(void) { return g_err.c_str(); }

const char* ftk_version(void) { return "ftk_mi355x 0.1 (gfx950)"; }

int64_t ftk_simplex_count(int32_t n, const int64_t* dims) {
  if ((n != 2 && n != 3) || !dims) return -1;
  for (int a = 0; a <= n; ++a)
    if (dims[a] < 2) return -1;
  return count_tested(n, dims);
}

void ftk_result_free(ftk_cp_result* r, const ftk_options* opt, ftk_stream_t stream) {
  if (!r) return;
  ftk_options o;
  resolve(opt, &o);
  Alloc al = make_alloc(o, (hipStream_t)stream);
  al.put(r->face_id);
  al.put(r->pos);
  al.put(r->mu);
  al.put(r->type);
  al.put(r->flags);
  al.put(r->label);
  std::memset(r, 0, sizeof(*r));
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------------------------
// 2D one-shot
// ---------------------------------------------------------------------------------------------------------------
namespace ftk {

ftk_status validate_options(const ftk_options& o) {
  if (o.quant_log2 < 0 || o.quant_log2 > 40) return fail(FTK_ERR_ARG, "quant_log2 must be in [0, 40]");
  if (o.precision != 0 && o.precision != 1) return fail(FTK_ERR_ARG, "precision must be 0 or 1");
  if ((o.alloc == nullptr) != (o.free == nullptr)) return fail(FTK_ERR_ARG, "alloc and free must be given together");
  if (o.tile_y != 0 && o.tile_y != 8 && o.tile_y != 16 && o.tile_y != 32)
    return fail(FTK_ERR_ARG, "tile_y must be 0, 8, 16 or 32");
  if (o.slab_depth < 0) return fail(FTK_ERR_ARG, "slab_depth must be >= 0");
  return FTK_OK;
}

// Results of the detection stage kept for emission.
struct Detect2 {
  uint16_t* masks = nullptr;
  long long* seg_off = nullptr;
  long long nseg = 0;
  bool wide = false;
  long long n_hits = 0;
};

static void tuned_tiles2(const ftk_options& o, int nt, int* ty, int* tt) {
  *ty = o.tile_y ? o.tile_y : 16;
  *tt = o.slab_depth ? o.slab_depth : 16;
  if (*tt > nt) *tt = nt;
}

ftk_status track2d_impl(const float* field, ftk_field_kind kind, int64_t nx, int64_t ny, int64_t nt,
                        const ftk_options& o, hipStream_t s, ftk_cp_result* out) {
  const Alloc al = make_alloc(o, s);
  Scratch sc(al);
  Grid2 g;
  g.f = field;
  g.kind = (int)kind;
  g.nx = (int)nx;
  g.ny = (int)ny;
  g.nt = (int)nt;
  g.nxt = (int)((nx + 63) / 64);
  g.qscale = std::ldexp(1.0f, o.quant_log2);
  g.precision = o.precision;
  const long long V = (long long)nx * ny * nt;
  const long long nseg = (long long)nt * ny * g.nxt;

  uint16_t* masks = sc.get<uint16_t>((size_t)V);
  int* seg_cnt = sc.get<int>((size_t)nseg);
  long long* seg_off = sc.get<long long>((size_t)nseg);
  long long* scan_tmp = sc.get<long long>(scan_tmp_elems(nseg));
  Ctl* dctl = sc.get<Ctl>(1);
  if (!masks || !seg_cnt || !seg_off || !scan_tmp || !dctl) return fail(FTK_ERR_OOM, "scratch allocation failed");
  HIP_TRY(hipMemsetAsync(dctl, 0, sizeof(Ctl), s));

  int ty, tt;
  tuned_tiles2(o, g.nt, &ty, &tt);
  Ctl h;
  bool wide = false;
  Phases ph;
  ph.init(o.profile != 0, s);
  ph.mark(0);
  HIP_TRY(launch_detect2d(g, ty, tt, false, masks, seg_cnt, &dctl->status, s));
  ph.mark(1);
  HIP_TRY(launch_scan(seg_cnt, seg_off, nseg, &dctl->total, scan_tmp, s));
  ph.mark(2);
  ftk_status st = read_ctl(&h, dctl, s);
  if (st) return st;
  if (h.status & ST_NONFINITE) return decode_status(h.status);
  if (h.status & ST_WIDE) {
    wide = true;
    HIP_TRY(hipMemsetAsync(dctl, 0, sizeof(Ctl), s));
    ph.mark(0);
    HIP_TRY(launch_detect2d(g, ty, tt, true, masks, seg_cnt, &dctl->status, s));
    ph.mark(1);
    HIP_TRY(launch_scan(seg_cnt, seg_off, nseg, &dctl->total, scan_tmp, s));
    ph.mark(2);
    st = read_ctl(&h, dctl, s);
    if (st) return st;
  }
  st = decode_status(h.status);
  if (st) return st;
  const long long nh = h.total;
  if (nh > 0xFFFFFFFELL) {
    out->n_hits = nh;
    return fail(FTK_ERR_CAPACITY, "%lld punctured simplices exceed the 32-bit hit index", nh);
  }

  ftk_cp_result r;
  std::memset(&r, 0, sizeof(r));
  r.n = 2;
  r.n_hits = nh;
  const unsigned outs = o.outputs;
  r.face_id = (int64_t*)al.get(sizeof(int64_t) * nh);
  if (outs & FTK_OUT_POS) r.pos = (float*)al.get(sizeof(float) * 3 * nh);
  if (outs & FTK_OUT_MU) r.mu = (float*)al.get(sizeof(float) * 3 * nh);
  if (outs & FTK_OUT_TYPE) r.type = (uint8_t*)al.get(nh);
  if (outs & FTK_OUT_FLAGS) r.flags = (uint8_t*)al.get(nh);
  if (outs & FTK_OUT_LABEL) r.label = (int64_t*)al.get(sizeof(int64_t) * nh);
  unsigned* parent = sc.get<unsigned>((size_t)nh);
  uint2* work = sc.get<uint2>((size_t)nh * 2);
  bool oom = !r.face_id || !parent || !work || ((outs & FTK_OUT_POS) && !r.pos) || ((outs & FTK_OUT_MU) && !r.mu) ||
             ((outs & FTK_OUT_TYPE) && !r.type) || ((outs & FTK_OUT_FLAGS) && !r.flags) ||
             ((outs & FTK_OUT_LABEL) && !r.label);
  if (oom) {
    ftk_result_free(&r, &o, (ftk_stream_t)s);
    return fail(FTK_ERR_OOM, "output allocation failed (%lld hits)", nh);
  }
  Out2 od;
  od.face_id = (long long*)r.face_id;
  od.pos = r.pos;
  od.mu = r.mu;
  od.type = r.type;
  od.flags = r.flags;
  od.parent = parent;
  od.work = work;
  hipError_t he = hipSuccess;
  ph.mark(3);
  if (nh > 0) {
    he = launch_emit2d(g, wide, masks, seg_off, nseg, od, &dctl->status, dctl->cnt, s);
    ph.mark(4);
    if (he == hipSuccess) he = launch_uf_hook(parent, work, &dctl->cnt[CNT_WORK], 2 * nh, s);
    if (he == hipSuccess) he = launch_uf_label(parent, od.face_id, (long long*)r.label, nh, dctl->cnt, s);
  } else {
    ph.mark(4);
  }
  ph.mark(5);
  if (he != hipSuccess) {
    ftk_result_free(&r, &o, (ftk_stream_t)s);
    return fail(FTK_ERR_HIP, "kernel launch: %s", hipGetErrorString(he));
  }
  st = read_ctl(&h, dctl, s);
  if (!st) st = decode_status(h.status);
  if (st) {
    ftk_result_free(&r, &o, (ftk_stream_t)s);
    return st;
  }
  r.n_trajectories = (long long)h.cnt[CNT_TRAJ];
  int64_t dims[3] = {nx, ny, nt};
  r.stats.simplices_tested = count_tested(2, dims);
  r.stats.cells_linked = (long long)h.cnt[CNT_LINKED];
  r.stats.fp64_fallbacks = (long long)h.cnt[CNT_FP64];
  r.stats.degenerate_sublocations = (long long)h.cnt[CNT_DEGEN];
  r.stats.wide_path = wide ? 1 : 0;
  r.stats.t_detect_ms = ph.ms(0, 1);
  r.stats.t_scan_ms = ph.ms(1, 2);
  r.stats.t_emit_ms = ph.ms(3, 4);
  r.stats.t_link_ms = ph.ms(4, 5);
  *out = r;
  return FTK_OK;
}

// ---------------------------------------------------------------------------------------------------------------
// 3D one-shot
// ---------------------------------------------------------------------------------------------------------------
ftk_status track3d_impl(const float* field, int64_t nx, int64_t ny, int64_t nz, int64_t nt, const ftk_options& o,
                        hipStream_t s, ftk_cp_result* out) {
  const Alloc al = make_alloc(o, s);
  Scratch sc(al);
  Grid3 g;
  g.f = field;
  g.nx = (int)nx;
  g.ny = (int)ny;
  g.nz = (int)nz;
  g.nt = (int)nt;
  g.nxt = (int)((nx + 15) / 16);
  g.qscale = std::ldexp(1.0f, o.quant_log2);
  g.precision = o.precision;
  const long long V = (long long)nx * ny * nz * nt;
  const long long nseg = (long long)nt * nz * ny * g.nxt;
  uint64_t* masks = sc.get<uint64_t>((size_t)V);
  int* seg_cnt = sc.get<int>((size_t)nseg);
  long long* seg_off = sc.get<long long>((size_t)nseg);
  long long* scan_tmp = sc.get<long long>(scan_tmp_elems(nseg));
  Ctl* dctl = sc.get<Ctl>(1);
  if (!masks || !seg_cnt || !seg_off || !scan_tmp || !dctl) return fail(FTK_ERR_OOM, "scratch allocation failed");
  HIP_TRY(hipMemsetAsync(dctl, 0, sizeof(Ctl), s));
  int tt = o.slab_depth ? o.slab_depth : 8;
  if (tt > g.nt) tt = g.nt;
  Ctl h;
  bool wide = false;
  Phases ph;
  ph.init(o.profile != 0, s);
  ph.mark(0);
  HIP_TRY(launch_detect3d(g, tt, false, masks, seg_cnt, &dctl->status, s));
  ph.mark(1);
  HIP_TRY(launch_scan(seg_cnt, seg_off, nseg, &dctl->total, scan_tmp, s));
  ph.mark(2);
  ftk_status st = read_ctl(&h, dctl, s);
  if (st) return st;
  if (h.status & ST_NONFINITE) return decode_status(h.status);
  if (h.status & ST_WIDE) {
    wide = true;
    HIP_TRY(hipMemsetAsync(dctl, 0, sizeof(Ctl), s));
    ph.mark(0);
    HIP_TRY(launch_detect3d(g, tt, true, masks, seg_cnt, &dctl->status, s));
    ph.mark(1);
    HIP_TRY(launch_scan(seg_cnt, seg_off, nseg, &dctl->total, scan_tmp, s));
    ph.mark(2);
    st = read_ctl(&h, dctl, s);
    if (st) return st;
  }
  st = decode_status(h.status);
  if (st) return st;
  const long long nh = h.total;
  if (nh > 0xFFFFFFFELL) {
    out->n_hits = nh;
    return fail(FTK_ERR_CAPACITY, "%lld punctured simplices exceed the 32-bit hit index", nh);
  }
  ftk_cp_result r;
  std::memset(&r, 0, sizeof(r));
  r.n = 3;
  r.n_hits = nh;
  const unsigned outs = o.outputs;
  r.face_id = (int64_t*)al.get(sizeof(int64_t) * nh);
  if (outs & FTK_OUT_POS) r.pos = (float*)al.get(sizeof(float) * 4 * nh);
  if (outs & FTK_OUT_MU) r.mu = (float*)al.get(sizeof(float) * 4 * nh);
  if (outs & FTK_OUT_TYPE) r.type = (uint8_t*)al.get(nh);
  if (outs & FTK_OUT_FLAGS) r.flags = (uint8_t*)al.get(nh);
  if (outs & FTK_OUT_LABEL) r.label = (int64_t*)al.get(sizeof(int64_t) * nh);
  unsigned* parent = sc.get<unsigned>((size_t)nh);
  uint2* work = sc.get<uint2>((size_t)nh);
  bool oom = !r.face_id || !parent || !work || ((outs & FTK_OUT_POS) && !r.pos) || ((outs & FTK_OUT_MU) && !r.mu) ||
             ((outs & FTK_OUT_TYPE) && !r.type) || ((outs & FTK_OUT_FLAGS) && !r.flags) ||
             ((outs & FTK_OUT_LABEL) && !r.label);
  if (oom) {
    ftk_result_free(&r, &o, (ftk_stream_t)s);
    return fail(FTK_ERR_OOM, "output allocation failed (%lld hits)", nh);
  }
  Out3 od;
  od.face_id = (long long*)r.face_id;
  od.pos = r.pos;
  od.mu = r.mu;
  od.type = r.type;
  od.flags = r.flags;
  od.parent = parent;
  od.work = work;
  hipError_t he = hipSuccess;
  ph.mark(3);
  if (nh > 0) {
    he = launch_emit3d(g, wide, masks, seg_off, nseg, od, &dctl->status, dctl->cnt, s);
    ph.mark(4);
    if (he == hipSuccess) he = launch_uf_hook(parent, work, &dctl->cnt[CNT_WORK], nh, s);
    if (he == hipSuccess) he = launch_uf_label(parent, od.face_id, (long long*)r.label, nh, dctl->cnt, s);
  } else {
    ph.mark(4);
  }
  ph.mark(5);
  if (he != hipSuccess) {
    ftk_result_free(&r, &o, (ftk_stream_t)s);
    return fail(FTK_ERR_HIP, "kernel launch: %s", hipGetErrorString(he));
  }
  st = read_ctl(&h, dctl, s);
  if (!st) st = decode_status(h.status);
  if (st) {
    ftk_result_free(&r, &o, (ftk_stream_t)s);
    return st;
  }
  r.n_trajectories = (long long)h.cnt[CNT_TRAJ];
  int64_t dims[4] = {nx, ny, nz, nt};
  r.stats.simplices_tested = count_tested(3, dims);
  r.stats.cells_linked = (long long)h.cnt[CNT_LINKED];
  r.stats.fp64_fallbacks = (long long)h.cnt[CNT_FP64];
  r.stats.degenerate_sublocations = (long long)h.cnt[CNT_DEGEN];
  r.stats.wide_path = wide ? 1 : 0;
  r.stats.t_detect_ms = ph.ms(0, 1);
  r.stats.t_scan_ms = ph.ms(1, 2);
  r.stats.t_emit_ms = ph.ms(3, 4);
  r.stats.t_link_ms = ph.ms(4, 5);
  *out = r;
  return FTK_OK;
}

}  // namespace ftk

extern "C" ftk_status ftk_track_cp3d(const float* field, ftk_field_kind kind, int64_t nx, int64_t ny, int64_t nz,
                                     int64_t nt, const ftk_options* opt, ftk_stream_t stream, ftk_cp_result* out) {
  g_err.clear();
  if (!out) return fail(FTK_ERR_ARG, "out is NULL");
  std::memset(out, 0, sizeof(*out));
  if (!field) return fail(FTK_ERR_ARG, "field is NULL");
  if (kind != FTK_SCALAR) return fail(FTK_ERR_ARG, "3D tracking takes a scalar field (kind FTK_SCALAR)");
  if (nx < 2 || ny < 2 || nz < 2 || nt < 2)
    return fail(FTK_ERR_ARG, "every dimension must be >= 2 (got %lld x %lld x %lld x %lld)", (long long)nx,
                (long long)ny, (long long)nz, (long long)nt);
  if (nx > (1 << 28) || ny > (1 << 28) || nz > (1 << 28) || nt > (1 << 28) || nx * ny * nz > (1ll << 36) ||
      nx * ny * nz * nt > (1ll << 40))
    return fail(FTK_ERR_ARG, "grid too large");
  ftk_options o;
  resolve(opt, &o);
  ftk_status st = ftk::validate_options(o);
  if (st) return st;
  return ftk::track3d_impl(field, nx, ny, nz, nt, o, (hipStream_t)stream, out);
}

extern "C" ftk_status ftk_track_cp2d(const float* field, ftk_field_kind kind, int64_t nx, int64_t ny, int64_t nt,
                                     const ftk_options* opt, ftk_stream_t stream, ftk_cp_result* out) {
  g_err.clear();
  if (!out) return fail(FTK_ERR_ARG, "out is NULL");
  std::memset(out, 0, sizeof(*out));
  if (!field) return fail(FTK_ERR_ARG, "field is NULL");
  if (kind != FTK_SCALAR && kind != FTK_VECTOR) return fail(FTK_ERR_ARG, "kind must be FTK_SCALAR or FTK_VECTOR");
  if (nx < 2 || ny < 2 || nt < 2) return fail(FTK_ERR_ARG, "every dimension must be >= 2 (got %lld x %lld x %lld)",
                                               (long long)nx, (long long)ny, (long long)nt);
  if (nx > (1 << 30) || ny > (1 << 30) || nt > (1 << 30) || nx * ny > (1ll << 40) || nx * ny * nt > (1ll << 42))
    return fail(FTK_ERR_ARG, "grid too large");
  ftk_options o;
  resolve(opt, &o);
  ftk_status st = ftk::validate_options(o);
  if (st) return st;
  return ftk::track2d_impl(field, kind, nx, ny, nt, o, (hipStream_t)stream, out);
}
