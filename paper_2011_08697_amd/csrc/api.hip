// api.hip -- the C ABI (include/ftk.h): argument checks, device memory, launch sequence, status decoding.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ftk.h"
#include "common.h"
#include "internal.h"
#include "offsets16.h"

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

// Scratch memory: a small cache of device blocks reused across calls (stream-ordered allocation costs tens of
// microseconds per call on this runtime).  A block is handed back only after the call has synchronised its
// stream, so no kernel can still be using it.
struct CachedBlock {
  void* p;
  size_t size;
  int dev;
};
std::mutex g_cache_mu;
std::vector<CachedBlock> g_cache;

void* cache_get(size_t bytes, size_t* got) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  bytes = (bytes + 4095) & ~size_t(4095);
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    int best = -1;
    for (int i = 0; i < (int)g_cache.size(); ++i) {
      const CachedBlock& b = g_cache[i];
      if (b.dev == dev && b.size >= bytes && b.size <= 2 * bytes + (64u << 20) &&
          (best < 0 || b.size < g_cache[best].size))
        best = i;
    }
    if (best >= 0) {
      CachedBlock b = g_cache[best];
      g_cache.erase(g_cache.begin() + best);
      *got = b.size;
      return b.p;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    // release cached blocks of this device and retry once
    std::vector<CachedBlock> drop;
    {
      std::lock_guard<std::mutex> lk(g_cache_mu);
      for (auto it = g_cache.begin(); it != g_cache.end();)
        if (it->dev == dev) {
          drop.push_back(*it);
          it = g_cache.erase(it);
        } else {
          ++it;
        }
    }
    for (auto& b : drop) (void)hipFree(b.p);
    p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  }
  *got = bytes;
  return p;
}

void cache_put(void* p, size_t size) {
  if (!p) return;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_cache.push_back(CachedBlock{p, size, dev});
}

// Scratch list released on scope exit: to the caller's allocator when the options carry one, else to the block
// cache.  Callers synchronise their stream before returning.
struct Scratch {
  static constexpr int kMax = 32;
  const Alloc& al;  // must outlive the Scratch (declare the Alloc as a named local first)
  void* p[kMax];
  size_t sz[kMax];
  int n = 0;
  explicit Scratch(const Alloc& a) : al(a) {}
  template <typename T>
  T* get(size_t count) {
    if (n >= kMax) return nullptr;  // callers report a failed scratch allocation
    size_t got = 0;
    void* q = nullptr;
    if (al.a) {  // the caller's allocator serves scratch too (and may refuse it)
      got = count * sizeof(T) + 16;
      q = al.get(got);
    } else {
      q = cache_get(count * sizeof(T) + 16, &got);
    }
    if (q) {
      p[n] = q;
      sz[n] = got;
      ++n;
    }
    return (T*)q;
  }
  ~Scratch() {
    if (n > 0) (void)hipStreamSynchronize(al.s);  // no-op on the normal path (already synchronised)
    for (int i = n - 1; i >= 0; --i) {
      if (al.a)
        al.put(p[i]);
      else
        cache_put(p[i], sz[i]);
    }
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
  unsigned status;   // status bits of the kernels (the streaming form: of its emissions, kept from create to finish)
  unsigned dstatus;  // status bits of the streaming form's per-push detection (cleared and read by every push)
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

// Test hooks of ftk_options.debug (FTK_DEBUG_*), carried into the 2D kernels.
void set_debug(Grid2& g, const ftk_options& o) {
  g.debug = o.debug & 0xFF;
  g.debug_step = (o.debug & FTK_DEBUG_INVARIANT) ? (int)((unsigned)o.debug >> 8) : -1;
}

// Emission form for a call (or a series of a batch): the sparse one (a wavefront per non-empty row segment) when
// hits are rare, below one per kSparseVertices vertices, else the tiled one.  Both give identical outputs; the
// FTK_DEBUG_TILED_EMIT / FTK_DEBUG_SPARSE_EMIT test hooks force either.
constexpr long long kSparseVertices = 128;
bool sparse_emission(const Grid2& g, long long n_hits, long long n_vertices) {
  if (g.debug & FTK_DEBUG_SPARSE_EMIT) return true;
  if (g.debug & (FTK_DEBUG_TILED_EMIT | FTK_DEBUG_SMALL_LDS)) return false;  // the hook tests the tiled form
  return n_hits * kSparseVertices < n_vertices;
}

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

// Detection tile rows and slab depth picked by ftk_autotune_cp2d, per (kind, nx, ny): consulted when the options
// leave them at 0.  Without an entry: 16 rows, 16 steps (within a few per cent of the best on the workloads here).
struct TuneKey {
  int kind;
  long long nx, ny;
  bool operator==(const TuneKey& k) const { return kind == k.kind && nx == k.nx && ny == k.ny; }
};
std::mutex g_tune_mu;
std::vector<std::pair<TuneKey, std::pair<int, int>>> g_tune;

static bool tune_lookup(int kind, long long nx, long long ny, int* ty, int* tt) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& e : g_tune)
    if (e.first == TuneKey{kind, nx, ny}) {
      *ty = e.second.first;
      *tt = e.second.second;
      return true;
    }
  return false;
}

static void tune_store(int kind, long long nx, long long ny, int ty, int tt) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& e : g_tune)
    if (e.first == TuneKey{kind, nx, ny}) {
      e.second = {ty, tt};
      return;
    }
  g_tune.push_back({TuneKey{kind, nx, ny}, {ty, tt}});
}

static void tuned_tiles2(const ftk_options& o, int kind, long long nx, long long ny, int nt, int* ty, int* tt) {
  int dty = 16, dtt = 16;
  tune_lookup(kind, nx, ny, &dty, &dtt);
  *ty = o.tile_y ? o.tile_y : dty;
  *tt = o.slab_depth ? o.slab_depth : dtt;
  if (*tt > nt) *tt = nt;
}

// Byte offsets of several arrays carved from one region (each 256-byte aligned).
struct Carve {
  size_t total = 0;
  template <typename T>
  size_t add(size_t count) {
    const size_t at = total;
    total += (count * sizeof(T) + 16 + 255) & ~size_t(255);
    return at;
  }
};

// Where a 2D tracking call takes its device memory: two scratch regions (group 0 before detection: masks, counts,
// offsets, scan temporaries, control block; group 1 once the hit count is known: union-find parents and the edge
// list) and the output arrays.
struct Mem2 {
  virtual ~Mem2() {}
  virtual char* scratch(int group, size_t bytes) = 0;  // null: refused (status from scratch_error)
  virtual ftk_status scratch_error(int group, size_t bytes) = 0;
  virtual ftk_status outputs(ftk_cp_result& r, long long nh, unsigned outs) = 0;
  virtual void drop_outputs(ftk_cp_result& r) = 0;
};

// The library's own memory: scratch from the caller's allocator hooks when given, else from the block cache;
// outputs from the hooks or the stream-ordered HIP allocator.
struct OwnMem2 : Mem2 {
  const ftk_options& o;
  hipStream_t s;
  const Alloc al;
  Scratch sc;
  OwnMem2(const ftk_options& opt, hipStream_t st) : o(opt), s(st), al(make_alloc(opt, st)), sc(al) {}
  char* scratch(int, size_t bytes) override { return sc.get<char>(bytes); }
  ftk_status scratch_error(int group, size_t bytes) override {
    return fail(FTK_ERR_OOM, "scratch allocation failed (%zu bytes, %s)", bytes,
                group == 0 ? "detection" : "union-find");
  }
  ftk_status outputs(ftk_cp_result& r, long long nh, unsigned outs) override {
    r.face_id = (int64_t*)al.get(sizeof(int64_t) * nh);
    if (outs & FTK_OUT_POS) r.pos = (float*)al.get(sizeof(float) * 3 * nh);
    if (outs & FTK_OUT_MU) r.mu = (float*)al.get(sizeof(float) * 3 * nh);
    if (outs & FTK_OUT_TYPE) r.type = (uint8_t*)al.get(nh);
    if (outs & FTK_OUT_FLAGS) r.flags = (uint8_t*)al.get(nh);
    if (outs & FTK_OUT_LABEL) r.label = (int64_t*)al.get(sizeof(int64_t) * nh);
    const bool oom = !r.face_id || ((outs & FTK_OUT_POS) && !r.pos) || ((outs & FTK_OUT_MU) && !r.mu) ||
                     ((outs & FTK_OUT_TYPE) && !r.type) || ((outs & FTK_OUT_FLAGS) && !r.flags) ||
                     ((outs & FTK_OUT_LABEL) && !r.label);
    if (oom) {
      drop_outputs(r);
      return fail(FTK_ERR_OOM, "output allocation failed (%lld hits)", nh);
    }
    return FTK_OK;
  }
  void drop_outputs(ftk_cp_result& r) override { ftk_result_free(&r, &o, (ftk_stream_t)s); }
};

__global__ void zero_words(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// n words set to v (a kernel rather than hipMemsetAsync: the 2D one-shot call may run under graph capture)
__global__ void fill_words(unsigned* p, unsigned v, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_words(unsigned* p, unsigned v, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  fill_words<<<(unsigned)blocks, 256, 0, s>>>(p, v, n);
  return hipGetLastError();
}

// Clears the control block with a kernel (no memset node, so the sequence is safe under stream capture too).
hipError_t clear_ctl(Ctl* d, hipStream_t s) {
  constexpr int n = (int)(sizeof(Ctl) / sizeof(unsigned));
  zero_words<<<1, 64, 0, s>>>((unsigned*)d, n);
  return hipGetLastError();
}

ftk_status track2d_core(const float* field, ftk_field_kind kind, int64_t nx, int64_t ny, int64_t nt,
                        const ftk_options& o, hipStream_t s, Mem2& mem, ftk_cp_result* out) {
  Grid2 g;
  g.f = field;
  g.kind = (int)kind;
  g.nx = (int)nx;
  g.ny = (int)ny;
  g.nt = (int)nt;
  g.nxt = (int)((nx + 63) / 64);
  g.qscale = std::ldexp(1.0f, o.quant_log2);
  g.precision = o.precision;
  g.t_begin = 0;
  g.t_end = (int)nt;
  g.f_ring = 0;
  g.m_ring = 0;
  set_debug(g, o);
  const long long V = (long long)nx * ny * nt;
  const long long nseg = (long long)nt * ny * g.nxt;

  Carve c0;
  const size_t o_masks = c0.add<uint16_t>((size_t)V);
  const size_t o_cnt = c0.add<int>((size_t)nseg);
  const size_t o_off = c0.add<long long>((size_t)nseg);
  const size_t o_tmp = c0.add<long long>(scan_tmp_elems(nseg));
  const size_t o_ctl = c0.add<Ctl>(1);
  char* b0 = mem.scratch(0, c0.total);
  if (!b0) return mem.scratch_error(0, c0.total);
  uint16_t* masks = (uint16_t*)(b0 + o_masks);
  int* seg_cnt = (int*)(b0 + o_cnt);
  long long* seg_off = (long long*)(b0 + o_off);
  long long* scan_tmp = (long long*)(b0 + o_tmp);
  Ctl* dctl = (Ctl*)(b0 + o_ctl);
  HIP_TRY(clear_ctl(dctl, s));

  int ty, tt;
  tuned_tiles2(o, g.kind, nx, ny, g.nt, &ty, &tt);
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
    HIP_TRY(clear_ctl(dctl, s));
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

  Carve c1;
  const size_t o_parent = c1.add<unsigned>((size_t)nh);
  const size_t o_work = c1.add<uint2>((size_t)nh * 2);
  char* b1 = mem.scratch(1, c1.total);
  if (!b1) {
    const ftk_status e = mem.scratch_error(1, c1.total);
    if (e == FTK_ERR_CAPACITY) out->n_hits = nh;
    return e;
  }
  unsigned* parent = (unsigned*)(b1 + o_parent);
  uint2* work = (uint2*)(b1 + o_work);

  ftk_cp_result r;
  std::memset(&r, 0, sizeof(r));
  r.n = 2;
  r.n_hits = nh;
  st = mem.outputs(r, nh, o.outputs);
  if (st) {
    if (st == FTK_ERR_CAPACITY) out->n_hits = nh;
    return st;
  }
  Out2 od;
  od.gbase = 0;
  od.label = (long long*)r.label;
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
    const bool sparse = sparse_emission(g, nh, V);
    if (sparse) {
      he = launch_fill_words(parent, 0xFFFFFFFFu, nh, s);
      if (he == hipSuccess)
        he = launch_emit2d_sparse(g, wide, masks, seg_cnt, seg_off, od, &dctl->status, dctl->cnt, s);
    } else {
      he = launch_emit2d(g, wide, masks, seg_cnt, seg_off, od, &dctl->status, dctl->cnt, s);
    }
    ph.mark(4);
    if (he == hipSuccess && sparse) he = launch_uf_compress(parent, nh, s);
    if (he == hipSuccess)
      he = sparse ? launch_uf_hook_slots(parent, work, nh, s)
                  : launch_uf_hook(parent, work, &dctl->cnt[CNT_WORK], 2 * nh, s);
    if (he == hipSuccess) he = launch_uf_label(parent, od.face_id, (long long*)r.label, nh, dctl->cnt, s);
  } else {
    ph.mark(4);
  }
  ph.mark(5);
  if (he != hipSuccess) {
    mem.drop_outputs(r);
    return fail(FTK_ERR_HIP, "kernel launch: %s", hipGetErrorString(he));
  }
  st = read_ctl(&h, dctl, s);
  if (!st) st = decode_status(h.status);
  if (st) {
    mem.drop_outputs(r);
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

ftk_status track2d_impl(const float* field, ftk_field_kind kind, int64_t nx, int64_t ny, int64_t nt,
                        const ftk_options& o, hipStream_t s, ftk_cp_result* out) {
  OwnMem2 mem(o, s);
  return track2d_core(field, kind, nx, ny, nt, o, s, mem, out);
}

// ---------------------------------------------------------------------------------------------------------------
// The 2D call that allocates nothing (ftk_track_cp2d_into): outputs in the caller's arrays, scratch carved from one
// fixed region per device.  The array below is a device symbol; host code reaches its memory only through the
// address hipGetSymbolAddress returns for the current device (the array's name is not a device address in host
// code).  Calls on one device share the region, so overlapping calls on one device race.
// ---------------------------------------------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = (size_t)FTK_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's region, looked up once per device.
ftk_status static_scratch(char** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(FTK_ERR_ARG, "device ordinal %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(FTK_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = (char*)p;
  }
  *out = g_scratch_ptr[dev];
  return FTK_OK;
}

// Scratch groups carved one after the other from the region; outputs are the caller's arrays.
struct StaticMem2 : Mem2 {
  char* base;
  size_t used = 0;
  const ftk_cp_result& io;  // the caller's output pointers
  long long capacity;
  StaticMem2(char* b, const ftk_cp_result& r, long long cap) : base(b), io(r), capacity(cap) {}
  char* scratch(int, size_t bytes) override {
    if (bytes > kStaticScratchBytes - used) return nullptr;
    char* p = base + used;
    used += bytes;
    return p;
  }
  ftk_status scratch_error(int group, size_t bytes) override {
    return fail(FTK_ERR_CAPACITY, "%s scratch of %zu bytes (after %zu in use) exceeds the %zu-byte static region",
                group == 0 ? "detection" : "union-find", bytes, used, kStaticScratchBytes);
  }
  ftk_status outputs(ftk_cp_result& r, long long nh, unsigned outs) override {
    if (nh > capacity)
      return fail(FTK_ERR_CAPACITY, "%lld punctured simplices exceed the output capacity of %lld", nh, capacity);
    r.face_id = io.face_id;
    r.pos = (outs & FTK_OUT_POS) ? io.pos : nullptr;
    r.mu = (outs & FTK_OUT_MU) ? io.mu : nullptr;
    r.type = (outs & FTK_OUT_TYPE) ? io.type : nullptr;
    r.flags = (outs & FTK_OUT_FLAGS) ? io.flags : nullptr;
    r.label = (outs & FTK_OUT_LABEL) ? io.label : nullptr;
    return FTK_OK;
  }
  void drop_outputs(ftk_cp_result& r) override { std::memset(&r, 0, sizeof(r)); }  // the caller's arrays
};

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
  g.t_begin = 0;
  g.t_end = (int)nt;
  g.f_ring = 0;
  g.m_ring = 0;
  const long long V = (long long)nx * ny * nz * nt;
  const long long nseg = (long long)nt * nz * ny * g.nxt;
  uint64_t* masks = sc.get<uint64_t>((size_t)V);
  int* seg_cnt = sc.get<int>((size_t)nseg);
  long long* seg_off = sc.get<long long>((size_t)nseg);
  long long* scan_tmp = sc.get<long long>(scan_tmp_elems(nseg));
  Ctl* dctl = sc.get<Ctl>(1);
  g.cert = sc.get<unsigned char>((size_t)(nt * cert3_plane(g)));
  if (!masks || !seg_cnt || !seg_off || !scan_tmp || !dctl || !g.cert)
    return fail(FTK_ERR_OOM, "scratch allocation failed");
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
  long long* list = sc.get<long long>((size_t)nh);  // row chunks with hits: at most one per hit
  bool oom = !r.face_id || !parent || !work || !list || ((outs & FTK_OUT_POS) && !r.pos) || ((outs & FTK_OUT_MU) && !r.mu) ||
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
    he = launch_emit3d(g, wide, masks, seg_cnt, seg_off, nh, od, &dctl->status, dctl->cnt, list, &dctl->cnt[CNT_LIST],
                       s);
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

// ---------------------------------------------------------------------------------------------------------------
// 2D batched: all series in one persistent launch per stage, concatenated scratch, one global union-find.
// ---------------------------------------------------------------------------------------------------------------
__global__ void gather_bases(const long long* __restrict__ seg_off, const long long* __restrict__ seg_start, int nser,
                             const long long* __restrict__ total, long long* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nser) out[i] = seg_off[seg_start[i]];
  if (i == nser) out[i] = *total;
}

ftk_status track2d_batched_impl(int nser, const float* const* fields, const int64_t* nx, const int64_t* ny,
                                const int64_t* nt, ftk_field_kind kind, const ftk_options& o, hipStream_t s,
                                ftk_cp_result* outs) {
  const Alloc al = make_alloc(o, s);
  Scratch sc(al);
  constexpr int TYD = 16, TYE = 8;
  // slab depth: the option, else the tuned one of the series with the most vertices, else 16 (rows fixed at 16)
  int ttd = o.slab_depth;
  if (!ttd) {
    int big = 0;
    for (int i = 1; i < nser; ++i)
      if (nx[i] * ny[i] * nt[i] > nx[big] * ny[big] * nt[big]) big = i;
    int tty = 16, ttt = 16;
    tune_lookup((int)kind, nx[big], ny[big], &tty, &ttt);
    ttd = ttt;
  }
  std::vector<Series2> ser(nser);
  std::vector<long long> mask_off(nser), seg_start(nser);
  std::vector<int> pre_d(nser + 1), pre_e(nser + 1);
  long long Vtot = 0, Stot = 0;
  pre_d[0] = pre_e[0] = 0;
  for (int i = 0; i < nser; ++i) {
    Grid2& g = ser[i].g;
    g.f = fields[i];
    g.kind = (int)kind;
    g.nx = (int)nx[i];
    g.ny = (int)ny[i];
    g.nt = (int)nt[i];
    g.nxt = (int)((nx[i] + 63) / 64);
    g.qscale = std::ldexp(1.0f, o.quant_log2);
    g.precision = o.precision;
    g.t_begin = 0;
    g.t_end = g.nt;
    g.f_ring = 0;
    g.m_ring = 0;
    set_debug(g, o);
    mask_off[i] = Vtot;
    seg_start[i] = Stot;
    Vtot += (long long)nx[i] * ny[i] * nt[i];
    Stot += (long long)nt[i] * ny[i] * g.nxt;
    const int tt = ttd < g.nt ? ttd : g.nt;
    pre_d[i + 1] = pre_d[i] + g.nxt * (int)((g.ny + TYD - 1) / TYD) * (int)((g.nt + tt - 1) / tt);
    pre_e[i + 1] = pre_e[i] + g.nxt * (int)((g.ny + TYE - 1) / TYE) * (int)((g.nt + 16 - 1) / 16);
  }
  uint16_t* masks = sc.get<uint16_t>((size_t)Vtot);
  int* seg_cnt = sc.get<int>((size_t)Stot);
  long long* seg_off = sc.get<long long>((size_t)Stot);
  long long* scan_tmp = sc.get<long long>(scan_tmp_elems(Stot));
  Ctl* dctl = sc.get<Ctl>(1);
  Series2* dser = sc.get<Series2>((size_t)nser);
  int* dpre = sc.get<int>((size_t)(2 * nser + 4));
  long long* dseg_start = sc.get<long long>((size_t)nser);
  long long* dbases = sc.get<long long>((size_t)nser + 1);
  unsigned long long* dcnt = sc.get<unsigned long long>((size_t)nser * CNT_N);
  int* dctr = sc.get<int>(4);
  if (!masks || !seg_cnt || !seg_off || !scan_tmp || !dctl || !dser || !dpre || !dseg_start || !dbases || !dcnt ||
      !dctr)
    return fail(FTK_ERR_OOM, "scratch allocation failed");
  for (int i = 0; i < nser; ++i) {
    ser[i].masks = masks + mask_off[i];
    ser[i].seg_cnt = seg_cnt + seg_start[i];
    ser[i].seg_off = seg_off + seg_start[i];
    ser[i].cnt = dcnt + (size_t)i * CNT_N;
    ser[i].wide = 0;
    std::memset(&ser[i].o, 0, sizeof(Out2));
  }
  HIP_TRY(hipMemsetAsync(dctl, 0, sizeof(Ctl), s));
  HIP_TRY(hipMemsetAsync(dcnt, 0, sizeof(unsigned long long) * CNT_N * nser, s));
  HIP_TRY(hipMemsetAsync(dctr, 0, sizeof(int) * 4, s));
  HIP_TRY(hipMemcpyAsync(dser, ser.data(), sizeof(Series2) * nser, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(dpre, pre_d.data(), sizeof(int) * (nser + 1), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(dpre + nser + 1, pre_e.data(), sizeof(int) * (nser + 1), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(dseg_start, seg_start.data(), sizeof(long long) * nser, hipMemcpyHostToDevice, s));
  Phases ph;
  ph.init(o.profile != 0, s);
  bool wide = false;
  Ctl h;
  std::vector<long long> bases(nser + 1);
  for (int pass = 0; pass < 2; ++pass) {
    ph.mark(0);
    HIP_TRY(launch_detect2d_batched(dser, dpre, nser, pre_d[nser], ttd, wide, dctr, &dctl->status, s));
    ph.mark(1);
    HIP_TRY(launch_scan(seg_cnt, seg_off, Stot, &dctl->total, scan_tmp, s));
    gather_bases<<<(nser + 256) / 256, 256, 0, s>>>(seg_off, dseg_start, nser, &dctl->total, dbases);
    HIP_TRY(hipGetLastError());
    ph.mark(2);
    HIP_TRY(hipMemcpyAsync(bases.data(), dbases, sizeof(long long) * (nser + 1), hipMemcpyDeviceToHost, s));
    ftk_status st = read_ctl(&h, dctl, s);
    if (st) return st;
    if (h.status & ST_NONFINITE) return decode_status(h.status);
    if (!(h.status & ST_WIDE) || wide) break;
    wide = true;
    HIP_TRY(hipMemsetAsync(dctl, 0, sizeof(Ctl), s));
    HIP_TRY(hipMemsetAsync(dctr, 0, sizeof(int) * 4, s));
  }
  ftk_status st = decode_status(h.status);
  if (st) return st;
  const long long total = h.total;
  if (total > 0xFFFFFFFELL) return fail(FTK_ERR_CAPACITY, "%lld punctured simplices in the batch exceed 2^32 - 2", total);
  unsigned* parent = sc.get<unsigned>((size_t)total);
  uint2* work = sc.get<uint2>((size_t)total * 2);
  unsigned* dgb = sc.get<unsigned>((size_t)nser + 1);
  long long* dpb = sc.get<long long>((size_t)nser + 1);
  if (!parent || !work || !dgb || !dpb) return fail(FTK_ERR_OOM, "scratch allocation failed");
  // emission form per series: tiled items (pre_e) for the dense ones, 64-segment blocks (pre_b) for the sparse ones
  std::vector<long long> pre_b(nser + 1);
  std::vector<char> sparse(nser);
  pre_b[0] = 0;
  for (int i = 0; i < nser; ++i) {
    const Grid2& g = ser[i].g;
    sparse[i] = sparse_emission(g, bases[i + 1] - bases[i], (long long)g.nx * g.ny * g.nt) ? 1 : 0;
    const int items = pre_e[i + 1] - pre_e[i];
    pre_e[i + 1] = pre_e[i] + (sparse[i] ? 0 : items);
    pre_b[i + 1] = pre_b[i] + (sparse[i] ? ((long long)g.nt * g.ny * g.nxt + 63) / 64 : 0);
  }
  // link slots of the sparse series (one per global hit index; cleared when tiled series leave some unwritten) and
  // their parents' initial value
  uint2* slots = nullptr;
  if (pre_b[nser] > 0) {
    slots = sc.get<uint2>((size_t)total);
    if (!slots) return fail(FTK_ERR_OOM, "scratch allocation failed");
    if (pre_e[nser] > 0) HIP_TRY(hipMemsetAsync(slots, 0, sizeof(uint2) * (size_t)total, s));
    HIP_TRY(hipMemsetAsync(parent, 0xFF, sizeof(unsigned) * (size_t)total, s));
  }
  std::vector<unsigned> gb(nser + 1);
  const unsigned outs_mask = o.outputs;
  bool oom = false;
  for (int i = 0; i < nser; ++i) {
    const long long nh = bases[i + 1] - bases[i];
    gb[i] = (unsigned)bases[i];
    ftk_cp_result& r = outs[i];
    std::memset(&r, 0, sizeof(r));
    r.n = 2;
    r.n_hits = nh;
    r.face_id = (int64_t*)al.get(sizeof(int64_t) * nh);
    if (outs_mask & FTK_OUT_POS) r.pos = (float*)al.get(sizeof(float) * 3 * nh);
    if (outs_mask & FTK_OUT_MU) r.mu = (float*)al.get(sizeof(float) * 3 * nh);
    if (outs_mask & FTK_OUT_TYPE) r.type = (uint8_t*)al.get(nh);
    if (outs_mask & FTK_OUT_FLAGS) r.flags = (uint8_t*)al.get(nh);
    if (outs_mask & FTK_OUT_LABEL) r.label = (int64_t*)al.get(sizeof(int64_t) * nh);
    oom = oom || !r.face_id || ((outs_mask & FTK_OUT_POS) && !r.pos) || ((outs_mask & FTK_OUT_MU) && !r.mu) ||
          ((outs_mask & FTK_OUT_TYPE) && !r.type) || ((outs_mask & FTK_OUT_FLAGS) && !r.flags) ||
          ((outs_mask & FTK_OUT_LABEL) && !r.label);
    Out2& od = ser[i].o;
    od.gbase = (unsigned)bases[i];
    od.face_id = (long long*)r.face_id;
    od.pos = r.pos;
    od.mu = r.mu;
    od.type = r.type;
    od.flags = r.flags;
    od.label = (long long*)r.label;
    od.parent = parent;
    od.work = sparse[i] ? slots : work;
    ser[i].wide = wide ? 1 : 0;
  }
  gb[nser] = (unsigned)total;
  auto free_all = [&]() {
    for (int i = 0; i < nser; ++i) ftk_result_free(&outs[i], &o, (ftk_stream_t)s);
  };
  if (oom) {
    free_all();
    return fail(FTK_ERR_OOM, "output allocation failed");
  }
  HIP_TRY(hipMemcpyAsync(dser, ser.data(), sizeof(Series2) * nser, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(dgb, gb.data(), sizeof(unsigned) * (nser + 1), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(dpre + nser + 1, pre_e.data(), sizeof(int) * (nser + 1), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(dpb, pre_b.data(), sizeof(long long) * (nser + 1), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(dctr, 0, sizeof(int) * 4, s));
  ph.mark(3);
  hipError_t he = hipSuccess;
  if (total > 0) {
    if (pre_e[nser] > 0)
      he = launch_emit2d_batched(dser, dpre + nser + 1, nser, pre_e[nser], wide, dctr, &dctl->status,
                                 &dctl->cnt[CNT_WORK], s);
    if (he == hipSuccess && pre_b[nser] > 0)
      he = launch_emit2d_sparse_batched(dser, dpb, nser, pre_b[nser], wide, &dctl->status, s);
    ph.mark(4);
    if (he == hipSuccess && slots) he = launch_uf_compress(parent, total, s);
    if (he == hipSuccess && pre_e[nser] > 0) he = launch_uf_hook(parent, work, &dctl->cnt[CNT_WORK], 2 * total, s);
    if (he == hipSuccess && slots) he = launch_uf_hook_slots(parent, slots, total, s);
    if (he == hipSuccess) he = launch_uf_label_batched(parent, dser, dgb, nser, total, s);
  } else {
    ph.mark(4);
  }
  ph.mark(5);
  if (he != hipSuccess) {
    free_all();
    return fail(FTK_ERR_HIP, "kernel launch: %s", hipGetErrorString(he));
  }
  std::vector<unsigned long long> hc((size_t)nser * CNT_N);
  HIP_TRY(hipMemcpyAsync(hc.data(), dcnt, sizeof(unsigned long long) * CNT_N * nser, hipMemcpyDeviceToHost, s));
  st = read_ctl(&h, dctl, s);
  if (!st) st = decode_status(h.status);
  if (st) {
    free_all();
    return st;
  }
  for (int i = 0; i < nser; ++i) {
    ftk_cp_result& r = outs[i];
    const unsigned long long* c = &hc[(size_t)i * CNT_N];
    r.n_trajectories = (long long)c[CNT_TRAJ];
    int64_t dims[3] = {nx[i], ny[i], nt[i]};
    r.stats.simplices_tested = count_tested(2, dims);
    r.stats.cells_linked = (long long)c[CNT_LINKED];
    r.stats.fp64_fallbacks = (long long)c[CNT_FP64];
    r.stats.degenerate_sublocations = (long long)c[CNT_DEGEN];
    r.stats.wide_path = wide ? 1 : 0;
    if (i == 0) {
      r.stats.t_detect_ms = ph.ms(0, 1);
      r.stats.t_scan_ms = ph.ms(1, 2);
      r.stats.t_emit_ms = ph.ms(3, 4);
      r.stats.t_link_ms = ph.ms(4, 5);
    }
  }
  return FTK_OK;
}

// ---------------------------------------------------------------------------------------------------------------
// Streaming (Sec. 3.2 "Ordinal and interval mesh elements": every simplex is visited with a sliding window of two
// time steps).  2D: the tracker keeps the last three steps in a ring; pushing step s detects the anchors of step
// s-1 (its ordinal simplices and the interval ones towards s) and emits step s-2, whose +t neighbour masks now
// exist.  finish() closes the series and runs the global union-find passes.  3D: the steps are accumulated on the
// device and the one-shot path runs at finish().
// ---------------------------------------------------------------------------------------------------------------
__global__ void add_plane_base(long long* __restrict__ off, long long n, const long long* __restrict__ running) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) off[i] += *running;
}
__global__ void bump_running(long long* running, const long long* plane_total) { *running += *plane_total; }

}  // namespace ftk

struct ftk_tracker {
  int n = 2;
  int64_t nx = 0, ny = 0, nz = 1;
  ftk_field_kind kind = FTK_SCALAR;
  ftk_options o{};
  hipStream_t s = nullptr;
  int steps = 0;
  int state = 0;  // 0 open, 1 finished, 2 failed
  size_t step_elems = 0;
  // window of the last steps (ring of 3): field steps, puncture masks (2D: 12 bits, 3D: 60 bits per vertex),
  // per-segment counts and offsets
  float* fring = nullptr;
  uint16_t* mring = nullptr;
  uint64_t* mring3 = nullptr;
  long long* list3 = nullptr;  // 3D emission: 64-vertex row chunks with hits of the emitted step
  unsigned char* cert3 = nullptr;  // 3D: certified detection tile-steps (ring of 3 planes)
  int* cring = nullptr;
  long long* oring = nullptr;
  long long* scan_tmp = nullptr;
  void* dctl = nullptr;
  long long* dplane = nullptr;
  long long nseg_plane = 0;
  int plane_wide[3] = {0, 0, 0};
  std::vector<long long> total_after;  // hits through step p
  long long emitted = 0;               // hits of the emitted steps
  // outputs and union-find scratch (grown on demand)
  long long cap = 0;
  long long* face_id = nullptr;
  float* pos = nullptr;
  float* mu = nullptr;
  uint8_t* type = nullptr;
  uint8_t* flags = nullptr;
  unsigned* parent = nullptr;
  uint2* work = nullptr;
};

namespace ftk {

static Alloc tracker_alloc(ftk_tracker* h) { return make_alloc(h->o, h->s); }

static void tracker_free_all(ftk_tracker* h) {
  const Alloc al = tracker_alloc(h);
  (void)hipStreamSynchronize(h->s);
  void* ps[] = {h->fring, h->mring, h->mring3, h->list3, h->cert3, h->cring, h->oring, h->scan_tmp, h->dctl,
                h->dplane, h->face_id, h->pos, h->mu, h->type, h->flags, h->parent, h->work};
  for (void* p : ps) al.put(p);
  h->fring = nullptr;
  h->mring = nullptr;
  h->mring3 = nullptr;
  h->list3 = nullptr;
  h->cert3 = nullptr;
  h->cring = nullptr;
  h->oring = nullptr;
  h->scan_tmp = nullptr;
  h->dctl = nullptr;
  h->dplane = nullptr;
  h->face_id = nullptr;
  h->pos = h->mu = nullptr;
  h->type = h->flags = nullptr;
  h->parent = nullptr;
  h->work = nullptr;
}

// Grow the output and union-find arrays to hold `need` hits, keeping the first `keep` entries.
static ftk_status tracker_reserve(ftk_tracker* h, long long need, long long keep) {
  if (need <= h->cap) return FTK_OK;
  const Alloc al = tracker_alloc(h);
  long long nc = h->cap ? h->cap : 1024;
  while (nc < need) nc = nc + nc / 2 + 1024;
  const unsigned outs = h->o.outputs;
  auto grow = [&](void** p, size_t elem, bool want) -> bool {
    if (!want) return true;
    void* q = al.get(elem * (size_t)nc);
    if (!q) return false;
    if (*p && keep > 0 && hipMemcpyAsync(q, *p, elem * (size_t)keep, hipMemcpyDeviceToDevice, h->s) != hipSuccess)
      return false;
    al.put(*p);
    *p = q;
    return true;
  };
  const size_t pe = 4 * (size_t)(h->n + 1);  // position / barycentric bytes per hit
  bool ok = grow((void**)&h->face_id, 8, true) && grow((void**)&h->pos, pe, (outs & FTK_OUT_POS) != 0) &&
            grow((void**)&h->mu, pe, (outs & FTK_OUT_MU) != 0) && grow((void**)&h->type, 1, (outs & FTK_OUT_TYPE) != 0) &&
            grow((void**)&h->flags, 1, (outs & FTK_OUT_FLAGS) != 0) && grow((void**)&h->parent, 4, true);
  if (ok) {
    // the edge list is rebuilt from the device counter, keep all of it
    void* q = al.get(sizeof(uint2) * 2 * (size_t)nc);
    if (!q) {
      ok = false;
    } else {
      if (h->work && hipMemcpyAsync(q, h->work, sizeof(uint2) * 2 * (size_t)h->cap, hipMemcpyDeviceToDevice, h->s) !=
                         hipSuccess)
        ok = false;
      al.put(h->work);
      h->work = (uint2*)q;
    }
  }
  if (!ok) return fail(FTK_ERR_OOM, "streaming output allocation failed (%lld hits)", need);
  h->cap = nc;
  return FTK_OK;
}

static Grid2 tracker_grid(ftk_tracker* h, int t_begin, int nt) {
  Grid2 g;
  g.f = h->fring;
  g.kind = (int)h->kind;
  g.nx = (int)h->nx;
  g.ny = (int)h->ny;
  g.nt = nt;
  g.nxt = (int)((h->nx + 63) / 64);
  g.qscale = std::ldexp(1.0f, h->o.quant_log2);
  g.precision = h->o.precision;
  g.t_begin = t_begin;
  g.t_end = t_begin + 1;
  g.f_ring = 3;
  g.m_ring = 3;
  set_debug(g, h->o);
  return g;
}

constexpr int kOpenNt = 1 << 29;  // "series still open": no step is the last one

// Detection + offsets of step p (anchors at p), nt = kOpenNt while open.
static ftk_status tracker_detect(ftk_tracker* h, int p, int nt) {
  Ctl* dctl = (Ctl*)h->dctl;
  Grid2 g = tracker_grid(h, p, nt);
  const int slot = p % 3;
  int* cnt = h->cring + (size_t)slot * h->nseg_plane;
  long long* off = h->oring + (size_t)slot * h->nseg_plane;
  int ty = h->o.tile_y ? h->o.tile_y : 16;
  for (int pass = 0; pass < 2; ++pass) {
    const bool wide = pass == 1;
    HIP_TRY(hipMemsetAsync(&dctl->dstatus, 0, sizeof(unsigned), h->s));
    HIP_TRY(launch_detect2d(g, ty, 1, wide, h->mring, h->cring, &dctl->dstatus, h->s));
    unsigned st = 0;
    HIP_TRY(hipMemcpyAsync(&st, &dctl->dstatus, sizeof(unsigned), hipMemcpyDeviceToHost, h->s));
    HIP_TRY(hipStreamSynchronize(h->s));
    if (st & ST_NONFINITE) return decode_status(st);
    if (st & ST_RANGE) return decode_status(st);
    if (!(st & ST_WIDE)) {
      h->plane_wide[slot] = wide ? 1 : 0;
      break;
    }
  }
  HIP_TRY(launch_scan(cnt, off, h->nseg_plane, h->dplane, h->scan_tmp, h->s));
  add_plane_base<<<(unsigned)((h->nseg_plane + 255) / 256), 256, 0, h->s>>>(off, h->nseg_plane, &dctl->total);
  bump_running<<<1, 1, 0, h->s>>>(&dctl->total, h->dplane);
  HIP_TRY(hipGetLastError());
  long long tot = 0;
  HIP_TRY(hipMemcpyAsync(&tot, &dctl->total, sizeof(long long), hipMemcpyDeviceToHost, h->s));
  HIP_TRY(hipStreamSynchronize(h->s));
  if (tot > 0xFFFFFFFELL) return fail(FTK_ERR_CAPACITY, "%lld punctured simplices exceed 2^32 - 2", tot);
  h->total_after.push_back(tot);
  return tracker_reserve(h, tot, h->emitted);
}

static ftk_status tracker_emit(ftk_tracker* h, int e, int nt) {
  Ctl* dctl = (Ctl*)h->dctl;
  Grid2 g = tracker_grid(h, e, nt);
  Out2 od;
  od.gbase = 0;
  od.face_id = h->face_id;
  od.pos = h->pos;
  od.mu = h->mu;
  od.type = h->type;
  od.flags = h->flags;
  od.parent = h->parent;
  od.work = h->work;
  od.label = nullptr;
  HIP_TRY(launch_emit2d_steps(g, h->plane_wide[e % 3] != 0, h->mring, h->cring, h->oring, od, &dctl->status, dctl->cnt, h->s));
  h->emitted = h->total_after[e];
  return FTK_OK;
}

// 3D window: the same schedule on the 4D Kuhn mesh.  Detecting the anchors of step p reads the field steps p and
// p + 1; emitting step e reads the field steps e and e + 1 and the masks and offsets of the steps e - 1 .. e + 1
// (the pentachora holding a tetrahedron reach one step either way), so three slots of each suffice.
static Grid3 tracker_grid3(ftk_tracker* h, int t_begin, int nt) {
  Grid3 g;
  g.f = h->fring;
  g.nx = (int)h->nx;
  g.ny = (int)h->ny;
  g.nz = (int)h->nz;
  g.nt = nt;
  g.nxt = (int)((h->nx + 15) / 16);
  g.qscale = std::ldexp(1.0f, h->o.quant_log2);
  g.precision = h->o.precision;
  g.t_begin = t_begin;
  g.t_end = t_begin + 1;
  g.f_ring = 3;
  g.m_ring = 3;
  g.cert = h->cert3;
  return g;
}

static ftk_status tracker_detect3(ftk_tracker* h, int p, int nt) {
  Ctl* dctl = (Ctl*)h->dctl;
  const Grid3 g = tracker_grid3(h, p, nt);
  const int slot = p % 3;
  int* cnt = h->cring + (size_t)slot * h->nseg_plane;
  long long* off = h->oring + (size_t)slot * h->nseg_plane;
  for (int pass = 0; pass < 2; ++pass) {
    const bool wide = pass == 1;
    zero_words<<<1, 64, 0, h->s>>>(&dctl->dstatus, 1);
    HIP_TRY(hipGetLastError());
    HIP_TRY(launch_detect3d(g, 1, wide, h->mring3, h->cring, &dctl->dstatus, h->s));
    unsigned st = 0;
    HIP_TRY(hipMemcpyAsync(&st, &dctl->dstatus, sizeof(unsigned), hipMemcpyDeviceToHost, h->s));
    HIP_TRY(hipStreamSynchronize(h->s));
    if (st & (ST_NONFINITE | ST_RANGE)) return decode_status(st);
    if (!(st & ST_WIDE)) {
      h->plane_wide[slot] = wide ? 1 : 0;
      break;
    }
  }
  HIP_TRY(launch_scan(cnt, off, h->nseg_plane, h->dplane, h->scan_tmp, h->s));
  add_plane_base<<<(unsigned)((h->nseg_plane + 255) / 256), 256, 0, h->s>>>(off, h->nseg_plane, &dctl->total);
  bump_running<<<1, 1, 0, h->s>>>(&dctl->total, h->dplane);
  HIP_TRY(hipGetLastError());
  long long tot = 0;
  HIP_TRY(hipMemcpyAsync(&tot, &dctl->total, sizeof(long long), hipMemcpyDeviceToHost, h->s));
  HIP_TRY(hipStreamSynchronize(h->s));
  if (tot > 0xFFFFFFFELL) return fail(FTK_ERR_CAPACITY, "%lld punctured simplices exceed 2^32 - 2", tot);
  h->total_after.push_back(tot);
  return tracker_reserve(h, tot, h->emitted);
}

static ftk_status tracker_emit3(ftk_tracker* h, int e, int nt) {
  Ctl* dctl = (Ctl*)h->dctl;
  const Grid3 g = tracker_grid3(h, e, nt);
  Out3 od;
  od.face_id = h->face_id;
  od.pos = h->pos;
  od.mu = h->mu;
  od.type = h->type;
  od.flags = h->flags;
  od.parent = h->parent;
  od.work = h->work;
  const long long step_hits = h->total_after[e] - (e > 0 ? h->total_after[e - 1] : 0);
  zero_words<<<1, 64, 0, h->s>>>((unsigned*)&dctl->cnt[CNT_LIST], 2);
  HIP_TRY(hipGetLastError());
  if (step_hits > 0)
    HIP_TRY(launch_emit3d(g, h->plane_wide[e % 3] != 0, h->mring3, h->cring, h->oring, step_hits, od, &dctl->status,
                          dctl->cnt, h->list3, &dctl->cnt[CNT_LIST], h->s));
  h->emitted = h->total_after[e];
  return FTK_OK;
}

}  // namespace ftk

extern "C" ftk_status ftk_cp_create(int32_t n, const int64_t* dims, ftk_field_kind kind, const ftk_options* opt,
                                    ftk_stream_t stream, ftk_tracker** out) {
  g_err.clear();
  if (!out) return fail(FTK_ERR_ARG, "tracker pointer is NULL");
  *out = nullptr;
  if ((n != 2 && n != 3) || !dims) return fail(FTK_ERR_ARG, "n must be 2 or 3 and dims given");
  for (int a = 0; a < n; ++a)
    if (dims[a] < 2 || dims[a] > (1 << 28)) return fail(FTK_ERR_ARG, "every spatial dimension must be in [2, 2^28]");
  if (n == 3 && kind != FTK_SCALAR) return fail(FTK_ERR_ARG, "3D tracking takes a scalar field");
  if (kind != FTK_SCALAR && kind != FTK_VECTOR) return fail(FTK_ERR_ARG, "bad kind");
  ftk_options o;
  resolve(opt, &o);
  ftk_status st = ftk::validate_options(o);
  if (st) return st;
  ftk_tracker* h = new ftk_tracker();
  h->n = n;
  h->nx = dims[0];
  h->ny = dims[1];
  h->nz = n == 3 ? dims[2] : 1;
  h->kind = kind;
  h->o = o;
  h->s = (hipStream_t)stream;
  h->step_elems = (size_t)h->nx * h->ny * h->nz * (kind == FTK_VECTOR ? 2 : 1);
  {
    const Alloc al = ftk::tracker_alloc(h);
    const long long plane = h->nx * h->ny * h->nz;  // vertices per step
    h->nseg_plane = n == 2 ? h->ny * ((h->nx + 63) / 64) : h->nz * h->ny * ((h->nx + 15) / 16);
    h->fring = (float*)al.get(sizeof(float) * 3 * h->step_elems);
    if (n == 2) {
      h->mring = (uint16_t*)al.get(sizeof(uint16_t) * 3 * plane);
    } else {
      h->mring3 = (uint64_t*)al.get(sizeof(uint64_t) * 3 * plane);
      h->list3 = (long long*)al.get(sizeof(long long) * h->nz * h->ny * ((h->nx + 63) / 64));
      ftk::Grid3 gd;
      gd.nx = (int)h->nx;
      gd.ny = (int)h->ny;
      gd.nz = (int)h->nz;
      h->cert3 = (unsigned char*)al.get((size_t)(3 * ftk::cert3_plane(gd)));
    }
    h->cring = (int*)al.get(sizeof(int) * 3 * h->nseg_plane);
    h->oring = (long long*)al.get(sizeof(long long) * 3 * h->nseg_plane);
    h->scan_tmp = (long long*)al.get(sizeof(long long) * ftk::scan_tmp_elems(h->nseg_plane));
    h->dctl = al.get(sizeof(Ctl));
    h->dplane = (long long*)al.get(sizeof(long long));
    const bool ring_ok =
        n == 2 ? h->mring != nullptr : (h->mring3 != nullptr && h->list3 != nullptr && h->cert3 != nullptr);
    if (!h->fring || !ring_ok || !h->cring || !h->oring || !h->scan_tmp || !h->dctl || !h->dplane) {
      ftk::tracker_free_all(h);
      delete h;
      return fail(FTK_ERR_OOM, "tracker allocation failed");
    }
    if (hipMemsetAsync(h->dctl, 0, sizeof(Ctl), h->s) != hipSuccess) {
      ftk::tracker_free_all(h);
      delete h;
      return fail(FTK_ERR_HIP, "hipMemsetAsync failed");
    }
  }
  *out = h;
  return FTK_OK;
}

extern "C" ftk_status ftk_cp_push(ftk_tracker* h, const float* step) {
  g_err.clear();
  if (!h) return fail(FTK_ERR_ARG, "tracker is NULL");
  if (h->state != 0) return fail(FTK_ERR_STATE, "tracker already finished or failed");
  if (!step) return fail(FTK_ERR_ARG, "step is NULL");
  if (h->steps >= (1 << 28)) return fail(FTK_ERR_ARG, "too many steps");
  const size_t bytes = sizeof(float) * h->step_elems;
  const int s = h->steps;
  HIP_TRY(hipMemcpyAsync(h->fring + (size_t)(s % 3) * h->step_elems, step, bytes, hipMemcpyDeviceToDevice, h->s));
  ftk_status st = FTK_OK;
  if (h->n == 2) {
    if (s >= 1) st = ftk::tracker_detect(h, s - 1, ftk::kOpenNt);
    if (!st && s >= 2) st = ftk::tracker_emit(h, s - 2, ftk::kOpenNt);
  } else {
    if (s >= 1) st = ftk::tracker_detect3(h, s - 1, ftk::kOpenNt);
    if (!st && s >= 2) st = ftk::tracker_emit3(h, s - 2, ftk::kOpenNt);
  }
  if (st) {
    h->state = 2;
    return st;
  }
  HIP_TRY(hipStreamSynchronize(h->s));  // the caller may reuse `step` on return
  ++h->steps;
  return FTK_OK;
}

extern "C" ftk_status ftk_cp_finish(ftk_tracker* h, ftk_cp_result* out) {
  g_err.clear();
  if (!h || !out) return fail(FTK_ERR_ARG, "tracker or result is NULL");
  std::memset(out, 0, sizeof(*out));
  if (h->state != 0) return fail(FTK_ERR_STATE, "tracker already finished or failed");
  if (h->steps < 2) return fail(FTK_ERR_STATE, "at least two steps must be pushed");
  h->state = 1;
  const int N = h->steps;
  Ctl* dctl = (Ctl*)h->dctl;
  ftk_status st;
  if (h->n == 2) {
    st = ftk::tracker_detect(h, N - 1, N);
    if (!st) st = ftk::tracker_emit(h, N - 2, N);
    if (!st) st = ftk::tracker_emit(h, N - 1, N);
  } else {
    st = ftk::tracker_detect3(h, N - 1, N);
    if (!st) st = ftk::tracker_emit3(h, N - 2, N);
    if (!st) st = ftk::tracker_emit3(h, N - 1, N);
  }
  if (st) return st;
  const long long nh = h->total_after[N - 1];
  const Alloc al = ftk::tracker_alloc(h);
  long long* label = nullptr;
  if ((h->o.outputs & FTK_OUT_LABEL) && !(label = (long long*)al.get(sizeof(long long) * (nh ? nh : 1))))
    return fail(FTK_ERR_OOM, "label allocation failed");
  if (nh > 0) {
    HIP_TRY(ftk::launch_uf_hook(h->parent, h->work, &dctl->cnt[ftk::CNT_WORK], 2 * h->cap, h->s));
    HIP_TRY(ftk::launch_uf_label(h->parent, h->face_id, label, nh, dctl->cnt, h->s));
  }
  Ctl hc;
  st = read_ctl(&hc, dctl, h->s);
  if (!st) st = decode_status(hc.status);
  if (st) {
    al.put(label);
    return st;
  }
  ftk_cp_result& r = *out;
  r.n = h->n;
  r.n_hits = nh;
  r.n_trajectories = (long long)hc.cnt[ftk::CNT_TRAJ];
  r.face_id = (int64_t*)h->face_id;
  r.pos = h->pos;
  r.mu = h->mu;
  r.type = h->type;
  r.flags = h->flags;
  r.label = (int64_t*)label;
  h->face_id = nullptr;
  h->pos = h->mu = nullptr;
  h->type = h->flags = nullptr;
  int64_t dims[4] = {h->nx, h->ny, h->n == 3 ? h->nz : N, N};
  r.stats.simplices_tested = count_tested(h->n, dims);
  r.stats.cells_linked = (long long)hc.cnt[ftk::CNT_LINKED];
  r.stats.fp64_fallbacks = (long long)hc.cnt[ftk::CNT_FP64];
  r.stats.degenerate_sublocations = (long long)hc.cnt[ftk::CNT_DEGEN];
  r.stats.wide_path = (h->plane_wide[0] | h->plane_wide[1] | h->plane_wide[2]) ? 1 : 0;
  return FTK_OK;
}

extern "C" void ftk_cp_destroy(ftk_tracker* h) {
  if (!h) return;
  ftk::tracker_free_all(h);
  delete h;
}

namespace ftk {

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

extern "C" ftk_status ftk_track_cp2d_batched(int32_t n_series, const float* const* fields, const int64_t* nx,
                                             const int64_t* ny, const int64_t* nt, ftk_field_kind kind,
                                             const ftk_options* opt, ftk_stream_t stream, ftk_cp_result* outs) {
  g_err.clear();
  if (n_series <= 0 || !fields || !nx || !ny || !nt || !outs) return fail(FTK_ERR_ARG, "bad batch arguments");
  if (n_series > 16384) return fail(FTK_ERR_ARG, "at most 16384 series per batch");
  if (kind != FTK_SCALAR && kind != FTK_VECTOR) return fail(FTK_ERR_ARG, "kind must be FTK_SCALAR or FTK_VECTOR");
  for (int i = 0; i < n_series; ++i) {
    std::memset(&outs[i], 0, sizeof(outs[i]));
    if (!fields[i]) return fail(FTK_ERR_ARG, "series %d: field is NULL", i);
    if (nx[i] < 2 || ny[i] < 2 || nt[i] < 2) return fail(FTK_ERR_ARG, "series %d: every dimension must be >= 2", i);
    if (nx[i] > (1 << 30) || ny[i] > (1 << 30) || nt[i] > (1 << 30) || nx[i] * ny[i] * nt[i] > (1ll << 40))
      return fail(FTK_ERR_ARG, "series %d: grid too large", i);
  }
  ftk_options o;
  resolve(opt, &o);
  ftk_status st = ftk::validate_options(o);
  if (st) return st;
  return ftk::track2d_batched_impl(n_series, fields, nx, ny, nt, kind, o, (hipStream_t)stream, outs);
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

extern "C" ftk_status ftk_track_cp2d_into(const float* field, ftk_field_kind kind, int64_t nx, int64_t ny,
                                          int64_t nt, const ftk_options* opt, ftk_stream_t stream, int64_t capacity,
                                          ftk_cp_result* io) {
  g_err.clear();
  if (!io) return fail(FTK_ERR_ARG, "io is NULL");
  if (!field) return fail(FTK_ERR_ARG, "field is NULL");
  if (kind != FTK_SCALAR && kind != FTK_VECTOR) return fail(FTK_ERR_ARG, "kind must be FTK_SCALAR or FTK_VECTOR");
  if (nx < 2 || ny < 2 || nt < 2) return fail(FTK_ERR_ARG, "every dimension must be >= 2 (got %lld x %lld x %lld)",
                                               (long long)nx, (long long)ny, (long long)nt);
  if (nx > (1 << 30) || ny > (1 << 30) || nt > (1 << 30) || nx * ny > (1ll << 40) || nx * ny * nt > (1ll << 42))
    return fail(FTK_ERR_ARG, "grid too large");
  if (capacity < 0) return fail(FTK_ERR_ARG, "capacity must be >= 0");
  ftk_options o;
  resolve(opt, &o);
  o.alloc = nullptr;  // nothing is allocated: the hooks and the phase timers are not used
  o.free = nullptr;
  o.alloc_ctx = nullptr;
  o.profile = 0;
  ftk_status st = ftk::validate_options(o);
  if (st) return st;
  const unsigned outs = o.outputs;
  if (capacity > 0 && (!io->face_id || ((outs & FTK_OUT_POS) && !io->pos) || ((outs & FTK_OUT_MU) && !io->mu) ||
                       ((outs & FTK_OUT_TYPE) && !io->type) || ((outs & FTK_OUT_FLAGS) && !io->flags) ||
                       ((outs & FTK_OUT_LABEL) && !io->label)))
    return fail(FTK_ERR_ARG, "io lacks an output array that opt->outputs asks for");
  char* base = nullptr;
  st = ftk::static_scratch(&base);
  if (st) return st;
  ftk_cp_result r = *io;  // the caller's pointers; *io is written only on success (n_hits also on CAPACITY)
  ftk::StaticMem2 mem(base, r, capacity);
  ftk_cp_result res;
  std::memset(&res, 0, sizeof(res));
  st = ftk::track2d_core(field, kind, nx, ny, nt, o, (hipStream_t)stream, mem, &res);
  if (st == FTK_OK) {
    *io = res;
  } else if (st == FTK_ERR_CAPACITY) {
    io->n_hits = res.n_hits;
  }
  return st;
}

// ---------------------------------------------------------------------------------------------------------------
// Trajectory post-processing (post.hip): trajectory table, slicing at a time step, loop filter.
// ---------------------------------------------------------------------------------------------------------------
namespace {

ftk_status check_post_args(const ftk_cp_result* r, int32_t n, const int64_t* dims) {
  if (!r || !dims) return fail(FTK_ERR_ARG, "result and dims must be given");
  if (n != 2 && n != 3) return fail(FTK_ERR_ARG, "n must be 2 or 3");
  if (r->n != n) return fail(FTK_ERR_ARG, "the result holds %dD faces, not %dD", (int)r->n, (int)n);
  for (int a = 0; a <= n; ++a)
    if (dims[a] < 2) return fail(FTK_ERR_ARG, "every dimension must be >= 2");
  if (r->n_hits < 0 || r->n_trajectories < 0) return fail(FTK_ERR_ARG, "negative counts in the result");
  if (r->n_hits > 0 && !r->face_id) return fail(FTK_ERR_ARG, "the result has no face_id array");
  return FTK_OK;
}

}  // namespace

extern "C" {

ftk_status ftk_traj_table_build(const ftk_cp_result* r, int32_t n, const int64_t* dims_with_t,
                                const ftk_options* opt, ftk_stream_t stream, ftk_traj_table* out) {
  g_err.clear();
  if (!out) return fail(FTK_ERR_ARG, "out is NULL");
  std::memset(out, 0, sizeof(*out));
  ftk_status st = check_post_args(r, n, dims_with_t);
  if (st) return st;
  if (r->n_hits > 0 && (!r->pos || !r->label))
    return fail(FTK_ERR_ARG, "the trajectory table needs the result's pos and label arrays");
  ftk_options o;
  resolve(opt, &o);
  if ((o.alloc == nullptr) != (o.free == nullptr)) return fail(FTK_ERR_ARG, "alloc and free must be given together");
  hipStream_t s = (hipStream_t)stream;
  const Alloc al = make_alloc(o, s);
  Scratch sc(al);
  const long long nh = r->n_hits, ntr = r->n_trajectories;
  ftk_traj_table t;
  std::memset(&t, 0, sizeof(t));
  t.n = ntr;
  t.label = (int64_t*)al.get(sizeof(int64_t) * ntr);
  t.n_points = (uint64_t*)al.get(sizeof(uint64_t) * ntr);
  t.t_min = (float*)al.get(sizeof(float) * ntr);
  t.t_max = (float*)al.get(sizeof(float) * ntr);
  t.n_ends = (int32_t*)al.get(sizeof(int32_t) * ntr);
  int* flag = sc.get<int>((size_t)nh);
  long long* off = sc.get<long long>((size_t)nh);
  long long* tmp = sc.get<long long>(ftk::scan_tmp_elems(nh));
  long long* rb = sc.get<long long>((size_t)ftk::row_buckets(n, dims_with_t) + 1);
  Ctl* dctl = sc.get<Ctl>(1);
  if (!t.label || !t.n_points || !t.t_min || !t.t_max || !t.n_ends || !flag || !off || !tmp || !rb || !dctl) {
    ftk_traj_table_free(&t, opt, stream);
    return fail(FTK_ERR_OOM, "trajectory table allocation failed");
  }
  hipError_t he = hipMemsetAsync(dctl, 0, sizeof(Ctl), s);
  if (he == hipSuccess)
    he = ftk::launch_traj_table(n, dims_with_t, (const long long*)r->face_id, (const long long*)r->label, r->pos, nh,
                                ntr, flag, off, &dctl->total, tmp, (long long*)t.label, rb,
                                (unsigned long long*)t.n_points, (int*)t.t_min, (int*)t.t_max, t.n_ends,
                                &dctl->status, s);
  Ctl h;
  if (he == hipSuccess) {
    st = read_ctl(&h, dctl, s);
  } else {
    st = fail(FTK_ERR_HIP, "kernel launch: %s", hipGetErrorString(he));
  }
  if (!st) st = decode_status(h.status);
  if (!st && nh > 0 && h.total != ntr)
    st = fail(FTK_ERR_INVARIANT, "%lld trajectory roots for %lld trajectories", h.total, ntr);
  if (st) {
    ftk_traj_table_free(&t, opt, stream);
    return st;
  }
  *out = t;
  return FTK_OK;
}

void ftk_traj_table_free(ftk_traj_table* tt, const ftk_options* opt, ftk_stream_t stream) {
  if (!tt) return;
  ftk_options o;
  resolve(opt, &o);
  Alloc al = make_alloc(o, (hipStream_t)stream);
  al.put(tt->label);
  al.put(tt->n_points);
  al.put(tt->t_min);
  al.put(tt->t_max);
  al.put(tt->n_ends);
  std::memset(tt, 0, sizeof(*tt));
}

ftk_status ftk_cp_slice(const ftk_cp_result* r, int32_t n, const int64_t* dims_with_t, int64_t t0,
                        const ftk_options* opt, ftk_stream_t stream, int64_t** idx, int64_t* count) {
  g_err.clear();
  if (!idx || !count) return fail(FTK_ERR_ARG, "idx and count must be given");
  *idx = nullptr;
  *count = 0;
  ftk_status st = check_post_args(r, n, dims_with_t);
  if (st) return st;
  if (t0 < 0 || t0 >= dims_with_t[n]) return fail(FTK_ERR_ARG, "t0 = %lld outside [0, nt)", (long long)t0);
  ftk_options o;
  resolve(opt, &o);
  if ((o.alloc == nullptr) != (o.free == nullptr)) return fail(FTK_ERR_ARG, "alloc and free must be given together");
  hipStream_t s = (hipStream_t)stream;
  const Alloc al = make_alloc(o, s);
  Scratch sc(al);
  const long long nh = r->n_hits;
  long long* range = sc.get<long long>(2);
  Ctl* dctl = sc.get<Ctl>(1);
  if (!range || !dctl) return fail(FTK_ERR_OOM, "scratch allocation failed");
  long long hr[2] = {0, 0};
  if (nh > 0) {
    HIP_TRY(ftk::launch_slice_range(n, dims_with_t, (const long long*)r->face_id, nh, t0, range, s));
    HIP_TRY(hipMemcpyAsync(hr, range, sizeof(hr), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  const long long lo = hr[0], cnt = hr[1] - hr[0];
  long long k = 0;
  int* flag = nullptr;
  long long* off = nullptr;
  if (cnt > 0) {
    flag = sc.get<int>((size_t)cnt);
    off = sc.get<long long>((size_t)cnt);
    long long* tmp = sc.get<long long>(ftk::scan_tmp_elems(cnt));
    if (!flag || !off || !tmp) return fail(FTK_ERR_OOM, "scratch allocation failed");
    HIP_TRY(hipMemsetAsync(dctl, 0, sizeof(Ctl), s));
    HIP_TRY(ftk::launch_slice_compact(n, dims_with_t, (const long long*)r->face_id, lo, cnt, flag, off, &dctl->total,
                                      tmp, nullptr, false, s));
    Ctl h;
    st = read_ctl(&h, dctl, s);
    if (st) return st;
    k = h.total;
  }
  int64_t* out = (int64_t*)al.get(sizeof(int64_t) * (size_t)(k > 0 ? k : 1));
  if (!out) return fail(FTK_ERR_OOM, "slice allocation failed");
  if (k > 0) {
    hipError_t he = ftk::launch_slice_compact(n, dims_with_t, (const long long*)r->face_id, lo, cnt, flag, off,
                                              nullptr, nullptr, (long long*)out, true, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) {
      al.put(out);
      return fail(FTK_ERR_HIP, "slice: %s", hipGetErrorString(he));
    }
  }
  *idx = out;
  *count = k;
  return FTK_OK;
}

ftk_status ftk_cp_filter_loops(const ftk_cp_result* r, const ftk_traj_table* tt, float min_duration,
                               ftk_stream_t stream, uint8_t* keep) {
  g_err.clear();
  if (!r || !tt) return fail(FTK_ERR_ARG, "result and table must be given");
  if (r->n_hits == 0) return FTK_OK;
  if (!keep) return fail(FTK_ERR_ARG, "keep must be given");
  if (!r->label) return fail(FTK_ERR_ARG, "the loop filter needs the result's label array");
  if (tt->n != r->n_trajectories || !tt->label || !tt->t_min || !tt->t_max || !tt->n_ends)
    return fail(FTK_ERR_ARG, "the trajectory table does not belong to this result");
  if (!(min_duration == min_duration)) return fail(FTK_ERR_ARG, "min_duration is NaN");
  HIP_TRY(ftk::launch_filter_loops((const long long*)r->label, r->n_hits, (const long long*)tt->label, tt->n,
                                   (const int*)tt->t_min, (const int*)tt->t_max, tt->n_ends, min_duration, keep,
                                   (hipStream_t)stream));
  return FTK_OK;
}

ftk_status ftk_traj_order(const ftk_cp_result* r, int32_t n, const int64_t* dims_with_t, const ftk_traj_table* tt,
                          const ftk_options* opt, ftk_stream_t stream, int64_t* order, int64_t* offsets) {
  g_err.clear();
  ftk_status st = check_post_args(r, n, dims_with_t);
  if (st) return st;
  if (!tt || !offsets) return fail(FTK_ERR_ARG, "table and offsets must be given");
  if (tt->n != r->n_trajectories || (tt->n > 0 && (!tt->label || !tt->n_points || !tt->n_ends)))
    return fail(FTK_ERR_ARG, "the trajectory table does not belong to this result");
  const long long nh = r->n_hits, ntr = r->n_trajectories;
  if (nh > 0 && (!order || !r->label)) return fail(FTK_ERR_ARG, "order and the result's label array must be given");
  if (nh > INT_MAX) return fail(FTK_ERR_CAPACITY, "ordering supports up to 2^31 - 1 points");
  ftk_options o;
  resolve(opt, &o);
  if ((o.alloc == nullptr) != (o.free == nullptr)) return fail(FTK_ERR_ARG, "alloc and free must be given together");
  hipStream_t s = (hipStream_t)stream;
  const Alloc al = make_alloc(o, s);
  Scratch sc(al);
  const size_t nz = (size_t)(nh > 0 ? nh : 1);
  int* nb = sc.get<int>(2 * nz);
  unsigned* seg = sc.get<unsigned>(4 * nz);
  unsigned char* is_ruler = sc.get<unsigned char>(nz);
  int* rid = sc.get<int>(nz);
  int* list = sc.get<int>(nz);
  int* flag = sc.get<int>(nz);
  long long* off = sc.get<long long>(nz);
  long long hB;
  long long* bstart = sc.get<long long>((size_t)ftk::hit_buckets(n, dims_with_t, nh, &hB) + 1);
  long long* rb = sc.get<long long>((size_t)ftk::row_buckets(n, dims_with_t) + 1);
  int* cnt = sc.get<int>((size_t)(ntr > 0 ? ntr : 1));
  long long* tmp = sc.get<long long>(ftk::scan_tmp_elems(nh > ntr ? nh : ntr));
  Ctl* dctl = sc.get<Ctl>(1);
  if (!nb || !seg || !is_ruler || !rid || !list || !flag || !off || !bstart || !rb || !cnt || !tmp || !dctl)
    return fail(FTK_ERR_OOM, "scratch allocation failed");
  HIP_TRY(hipMemsetAsync(dctl, 0, sizeof(Ctl), s));
  HIP_TRY(ftk::launch_order_setup(n, dims_with_t, (const long long*)r->face_id, (const long long*)r->label, nh,
                                  (const long long*)tt->label, (const unsigned long long*)tt->n_points, tt->n_ends,
                                  ntr, nb, seg, is_ruler, rid, list, bstart, rb, flag, off, &dctl->total, cnt,
                                  (long long*)offsets, tmp, &dctl->status, s));
  Ctl h;
  st = read_ctl(&h, dctl, s);
  if (st) return st;
  if (h.status) return decode_status(h.status);
  if (nh > 0) {
    const long long nr = h.total;
    const size_t nrz = (size_t)(nr > 0 ? nr : 1);
    int* st0 = sc.get<int>(8 * nrz);
    int* st1 = sc.get<int>(8 * nrz);
    int* act0 = sc.get<int>(nrz);
    int* act1 = sc.get<int>(nrz);
    if (!st0 || !st1 || !act0 || !act1) return fail(FTK_ERR_OOM, "scratch allocation failed");
    HIP_TRY(ftk::launch_order_walk(nb, is_ruler, list, nr, nh, seg, st0, &dctl->status, s));
    // pointer jumping over the rulers: the reach of every open arm doubles per round, so a path of L rulers closes
    // within ceil(log2 L) + 2 rounds (one more to copy the final states); an arm that walks past n_hits steps is
    // closed as an invariant error
    int* in = st0;
    int* out = st1;
    const int* act = nullptr;
    long long n_act = nr;
    int* lists[2] = {act0, act1};
    for (int round = 0; n_act > 0; ++round) {
      if (round >= 64) return fail(FTK_ERR_INVARIANT, "trajectory walk did not close (internal error)");
      HIP_TRY(hipMemsetAsync(&dctl->cnt[0], 0, sizeof(unsigned long long), s));
      int* next = lists[round & 1];
      HIP_TRY(ftk::launch_order_jump(nb, rid, act, n_act, nh, in, out, next, (unsigned long long*)&dctl->cnt[0],
                                     &dctl->status, s));
      st = read_ctl(&h, dctl, s);
      if (st) return st;
      if (h.status) return decode_status(h.status);
      n_act = (long long)h.cnt[0];
      act = next;
      int* x = in;
      in = out;
      out = x;
    }
    HIP_TRY(ftk::launch_order_place(n, dims_with_t, (const long long*)r->label, nh, (const long long*)tt->label, rb,
                                    (const long long*)offsets, is_ruler, rid, seg, in, (long long*)order,
                                    &dctl->status, s));
  }
  st = read_ctl(&h, dctl, s);
  if (st) return st;
  return decode_status(h.status);
}

namespace {

ftk_status check_walk_args(const ftk_cp_result* r, const ftk_traj_table* tt, const int64_t* order,
                           const int64_t* offsets, const uint8_t* type_in, const uint8_t* type_out) {
  if (!r || !tt) return fail(FTK_ERR_ARG, "result and table must be given");
  if (r->n != 2 && r->n != 3) return fail(FTK_ERR_ARG, "the result holds no 2D or 3D faces");
  if (tt->n != r->n_trajectories || (tt->n > 0 && !tt->n_ends))
    return fail(FTK_ERR_ARG, "the trajectory table does not belong to this result");
  if (r->n_hits == 0) return FTK_OK;
  if (!order || !offsets || !type_in || !type_out) return fail(FTK_ERR_ARG, "order, offsets and types must be given");
  const uint8_t* a = type_in;
  const uint8_t* b = type_out;
  if (a < b + r->n_hits && b < a + r->n_hits) return fail(FTK_ERR_ARG, "type_out must not overlap type_in");
  return FTK_OK;
}

}  // namespace

ftk_status ftk_traj_smooth_types(const ftk_cp_result* r, const ftk_traj_table* tt, const int64_t* order,
                                 const int64_t* offsets, const uint8_t* type_in, int32_t half_window,
                                 const ftk_options* opt, ftk_stream_t stream, uint8_t* type_out) {
  g_err.clear();
  ftk_status st = check_walk_args(r, tt, order, offsets, type_in, type_out);
  if (st || r->n_hits == 0) return st;
  if (half_window < 0) return fail(FTK_ERR_ARG, "half_window must be >= 0");
  ftk_options o;
  resolve(opt, &o);
  if ((o.alloc == nullptr) != (o.free == nullptr)) return fail(FTK_ERR_ARG, "alloc and free must be given together");
  hipStream_t s = (hipStream_t)stream;
  const Alloc al = make_alloc(o, s);
  Scratch sc(al);
  const long long nh = r->n_hits;
  int* head = sc.get<int>((size_t)nh);
  long long* heads = sc.get<long long>((size_t)nh);
  long long* tmp = sc.get<long long>(ftk::scan_tmp_elems(nh));
  Ctl* dctl = sc.get<Ctl>(1);
  if (!head || !heads || !tmp || !dctl) return fail(FTK_ERR_OOM, "scratch allocation failed");
  HIP_TRY(hipMemsetAsync(dctl, 0, sizeof(Ctl), s));
  HIP_TRY(ftk::launch_smooth((const long long*)order, (const long long*)offsets, tt->n_ends, tt->n, nh, type_in,
                             half_window, head, heads, &dctl->total, tmp, type_out, &dctl->status, s));
  Ctl h;
  st = read_ctl(&h, dctl, s);
  if (st) return st;
  return decode_status(h.status);
}

ftk_status ftk_traj_simplify_types(const ftk_cp_result* r, const ftk_traj_table* tt, const int64_t* order,
                                   const int64_t* offsets, const uint8_t* type_in, float min_persistence,
                                   const ftk_options* opt, ftk_stream_t stream, uint8_t* type_out) {
  g_err.clear();
  ftk_status st = check_walk_args(r, tt, order, offsets, type_in, type_out);
  if (st || r->n_hits == 0) return st;
  if (!r->pos) return fail(FTK_ERR_ARG, "simplification needs the result's pos array");
  if (!(min_persistence == min_persistence)) return fail(FTK_ERR_ARG, "min_persistence is NaN");
  ftk_options o;
  resolve(opt, &o);
  if ((o.alloc == nullptr) != (o.free == nullptr)) return fail(FTK_ERR_ARG, "alloc and free must be given together");
  hipStream_t s = (hipStream_t)stream;
  const Alloc al = make_alloc(o, s);
  Scratch sc(al);
  const long long nh = r->n_hits;
  long long* rot = sc.get<long long>((size_t)(tt->n > 0 ? tt->n : 1));
  int* flag = sc.get<int>((size_t)nh);
  long long* run_off = sc.get<long long>((size_t)nh);
  long long* tmp = sc.get<long long>(ftk::scan_tmp_elems(nh));
  int* tmin = sc.get<int>((size_t)nh);
  int* tmax = sc.get<int>((size_t)nh);
  uint8_t* run_type = sc.get<uint8_t>((size_t)nh);
  uint8_t* new_type = sc.get<uint8_t>((size_t)nh);
  int* head = sc.get<int>((size_t)nh);
  long long* heads = sc.get<long long>((size_t)nh);
  Ctl* dctl = sc.get<Ctl>(1);
  if (!rot || !flag || !run_off || !tmp || !tmin || !tmax || !run_type || !new_type || !head || !heads || !dctl)
    return fail(FTK_ERR_OOM, "scratch allocation failed");
  HIP_TRY(hipMemsetAsync(dctl, 0, sizeof(Ctl), s));
  HIP_TRY(ftk::launch_simplify(r->n, r->pos, (const long long*)order, (const long long*)offsets, tt->n_ends, tt->n, nh,
                               type_in, min_persistence, rot, flag, run_off, head, heads, &dctl->total, tmp, tmin,
                               tmax, run_type, new_type, type_out, &dctl->status, s));
  Ctl h;
  st = read_ctl(&h, dctl, s);
  if (st) return st;
  return decode_status(h.status);
}

int64_t ftk_edge_count(const int64_t* d) {
  if (!d) return -1;
  for (int a = 0; a < 4; ++a)
    if (d[a] < 2) return -1;
  int64_t tot = 0;
  for (int M = 1; M < 16; ++M) {
    int64_t p = 1;
    for (int a = 0; a < 4; ++a) p *= d[a] - ((M >> a) & 1);
    tot += p;
  }
  return tot;
}

void ftk_iso_result_free(ftk_iso_result* r, const ftk_options* opt, ftk_stream_t stream) {
  if (!r) return;
  ftk_options o;
  resolve(opt, &o);
  const Alloc al = make_alloc(o, (hipStream_t)stream);
  al.put(r->edge_id);
  al.put(r->pos);
  al.put(r->label);
  al.put(r->tets);
  std::memset(r, 0, sizeof(*r));
}

ftk_status ftk_track_iso3d(const float* field, int64_t nx, int64_t ny, int64_t nz, int64_t nt, float isovalue,
                           const ftk_options* opt, ftk_stream_t stream, ftk_iso_result* out) {
  g_err.clear();
  if (!out) return fail(FTK_ERR_ARG, "out is NULL");
  std::memset(out, 0, sizeof(*out));
  if (!field) return fail(FTK_ERR_ARG, "field is NULL");
  if (nx < 2 || ny < 2 || nz < 2 || nt < 2) return fail(FTK_ERR_ARG, "every dimension must be >= 2");
  if (nx > (1 << 30) || ny > 65535 || nz * nt > 65535) return fail(FTK_ERR_ARG, "grid too large (ny and nz * nt <= 65535)");
  if (!std::isfinite(isovalue)) return fail(FTK_ERR_ARG, "isovalue must be finite");
  ftk_options o;
  resolve(opt, &o);
  if ((o.alloc == nullptr) != (o.free == nullptr)) return fail(FTK_ERR_ARG, "alloc and free must be given together");
  hipStream_t s = (hipStream_t)stream;
  const Alloc al = make_alloc(o, s);
  Scratch sc(al);
  const long long V = nx * ny * nz * nt;
  const long long G = (V + 15) / 16;  // groups of 16 vertices (offsets: one base per group)
  unsigned short* emask = sc.get<unsigned short>((size_t)V);
  unsigned char* hcnt = sc.get<unsigned char>((size_t)G * 16);
  unsigned char* tcnt = sc.get<unsigned char>((size_t)G * 16);
  int* gsum = sc.get<int>((size_t)G);
  long long* hbase = sc.get<long long>((size_t)G);
  long long* tbase = sc.get<long long>((size_t)G);
  long long* abase = sc.get<long long>((size_t)G);
  unsigned long long* bits = sc.get<unsigned long long>((size_t)((nx + 63) / 64) * ny * nz * nt);
  long long* tmp = sc.get<long long>(ftk::scan_tmp_elems(G));
  Ctl* dctl = sc.get<Ctl>(1);
  if (!emask || !hcnt || !tcnt || !gsum || !hbase || !tbase || !abase || !bits || !tmp || !dctl)
    return fail(FTK_ERR_OOM, "scratch allocation failed");
  HIP_TRY(hipMemsetAsync(dctl, 0, sizeof(Ctl), s));
  HIP_TRY(ftk::launch_iso_count(field, (int)nx, (int)ny, (int)nz, (int)nt, isovalue, bits, emask, hcnt, tcnt,
                                &dctl->status, s));
  HIP_TRY(ftk::launch_group16_bases(hcnt, V, false, gsum, hbase, &dctl->total, tmp, s));
  HIP_TRY(ftk::launch_group16_bases(tcnt, V, false, gsum, tbase, (long long*)&dctl->cnt[ftk::CNT_LIST], tmp, s));
  HIP_TRY(ftk::launch_group16_bases(tcnt, V, true, gsum, abase, (long long*)&dctl->cnt[ftk::CNT_WORK], tmp, s));
  Ctl h;
  ftk_status st = read_ctl(&h, dctl, s);
  if (st) return st;
  st = decode_status(h.status);
  if (st) return st;
  const long long nh = h.total, ntets = (long long)h.cnt[ftk::CNT_LIST], nact = (long long)h.cnt[ftk::CNT_WORK];
  if (nh > 0x7fffffffll) return fail(FTK_ERR_CAPACITY, "%lld crossed edges exceed the 32-bit tetrahedron indices", nh);
  ftk_iso_result r;
  std::memset(&r, 0, sizeof(r));
  r.n_hits = nh;
  r.n_tets = ntets;
  r.edge_id = (int64_t*)al.get(sizeof(int64_t) * (size_t)(nh > 0 ? nh : 1));
  r.pos = (float*)al.get(sizeof(float) * 4 * (size_t)(nh > 0 ? nh : 1));
  r.label = (int64_t*)al.get(sizeof(int64_t) * (size_t)(nh > 0 ? nh : 1));
  r.tets = (int32_t*)al.get(sizeof(int32_t) * 4 * (size_t)(ntets > 0 ? ntets : 1));
  unsigned* parent = sc.get<unsigned>((size_t)(nh > 0 ? nh : 1));
  long long* active = sc.get<long long>((size_t)(nact > 0 ? nact : 1));
  if (!r.edge_id || !r.pos || !r.label || !r.tets || !parent || !active) {
    ftk_iso_result_free(&r, opt, stream);
    return fail(FTK_ERR_OOM, "output allocation failed");
  }
  if ((((uintptr_t)r.tets | (uintptr_t)r.pos) & 15u) != 0) {  // tetrahedra and points: 16-byte stores
    ftk_iso_result_free(&r, opt, stream);
    return fail(FTK_ERR_ARG, "the allocator returned a point or tetrahedron array not aligned to 16 bytes");
  }
  hipError_t he = hipSuccess;
  if (nh > 0) {
    he = ftk::launch_iso_emit(field, (int)nx, (int)ny, (int)nz, (int)nt, isovalue, emask, hbase, hcnt,
                              (long long*)r.edge_id, r.pos, parent, s);
    if (he == hipSuccess) he = ftk::launch_iso_active(tcnt, abase, V, active, s);
    if (he == hipSuccess)
      he = ftk::launch_iso_unite(field, (int)nx, (int)ny, (int)nz, (int)nt, isovalue, bits, active, nact, emask, hbase,
                                 hcnt, tcnt, tbase, parent, (int*)r.tets, &dctl->status, s);
    if (he == hipSuccess)
      he = ftk::launch_uf_label(parent, (const long long*)r.edge_id, (long long*)r.label, nh, dctl->cnt, s);
  }
  if (he != hipSuccess) {
    ftk_iso_result_free(&r, opt, stream);
    return fail(FTK_ERR_HIP, "kernel launch: %s", hipGetErrorString(he));
  }
  st = read_ctl(&h, dctl, s);
  if (!st) st = decode_status(h.status);
  if (st) {
    ftk_iso_result_free(&r, opt, stream);
    return st;
  }
  r.n_components = (long long)h.cnt[ftk::CNT_TRAJ];
  *out = r;
  return FTK_OK;
}

int64_t ftk_triangle_count(const int64_t* d) {
  if (!d) return -1;
  for (int a = 0; a < 4; ++a)
    if (d[a] < 2) return -1;
  int64_t tot = 0;
  for (int ty = 0; ty < ftk::kTri3.count; ++ty) {
    const int u = ftk::kTri3.m[ty][0] | ftk::kTri3.m[ty][1];
    int64_t p = 1;
    for (int a = 0; a < 4; ++a) p *= d[a] - ((u >> a) & 1);
    tot += p;
  }
  return tot;
}

void ftk_vortex_result_free(ftk_vortex_result* r, const ftk_options* opt, ftk_stream_t stream) {
  if (!r) return;
  ftk_options o;
  resolve(opt, &o);
  const Alloc al = make_alloc(o, (hipStream_t)stream);
  al.put(r->tri_id);
  al.put(r->pos);
  al.put(r->label);
  std::memset(r, 0, sizeof(*r));
}

ftk_status ftk_track_vortex3d(const float* psi, int64_t nx, int64_t ny, int64_t nz, int64_t nt,
                              const ftk_options* opt, ftk_stream_t stream, ftk_vortex_result* out) {
  g_err.clear();
  if (!out) return fail(FTK_ERR_ARG, "out is NULL");
  std::memset(out, 0, sizeof(*out));
  if (!psi) return fail(FTK_ERR_ARG, "psi is NULL");
  if (nx < 2 || ny < 2 || nz < 2 || nt < 2) return fail(FTK_ERR_ARG, "every dimension must be >= 2");
  if (nx > (1 << 30) || ny > 65535 || nz * nt > 65535) return fail(FTK_ERR_ARG, "grid too large (ny and nz * nt <= 65535)");
  ftk_options o;
  resolve(opt, &o);
  ftk_status st = ftk::validate_options(o);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  const Alloc al = make_alloc(o, s);
  Scratch sc(al);
  const long long V = nx * ny * nz * nt;
  unsigned short* emask = sc.get<unsigned short>((size_t)V);
  unsigned long long* tmask = sc.get<unsigned long long>((size_t)V);
  unsigned char* cnt = sc.get<unsigned char>((size_t)V);
  long long* hoff = sc.get<long long>((size_t)V);
  long long* tmp = sc.get<long long>(ftk::scan_tmp_elems(V));
  Ctl* dctl = sc.get<Ctl>(1);
  if (!emask || !tmask || !cnt || !hoff || !tmp || !dctl) return fail(FTK_ERR_OOM, "scratch allocation failed");
  const float qscale = std::ldexp(1.0f, o.quant_log2);
  HIP_TRY(hipMemsetAsync(dctl, 0, sizeof(Ctl), s));
  HIP_TRY(ftk::launch_vx_detect(psi, (int)nx, (int)ny, (int)nz, (int)nt, qscale, emask, tmask, cnt, &dctl->status, s));
  HIP_TRY(ftk::launch_scan_u8(cnt, hoff, V, &dctl->total, tmp, s));
  Ctl h;
  st = read_ctl(&h, dctl, s);
  if (st) return st;
  st = decode_status(h.status);
  if (st) return st;
  const long long nh = h.total;
  if (nh >= 0xffffffffll) return fail(FTK_ERR_CAPACITY, "%lld positive triangles exceed the 32-bit union-find", nh);
  ftk_vortex_result r;
  std::memset(&r, 0, sizeof(r));
  r.n_hits = nh;
  r.tri_id = (int64_t*)al.get(sizeof(int64_t) * (size_t)(nh > 0 ? nh : 1));
  r.pos = (float*)al.get(sizeof(float) * 4 * (size_t)(nh > 0 ? nh : 1));
  r.label = (int64_t*)al.get(sizeof(int64_t) * (size_t)(nh > 0 ? nh : 1));
  unsigned* parent = sc.get<unsigned>((size_t)(nh > 0 ? nh : 1));
  if (!r.tri_id || !r.pos || !r.label || !parent) {
    ftk_vortex_result_free(&r, opt, stream);
    return fail(FTK_ERR_OOM, "output allocation failed");
  }
  hipError_t he = hipSuccess;
  if (nh > 0) {
    he = ftk::launch_vx_emit(psi, (int)nx, (int)ny, (int)nz, (int)nt, qscale, tmask, hoff, (long long*)r.tri_id, r.pos,
                             parent, s);
    if (he == hipSuccess)
      he = ftk::launch_uf_label(parent, (const long long*)r.tri_id, (long long*)r.label, nh, dctl->cnt, s);
  }
  if (he != hipSuccess) {
    ftk_vortex_result_free(&r, opt, stream);
    return fail(FTK_ERR_HIP, "kernel launch: %s", hipGetErrorString(he));
  }
  st = read_ctl(&h, dctl, s);
  if (!st) st = decode_status(h.status);
  if (st) {
    ftk_vortex_result_free(&r, opt, stream);
    return st;
  }
  r.n_components = (long long)h.cnt[ftk::CNT_TRAJ];
  *out = r;
  return FTK_OK;
}

}  // extern "C"

struct ftk_mesh {
  const float* xy = nullptr;  // caller's device array, referenced (not copied)
  long long nv = 0, nf = 0, ne = 0;
  int* tri = nullptr;       // [nf][3] ascending per row
  int* edge = nullptr;      // [ne][2] a < b, ascending
  int* tri_edge = nullptr;  // [nf][3] edges (v0 v1), (v1 v2), (v0 v2)
  int* edge_tri = nullptr;  // [ne][2] triangles of each edge (-1: none); null if an edge has more than two
};

extern "C" {

void ftk_mesh_result_free(ftk_mesh_result* r, const ftk_options* opt, ftk_stream_t stream) {
  if (!r) return;
  ftk_options o;
  resolve(opt, &o);
  const Alloc al = make_alloc(o, (hipStream_t)stream);
  al.put(r->face_id);
  al.put(r->pos);
  al.put(r->label);
  std::memset(r, 0, sizeof(*r));
}

ftk_status ftk_mesh_create(const float* xy, int64_t nv, const int32_t* tri, int64_t nf, ftk_stream_t stream,
                           ftk_mesh** out) {
  g_err.clear();
  if (!out) return fail(FTK_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!xy || !tri) return fail(FTK_ERR_ARG, "xy and tri must be given");
  if (nv < 3 || nf < 1) return fail(FTK_ERR_ARG, "need nv >= 3 and nf >= 1");
  if (nv >= (1ll << 31) || nf >= (1ll << 29)) return fail(FTK_ERR_ARG, "mesh too large");
  hipStream_t s = (hipStream_t)stream;
  // mesh topology on the host: rows sorted, unique edges (a < b) ascending, edges (v0 v1), (v1 v2), (v0 v2) per row
  std::vector<int> ht((size_t)(3 * nf));
  HIP_TRY(hipMemcpyAsync(ht.data(), tri, sizeof(int) * 3 * (size_t)nf, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::vector<unsigned long long> keys((size_t)(3 * nf));
  for (long long T = 0; T < nf; ++T) {
    int* r = &ht[(size_t)(3 * T)];
    for (int k = 0; k < 3; ++k)
      if (r[k] < 0 || r[k] >= nv) return fail(FTK_ERR_ARG, "triangle %lld: vertex index out of range", T);
    std::sort(r, r + 3);
    if (r[0] == r[1] || r[1] == r[2]) return fail(FTK_ERR_ARG, "triangle %lld repeats a vertex", T);
    keys[(size_t)(3 * T)] = ((unsigned long long)r[0] << 32) | (unsigned)r[1];
    keys[(size_t)(3 * T + 1)] = ((unsigned long long)r[1] << 32) | (unsigned)r[2];
    keys[(size_t)(3 * T + 2)] = ((unsigned long long)r[0] << 32) | (unsigned)r[2];
  }
  std::vector<unsigned long long> ukeys(keys);
  std::sort(ukeys.begin(), ukeys.end());
  ukeys.erase(std::unique(ukeys.begin(), ukeys.end()), ukeys.end());
  const long long ne = (long long)ukeys.size();
  std::vector<int> he((size_t)(2 * ne)), hte((size_t)(3 * nf));
  for (long long E = 0; E < ne; ++E) {
    he[(size_t)(2 * E)] = (int)(ukeys[(size_t)E] >> 32);
    he[(size_t)(2 * E + 1)] = (int)(ukeys[(size_t)E] & 0xffffffffull);
  }
  for (size_t k = 0; k < keys.size(); ++k)
    hte[k] = (int)(std::lower_bound(ukeys.begin(), ukeys.end(), keys[k]) - ukeys.begin());
  std::vector<int> het((size_t)(2 * ne), -1);  // triangles of each edge
  bool two_per_edge = true;
  for (long long T = 0; T < nf && two_per_edge; ++T)
    for (int k = 0; k < 3; ++k) {
      int* slot = &het[(size_t)(2 * hte[(size_t)(3 * T + k)])];
      if (slot[0] < 0)
        slot[0] = (int)T;
      else if (slot[1] < 0)
        slot[1] = (int)T;
      else
        two_per_edge = false;
    }
  ftk_mesh* m = new ftk_mesh();
  m->xy = xy;
  m->nv = nv;
  m->nf = nf;
  m->ne = ne;
  hipError_t e = hipMalloc((void**)&m->tri, sizeof(int) * 3 * (size_t)nf);
  if (e == hipSuccess) e = hipMalloc((void**)&m->edge, sizeof(int) * 2 * (size_t)ne);
  if (e == hipSuccess) e = hipMalloc((void**)&m->tri_edge, sizeof(int) * 3 * (size_t)nf);
  if (e == hipSuccess) e = hipMemcpyAsync(m->tri, ht.data(), sizeof(int) * 3 * (size_t)nf, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(m->edge, he.data(), sizeof(int) * 2 * (size_t)ne, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(m->tri_edge, hte.data(), sizeof(int) * 3 * (size_t)nf, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && two_per_edge) {
    e = hipMalloc((void**)&m->edge_tri, sizeof(int) * 2 * (size_t)ne);
    if (e == hipSuccess)
      e = hipMemcpyAsync(m->edge_tri, het.data(), sizeof(int) * 2 * (size_t)ne, hipMemcpyHostToDevice, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host vectors die on return
  if (e != hipSuccess) {
    ftk_mesh_destroy(m);
    return fail(FTK_ERR_HIP, "mesh upload: %s", hipGetErrorString(e));
  }
  *out = m;
  return FTK_OK;
}

void ftk_mesh_destroy(ftk_mesh* m) {
  if (!m) return;
  if (m->tri) (void)hipFree(m->tri);
  if (m->edge) (void)hipFree(m->edge);
  if (m->tri_edge) (void)hipFree(m->tri_edge);
  if (m->edge_tri) (void)hipFree(m->edge_tri);
  delete m;
}

ftk_status ftk_track_cp_mesh(const ftk_mesh* m, const float* field, int64_t nt, const ftk_options* opt,
                             ftk_stream_t stream, ftk_mesh_result* out) {
  g_err.clear();
  if (!out) return fail(FTK_ERR_ARG, "out is NULL");
  std::memset(out, 0, sizeof(*out));
  if (!m || !field) return fail(FTK_ERR_ARG, "mesh and field must be given");
  if (nt < 2 || nt > 65535) return fail(FTK_ERR_ARG, "need 2 <= nt <= 65535");
  ftk_options o;
  resolve(opt, &o);
  ftk_status st = ftk::validate_options(o);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  const long long nv = m->nv, nf = m->nf, ne = m->ne;
  const long long S = 3 * nf + 2 * ne, NF = S * nt;
  const Alloc al = make_alloc(o, s);
  Scratch sc(al);
  const long long G = (NF + 15) / 16;  // groups of 16 faces: the offsets keep one base per group
  unsigned char* flag = sc.get<unsigned char>((size_t)G * 16);
  int* gsum = sc.get<int>((size_t)G);
  long long* base = sc.get<long long>((size_t)G);
  long long* tmp = sc.get<long long>(ftk::scan_tmp_elems(G));
  Ctl* dctl = sc.get<Ctl>(1);
  float* ft = sc.get<float>((size_t)(2 * nv * nt));
  if (!flag || !gsum || !base || !tmp || !dctl || !ft) return fail(FTK_ERR_OOM, "scratch allocation failed");
  HIP_TRY(hipMemsetAsync(dctl, 0, sizeof(Ctl), s));
  const float qscale = std::ldexp(1.0f, o.quant_log2);
  HIP_TRY(ftk::launch_pm_test(m->xy, m->tri, m->edge, m->tri_edge, field, nv, nf, ne, (int)nt, qscale, ft, flag,
                              &dctl->status, s));
  HIP_TRY(ftk::launch_group16_bases(flag, NF, false, gsum, base, &dctl->total, tmp, s));
  Ctl h;
  st = read_ctl(&h, dctl, s);
  if (st) return st;
  st = decode_status(h.status);
  if (st) return st;
  const long long nh = h.total;
  if (nh >= 0xffffffffll) return fail(FTK_ERR_CAPACITY, "%lld punctured faces exceed the 32-bit union-find", nh);
  ftk_mesh_result r;
  std::memset(&r, 0, sizeof(r));
  r.n_hits = nh;
  r.faces_per_step = S;
  r.n_edges = ne;
  r.face_id = (int64_t*)al.get(sizeof(int64_t) * (size_t)(nh > 0 ? nh : 1));
  r.pos = (float*)al.get(sizeof(float) * 3 * (size_t)(nh > 0 ? nh : 1));
  r.label = (int64_t*)al.get(sizeof(int64_t) * (size_t)(nh > 0 ? nh : 1));
  unsigned* parent = sc.get<unsigned>((size_t)(nh > 0 ? nh : 1));
  if (!r.face_id || !r.pos || !r.label || !parent) {
    ftk_mesh_result_free(&r, opt, stream);
    return fail(FTK_ERR_OOM, "output allocation failed");
  }
  hipError_t hr = hipSuccess;
  if (nh > 0) {
    hr = ftk::launch_pm_emit(m->xy, m->tri, m->edge, m->tri_edge, m->edge_tri, field, nv, nf, ne, (int)nt, qscale,
                             flag, base, nh, (long long*)r.face_id, r.pos, parent, &dctl->status, s);
    if (hr == hipSuccess)
      hr = ftk::launch_uf_label(parent, (const long long*)r.face_id, (long long*)r.label, nh, dctl->cnt, s);
  }
  if (hr != hipSuccess) {
    ftk_mesh_result_free(&r, opt, stream);
    return fail(FTK_ERR_HIP, "kernel launch: %s", hipGetErrorString(hr));
  }
  st = read_ctl(&h, dctl, s);
  if (!st) st = decode_status(h.status);
  if (st) {
    ftk_mesh_result_free(&r, opt, stream);
    return st;
  }
  r.n_trajectories = (long long)h.cnt[ftk::CNT_TRAJ];
  *out = r;
  return FTK_OK;
}

ftk_status ftk_track_cp_mesh2d(const float* xy, int64_t nv, const int32_t* tri, int64_t nf, const float* field,
                               int64_t nt, const ftk_options* opt, ftk_stream_t stream, ftk_mesh_result* out) {
  g_err.clear();
  if (!out) return fail(FTK_ERR_ARG, "out is NULL");
  std::memset(out, 0, sizeof(*out));
  if (!field) return fail(FTK_ERR_ARG, "field must be given");
  if (nt < 2 || nt > 65535) return fail(FTK_ERR_ARG, "need 2 <= nt <= 65535");
  ftk_mesh* m = nullptr;
  ftk_status st = ftk_mesh_create(xy, nv, tri, nf, stream, &m);
  if (st) return st;
  st = ftk_track_cp_mesh(m, field, nt, opt, stream, out);
  (void)hipStreamSynchronize((hipStream_t)stream);
  ftk_mesh_destroy(m);
  return st;
}

void ftk_buffer_free(void* p, const ftk_options* opt, ftk_stream_t stream) {
  if (!p) return;
  ftk_options o;
  resolve(opt, &o);
  make_alloc(o, (hipStream_t)stream).put(p);
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------------------------
// Autotuning of the 2D detection tiling (tile rows x slab depth) on the caller's field.
// ---------------------------------------------------------------------------------------------------------------
extern "C" ftk_status ftk_autotune_cp2d(const float* field, ftk_field_kind kind, int64_t nx, int64_t ny, int64_t nt,
                                         const ftk_options* opt, ftk_stream_t stream, ftk_options* tuned) {
  g_err.clear();
  if (!field || !tuned) return fail(FTK_ERR_ARG, "field and tuned must be given");
  if (kind != FTK_SCALAR && kind != FTK_VECTOR) return fail(FTK_ERR_ARG, "kind must be FTK_SCALAR or FTK_VECTOR");
  if (nx < 2 || ny < 2 || nt < 2) return fail(FTK_ERR_ARG, "nx, ny, nt must be >= 2");
  if (nx > (1 << 30) || ny > (1 << 30) || nt > (1 << 30)) return fail(FTK_ERR_ARG, "dimension too large");
  ftk_options o;
  resolve(opt, &o);
  ftk_status st = ftk::validate_options(o);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  const Alloc al = make_alloc(o, s);
  Scratch sc(al);
  ftk::Grid2 g;
  g.f = field;
  g.kind = (int)kind;
  g.nx = (int)nx;
  g.ny = (int)ny;
  g.nt = (int)nt;
  g.nxt = (int)((nx + 63) / 64);
  g.qscale = std::ldexp(1.0f, o.quant_log2);
  g.precision = o.precision;
  g.t_begin = 0;
  g.t_end = (int)nt;
  g.f_ring = 0;
  g.m_ring = 0;
  set_debug(g, o);
  const long long V = (long long)nx * ny * nt, nseg = (long long)nt * ny * g.nxt;
  uint16_t* masks = sc.get<uint16_t>((size_t)V);
  int* seg_cnt = sc.get<int>((size_t)nseg);
  Ctl* dctl = sc.get<Ctl>(1);
  if (!masks || !seg_cnt || !dctl) return fail(FTK_ERR_OOM, "scratch allocation failed");
  HIP_TRY(hipMemsetAsync(dctl, 0, sizeof(Ctl), s));
  Phases ph;
  ph.init(true, s);
  if (!ph.on) return fail(FTK_ERR_HIP, "event creation failed");
  const int rows[3] = {8, 16, 32}, slabs[3] = {8, 16, 32};
  int best_ty = 16, best_tt = 16;
  float best = 1e30f;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const int ty = rows[a], tt = slabs[b] < nt ? slabs[b] : (int)nt;
      if (b > 0 && slabs[b - 1] >= nt) continue;  // same clamped depth as the previous candidate
      HIP_TRY(ftk::launch_detect2d(g, ty, tt, false, masks, seg_cnt, &dctl->status, s));  // warm-up
      ph.mark(0);
      for (int r = 0; r < 2; ++r) HIP_TRY(ftk::launch_detect2d(g, ty, tt, false, masks, seg_cnt, &dctl->status, s));
      ph.mark(1);
      HIP_TRY(hipStreamSynchronize(s));
      const float ms = ph.ms(0, 1);
      if (ms < best) {
        best = ms;
        best_ty = ty;
        best_tt = tt;
      }
    }
  Ctl h;
  st = read_ctl(&h, dctl, s);
  if (st) return st;
  if (h.status & ftk::ST_NONFINITE) return decode_status(h.status);
  ftk::tune_store((int)kind, nx, ny, best_ty, best_tt);
  *tuned = o;
  tuned->tile_y = best_ty;
  tuned->slab_depth = best_tt;
  return FTK_OK;
}
