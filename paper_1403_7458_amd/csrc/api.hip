// C ABI of libspamm: argument checks, handle management, device memory,
// kernel timing and the host side of SpAMM (Eq. 4) and SP2 (Sec. 4).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace spamm {

namespace {

thread_local std::string g_last_error;

int fail(const Error& e) {
  g_last_error = e.msg;
  return e.code;
}
int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}
Error err(int code, const std::string& msg) { return Error{code, msg}; }

std::mutex g_pool_mu;
bool g_pool_ready[64] = {};

void configure_pool(int dev) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (dev < 0 || dev >= 64 || g_pool_ready[dev]) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t keep = UINT64_MAX;  // keep freed blocks cached in the pool
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  }
  (void)hipGetLastError();
  g_pool_ready[dev] = true;
}

// ---- kernel timing ----------------------------------------------------------

struct TimedSpan {
  int phase;
  hipEvent_t a, b;
  int64_t products;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<TimedSpan> g_spans;
spamm_profile g_prof_acc{};

// Pinned staging for small device-to-host reads on this thread.  Kept for
// the life of the process (no HIP call from static destructors).
thread_local void* g_stage = nullptr;

void* staging() {
  if (!g_stage && hipHostMalloc(&g_stage, 4096, 0) != hipSuccess) {
    (void)hipGetLastError();
    g_stage = nullptr;
  }
  return g_stage;
}

Error read_small(void* host, const void* dev, size_t bytes, hipStream_t s) {
  void* st = bytes <= 4096 ? staging() : nullptr;
  if (st) {
    SPAMM_HIP(hipMemcpyAsync(st, dev, bytes, hipMemcpyDeviceToHost, s));
    SPAMM_HIP(hipStreamSynchronize(s));
    std::memcpy(host, st, bytes);
  } else {
    SPAMM_HIP(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s));
    SPAMM_HIP(hipStreamSynchronize(s));
  }
  return Error{};
}

// Pointer kind: device memory of the current device, or host memory.
bool is_device_ptr(const void* p) {
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof(attr));
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice;
}

int current_device() {
  int d = 0;
  (void)hipGetDevice(&d);
  return d;
}

// A dense FP64 input on the device: either the caller's pointer or a
// staged copy of host memory (owned here).
struct DenseIn {
  const double* p = nullptr;
  int64_t ld = 0;
  double* owned = nullptr;
  hipStream_t s = nullptr;
  Error take(const double* src, int64_t n, int64_t ld_src, hipStream_t st) {
    s = st;
    if (is_device_ptr(src)) {
      p = src;
      ld = ld_src;
      return Error{};
    }
    SPAMM_TRY(dev_alloc_n(&owned, n * n, st));
    SPAMM_HIP(hipMemcpy2DAsync(owned, size_t(n) * 8, src, size_t(ld_src) * 8, size_t(n) * 8,
                               size_t(n), hipMemcpyHostToDevice, st));
    p = owned;
    ld = n;
    return Error{};
  }
  ~DenseIn() {
    if (owned) dev_free(owned, s);
  }
};

// Per-thread reusable workspace of the culling pass, kept for the life of
// the thread (never destroyed, so no HIP call runs from a static destructor).
struct Workspace {
  CullWork cull;
  hipStream_t last = nullptr;
  bool used = false;
  int device = -1;
  void bind(hipStream_t s) {
    const int d = current_device();
    if (device != d) {
      if (used) cull.release(last);
      device = d;
    }
    if (used && last != s) (void)hipStreamSynchronize(last);
    last = s;
    used = true;
  }
};
thread_local Workspace* g_ws_ptr = nullptr;
Workspace& ws() {
  if (!g_ws_ptr) g_ws_ptr = new Workspace();
  return *g_ws_ptr;
}

bool valid_prec(int p) { return p >= SPAMM_FP64 && p <= SPAMM_FP16X3; }

// ---- matrices ----------------------------------------------------------------

Error build_from_dense(const double* a_dev, int64_t lda, int64_t n, int prec, Scale* scale,
                       double* trace_part, hipStream_t s, spamm_matrix** out, Scale* scale_host,
                       int64_t* count_dev) {
  spamm_matrix* m = nullptr;
  SPAMM_TRY(new_matrix(n, prec, s, &m));
  {
    PhaseTimer timer(SPAMM_PHASE_TREE, s);
    launch_leaf_norms_dense(a_dev, lda, m, scale, s);
    Error e = compact_nonzero_blocks(m, count_dev, s);
    if (!e.ok()) {
      free_matrix(m);
      return e;
    }
  }
  struct {
    int64_t count[2];
  } cnt;
  Error e = read_small(&cnt, count_dev, sizeof(cnt), s);
  if (e.ok()) e = read_small(scale_host, scale, sizeof(Scale), s);
  if (!e.ok()) {
    free_matrix(m);
    return e;
  }
  if (scale_host->nonfinite) {
    free_matrix(m);
    return err(SPAMM_ERR_NONFINITE, "input holds NaN or Inf");
  }
  if ((prec == SPAMM_FP16 || prec == SPAMM_FP16X3) && scale_host->max_val > 65504.0) {
    free_matrix(m);
    return err(SPAMM_ERR_INVALID_ARG, "FP16 forms need |entries| <= 65504");
  }
  m->n_blocks = cnt.count[0];
  e = alloc_pool(m, std::max<int64_t>(m->n_blocks, 1), s);
  if (!e.ok()) {
    free_matrix(m);
    return e;
  }
  {
    PhaseTimer timer(SPAMM_PHASE_TREE, s);
    if (trace_part) launch_fill_f64(trace_part, m->nb, 0.0, s);
    launch_write_tiles(a_dev, lda, m, scale, trace_part, s);
  }
  launch_pyramid(m, s);
  *out = m;
  return Error{};
}

Error check_tau(double tau) {
  if (!std::isfinite(tau) || tau < 0.0) return err(SPAMM_ERR_INVALID_ARG, "tau must be finite and >= 0");
  return Error{};
}

Error multiply_impl(const spamm_matrix* a, const spamm_matrix* b, double tau, hipStream_t s,
                    spamm_matrix** c_out, spamm_mult_stats* st) {
  if (!a || !b || !c_out) return err(SPAMM_ERR_INVALID_ARG, "NULL handle");
  SPAMM_TRY(check_tau(tau));
  if (a->n != b->n || a->prec != b->prec)
    return err(SPAMM_ERR_SHAPE, "operands differ in size or precision");
  ws().bind(s);
  CullResult cr;
  SPAMM_TRY(run_cull(ws().cull, a, b, tau, st != nullptr, s, &cr));
  spamm_matrix* c = nullptr;
  SPAMM_TRY(new_matrix(a->n, a->prec, s, &c));
  Error e = alloc_pool(c, std::max<int64_t>(cr.n_cblocks, 1), s);
  if (!e.ok()) {
    free_matrix(c);
    return e;
  }
  c->n_blocks = cr.n_cblocks;
  const int64_t cells = int64_t(c->nb) * c->nb;
  launch_fill_i32(c->map, cells, -1, s);
  launch_fill_f64(c->norms + tier_offset(c->depth), cells, 0.0, s);
  GemmArgs g{};
  g.nb = a->nb;
  g.n_nodes = cr.n_cblocks;
  g.nodes = cr.nodes;
  g.nptr = cr.nptr;
  g.ks = cr.ks;
  g.n_super = cr.n_super;
  g.sup_nodes = cr.sup_nodes;
  g.sup_nptr = cr.sup_nptr;
  g.sup_ks = cr.sup_ks;
  g.sup_bits = cr.sup_bits;
  g.sup_cnt4 = cr.sup_cnt4;
  g.sup_noff = cr.sup_noff;
  if (a->prec == SPAMM_FP32 && cr.n_quad > 0 && leaf_kernel_choice() == kLeaf4x4) {
    launch_quad_masks(cr, a, b, tau, s);
    launch_scatter_nodes(cr.nodes, cr.n_cblocks, c->nb, c->map, c->coords, s);
    g.n_quad = cr.n_quad;
    g.quad_nodes = cr.quad_nodes;
    g.quad_nptr = cr.quad_nptr;
    g.quad_ks = cr.quad_ks;
    g.quad_masks = cr.quad_masks;
  }
  g.pool_a = a->pool;
  g.map_a = a->map;
  g.pool_b = b->pool;
  g.map_b = b->map;
  g.pool_c = c->pool;
  g.map_c = c->map;
  g.coords_c = c->coords;
  g.norm_c = c->norms + tier_offset(c->depth);
  const bool fp16 = a->prec == SPAMM_FP16 || a->prec == SPAMM_FP16X3;
  int32_t* overflow = reinterpret_cast<int32_t*>(&ws().cull.ctl_dev->scratch[2]);
  if (fp16) {
    launch_fill_i32(overflow, 2, 0, s);
    g.overflow = overflow;
  }
  {
    PhaseTimer timer(SPAMM_PHASE_GEMM, s, cr.n_tasks);
    launch_leaf_gemm(a->prec, g, s);
  }
  launch_pyramid(c, s);
  if (fp16) {
    int32_t flag = 0;
    Error e2 = read_small(&flag, overflow, sizeof(flag), s);
    if (e2.ok() && flag) e2 = err(SPAMM_ERR_NONFINITE, "product leaves FP16's finite range");
    if (!e2.ok()) {
      free_matrix(c);
      return e2;
    }
  }
  if (st) {
    st->n_exec = cr.n_tasks;
    st->n_cblocks = cr.n_cblocks;
    st->n_nonzero_pairs = cr.nonzero_pairs;
    st->n_dense = int64_t(a->nb) * a->nb * a->nb;
    st->err_bound = cr.err_bound;
    st->cull_restarts = cr.restarts;
    st->reserved = 0;
  }
  *c_out = c;
  return Error{};
}

}  // namespace

// ---- shared helpers ---------------------------------------------------------

Error hip_error(hipError_t e, const char* what) {
  (void)hipGetLastError();
  return Error{e == hipErrorOutOfMemory ? SPAMM_ERR_OOM : SPAMM_ERR_DEVICE,
               std::string(what) + ": " + hipGetErrorString(e)};
}

Error dev_alloc(void** p, size_t bytes, hipStream_t s) {
  configure_pool(current_device());
  hipError_t e = hipMallocAsync(p, bytes, s);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return Error{e == hipErrorOutOfMemory ? SPAMM_ERR_OOM : SPAMM_ERR_DEVICE,
                 "device allocation of " + std::to_string(bytes) + " bytes failed: " +
                     hipGetErrorString(e)};
  }
  return Error{};
}

void dev_free(void* p, hipStream_t s) {
  if (p) (void)hipFreeAsync(p, s);
}

Error DevBuf::reserve(size_t want, hipStream_t s) {
  if (want <= bytes && p) return Error{};
  dev_free(p, s);
  p = nullptr;
  bytes = 0;
  const size_t grown = std::max(want, size_t(256));
  SPAMM_TRY(dev_alloc(&p, grown, s));
  bytes = grown;
  return Error{};
}

void DevBuf::release(hipStream_t s) {
  dev_free(p, s);
  p = nullptr;
  bytes = 0;
}

bool profiling_on() { return g_prof_on; }

PhaseTimer::PhaseTimer(int ph, hipStream_t s, int64_t prod) : phase(ph), stream(s), products(prod) {
  if (!g_prof_on) return;
  if (hipEventCreate(&start) != hipSuccess || hipEventRecord(start, s) != hipSuccess) {
    (void)hipGetLastError();
    start = nullptr;
  }
}

PhaseTimer::~PhaseTimer() {
  if (!start) return;
  hipEvent_t stop = nullptr;
  if (hipEventCreate(&stop) != hipSuccess || hipEventRecord(stop, stream) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipEventDestroy(start);
    return;
  }
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_spans.push_back(TimedSpan{phase, start, stop, products});
}

Error new_matrix(int64_t n, int prec, hipStream_t s, spamm_matrix** out) {
  int nb = 1, depth = 0;
  while (int64_t(kLeaf) * nb < n) {
    nb *= 2;
    ++depth;
    if (depth > SPAMM_MAX_DEPTH) return err(SPAMM_ERR_INVALID_ARG, "matrix too large");
  }
  spamm_matrix* m = new spamm_matrix();
  m->n = n;
  m->nb = nb;
  m->depth = depth;
  m->n_pad = int64_t(kLeaf) * nb;
  m->prec = prec;
  m->device = current_device();
  m->stream = s;
  Error e = dev_alloc_n(&m->map, int64_t(nb) * nb, s);
  if (e.ok()) e = dev_alloc_n(&m->norms, norms_size(depth), s);
  if (!e.ok()) {
    free_matrix(m);
    return e;
  }
  *out = m;
  return Error{};
}

// Tile pool of cap_blocks tiles; the slot -> block array too unless the
// compaction of a tree build already made one (sized nb * nb).
Error alloc_pool(spamm_matrix* m, int64_t cap_blocks, hipStream_t s) {
  SPAMM_TRY(dev_alloc(&m->pool, size_t(cap_blocks) * tile_bytes(m->prec), s));
  if (m->coords == nullptr) {
    Error e = dev_alloc_n(&m->coords, cap_blocks, s);
    if (!e.ok()) {
      dev_free(m->pool, s);
      m->pool = nullptr;
      return e;
    }
  }
  m->cap_blocks = cap_blocks;
  return Error{};
}

void free_matrix(spamm_matrix* m) {
  if (!m) return;
  dev_free(m->pool, m->stream);
  dev_free(m->coords, m->stream);
  dev_free(m->map, m->stream);
  dev_free(m->norms, m->stream);
  delete m;
}

}  // namespace spamm

using namespace spamm;

extern "C" {

void sp2_options_default(sp2_options* o) {
  if (!o) return;
  o->precision = SPAMM_FP32;
  o->max_iter = 100;
  o->min_iter = 0;
  o->stall_rule = 1;
  o->tol = 1e-8;
  o->stall_floor = 0.0;
}

const char* spamm_last_error(void) { return g_last_error.c_str(); }

const char* spamm_version(void) { return "spamm-mi355x 0.1 (gfx950)"; }

int spamm_tree_build(const double* a, int64_t n, int64_t lda, int32_t prec, void* stream,
                     spamm_matrix** out) {
  if (out) *out = nullptr;
  if (!a || !out) return fail(SPAMM_ERR_INVALID_ARG, "NULL pointer");
  if (n < 1 || lda < n) return fail(SPAMM_ERR_INVALID_ARG, "need n >= 1 and lda >= n");
  if (!valid_prec(prec)) return fail(SPAMM_ERR_INVALID_ARG, "unsupported precision");
  hipStream_t s = static_cast<hipStream_t>(stream);
  DenseIn in;
  Error e = in.take(a, n, lda, s);
  if (!e.ok()) return fail(e);
  Scale* scale = nullptr;
  int64_t* cnt = nullptr;
  e = dev_alloc_n(&scale, 1, s);
  if (e.ok()) e = dev_alloc_n(&cnt, 2, s);
  if (e.ok()) {
    launch_init_scale(scale, s);
    Scale sh;
    e = build_from_dense(in.p, in.ld, n, prec, scale, nullptr, s, out, &sh, cnt);
  }
  dev_free(scale, s);
  dev_free(cnt, s);
  return e.ok() ? SPAMM_OK : fail(e);
}

int spamm_multiply(const spamm_matrix* a, const spamm_matrix* b, double tau, void* stream,
                   spamm_matrix** c, spamm_mult_stats* st) {
  if (c) *c = nullptr;
  Error e = multiply_impl(a, b, tau, static_cast<hipStream_t>(stream), c, st);
  return e.ok() ? SPAMM_OK : fail(e);
}

}  // extern "C"

struct spamm_tasks {
  int64_t n_cblocks = 0, n_tasks = 0;
  int32_t* nodes = nullptr;
  int64_t* nptr = nullptr;
  int32_t* ks = nullptr;
  hipStream_t stream = nullptr;
};

namespace {

__global__ void k_unpack_nodes(const int32_t* nodes, int64_t n, int32_t* ci, int32_t* cj) {
  const int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (x >= n) return;
  ci[x] = unpack_i(nodes[x]);
  cj[x] = unpack_j(nodes[x]);
}

void free_tasks(spamm_tasks* t) {
  if (!t) return;
  dev_free(t->nodes, t->stream);
  dev_free(t->nptr, t->stream);
  dev_free(t->ks, t->stream);
  delete t;
}

Error copy_out(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return Error{};
  if (is_device_ptr(dst)) {
    SPAMM_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
  } else {
    SPAMM_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
    SPAMM_HIP(hipStreamSynchronize(s));
  }
  return Error{};
}

Error cull_impl(const spamm_matrix* a, const spamm_matrix* b, double tau, hipStream_t s,
                spamm_tasks** out) {
  if (!a || !b || !out) return err(SPAMM_ERR_INVALID_ARG, "NULL handle");
  SPAMM_TRY(check_tau(tau));
  if (a->n != b->n || a->prec != b->prec)
    return err(SPAMM_ERR_SHAPE, "operands differ in size or precision");
  ws().bind(s);
  CullResult cr;
  SPAMM_TRY(run_cull(ws().cull, a, b, tau, false, s, &cr));
  spamm_tasks* t = new spamm_tasks();
  t->stream = s;
  t->n_cblocks = cr.n_cblocks;
  t->n_tasks = cr.n_tasks;
  Error e = dev_alloc_n(&t->nodes, cr.n_cblocks, s);
  if (e.ok()) e = dev_alloc_n(&t->nptr, cr.n_cblocks + 1, s);
  if (e.ok()) e = dev_alloc_n(&t->ks, cr.n_tasks, s);
  if (!e.ok()) {
    free_tasks(t);
    return e;
  }
  hipError_t h = hipSuccess;
  if (cr.n_cblocks > 0)
    h = hipMemcpyAsync(t->nodes, cr.nodes, size_t(cr.n_cblocks) * 4, hipMemcpyDeviceToDevice, s);
  if (h == hipSuccess)
    h = hipMemcpyAsync(t->nptr, cr.nptr, size_t(cr.n_cblocks + 1) * 8, hipMemcpyDeviceToDevice, s);
  if (h == hipSuccess && cr.n_tasks > 0)
    h = hipMemcpyAsync(t->ks, cr.ks, size_t(cr.n_tasks) * 4, hipMemcpyDeviceToDevice, s);
  if (h != hipSuccess) {
    free_tasks(t);
    return hip_error(h, "hipMemcpyAsync");
  }
  *out = t;
  return Error{};
}

}  // namespace

extern "C" {

int spamm_cull(const spamm_matrix* a, const spamm_matrix* b, double tau, void* stream,
               spamm_tasks** out) {
  if (out) *out = nullptr;
  Error e = cull_impl(a, b, tau, static_cast<hipStream_t>(stream), out);
  return e.ok() ? SPAMM_OK : fail(e);
}

int spamm_tasks_info(const spamm_tasks* t, int64_t* n_cblocks, int64_t* n_tasks) {
  if (!t) return fail(SPAMM_ERR_INVALID_ARG, "NULL handle");
  if (n_cblocks) *n_cblocks = t->n_cblocks;
  if (n_tasks) *n_tasks = t->n_tasks;
  return SPAMM_OK;
}

int spamm_tasks_copy(const spamm_tasks* t, int32_t* c_i, int32_t* c_j, int64_t* c_ptr, int32_t* k,
                     void* stream) {
  if (!t || !c_i || !c_j || !c_ptr || !k) return fail(SPAMM_ERR_INVALID_ARG, "NULL pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int32_t* tmp = nullptr;
  Error e = dev_alloc_n(&tmp, 2 * std::max<int64_t>(t->n_cblocks, 1), s);
  if (!e.ok()) return fail(e);
  if (t->n_cblocks > 0)
    k_unpack_nodes<<<unsigned((t->n_cblocks + 255) / 256), 256, 0, s>>>(
        t->nodes, t->n_cblocks, tmp, tmp + t->n_cblocks);
  e = copy_out(c_i, tmp, size_t(t->n_cblocks) * 4, s);
  if (e.ok()) e = copy_out(c_j, tmp + t->n_cblocks, size_t(t->n_cblocks) * 4, s);
  if (e.ok()) e = copy_out(c_ptr, t->nptr, size_t(t->n_cblocks + 1) * 8, s);
  if (e.ok()) e = copy_out(k, t->ks, size_t(t->n_tasks) * 4, s);
  dev_free(tmp, s);
  return e.ok() ? SPAMM_OK : fail(e);
}

void spamm_tasks_destroy(spamm_tasks* t) { free_tasks(t); }

int spamm_to_dense(const spamm_matrix* m, double* out, int64_t ld, void* stream) {
  if (!m || !out) return fail(SPAMM_ERR_INVALID_ARG, "NULL pointer");
  if (ld < m->n) return fail(SPAMM_ERR_INVALID_ARG, "ld < n");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (is_device_ptr(out)) {
    launch_to_dense(m, out, ld, s);
    return SPAMM_OK;
  }
  double* tmp = nullptr;
  Error e = dev_alloc_n(&tmp, m->n * m->n, s);
  if (!e.ok()) return fail(e);
  launch_to_dense(m, tmp, m->n, s);
  hipError_t h = hipMemcpy2DAsync(out, size_t(ld) * 8, tmp, size_t(m->n) * 8, size_t(m->n) * 8,
                                  size_t(m->n), hipMemcpyDeviceToHost, s);
  if (h == hipSuccess) h = hipStreamSynchronize(s);
  dev_free(tmp, s);
  if (h != hipSuccess) return fail(hip_error(h, "hipMemcpy2DAsync"));
  return SPAMM_OK;
}

int spamm_matrix_info(const spamm_matrix* m, spamm_info* info) {
  if (!m || !info) return fail(SPAMM_ERR_INVALID_ARG, "NULL pointer");
  double root = 0.0;
  Error e = read_small(&root, m->norms, sizeof(double), m->stream);
  if (!e.ok()) return fail(e);
  info->n = m->n;
  info->n_pad = m->n_pad;
  info->nb = m->nb;
  info->depth = m->depth;
  info->precision = m->prec;
  info->reserved = 0;
  info->n_blocks = m->n_blocks;
  info->frobenius = root;
  return SPAMM_OK;
}

int spamm_matrix_norms(const spamm_matrix* m, double* out, void* stream) {
  if (!m || !out) return fail(SPAMM_ERR_INVALID_ARG, "NULL pointer");
  Error e = copy_out(out, m->norms, size_t(norms_size(m->depth)) * 8,
                     static_cast<hipStream_t>(stream));
  return e.ok() ? SPAMM_OK : fail(e);
}

void spamm_matrix_destroy(spamm_matrix* m) { free_matrix(m); }

int spamm_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return SPAMM_OK;
}

int spamm_profile_reset(void) {
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& sp : g_spans) {
    (void)hipEventDestroy(sp.a);
    (void)hipEventDestroy(sp.b);
  }
  g_spans.clear();
  std::memset(&g_prof_acc, 0, sizeof(g_prof_acc));
  return SPAMM_OK;
}

int spamm_profile_read(spamm_profile* out) {
  if (!out) return fail(SPAMM_ERR_INVALID_ARG, "NULL pointer");
  hipError_t h = hipDeviceSynchronize();
  if (h != hipSuccess) return fail(hip_error(h, "hipDeviceSynchronize"));
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& sp : g_spans) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, sp.a, sp.b) == hipSuccess) {
      g_prof_acc.launches[sp.phase] += 1;
      g_prof_acc.ms[sp.phase] += ms;
      if (sp.phase == SPAMM_PHASE_GEMM) g_prof_acc.gemm_products += sp.products;
    } else {
      (void)hipGetLastError();
    }
    (void)hipEventDestroy(sp.a);
    (void)hipEventDestroy(sp.b);
  }
  g_spans.clear();
  *out = g_prof_acc;
  return SPAMM_OK;
}

}  // extern "C"

// ---- SP2 -----------------------------------------------------------------------

namespace {

struct Sp2Buffers {
  hipStream_t s = nullptr;
  double* row = nullptr;      // 3 n: Gershgorin lo, hi, max
  Scale* scale = nullptr;
  int64_t* cnt = nullptr;
  double* trace_part = nullptr;
  double* err_part = nullptr;
  ~Sp2Buffers() {
    dev_free(row, s);
    dev_free(scale, s);
    dev_free(cnt, s);
    dev_free(trace_part, s);
    dev_free(err_part, s);
  }
};

// Gershgorin bounds and input checks of F, then the tree of
// X_0 = (eps_max I - F) / (eps_max - eps_min) (the SP2 scaling; Sec. 4):
// leaf norms of the FP64 values of X_0, then its tiles, with the diagonal
// sums of the stored values in buf.trace_part.
Error sp2_ingest(const double* f, int64_t ldf, int64_t n, int prec, Sp2Buffers& buf,
                 hipStream_t s, spamm_matrix** x, Scale* sh) {
  int nb = 1;
  while (int64_t(kLeaf) * nb < n) nb *= 2;
  SPAMM_TRY(dev_alloc_n(&buf.row, 3 * n, s));
  SPAMM_TRY(dev_alloc_n(&buf.scale, 1, s));
  SPAMM_TRY(dev_alloc_n(&buf.cnt, 2, s));
  SPAMM_TRY(dev_alloc_n(&buf.trace_part, nb, s));
  {
    PhaseTimer timer(SPAMM_PHASE_TREE, s);
    launch_init_scale(buf.scale, s);
    launch_gershgorin_scale(f, n, ldf, buf.row, buf.row + n, buf.row + 2 * n, buf.scale, s);
    launch_asymmetry(f, n, ldf, buf.scale, s);
  }
  // Reject bad input before building anything.
  SPAMM_TRY(read_small(sh, buf.scale, sizeof(Scale), s));
  if (sh->nonfinite) return err(SPAMM_ERR_NONFINITE, "F holds NaN or Inf");
  if (sh->max_asym > 1e-12 * sh->max_abs)
    return err(SPAMM_ERR_NOT_SYMMETRIC, "F is not symmetric (max|F - F^T| > 1e-12 max|F|)");
  if (sh->bad_bounds)
    return err(SPAMM_ERR_INVALID_ARG, "degenerate spectrum bounds (eps_max <= eps_min)");
  return build_from_dense(f, ldf, n, prec, buf.scale, buf.trace_part, s, x, sh, buf.cnt);
}

Error sp2_impl(const double* f, int64_t n, int64_t ldf, int64_t n_occ, double tau,
               const sp2_options* opt_in, hipStream_t s, double* p, int64_t ldp, sp2_stats* st,
               int* status) {
  sp2_options opt;
  sp2_options_default(&opt);
  if (opt_in) opt = *opt_in;
  if (!f || !p) return err(SPAMM_ERR_INVALID_ARG, "NULL pointer");
  if (n < 1 || ldf < n || ldp < n) return err(SPAMM_ERR_INVALID_ARG, "need n >= 1, ldf >= n, ldp >= n");
  if (n_occ < 0 || n_occ > n) return err(SPAMM_ERR_INVALID_ARG, "need 0 <= n_occ <= n");
  SPAMM_TRY(check_tau(tau));
  if (!valid_prec(opt.precision)) return err(SPAMM_ERR_INVALID_ARG, "unsupported precision");
  if (opt.max_iter < 1 || opt.max_iter > SP2_MAX_ITER || opt.min_iter < 0 ||
      !(opt.tol >= 0.0) || !(opt.stall_floor >= 0.0))
    return err(SPAMM_ERR_INVALID_ARG, "bad sp2 options");
  ws().bind(s);
  CullWork& w = ws().cull;
  SPAMM_TRY(ensure_control(w));
  DenseIn in;
  SPAMM_TRY(in.take(f, n, ldf, s));
  Sp2Buffers buf;
  buf.s = s;
  Scale sh;
  spamm_matrix* x = nullptr;
  SPAMM_TRY(sp2_ingest(in.p, in.ld, n, opt.precision, buf, s, &x, &sh));
  const int64_t cells = int64_t(x->nb) * x->nb;
  Error e0 = dev_alloc_n(&buf.err_part, cells, s);
  if (!e0.ok()) {
    free_matrix(x);
    return e0;
  }
  const int nb = x->nb;
  Control* ctl = w.ctl_dev;
  launch_sp2_reduce(nb, buf.trace_part, nullptr, nullptr, ctl, s);
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->eps_min = sh.eps_min;
    st->eps_max = sh.eps_max;
  }
  CullResult cr;
  Error e = run_cull(w, x, x, tau, false, s, &cr);
  if (!e.ok()) {
    free_matrix(x);
    return e;
  }
  double t_n = w.ctl_host->sp2_trace;
  std::vector<double> errs;
  // The stall rule acts below stall_floor * ||P||_F, ||P||_F = sqrt(n_occ);
  // stall_floor = 0 picks max(1e-3, 4 u) for the leaf precision's unit
  // roundoff u, since the floor of e_n grows with u.
  double floor_rel = opt.stall_floor;
  if (floor_rel == 0.0) {
    static const double unit[] = {0x1p-53, 0x1p-24, 0x1p-8, 0x1p-11, 0x1p-16, 0x1p-22};
    floor_rel = std::max(1e-3, 4.0 * unit[opt.precision]);
  }
  const double stall_at = floor_rel * std::sqrt(double(std::max<int64_t>(n_occ, 1)));
  int stop = SP2_STOP_MAX_ITER;
  int it = 0;
  int64_t total_exec = 0;
  for (it = 0; it < opt.max_iter; ++it) {
    const bool square = t_n > double(n_occ);
    spamm_matrix* y = nullptr;
    e = new_matrix(n, opt.precision, s, &y);
    if (e.ok()) e = alloc_pool(y, std::max<int64_t>(cr.n_cblocks + (square ? 0 : x->n_blocks), 1), s);
    if (!e.ok()) {
      free_matrix(y);
      free_matrix(x);
      return e;
    }
    launch_sp2_prepare(y->map, y->norms + tier_offset(y->depth), buf.err_part, nb,
                       buf.trace_part, &ctl->scratch[1], s);
    GemmArgs g{};
    g.nb = nb;
    g.n_nodes = cr.n_cblocks;
    g.nodes = cr.nodes;
    g.nptr = cr.nptr;
    g.ks = cr.ks;
    g.n_super = cr.n_super;
    g.sup_nodes = cr.sup_nodes;
    g.sup_nptr = cr.sup_nptr;
    g.sup_ks = cr.sup_ks;
    g.sup_bits = cr.sup_bits;
    g.sup_cnt4 = cr.sup_cnt4;
    g.sup_noff = cr.sup_noff;
    if (opt.precision == SPAMM_FP32 && cr.n_quad > 0 && leaf_kernel_choice() == kLeaf4x4) {
      launch_quad_masks(cr, x, x, tau, s);
      launch_scatter_nodes(cr.nodes, cr.n_cblocks, nb, y->map, y->coords, s);
      g.n_quad = cr.n_quad;
      g.quad_nodes = cr.quad_nodes;
      g.quad_nptr = cr.quad_nptr;
      g.quad_ks = cr.quad_ks;
      g.quad_masks = cr.quad_masks;
    }
    g.pool_a = x->pool;
    g.map_a = x->map;
    g.pool_b = x->pool;
    g.map_b = x->map;
    g.pool_c = y->pool;
    g.map_c = y->map;
    g.coords_c = y->coords;
    g.norm_c = y->norms + tier_offset(y->depth);
    g.sp2 = 1;
    g.square = square ? 1 : 0;
    g.pool_x = x->pool;
    g.map_x = x->map;
    g.trace_part = buf.trace_part;
    g.err_part = buf.err_part;
    g.overflow = reinterpret_cast<int32_t*>(&ctl->scratch[2]);
    {
      PhaseTimer timer(SPAMM_PHASE_GEMM, s, cr.n_tasks);
      launch_leaf_gemm(opt.precision, g, s);
    }
    {
      PhaseTimer timer(SPAMM_PHASE_EPILOGUE, s);
      RestArgs r{};
      r.nb = nb;
      r.square = g.square;
      r.n_x = x->n_blocks;
      r.pool_x = x->pool;
      r.coords_x = x->coords;
      r.base_slot = cr.n_cblocks;
      r.pool_out = y->pool;
      r.map_out = y->map;
      r.coords_out = y->coords;
      r.norm_out = y->norms + tier_offset(y->depth);
      r.trace_part = buf.trace_part;
      r.err_part = buf.err_part;
      r.counter = &ctl->scratch[1];
      launch_sp2_rest(opt.precision, r, s);
      launch_sp2_reduce(nb, buf.trace_part, buf.err_part, nullptr, ctl, s);
    }
    launch_pyramid(y, s);
    const int64_t n_exec = cr.n_tasks, y_direct = cr.n_cblocks;
    total_exec += n_exec;
    if (st) {
      st->branch[it] = square ? 1 : 0;
      st->trace[it] = t_n;
      st->n_exec[it] = n_exec;
      st->n_blocks[it] = x->n_blocks;
    }
    // The next product's occlusion pass is queued before the one
    // synchronisation of this iteration, which also brings back t_{n+1}
    // and e_n.
    if (it + 1 < opt.max_iter) {
      e = run_cull(w, y, y, tau, false, s, &cr);
    } else {
      e = read_small(w.ctl_host, ctl, sizeof(Control), s);
    }
    if (!e.ok()) {
      free_matrix(y);
      free_matrix(x);
      return e;
    }
    if (w.ctl_host->scratch[2] != 0) {
      free_matrix(y);
      free_matrix(x);
      return err(SPAMM_ERR_NONFINITE, "SP2 iterate is not finite or leaves FP16's range");
    }
    const double e_n = std::sqrt(w.ctl_host->sp2_err2);
    t_n = w.ctl_host->sp2_trace;
    y->n_blocks = y_direct + w.ctl_host->extra_blocks;
    errs.push_back(e_n);
    if (st) st->err[it] = e_n;
    free_matrix(x);
    x = y;
    if (it + 1 >= opt.min_iter) {
      if (e_n < opt.tol) {
        stop = SP2_STOP_CONVERGED;
        break;
      }
      if (opt.stall_rule && it >= 2 && e_n < stall_at && e_n >= errs[it - 2]) {
        stop = SP2_STOP_STALLED;
        break;
      }
    }
  }
  const int iters = std::min(it + 1, opt.max_iter);
  if (st) {
    st->iterations = iters;
    st->stop_reason = stop;
    st->trace_final = t_n;
    st->n_exec_total = total_exec;
  }
  // P = X_{n+1} of the stopping iteration, unpadded to FP64.
  if (is_device_ptr(p)) {
    launch_to_dense(x, p, ldp, s);
    hipError_t h = hipStreamSynchronize(s);
    free_matrix(x);
    if (h != hipSuccess) return hip_error(h, "hipStreamSynchronize");
  } else {
    double* tmp = nullptr;
    e = dev_alloc_n(&tmp, n * n, s);
    if (!e.ok()) {
      free_matrix(x);
      return e;
    }
    launch_to_dense(x, tmp, n, s);
    hipError_t h = hipMemcpy2DAsync(p, size_t(ldp) * 8, tmp, size_t(n) * 8, size_t(n) * 8,
                                    size_t(n), hipMemcpyDeviceToHost, s);
    if (h == hipSuccess) h = hipStreamSynchronize(s);
    dev_free(tmp, s);
    free_matrix(x);
    if (h != hipSuccess) return hip_error(h, "hipMemcpy2DAsync");
  }
  *status = stop == SP2_STOP_MAX_ITER ? SPAMM_NOT_CONVERGED : SPAMM_OK;
  return Error{};
}

}  // namespace

extern "C" int sp2_solve(const double* f, int64_t n, int64_t ldf, int64_t n_occ, double tau,
                         const sp2_options* opt, void* stream, double* p, int64_t ldp,
                         sp2_stats* st) {
  int status = SPAMM_OK;
  Error e = sp2_impl(f, n, ldf, n_occ, tau, opt, static_cast<hipStream_t>(stream), p, ldp, st,
                     &status);
  if (!e.ok()) return fail(e);
  if (status == SPAMM_NOT_CONVERGED) g_last_error = "SP2 reached max_iter without converging";
  return status;
}

extern "C" int sp2_initial_guess(const double* f, int64_t n, int64_t ldf, int32_t prec,
                                 void* stream, spamm_matrix** x0, double* eps_min,
                                 double* eps_max) {
  if (x0) *x0 = nullptr;
  if (!f || !x0) return fail(SPAMM_ERR_INVALID_ARG, "NULL pointer");
  if (n < 1 || ldf < n) return fail(SPAMM_ERR_INVALID_ARG, "need n >= 1 and ldf >= n");
  if (!valid_prec(prec)) return fail(SPAMM_ERR_INVALID_ARG, "unsupported precision");
  hipStream_t s = static_cast<hipStream_t>(stream);
  DenseIn in;
  Error e = in.take(f, n, ldf, s);
  if (!e.ok()) return fail(e);
  Sp2Buffers buf;
  buf.s = s;
  Scale sh;
  e = sp2_ingest(in.p, in.ld, n, prec, buf, s, x0, &sh);
  if (!e.ok()) return fail(e);
  if (eps_min) *eps_min = sh.eps_min;
  if (eps_max) *eps_max = sh.eps_max;
  return SPAMM_OK;
}
