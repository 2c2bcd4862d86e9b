// C ABI of libspamm: argument checks, handle management, device memory,
// kernel timing and the host side of SpAMM (Eq. 4).  SP2 and the serving
// form are in sp2.hip.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace spamm {

thread_local std::string g_last_error;

void set_last_error(const std::string& m) { g_last_error = m; }

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
  int phase, device;
  hipEvent_t a, b;
  int64_t products;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
unsigned g_prof_mask = (1u << SPAMM_N_PHASES) - 1;
std::vector<TimedSpan> g_spans;
spamm_profile g_prof_acc{};
// Recorded events go back to a per-device pool when read: creating events
// inside the timed work costs host time between launches.
std::map<int, std::vector<hipEvent_t>> g_event_pool;

// A timing event of the current device.  Without the system-scope fence a
// record is a plain timestamp, with no cache write-back between the kernels
// it separates; the spans are only read after a device synchronisation.
hipEvent_t take_event(int device) {
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    auto& pool = g_event_pool[device];
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

// Caller holds g_prof_mu.
void return_span(const TimedSpan& sp) {
  auto& pool = g_event_pool[sp.device];
  pool.push_back(sp.a);
  pool.push_back(sp.b);
}

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

Workspace& ws() {
  static thread_local Workspace* w = nullptr;
  if (!w) w = new Workspace();  // never destroyed: no HIP call from static destructors
  return *w;
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

PhaseTimer::PhaseTimer(int ph, hipStream_t s, int64_t prod) : phase(ph), stream(s), products(prod) {
  if (!g_prof_on || !(g_prof_mask >> ph & 1u)) return;
  start = take_event(current_device());
  if (start && hipEventRecord(start, s) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipEventDestroy(start);
    start = nullptr;
  }
}

PhaseTimer::~PhaseTimer() {
  if (!start) return;
  const int device = current_device();
  hipEvent_t stop = take_event(device);
  if (!stop || hipEventRecord(stop, stream) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipEventDestroy(start);
    if (stop) (void)hipEventDestroy(stop);
    return;
  }
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_spans.push_back(TimedSpan{phase, device, start, stop, products});
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
  if (!m->owns) {
    delete m;
    return;
  }
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
  o->symmetric = 1;
  o->reserved = 0;
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

int spamm_profile_phases(unsigned mask) {
  if (mask == 0 || (mask >> SPAMM_N_PHASES) != 0) return fail(SPAMM_ERR_INVALID_ARG, "bad phase mask");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_mask = mask;
  return SPAMM_OK;
}

int spamm_profile_reset(void) {
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& sp : g_spans) return_span(sp);
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
    return_span(sp);
  }
  g_spans.clear();
  *out = g_prof_acc;
  return SPAMM_OK;
}

}  // extern "C"
