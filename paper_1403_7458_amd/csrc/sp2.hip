// SP2 spectral projection (Sec. 4) on the host side, and the serving form
// that iterates many SP2 solves together on one stream.
//
// One solve is a chain of stream-ordered phases with a single host
// synchronisation per iteration (Sp2Job).  The synchronous sp2_solve drives
// one job; the server drives all its admitted jobs in lockstep, one
// iteration each per step, with the leaf products of a step in one launch
// per precision and one synchronisation per step.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"

namespace spamm {

namespace {

// Unit roundoff of each leaf precision: FP64, FP32, BF16, FP16, BF16 hi+lo,
// FP16 hi+lo (low part scaled by 2^11).
constexpr double kUnit[] = {0x1p-53, 0x1p-24, 0x1p-8, 0x1p-11, 0x1p-16, 0x1p-22};

Error check_sp2(const double* f, int64_t n, int64_t ldf, int64_t n_occ, double tau,
                const sp2_options& opt) {
  if (!f) return err(SPAMM_ERR_INVALID_ARG, "NULL pointer");
  if (n < 1 || ldf < n) return err(SPAMM_ERR_INVALID_ARG, "need n >= 1 and ldf >= n");
  if (n_occ < 0 || n_occ > n) return err(SPAMM_ERR_INVALID_ARG, "need 0 <= n_occ <= n");
  SPAMM_TRY(check_tau(tau));
  if (!valid_prec(opt.precision)) return err(SPAMM_ERR_INVALID_ARG, "unsupported precision");
  if (opt.max_iter < 1 || opt.max_iter > SP2_MAX_ITER || opt.min_iter < 0 ||
      !(opt.tol >= 0.0) || !(opt.stall_floor >= 0.0) || (opt.symmetric != 0 && opt.symmetric != 1))
    return err(SPAMM_ERR_INVALID_ARG, "bad sp2 options");
  return Error{};
}

struct Sp2Buffers {
  hipStream_t s = nullptr;
  double* row = nullptr;  // 3 n: Gershgorin lo, hi, max
  Scale* scale = nullptr;
  int64_t* cnt = nullptr;
  double* trace_part = nullptr;
  double* err_part = nullptr;
  float* colq0 = nullptr;  // column-quad copy of X_0's tiles (FP32 symmetric squares)
  ~Sp2Buffers() {
    dev_free(row, s);
    dev_free(scale, s);
    dev_free(cnt, s);
    dev_free(trace_part, s);
    dev_free(err_part, s);
    dev_free(colq0, s);
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

// One SP2 solve.  Per iteration n (square = t_n > n_occ):
//   front    X_{n+1}'s buffers and the leaf-product arguments of C = X_n X_n
//   (caller) the leaf products with the fused update, alone or batched
//   back     blocks of X_n without products, the fixed-order reductions of
//            tr X_{n+1} and e_n, X_{n+1}'s pyramid, and the occlusion pass of
//            the next square (or, at max_iter, the copy of the scalars)
//   (caller) synchronise the stream
//   end_iter the scalars, the branch of the next iteration and the stop test
class Sp2Job {
 public:
  Sp2Job(int64_t n, int64_t n_occ, double tau, const sp2_options& opt, hipStream_t s,
         Sp2Work* work)
      : n_(n), n_occ_(n_occ), tau_(tau), opt_(opt), s_(s), w_(&work->cull), iter_(work->iter) {
    buf_.s = s;
    std::memset(&st_, 0, sizeof(st_));
    double floor_rel = opt.stall_floor;
    // stall_floor = 0 picks max(1e-3, 4 u) for the leaf precision's unit
    // roundoff u: the floor of e_n grows with u.  The rule acts below
    // floor_rel * ||P||_F with ||P||_F = sqrt(n_occ).
    if (floor_rel == 0.0) floor_rel = std::max(1e-3, 4.0 * kUnit[opt.precision]);
    stall_at_ = floor_rel * std::sqrt(double(std::max<int64_t>(n_occ, 1)));
  }
  ~Sp2Job() {
    free_matrix(y_);
    free_matrix(x_);
  }
  Sp2Job(const Sp2Job&) = delete;
  Sp2Job& operator=(const Sp2Job&) = delete;

  // Input checks (one synchronisation), the tree of X_0, tr X_0 and the
  // first occlusion pass, queued.  f: device, row-major, ldf.
  Error begin(const double* f, int64_t ldf) {
    SPAMM_TRY(ensure_control(*w_));
    SPAMM_TRY(sp2_ingest(f, ldf, n_, opt_.precision, buf_, s_, &x_, &sh_));
    SPAMM_TRY(dev_alloc_n(&buf_.err_part, int64_t(x_->nb) * x_->nb, s_));
    st_.eps_min = sh_.eps_min;
    st_.eps_max = sh_.eps_max;
    // Exactly symmetric F gives exactly symmetric X_0 (each entry is scaled
    // on its own), and squares computed on the upper triangle and mirrored
    // keep every X_n exactly symmetric.  The LDS-staged FP32 variants have
    // no mirrored epilogue.
    const int choice = leaf_kernel_choice();
    sym_ = opt_.symmetric && sh_.max_asym == 0.0 &&
           !(opt_.precision == SPAMM_FP32 && (choice == kLeaf2x2 || choice == kLeaf4x4));
    st_.symmetric = sym_ ? 1 : 0;
    // FP32 symmetric squares on the 2 x 2 kernels read their operands from
    // column-quad copies of the tiles (coalesced loads); every iterate
    // carries one, written next to its row-major tiles.
    colq_ = sym_ && opt_.precision == SPAMM_FP32 && x_->depth >= 1 &&
            (choice == kLeafW2x2 || choice == kLeafW2x2s);
    if (colq_) {
      SPAMM_TRY(dev_alloc_n(&buf_.colq0, std::max<int64_t>(x_->n_blocks, 1) * kLeaf2, s_));
      launch_tiles_to_colq(x_->pool, x_->n_blocks, buf_.colq0, s_);
      x_->colq = buf_.colq0;
    }
    launch_sp2_reduce(x_->nb, buf_.trace_part, nullptr, nullptr, w_->ctl_dev, s_);
    return cull_launch(*w_, x_, x_, tau_, false, s_, sym_);
  }
  // After the synchronisation: the first task list and t_0.
  Error begun() {
    SPAMM_TRY(cull_finish(*w_, x_, x_, tau_, false, s_, &cr_));
    t_n_ = w_->ctl_host->sp2_trace;
    return Error{};
  }

  Error front(GemmArgs* g, int64_t* products) {
    square_ = t_n_ > double(n_occ_);
    const int nb = x_->nb;
    Control* ctl = w_->ctl_dev;
    // The direct C blocks, their mirrors (symmetric squares), then the
    // blocks of X_n carried over.
    const int64_t direct = cr_.n_cblocks + cr_.n_mirrors;
    SPAMM_TRY(iterate(iter_[it_ & 1],
                      std::max<int64_t>(direct + (square_ ? 0 : x_->n_blocks), 1), &y_));
    if (!prepared_)
      launch_sp2_prepare(y_->map, y_->norms + tier_offset(y_->depth), buf_.err_part, nb,
                         buf_.trace_part, &ctl->scratch[1], s_);
    prepared_ = false;
    *g = GemmArgs{};
    g->nb = nb;
    g->n_nodes = cr_.n_cblocks;
    g->nodes = cr_.nodes;
    g->nptr = cr_.nptr;
    g->ks = cr_.ks;
    g->n_super = cr_.n_super;
    g->sup_nodes = cr_.sup_nodes;
    g->sup_nptr = cr_.sup_nptr;
    g->sup_ks = cr_.sup_ks;
    g->sup_bits = cr_.sup_bits;
    g->sup_cnt4 = cr_.sup_cnt4;
    g->sup_noff = cr_.sup_noff;
    if (!sym_ && opt_.precision == SPAMM_FP32 && cr_.n_quad > 0 &&
        leaf_kernel_choice() == kLeaf4x4) {
      launch_quad_masks(cr_, x_, x_, tau_, s_);
      launch_scatter_nodes(cr_.nodes, cr_.n_cblocks, nb, y_->map, y_->coords, s_);
      g->n_quad = cr_.n_quad;
      g->quad_nodes = cr_.quad_nodes;
      g->quad_nptr = cr_.quad_nptr;
      g->quad_ks = cr_.quad_ks;
      g->quad_masks = cr_.quad_masks;
    }
    g->pool_a = x_->pool;
    g->map_a = x_->map;
    g->pool_b = x_->pool;
    g->map_b = x_->map;
    g->pool_c = y_->pool;
    g->map_c = y_->map;
    g->coords_c = y_->coords;
    g->norm_c = y_->norms + tier_offset(y_->depth);
    g->sp2 = 1;
    g->square = square_ ? 1 : 0;
    g->pool_x = x_->pool;
    g->map_x = x_->map;
    g->trace_part = buf_.trace_part;
    g->err_part = buf_.err_part;
    g->overflow = reinterpret_cast<int32_t*>(&ctl->scratch[2]);
    g->sym = sym_ ? 1 : 0;
    g->moff = cr_.moff;
    g->colq_a = x_->colq;
    g->colq_c = y_->colq;
    *products = cr_.n_tasks;
    return Error{};
  }

  Error back() {
    Control* ctl = w_->ctl_dev;
    {
      PhaseTimer timer(SPAMM_PHASE_EPILOGUE, s_);
      RestArgs r{};
      r.nb = x_->nb;
      r.square = square_ ? 1 : 0;
      r.n_x = x_->n_blocks;
      r.pool_x = x_->pool;
      r.coords_x = x_->coords;
      r.base_slot = cr_.n_cblocks + cr_.n_mirrors;
      r.pool_out = y_->pool;
      r.map_out = y_->map;
      r.coords_out = y_->coords;
      r.norm_out = y_->norms + tier_offset(y_->depth);
      r.trace_part = buf_.trace_part;
      r.err_part = buf_.err_part;
      r.counter = &ctl->scratch[1];
      r.colq_x = x_->colq;
      r.colq_out = y_->colq;
      launch_sp2_rest(opt_.precision, r, s_);
      launch_sp2_reduce(x_->nb, buf_.trace_part, buf_.err_part, nullptr, ctl, s_);
    }
    // The next square's occlusion pass is queued before the one
    // synchronisation of this iteration, which also brings back t_{n+1}
    // and e_n; its first launch also finishes X_{n+1}'s pyramid.
    culled_ = it_ + 1 < opt_.max_iter;
    const int pyr_top = launch_pyramid(y_, s_, culled_);
    const int it = it_;
    st_.branch[it] = square_ ? 1 : 0;
    st_.trace[it] = t_n_;
    st_.n_exec[it] = cr_.n_tasks;
    st_.n_blocks[it] = x_->n_blocks;
    total_exec_ += cr_.n_tasks;
    y_direct_ = cr_.n_cblocks + cr_.n_mirrors;
    if (!culled_) {
      SPAMM_HIP(hipMemcpyAsync(w_->ctl_host, ctl, sizeof(Control), hipMemcpyDeviceToHost, s_));
      return Error{};
    }
    SPAMM_TRY(cull_launch(*w_, y_, y_, tau_, false, s_, sym_, pyr_top));
    // The next iterate's map, pyramid and partial sums are cleared now, so
    // that after the synchronisation only the leaf products remain to be
    // queued.  Its buffers are those of X_n, whose last reader (this
    // iteration's rest of X_n) is already queued.
    IterBuf& nb = iter_[(it + 1) & 1];
    SPAMM_TRY(nb.map.grow(size_t(x_->nb) * x_->nb * sizeof(int32_t), s_));
    SPAMM_TRY(nb.norms.grow(size_t(norms_size(x_->depth)) * sizeof(double), s_));
    launch_sp2_prepare(static_cast<int32_t*>(nb.map.p),
                       static_cast<double*>(nb.norms.p) + tier_offset(x_->depth), buf_.err_part,
                       x_->nb, buf_.trace_part, &ctl->scratch[1], s_);
    prepared_ = true;
    return Error{};
  }

  Error end_iter() {
    if (culled_) SPAMM_TRY(cull_finish(*w_, y_, y_, tau_, false, s_, &cr_));
    const Control& h = *w_->ctl_host;
    if (h.scratch[2] != 0)
      return err(SPAMM_ERR_NONFINITE, "SP2 iterate is not finite or leaves FP16's range");
    const double e_n = std::sqrt(h.sp2_err2);
    t_n_ = h.sp2_trace;
    y_->n_blocks = y_direct_ + h.extra_blocks;
    errs_.push_back(e_n);
    st_.err[it_] = e_n;
    free_matrix(x_);
    x_ = y_;
    y_ = nullptr;
    const int it = it_++;
    if (it + 1 >= opt_.min_iter) {
      if (e_n < opt_.tol) {
        stop_ = SP2_STOP_CONVERGED;
        done_ = true;
      } else if (opt_.stall_rule && it >= 2 && e_n < stall_at_ && e_n >= errs_[it - 2]) {
        stop_ = SP2_STOP_STALLED;
        done_ = true;
      }
    }
    if (it_ >= opt_.max_iter) done_ = true;
    if (done_) {
      st_.iterations = it_;
      st_.stop_reason = stop_;
      st_.trace_final = t_n_;
      st_.n_exec_total = total_exec_;
    }
    return Error{};
  }

  // P = X_{n+1} of the stopping iteration, unpadded to FP64 (queued).
  void output(double* p_dev, int64_t ldp) { launch_to_dense(x_, p_dev, ldp, s_); }

  bool done() const { return done_; }
  int64_t next_products() const { return cr_.n_tasks; }
  int status() const { return stop_ == SP2_STOP_MAX_ITER ? SPAMM_NOT_CONVERGED : SPAMM_OK; }
  const sp2_stats& stats() const { return st_; }
  int prec() const { return opt_.precision; }
  const Scale& scale() const { return sh_; }
  spamm_matrix* release_x() {
    spamm_matrix* m = x_;
    x_ = nullptr;
    return m;
  }

 private:
  // X_{n+1} in the workspace buffers b (those of X_{n-1}, whose last reader
  // ran earlier on the stream), grown to hold `cap` blocks.
  Error iterate(IterBuf& b, int64_t cap, spamm_matrix** out) {
    const int nb = x_->nb, depth = x_->depth;
    // At most twice the real blocks: C's blocks plus X_n's.
    const int64_t rb = (n_ + kLeaf - 1) / kLeaf, most = 2 * rb * rb;
    SPAMM_TRY(b.map.grow(size_t(nb) * nb * sizeof(int32_t), s_));
    SPAMM_TRY(b.norms.grow(size_t(norms_size(depth)) * sizeof(double), s_));
    // With column-quad copies the pool holds cap tiles, then their copies.
    const size_t tb = tile_bytes(opt_.precision) * (colq_ ? 2 : 1);
    SPAMM_TRY(b.pool.grow(size_t(cap) * tb, s_, size_t(most) * tb));
    SPAMM_TRY(b.coords.grow(size_t(cap) * sizeof(int32_t), s_, size_t(most) * sizeof(int32_t)));
    spamm_matrix* m = new spamm_matrix();
    m->n = n_;
    m->n_pad = x_->n_pad;
    m->nb = nb;
    m->depth = depth;
    m->prec = opt_.precision;
    m->device = x_->device;
    m->stream = s_;
    m->cap_blocks = cap;
    m->pool = b.pool.p;
    m->map = static_cast<int32_t*>(b.map.p);
    m->coords = static_cast<int32_t*>(b.coords.p);
    m->norms = static_cast<double*>(b.norms.p);
    m->owns = false;
    m->colq = colq_ ? static_cast<char*>(b.pool.p) + size_t(cap) * tile_bytes(opt_.precision)
                    : nullptr;
    *out = m;
    return Error{};
  }

  int64_t n_, n_occ_;
  double tau_;
  sp2_options opt_;
  hipStream_t s_;
  CullWork* w_;
  IterBuf* iter_;
  Sp2Buffers buf_;
  Scale sh_{};
  spamm_matrix* x_ = nullptr;  // X_n
  spamm_matrix* y_ = nullptr;  // X_{n+1} while iteration n is in flight
  CullResult cr_;
  sp2_stats st_;
  std::vector<double> errs_;
  double t_n_ = 0.0, stall_at_ = 0.0;
  int it_ = 0;
  int stop_ = SP2_STOP_MAX_ITER;
  bool done_ = false, square_ = false, culled_ = false, sym_ = false, prepared_ = false;
  bool colq_ = false;
  int64_t total_exec_ = 0, y_direct_ = 0;
};

Error sync(hipStream_t s) {
  SPAMM_HIP(hipStreamSynchronize(s));
  return Error{};
}

Error sp2_impl(const double* f, int64_t n, int64_t ldf, int64_t n_occ, double tau,
               const sp2_options* opt_in, hipStream_t s, double* p, int64_t ldp, sp2_stats* st,
               int* status) {
  sp2_options opt;
  sp2_options_default(&opt);
  if (opt_in) opt = *opt_in;
  SPAMM_TRY(check_sp2(f, n, ldf, n_occ, tau, opt));
  if (!p) return err(SPAMM_ERR_INVALID_ARG, "NULL pointer");
  if (ldp < n) return err(SPAMM_ERR_INVALID_ARG, "need ldp >= n");
  ws().bind(s);
  DenseIn in;
  SPAMM_TRY(in.take(f, n, ldf, s));
  Sp2Job job(n, n_occ, tau, opt, s, &ws().sp2);
  SPAMM_TRY(job.begin(in.p, in.ld));
  SPAMM_TRY(sync(s));
  SPAMM_TRY(job.begun());
  while (!job.done()) {
    GemmArgs g;
    int64_t products = 0;
    SPAMM_TRY(job.front(&g, &products));
    {
      PhaseTimer timer(SPAMM_PHASE_GEMM, s, products);
      launch_leaf_gemm(opt.precision, g, s);
    }
    SPAMM_TRY(job.back());
    SPAMM_TRY(sync(s));
    SPAMM_TRY(job.end_iter());
  }
  if (st) *st = job.stats();
  if (is_device_ptr(p)) {
    job.output(p, ldp);
    SPAMM_TRY(sync(s));
  } else {
    double* tmp = nullptr;
    SPAMM_TRY(dev_alloc_n(&tmp, n * n, s));
    job.output(tmp, n);
    hipError_t h = hipMemcpy2DAsync(p, size_t(ldp) * 8, tmp, size_t(n) * 8, size_t(n) * 8,
                                    size_t(n), hipMemcpyDeviceToHost, s);
    if (h == hipSuccess) h = hipStreamSynchronize(s);
    dev_free(tmp, s);
    if (h != hipSuccess) return hip_error(h, "hipMemcpy2DAsync");
  }
  *status = job.status();
  return Error{};
}

}  // namespace

// Device memory an SP2 solve of order n holds at its peak (an upper bound
// over the fill-in SpAMM allows): the two iterate buffers (each up to twice
// the real blocks: C's blocks plus X_n's in the 2X - X^2 branch), both
// trees' maps and pyramids, a dense FP64 staging copy of F and the dense
// result, the SP2 partial sums and a culling workspace sized for the dense
// task count.
size_t footprint_bytes(int64_t n, int prec) {
  int nb = 1, depth = 0;
  while (int64_t(kLeaf) * nb < n) {
    nb *= 2;
    ++depth;
  }
  const double rb = double((n + kLeaf - 1) / kLeaf);
  const double cells = double(nb) * nb;
  // FP32 iterates also hold column-quad copies of their tiles, and X_0 one
  // of its own.
  const double tb = double(tile_bytes(prec)) * (prec == SPAMM_FP32 ? 2.0 : 1.0);
  double b = 4.0 * rb * rb * (tb + 4.0);
  if (prec == SPAMM_FP32) b += rb * rb * double(tile_bytes(prec));
  b += 2.0 * (cells * 8.0 + double(norms_size(depth)) * 8.0);
  b += 2.0 * double(n) * double(n) * 8.0;
  b += cells * 8.0 + double(nb) * 8.0 + 3.0 * double(n) * 8.0;
  b += 8.0 * rb * rb * rb + 64.0 * cells + double(1 << 20);
  return size_t(b);
}

}  // namespace spamm

using namespace spamm;

extern "C" int sp2_solve(const double* f, int64_t n, int64_t ldf, int64_t n_occ, double tau,
                         const sp2_options* opt, void* stream, double* p, int64_t ldp,
                         sp2_stats* st) {
  int status = SPAMM_OK;
  Error e = sp2_impl(f, n, ldf, n_occ, tau, opt, static_cast<hipStream_t>(stream), p, ldp, st,
                     &status);
  if (!e.ok()) return fail(e);
  if (status == SPAMM_NOT_CONVERGED) set_last_error("SP2 reached max_iter without converging");
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

extern "C" size_t sp2_footprint_bytes(int64_t n, int32_t prec) {
  if (n < 1 || !valid_prec(prec)) return 0;
  return footprint_bytes(n, prec);
}

// ---- serving --------------------------------------------------------------------

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t id = 0;
  int64_t n = 0, n_occ = 0;
  double tau = 0.0;
  sp2_options opt{};
  const double* f_dev = nullptr;  // caller's device input
  int64_t ldf = 0;
  std::vector<double> f_host;     // copy of a host input
  size_t reserve = 0;
  size_t accounted = 0;           // bytes counted in used_bytes while running
  // Running.
  std::unique_ptr<Sp2Work> work;
  std::unique_ptr<Sp2Job> job;
  GemmArgs g{};
  int64_t products = 0;
  bool failed = false;
  // Finished.
  bool finished = false;
  int status = SPAMM_PENDING;
  std::string msg;
  double* p_dev = nullptr;        // n x n result, held until polled
  size_t held = 0;
  sp2_stats stats{};
};

}  // namespace

struct spamm_server {
  size_t budget = 0;
  spamm_server_options opt{};
  int device = 0;
  hipStream_t stream = nullptr;   // the worker's
  hipStream_t copy = nullptr;     // callers' result copies
  GemmArgs* args_host = nullptr;  // pinned, max_active
  GemmArgs* args_dev = nullptr;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::map<uint64_t, Request*> all;  // every request not yet polled
  // Workspaces of finished requests, kept with their buffers (counted in
  // cached_bytes) so that later requests reuse them instead of allocating.
  std::vector<std::unique_ptr<Sp2Work>> spare;
  uint64_t next_id = 1;
  bool stopping = false;
  spamm_server_info st{};
  std::thread worker;

  void run();
  void finish(Request* r, const Error& e);
  Error start(Request* r);
  // Under mu: whether q fits with the newest spare workspace, then takes it.
  bool fits(const Request* q) const {
    const size_t h = spare.empty() ? 0 : spare.back()->held_bytes();
    const size_t acc = std::max(q->reserve, h);
    return st.used_bytes + acc + (st.cached_bytes - h) <= budget;
  }
  void admit(Request* r) {
    const size_t h = spare.empty() ? 0 : spare.back()->held_bytes();
    if (!spare.empty()) {
      r->work = std::move(spare.back());
      spare.pop_back();
    }
    st.cached_bytes -= h;
    r->accounted = std::max(r->reserve, h);
    st.used_bytes += r->accounted;
    st.queued -= 1;
    st.active += 1;
    st.peak_used_bytes = std::max(st.peak_used_bytes, st.used_bytes + st.cached_bytes);
  }
  void trim_cache() {
    for (auto& w : spare) w->release(stream);
    st.cached_bytes = 0;
  }
};

namespace {

// H2D staging of a host input on the worker's stream.
Error stage_host_input(Request* r, hipStream_t s, double** f_dev) {
  SPAMM_TRY(dev_alloc_n(f_dev, r->n * r->n, s));
  SPAMM_HIP(hipMemcpyAsync(*f_dev, r->f_host.data(), size_t(r->n) * r->n * 8,
                           hipMemcpyHostToDevice, s));
  return Error{};
}

}  // namespace

Error spamm_server::start(Request* r) {
  if (!r->work) r->work.reset(new Sp2Work());
  r->job.reset(new Sp2Job(r->n, r->n_occ, r->tau, r->opt, stream, r->work.get()));
  double* staged = nullptr;
  const double* f = r->f_dev;
  int64_t ldf = r->ldf;
  if (!f) {
    SPAMM_TRY(stage_host_input(r, stream, &staged));
    f = staged;
    ldf = r->n;
  }
  Error e = r->job->begin(f, ldf);
  if (e.ok()) e = sync(stream);
  if (staged) dev_free(staged, stream);
  std::vector<double>().swap(r->f_host);
  if (e.ok()) e = r->job->begun();
  return e;
}

// Publishes the outcome of a request leaving the running set (its result,
// if any, is already on the device and synchronised).
void spamm_server::finish(Request* r, const Error& e) {
  if (r->job) {
    if (e.ok()) r->stats = r->job->stats();
    r->job.reset();
  }
  std::unique_ptr<Sp2Work> w = std::move(r->work);
  std::lock_guard<std::mutex> lk(mu);
  if (w) {
    st.cached_bytes += w->held_bytes();
    spare.push_back(std::move(w));
  }
  r->status = e.ok() ? r->status : e.code;
  r->msg = e.ok() ? r->msg : e.msg;
  if (!e.ok() && r->p_dev) {
    dev_free(r->p_dev, stream);
    r->p_dev = nullptr;
  }
  st.used_bytes -= r->accounted;
  r->held = r->p_dev ? size_t(r->n) * r->n * 8 : 0;
  st.used_bytes += r->held;
  st.peak_used_bytes = std::max(st.peak_used_bytes, st.used_bytes + st.cached_bytes);
  st.active -= 1;
  st.completed += 1;
  if (!e.ok()) st.failed += 1;
  st.solve_iterations += r->stats.iterations;
  r->finished = true;
  cv_done.notify_all();
}

void spamm_server::run() {
  (void)hipSetDevice(device);
  std::vector<Request*> running;
  for (;;) {
    // Admission, first come first served: the head of the queue starts when
    // its footprint fits in what the budget has left, a slot is free and
    // the running requests' leaf products per step are below fill_products
    // (so a request that fills the device alone runs alone, and small ones
    // share steps).
    bool stop_now = false;
    for (;;) {
      Request* r = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
          if (stopping) {
            stop_now = true;
            break;
          }
          int64_t load = 0;
          for (const Request* q : running) load += q->products;
          if (!queue.empty() && int64_t(running.size()) < opt.max_active &&
              (opt.fill_products <= 0 || running.empty() || load < opt.fill_products)) {
            if (!fits(queue.front()) && st.cached_bytes > 0) trim_cache();
            if (fits(queue.front())) {
              r = queue.front();
              queue.pop_front();
              admit(r);
              break;
            }
          }
          if (!running.empty()) break;
          cv_work.wait(lk);
        }
      }
      if (stop_now || !r) break;
      Error e = start(r);
      if (e.ok()) {
        r->products = r->job->next_products();
        running.push_back(r);
      } else {
        (void)hipStreamSynchronize(stream);
        finish(r, e);
      }
    }
    if (stop_now) break;
    if (running.empty()) continue;
    // One iteration of every running solve: the leaf products of each
    // precision in one launch.
    std::stable_sort(running.begin(), running.end(),
                     [](const Request* a, const Request* b) { return a->job->prec() < b->job->prec(); });
    for (Request* r : running) {
      r->failed = false;
      Error e = r->job->front(&r->g, &r->products);
      if (!e.ok()) {
        r->failed = true;
        r->msg = e.msg;
        r->status = e.code;
      }
    }
    size_t i0 = 0;
    while (i0 < running.size()) {
      const int prec = running[i0]->job->prec();
      size_t i1 = i0;
      int64_t products = 0;
      int cnt = 0;
      while (i1 < running.size() && running[i1]->job->prec() == prec) {
        if (!running[i1]->failed) {
          args_host[i0 + cnt] = running[i1]->g;
          products += running[i1]->products;
          ++cnt;
        }
        ++i1;
      }
      if (cnt > 0 && opt.batch_gemm) {
        // The pinned arguments are rewritten only after this step's
        // synchronisation.
        hipError_t h = hipMemcpyAsync(args_dev + i0, args_host + i0, size_t(cnt) * sizeof(GemmArgs),
                                      hipMemcpyHostToDevice, stream);
        if (h != hipSuccess) {
          (void)hipGetLastError();
          for (size_t k = i0; k < i1; ++k) {
            running[k]->failed = true;
            running[k]->status = SPAMM_ERR_DEVICE;
            running[k]->msg = "copy of the leaf-product arguments failed";
          }
          cnt = 0;
        }
      }
      if (cnt > 0) {
        PhaseTimer timer(SPAMM_PHASE_GEMM, stream, products);
        if (opt.batch_gemm) {
          launch_leaf_gemm_batch(prec, args_host + i0, args_dev + i0, cnt, stream);
          std::lock_guard<std::mutex> lk(mu);
          st.gemm_launches += 1;
        } else {
          for (int k = 0; k < cnt; ++k) launch_leaf_gemm(prec, args_host[i0 + k], stream);
          std::lock_guard<std::mutex> lk(mu);
          st.gemm_launches += cnt;
        }
      }
      i0 = i1;
    }
    for (Request* r : running) {
      if (r->failed) continue;
      Error e = r->job->back();
      if (!e.ok()) {
        r->failed = true;
        r->msg = e.msg;
        r->status = e.code;
      }
    }
    Error es = sync(stream);
    {
      std::lock_guard<std::mutex> lk(mu);
      st.steps += 1;
    }
    std::vector<Request*> next, retire;
    for (Request* r : running) {
      Error e = es;
      if (e.ok() && r->failed) e = Error{r->status, r->msg};
      if (e.ok()) e = r->job->end_iter();
      if (e.ok() && r->job->done()) {
        e = dev_alloc_n(&r->p_dev, r->n * r->n, stream);
        if (e.ok()) {
          r->job->output(r->p_dev, r->n);
          r->status = r->job->status();
          if (r->status == SPAMM_NOT_CONVERGED) r->msg = "SP2 reached max_iter without converging";
        }
      }
      if (!e.ok()) {
        r->status = e.code;
        r->msg = e.msg;
        r->failed = true;
        retire.push_back(r);
      } else if (r->job->done()) {
        retire.push_back(r);
      } else {
        next.push_back(r);
      }
    }
    if (!retire.empty()) {
      Error e = sync(stream);
      for (Request* r : retire) finish(r, r->failed ? Error{r->status, r->msg} : e);
    }
    running.swap(next);
  }
  // Stopping: drop what is still running.
  for (Request* r : running) {
    r->job.reset();
    if (r->work) r->work->release(stream);
    r->work.reset();
  }
  (void)hipStreamSynchronize(stream);
}

extern "C" {

void spamm_server_options_default(spamm_server_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->max_active = 64;
  o->batch_gemm = 1;
  o->device = -1;
  o->fill_products = 1 << 18;
}

int spamm_server_create(size_t hbm_budget_bytes, const spamm_server_options* o,
                        spamm_server** out) {
  if (out) *out = nullptr;
  if (!out) return fail(SPAMM_ERR_INVALID_ARG, "NULL pointer");
  spamm_server_options opt;
  spamm_server_options_default(&opt);
  if (o) opt = *o;
  if (opt.max_active < 1 || opt.max_active > 1024)
    return fail(SPAMM_ERR_INVALID_ARG, "need 1 <= max_active <= 1024");
  if (opt.fill_products < 0) return fail(SPAMM_ERR_INVALID_ARG, "need fill_products >= 0");
  if (hbm_budget_bytes == 0) return fail(SPAMM_ERR_INVALID_ARG, "budget must be > 0");
  int dev = opt.device;
  if (dev < 0) dev = current_device();
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || dev >= count) {
    (void)hipGetLastError();
    return fail(SPAMM_ERR_INVALID_ARG, "no such device");
  }
  int prev = current_device();
  if (hipSetDevice(dev) != hipSuccess) return fail(hip_error(hipGetLastError(), "hipSetDevice"));
  std::unique_ptr<spamm_server> sv(new spamm_server());
  sv->budget = hbm_budget_bytes;
  sv->opt = opt;
  sv->device = dev;
  sv->st.budget_bytes = hbm_budget_bytes;
  Error e;
  hipError_t h = hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking);
  if (h == hipSuccess) h = hipStreamCreateWithFlags(&sv->copy, hipStreamNonBlocking);
  if (h == hipSuccess)
    h = hipHostMalloc(reinterpret_cast<void**>(&sv->args_host), sizeof(GemmArgs) * opt.max_active, 0);
  if (h == hipSuccess)
    h = hipMalloc(reinterpret_cast<void**>(&sv->args_dev), sizeof(GemmArgs) * opt.max_active);
  (void)hipSetDevice(prev);
  if (h != hipSuccess) {
    e = hip_error(h, "server set-up");
    if (sv->args_dev) (void)hipFree(sv->args_dev);
    if (sv->args_host) (void)hipHostFree(sv->args_host);
    if (sv->copy) (void)hipStreamDestroy(sv->copy);
    if (sv->stream) (void)hipStreamDestroy(sv->stream);
    return fail(e);
  }
  spamm_server* raw = sv.get();
  raw->worker = std::thread([raw] { raw->run(); });
  *out = sv.release();
  return SPAMM_OK;
}

int spamm_server_submit(spamm_server* sv, const double* f, int64_t n, int64_t ldf, int64_t n_occ,
                        double tau, const sp2_options* opt_in, uint64_t* request_id) {
  if (request_id) *request_id = 0;
  if (!sv || !request_id) return fail(SPAMM_ERR_INVALID_ARG, "NULL pointer");
  sp2_options opt;
  sp2_options_default(&opt);
  if (opt_in) opt = *opt_in;
  Error e = check_sp2(f, n, ldf, n_occ, tau, opt);
  if (!e.ok()) return fail(e);
  std::unique_ptr<Request> r(new Request());
  r->n = n;
  r->n_occ = n_occ;
  r->tau = tau;
  r->opt = opt;
  r->ldf = ldf;
  r->reserve = footprint_bytes(n, opt.precision);
  if (r->reserve > sv->budget)
    return fail(SPAMM_ERR_OOM, "request needs " + std::to_string(r->reserve) +
                                   " bytes of device memory, more than the server's budget");
  int prev = current_device();
  (void)hipSetDevice(sv->device);
  const bool on_device = is_device_ptr(f);
  (void)hipSetDevice(prev);
  if (on_device) {
    r->f_dev = f;
  } else {
    r->f_host.resize(size_t(n) * n);
    for (int64_t i = 0; i < n; ++i)
      std::memcpy(r->f_host.data() + i * n, f + i * ldf, size_t(n) * 8);
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->stopping) return fail(SPAMM_ERR_INVALID_ARG, "server is shutting down");
  r->id = sv->next_id++;
  *request_id = r->id;
  sv->st.submitted += 1;
  sv->st.queued += 1;
  sv->all[r->id] = r.get();
  sv->queue.push_back(r.release());
  sv->cv_work.notify_one();
  return SPAMM_OK;
}

namespace {

// Copies a finished request's result out and forgets the request.
int collect(spamm_server* sv, std::unique_lock<std::mutex>& lk, Request* r, double* p,
            int64_t ldp, sp2_stats* st) {
  sv->all.erase(r->id);
  lk.unlock();
  std::unique_ptr<Request> own(r);
  Error e;
  if (r->p_dev) {
    int prev = current_device();
    (void)hipSetDevice(sv->device);
    const bool dev_out = is_device_ptr(p);
    hipError_t h = hipMemcpy2DAsync(p, size_t(ldp) * 8, r->p_dev, size_t(r->n) * 8,
                                    size_t(r->n) * 8, size_t(r->n),
                                    dev_out ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                    sv->copy);
    if (h == hipSuccess) h = hipStreamSynchronize(sv->copy);
    if (h != hipSuccess) e = hip_error(h, "result copy");
    dev_free(r->p_dev, sv->copy);
    (void)hipStreamSynchronize(sv->copy);
    (void)hipSetDevice(prev);
  }
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->st.used_bytes -= r->held;
  }
  sv->cv_work.notify_one();
  if (!e.ok()) return fail(e);
  if (st) *st = r->stats;
  if (r->status != SPAMM_OK) set_last_error(r->msg);
  return r->status;
}

int poll_impl(spamm_server* sv, uint64_t id, double* p, int64_t ldp, sp2_stats* st, bool wait) {
  if (!sv) return fail(SPAMM_ERR_INVALID_ARG, "NULL server");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->all.find(id);
  if (it == sv->all.end()) return fail(SPAMM_ERR_INVALID_ARG, "unknown request id");
  Request* r = it->second;
  // The worker writes a request's outcome before it sets `finished` under
  // the lock, and never touches the request afterwards.
  const bool out_ok = p && ldp >= r->n;
  if (!r->finished) {
    if (!out_ok) return fail(SPAMM_ERR_INVALID_ARG, "need p and ldp >= n");
    if (!wait) return SPAMM_PENDING;
    sv->cv_done.wait(lk, [&] { return r->finished; });
  }
  if (r->p_dev && !out_ok) return fail(SPAMM_ERR_INVALID_ARG, "need p and ldp >= n");
  return collect(sv, lk, r, p, ldp, st);
}

}  // namespace

int spamm_server_poll(spamm_server* sv, uint64_t id, double* p, int64_t ldp, sp2_stats* st) {
  return poll_impl(sv, id, p, ldp, st, false);
}

int spamm_server_wait(spamm_server* sv, uint64_t id, double* p, int64_t ldp, sp2_stats* st) {
  return poll_impl(sv, id, p, ldp, st, true);
}

int spamm_server_stats(spamm_server* sv, spamm_server_info* out) {
  if (!sv || !out) return fail(SPAMM_ERR_INVALID_ARG, "NULL pointer");
  std::lock_guard<std::mutex> lk(sv->mu);
  *out = sv->st;
  return SPAMM_OK;
}

void spamm_server_destroy(spamm_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stopping = true;
  }
  sv->cv_work.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  int prev = current_device();
  (void)hipSetDevice(sv->device);
  for (auto& kv : sv->all) {
    Request* r = kv.second;
    if (r->p_dev) dev_free(r->p_dev, sv->stream);
    delete r;
  }
  for (auto& w : sv->spare) w->release(sv->stream);
  sv->spare.clear();
  (void)hipStreamSynchronize(sv->stream);
  (void)hipFree(sv->args_dev);
  (void)hipHostFree(sv->args_host);
  (void)hipStreamDestroy(sv->copy);
  (void)hipStreamDestroy(sv->stream);
  (void)hipSetDevice(prev);
  delete sv;
}

}  // extern "C"
