// Internal declarations shared by the translation units of libspamm.
// Device layout of a SpAMM matrix (one per handle):
//   pool    tiles of 32 x 32 elements in the working precision, each tile
//           contiguous and row-major; tile s holds block coords[s]
//   map     int32[nb * nb], row-major over (i, j): tile slot or -1
//   coords  int32[cap], slot -> (i << 16) | j
//   norms   FP64 Frobenius norms of every quadtree tier; tier t is a
//           2^t x 2^t row-major array at offset (4^t - 1) / 3 (Eqs. 2-3)
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/spamm.h"

namespace spamm {

constexpr int kLeaf = 32;
constexpr int kLeaf2 = kLeaf * kLeaf;
constexpr int kMaxTiers = SPAMM_MAX_DEPTH + 1;

__host__ __device__ inline int64_t tier_offset(int t) { return ((int64_t(1) << (2 * t)) - 1) / 3; }
inline int64_t norms_size(int depth) { return tier_offset(depth + 1); }

// Column-quad order of an FP32 32 x 32 tile, the operand layout of the
// 2 x 2 leaf kernels: element (r, c) at ((r % 16) / 4 * 64 + r / 16 * 32 + c)
// * 4 + r % 4, so that 16-byte load q of lane l = 32 kk + c holds rows
// 16 kk + 4 q .. 16 kk + 4 q + 3 of column c, and each load of a wave reads
// 1 KiB contiguously.
__host__ __device__ inline int colq_index(int r, int c) {
  return (((r & 15) >> 2) * 64 + (r >> 4) * 32 + c) * 4 + (r & 3);
}

// Parents of tier t from tier t+1: n^2(parent) = sum of the 4 children's
// squared norms, added in the order (0,0), (0,1), (1,0), (1,1) (Eq. 3).
__device__ inline double parent_norm(const double* ch, int64_t w2, int64_t I, int64_t J) {
  const double a = ch[(2 * I) * w2 + 2 * J], b = ch[(2 * I) * w2 + 2 * J + 1];
  const double c = ch[(2 * I + 1) * w2 + 2 * J], d = ch[(2 * I + 1) * w2 + 2 * J + 1];
  return sqrt(a * a + b * b + c * c + d * d);
}

// Tiers t_top .. 0 of a norm pyramid by one workgroup (each tier reads the
// one below, written by this workgroup before the barrier).  Every thread
// of the workgroup calls it.
__device__ inline void pyramid_tiers(double* __restrict__ norms, int t_top) {
  for (int t = t_top; t >= 0; --t) {
    const int64_t w = int64_t(1) << t;
    for (int64_t x = threadIdx.x; x < w * w; x += blockDim.x)
      norms[tier_offset(t) + x] = parent_norm(norms + tier_offset(t + 1), 2 * w, x / w, x % w);
    __syncthreads();
  }
}
// Bytes of one stored 32 x 32 tile: FP64 8 KiB, FP32 4 KiB; 16-bit forms keep
// the block and its transpose (4 KiB), split forms also the low part (8 KiB).
inline size_t tile_bytes(int prec) {
  switch (prec) {
    case SPAMM_FP64: return 8 * kLeaf2;
    case SPAMM_FP32: return 4 * kLeaf2;
    case SPAMM_BF16:
    case SPAMM_FP16: return 2 * 2 * kLeaf2;
    default: return 4 * 2 * kLeaf2;
  }
}

__host__ __device__ inline int32_t pack_ij(int i, int j) { return (i << 16) | j; }
__host__ __device__ inline int unpack_i(int32_t p) { return p >> 16; }
__host__ __device__ inline int unpack_j(int32_t p) { return p & 0xffff; }

// Error carried from a failing step to the C ABI.
struct Error {
  int code = SPAMM_OK;
  std::string msg;
  bool ok() const { return code == SPAMM_OK; }
};

Error hip_error(hipError_t e, const char* what);
#define SPAMM_HIP(call)                                    \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return ::spamm::hip_error(e_, #call); \
  } while (0)
#define SPAMM_TRY(expr)               \
  do {                                \
    ::spamm::Error r_ = (expr);       \
    if (!r_.ok()) return r_;          \
  } while (0)

// Stream-ordered device allocation (hipMallocAsync on the device's default
// pool, kept cached between calls).
Error dev_alloc(void** p, size_t bytes, hipStream_t s);
void dev_free(void* p, hipStream_t s);

template <class T>
Error dev_alloc_n(T** p, int64_t n, hipStream_t s) {
  return dev_alloc(reinterpret_cast<void**>(p), size_t(n > 0 ? n : 1) * sizeof(T), s);
}

// Grow-only device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  Error reserve(size_t want, hipStream_t s);
  // As reserve, but a regrowth takes 25% headroom (buffers that creep up),
  // never past `limit` bytes.
  Error grow(size_t want, hipStream_t s, size_t limit = SIZE_MAX) {
    if (want <= bytes && p) return Error{};
    return reserve(std::max(want, std::min(want + want / 4, limit)), s);
  }
  void release(hipStream_t s);
};

// Kernel timing (phase totals over HIP events).
struct PhaseTimer {
  int phase;
  hipStream_t stream;
  hipEvent_t start = nullptr;
  int64_t products;
  PhaseTimer(int ph, hipStream_t s, int64_t prod = 0);
  ~PhaseTimer();
};

}  // namespace spamm

// The matrix handle.
struct spamm_matrix {
  int64_t n = 0, n_pad = 0;
  int nb = 0, depth = 0, prec = SPAMM_FP32;
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t n_blocks = 0;
  int64_t cap_blocks = 0;
  void* pool = nullptr;
  int32_t* map = nullptr;
  int32_t* coords = nullptr;
  double* norms = nullptr;
  double frob = 0.0;
  bool owns = true;  // false: the buffers belong to a workspace (SP2 iterates)
  void* colq = nullptr;  // FP32 SP2 operands: column-quad copy of the pool (never owned)
};

namespace spamm {

// ---- tree.hip --------------------------------------------------------------

// Scaling applied while ingesting: value = (diag * [i == j] + sign * a_ij) / div
// for i, j < n, zero in the padding.  Lives in device memory so that SP2's
// Gershgorin bounds never leave the device before the tiles are written.
struct Scale {
  double diag, sign, div;
  double eps_min, eps_max;
  double max_abs, max_asym;
  double max_val;  // max |scaled value| (for the 16-bit range check)
  int32_t nonfinite;
  int32_t bad_bounds;
};

Error new_matrix(int64_t n, int prec, hipStream_t s, spamm_matrix** out);
void free_matrix(spamm_matrix* m);
Error alloc_pool(spamm_matrix* m, int64_t cap_blocks, hipStream_t s);

// Leaf norms of the scaled input into m->norms (leaf tier), the non-finite
// flag into scale->nonfinite.  a: device, n x n, lda.
void launch_leaf_norms_dense(const double* a, int64_t lda, const spamm_matrix* m,
                             Scale* scale, hipStream_t s);
// Slots for the blocks with non-zero norm: fills m->map and m->coords
// (capacity nb*nb) and writes the count into *count_dev.
Error compact_nonzero_blocks(spamm_matrix* m, int64_t* count_dev, hipStream_t s);
// Scaled, converted tiles of every stored block; diagonal-block traces of
// the stored values into trace_part[nb] when non-NULL.
void launch_write_tiles(const double* a, int64_t lda, const spamm_matrix* m, const Scale* scale,
                        double* trace_part, hipStream_t s);
// Tier norms above the leaves (Eq. 3).
// Tiers depth-1 .. 0 of m's pyramid from its leaf norms.  With leave_top,
// the tiers that one workgroup computes are left out and their top tier is
// returned (-1 when none are left): the occlusion pass computes them at its
// start (cull_launch's pyr_top).
int launch_pyramid(const spamm_matrix* m, hipStream_t s, bool leave_top = false);
// Gershgorin bounds, max |F| and the non-finite flag, then the scale of
// X_0 = (eps_max I - F) / (eps_max - eps_min).
void launch_gershgorin_scale(const double* f, int64_t n, int64_t ldf, double* row_lo,
                             double* row_hi, double* row_max, Scale* scale, hipStream_t s);
// max |F_ij - F_ji| into scale->max_asym.
void launch_asymmetry(const double* f, int64_t n, int64_t ldf, Scale* scale, hipStream_t s);
void launch_init_scale(Scale* scale, hipStream_t s);  // plain: diag 0, sign 1, div 1
void launch_to_dense(const spamm_matrix* m, double* out, int64_t ld, hipStream_t s);
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
void launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);

// ---- scan.hip --------------------------------------------------------------

// Exclusive scans of cnt[0..L) and of [cnt > 0], with L = mult * (*len_dev)
// when len_dev is non-NULL (else len_host), optionally masked to zero when
// *len_dev exceeds len_cap.  Totals go to *tot_cnt and *tot_nz; the sum of
// err[0..L/mult) (fixed order) to *tot_err when err is non-NULL.
struct ScanWork {
  DevBuf part;
};
Error launch_scan(const int32_t* cnt, int64_t* off_cnt, int32_t* off_nz, const double* err,
                 const int64_t* len_dev, int64_t len_cap, int mult, int64_t len_host,
                 int64_t* tot_cnt, int64_t* tot_nz, double* tot_err, ScanWork& w,
                 hipStream_t s);

// ---- cull.hip --------------------------------------------------------------

// Control block shared by the culling pass and the SP2 reductions, copied
// to the host in one transfer per synchronisation.
struct Control {
  int64_t n_nodes[kMaxTiers];
  int64_t n_tasks[kMaxTiers];
  double err[kMaxTiers];
  int64_t nonzero_pairs;
  int64_t extra_blocks;   // SP2: blocks of X_n carried into X_{n+1} without products
  double sp2_trace;       // tr X_{n+1}
  double sp2_err2;        // ||C - X_n||_F^2
  double frob2;           // ||X_{n+1}||_F^2
  int64_t scratch[4];
};

struct CullWork {
  int depth = -1;
  int64_t cap_nodes[kMaxTiers] = {};
  int64_t cap_tasks[kMaxTiers] = {};
  DevBuf nodes[kMaxTiers], nptr[kMaxTiers], ks[kMaxTiers];
  DevBuf cnt4, toff, noff, part, bits, quad;
  DevBuf mflag, moff;  // symmetric products: off-diagonal flags, mirror offsets
  ScanWork mscan;
  bool upper = false;  // the pass keeps only C nodes with I <= J
  int64_t cap_count = 0;
  Control* ctl_dev = nullptr;
  Control* ctl_host = nullptr;  // pinned
  void release(hipStream_t s);
  size_t held_bytes() const {
    size_t b = cnt4.bytes + toff.bytes + noff.bytes + part.bytes + bits.bytes + quad.bytes +
               mflag.bytes + moff.bytes + mscan.part.bytes;
    for (int t = 0; t < kMaxTiers; ++t) b += nodes[t].bytes + nptr[t].bytes + ks[t].bytes;
    return b;
  }
  ~CullWork();
};

struct CullResult {
  int64_t n_cblocks = 0, n_tasks = 0, nonzero_pairs = 0;
  // Passes with `upper`: the off-diagonal C blocks (their mirrors) and, per
  // C block, the number of off-diagonal ones before it.
  int64_t n_mirrors = 0;
  const int64_t* moff = nullptr;
  double err_bound = 0.0;
  int restarts = 0;
  const int32_t* nodes = nullptr;
  const int64_t* nptr = nullptr;
  const int32_t* ks = nullptr;
  // Tier d-1 (depth >= 1): the 2 x 2 groups of C blocks, each with its
  // ascending K list, the 8 pass bits of every entry (bit 2q + c for child
  // C block q = 2a + b and leaf k = 2K + c), and per child q its leaf task
  // count and C-block index (cnt4[4p + q], noff[4p + q]).
  int64_t n_super = 0;
  const int32_t* sup_nodes = nullptr;
  const int64_t* sup_nptr = nullptr;
  const int32_t* sup_ks = nullptr;
  const uint8_t* sup_bits = nullptr;
  const int32_t* sup_cnt4 = nullptr;
  const int64_t* sup_noff = nullptr;
  // Tier d-2 (depth >= 2): the 4 x 4 groups of C blocks with their K lists
  // and, per entry, the 64 pass bits of its leaf products (bit 16c + 4a + b
  // for C block (4I + a, 4J + b) and leaf k = 4K + c), filled by
  // launch_quad_masks.
  int64_t n_quad = 0;
  const int32_t* quad_nodes = nullptr;
  const int64_t* quad_nptr = nullptr;
  const int32_t* quad_ks = nullptr;
  uint64_t* quad_masks = nullptr;
};

// Runs the occlusion pass tier by tier and synchronises `s` once (plus once
// per regrowth of the frontier buffers).  With want_pairs the count of
// non-zero block pairs and the complete culled-product bound (err_bound)
// are computed too; without, err_bound misses the top tiers.
Error run_cull(CullWork& w, const spamm_matrix* a, const spamm_matrix* b, double tau,
               bool want_pairs, hipStream_t s, CullResult* out);
// The same in two halves: cull_launch queues the pass and the copy of the
// control block to w.ctl_host; after the caller has synchronised `s`,
// cull_finish regrows and resumes where needed and fills `out`.
// With `upper` only the C blocks (i, j) with i <= j are kept (products
// known to be symmetric: the other blocks are their mirrors).  With
// pyr_top >= 0 (a == b) the pass first computes a's pyramid tiers
// pyr_top .. 0, which launch_pyramid(..., leave_top) left out.
Error cull_launch(CullWork& w, const spamm_matrix* a, const spamm_matrix* b, double tau,
                  bool want_pairs, hipStream_t s, bool upper = false, int pyr_top = -1);
Error cull_finish(CullWork& w, const spamm_matrix* a, const spamm_matrix* b, double tau,
                  bool want_pairs, hipStream_t s, CullResult* out);
Error ensure_control(CullWork& w);

// The 64-bit leaf masks of the tier d-2 frontier (see CullResult).  Each bit
// repeats the decisions the tier walk took for that leaf product and its
// tier d-1 parent.
void launch_quad_masks(const CullResult& r, const spamm_matrix* a, const spamm_matrix* b,
                       double tau, hipStream_t s);
// map_c[i * nb + j] = x and coords_c[x] = (i, j) for the C blocks of a task list.
void launch_scatter_nodes(const int32_t* nodes, int64_t n, int nb, int32_t* map_c,
                          int32_t* coords_c, hipStream_t s);

// ---- leafgemm.hip ----------------------------------------------------------

struct GemmArgs {
  int nb;
  int64_t n_nodes;
  const int32_t* nodes;
  const int64_t* nptr;
  const int32_t* ks;
  // 2 x 2 block groups of tier d-1 (see CullResult); n_super = 0 selects
  // one wave per C block over the leaf task list instead.
  int64_t n_super;
  const int32_t* sup_nodes;
  const int64_t* sup_nptr;
  const int32_t* sup_ks;
  const uint8_t* sup_bits;
  const int32_t* sup_cnt4;
  const int64_t* sup_noff;
  // 4 x 4 block groups of tier d-2 (see CullResult); used when n_quad > 0.
  // map_c must then already hold the C blocks (launch_scatter_nodes).
  int64_t n_quad;
  const int32_t* quad_nodes;
  const int64_t* quad_nptr;
  const int32_t* quad_ks;
  const uint64_t* quad_masks;
  const void* pool_a;
  const int32_t* map_a;
  const void* pool_b;
  const int32_t* map_b;
  void* pool_c;
  int32_t* map_c;
  int32_t* coords_c;
  double* norm_c;        // leaf tier of C's norms, [nb * nb]
  // Fused SP2 update (sp2 != 0): X_{n+1} = C (square) or 2 X_n - C.
  int sp2;
  int square;
  const void* pool_x;
  const int32_t* map_x;
  double* trace_part;    // [nb]
  double* err_part;      // [nb * nb]
  // FP16 forms: set to 1 when a stored value leaves FP16's finite range.
  int32_t* overflow;
  // Symmetric products (sym != 0): the task list holds only C blocks with
  // i <= j; each off-diagonal block is also stored transposed as block
  // (j, i) in slot n_nodes + moff[node], with the same norm and partials.
  int sym;
  const int64_t* moff;
  // FP32 symmetric squares: the operands' column-quad copy (colq_a, see
  // colq_index; A_ik is read as the columns of its stored transpose (k, i)),
  // and where C's column-quad copy goes (colq_c, with its mirror's).  Null:
  // operands are read from the row-major pools.
  const void* colq_a;
  void* colq_c;
};
// Slot of the mirror of C block `node` = (i, j), or -1.
__device__ inline int64_t mirror_slot(const GemmArgs& g, int64_t node, int i, int j) {
  return (g.sym && i != j) ? g.n_nodes + g.moff[node] : -1;
}
// Leaf-product kernels (all add the same products in the same order):
//   block  one wave per C block;
//   2x2    4 waves per 2 x 2 group of C blocks, operands staged in LDS;
//   4x4    4 waves per 4 x 4 group, operands staged in LDS;
//   w2x2   one wave per 2 x 2 group, operands in registers, next step's
//          loads in flight; w2x2s the same with one operand set (default:
//          fastest measured on the 150-molecule workload).
enum { kLeafBlock = 0, kLeaf2x2 = 1, kLeaf4x4 = 2, kLeafW2x2 = 3, kLeafW2x2s = 4,
       kLeafDefault = kLeafW2x2s };
int leaf_kernel_choice();
// Waves per workgroup of the 2 x 2 kernels for a launch of `groups` groups.
constexpr int64_t kManyGroups = 16384;
int w2x2_waves(int64_t groups);
void launch_leaf_gemm(int prec, const GemmArgs& g, hipStream_t s);
// 16-bit forms (leafgemm16.hip).
void launch_leaf_gemm_half(int prec, const GemmArgs& g, hipStream_t s);

// Batched launch: the leaf products of several independent products of one
// precision in one grid.  Product job[r] owns workgroups [first[r],
// first[r + 1]), a multiple of the XCD count, and its first items[r] waves
// do exactly the work a launch of that product alone gives them, so the
// results are bitwise those of separate launches.  Within its range each
// product's workgroups map to its items XCD by XCD in contiguous runs, as in
// a solo launch: workgroups are dispatched to the XCDs round-robin, so every
// XCD gets an equal share of every product, whatever their sizes.
constexpr int kMaxBatch = 64;
constexpr int kBatchXcds = 8;
struct GemmBatch {
  const GemmArgs* args;            // device array
  int32_t n;
  int32_t waves_per_group;
  int32_t job[kMaxBatch];
  int64_t items[kMaxBatch];
  int64_t first[kMaxBatch + 1];
};
// The product of this wave (its item index in `item`), or NULL if the wave
// has no work.
__device__ inline const GemmArgs* batch_locate(const GemmBatch& b, int wave, int64_t& item) {
  const int64_t wg = blockIdx.x;
  if (wg >= b.first[b.n]) return nullptr;
  int lo = 0, hi = b.n - 1;  // largest r with first[r] <= wg
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.first[mid] <= wg)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int64_t local = wg - b.first[lo];
  const int64_t per_xcd = (b.first[lo + 1] - b.first[lo]) / kBatchXcds;
  const int64_t c = (local % kBatchXcds) * per_xcd + local / kBatchXcds;
  // The wave index is uniform across the wave; saying so keeps the item,
  // and every branch and address derived from it, in scalar registers.
  item = c * b.waves_per_group + __builtin_amdgcn_readfirstlane(wave);
  if (item >= b.items[lo]) return nullptr;
  // The arguments are read through the constant address space, as kernel
  // arguments are: no store of the kernel can change them, so the compiler
  // reads them with scalar loads and branches on them uniformly.
  typedef const __attribute__((address_space(4))) GemmArgs ConstArgs;
  return (const GemmArgs*)((ConstArgs*)(b.args) + b.job[lo]);
}
// host[r] and dev[r] hold the same arguments, on the host and the device;
// every product is of precision prec.  Products whose kernel has no batched
// form (the LDS-staged FP32 variants) are launched one by one.
void launch_leaf_gemm_batch(int prec, const GemmArgs* host, const GemmArgs* dev, int n,
                            hipStream_t s);
void launch_leaf_gemm_half_batch(int prec, const GemmArgs* host, const GemmArgs* dev, int n,
                                 hipStream_t s);
// Fills batches of at most kMaxBatch products of one kind: items(r) is the
// number of waves product r needs (0: skipped), waves_per_group the waves
// of a workgroup; emit(batch) launches first[n] workgroups.
template <class Items, class Emit>
void for_each_batch(const GemmArgs* dev, int n, int waves_per_group, Items items, Emit emit) {
  GemmBatch b{};
  b.args = dev;
  b.n = 0;
  b.waves_per_group = waves_per_group;
  b.first[0] = 0;
  for (int r = 0; r < n; ++r) {
    const int64_t w = items(r);
    if (w <= 0) continue;
    const int64_t groups = (w + waves_per_group - 1) / waves_per_group;
    b.job[b.n] = r;
    b.items[b.n] = w;
    b.first[b.n + 1] = b.first[b.n] + (groups + kBatchXcds - 1) / kBatchXcds * kBatchXcds;
    if (++b.n == kMaxBatch) {
      emit(b);
      b.n = 0;
    }
  }
  if (b.n > 0) emit(b);
}

// SP2: blocks of X_n without any executed product.
struct RestArgs {
  int nb;
  int square;
  int64_t n_x;
  const void* pool_x;
  const int32_t* coords_x;
  int64_t base_slot;     // first free slot of the output pool (= C blocks)
  void* pool_out;
  int32_t* map_out;
  int32_t* coords_out;
  double* norm_out;
  double* trace_part;
  double* err_part;
  int64_t* counter;      // appended blocks
  const void* colq_x;    // FP32: column-quad copies of X_n and of the output, or null
  void* colq_out;
};
void launch_sp2_rest(int prec, const RestArgs& r, hipStream_t s);
// Column-quad copies (colq_index) of n FP32 row-major tiles.
void launch_tiles_to_colq(const void* pool, int64_t n, void* colq, hipStream_t s);
void launch_sp2_rest_half(int prec, const RestArgs& r, hipStream_t s);
// map(-1), leaf norms, err_part (nb*nb), trace_part (nb) and the counter
// cleared for one SP2 iteration.
void launch_sp2_prepare(int32_t* map, double* norm_leaf, double* err_part, int nb,
                        double* trace_part, int64_t* counter, hipStream_t s);
// Fixed-order sums of trace_part[nb], err_part[nb*nb] and the squared leaf
// norms into ctl->sp2_trace, sp2_err2, frob2.
void launch_sp2_reduce(int nb, const double* trace_part, const double* err_part,
                       const double* norm_leaf, Control* ctl, hipStream_t s);

// ---- api.hip: host helpers shared by the C ABI's translation units ----------

Error err(int code, const std::string& msg);
int fail(const Error& e);                       // records e.msg, returns e.code
int fail(int code, const std::string& msg);
void set_last_error(const std::string& m);      // this thread's spamm_last_error()
// Small device-to-host read through pinned staging; synchronises s.
Error read_small(void* host, const void* dev, size_t bytes, hipStream_t s);
bool is_device_ptr(const void* p);              // device memory (else host memory)
int current_device();
bool valid_prec(int p);
Error check_tau(double tau);

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
// Grow-only buffers of one SP2 iterate (block map, norm pyramid, tile pool,
// slot coordinates), reused from iteration to iteration: X_{n+1} takes the
// buffers X_{n-1} held.
struct IterBuf {
  DevBuf map, norms, pool, coords;  // pool: the tiles, then their column-quad copies if any
  void release(hipStream_t s) {
    map.release(s);
    norms.release(s);
    pool.release(s);
    coords.release(s);
  }
  size_t held_bytes() const { return map.bytes + norms.bytes + pool.bytes + coords.bytes; }
};
// What one SP2 solve reuses: the culling workspace and two iterate buffers.
struct Sp2Work {
  CullWork cull;
  IterBuf iter[2];
  void release(hipStream_t s) {
    cull.release(s);
    iter[0].release(s);
    iter[1].release(s);
  }
  size_t held_bytes() const {
    return cull.held_bytes() + iter[0].held_bytes() + iter[1].held_bytes();
  }
};

struct Workspace {
  Sp2Work sp2;
  CullWork& cull = sp2.cull;
  hipStream_t last = nullptr;
  bool used = false;
  int device = -1;
  void bind(hipStream_t s) {
    const int d = current_device();
    if (device != d) {
      if (used) sp2.release(last);
      device = d;
    }
    if (used && last != s) (void)hipStreamSynchronize(last);
    last = s;
    used = true;
  }
};
Workspace& ws();  // this thread's, kept for the life of the thread

// Tree of a dense FP64 device matrix under `scale` (leaf norms, compaction,
// tiles, pyramid); the Scale read back into *scale_host.  With trace_part
// the diagonal-block sums of the stored values land there.
Error build_from_dense(const double* a_dev, int64_t lda, int64_t n, int prec, Scale* scale,
                       double* trace_part, hipStream_t s, spamm_matrix** out, Scale* scale_host,
                       int64_t* count_dev);

}  // namespace spamm
