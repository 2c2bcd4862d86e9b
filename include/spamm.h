/*
 * spamm.h -- C ABI of the MI355X (gfx950) Sparse Approximate Matrix Multiply
 * (SpAMM) and of second-order spectral projection (SP2) built on it.
 *
 * The operations follow Bock, Challacombe & Kale, "Solvers for O(N)
 * Electronic Structure in the Strong Scaling Limit":
 *   - a matrix is a quadtree whose nodes carry Frobenius norms (Sec. 2,
 *     Eqs. 1-3), stored here as 32 x 32 dense leaf blocks of a matrix
 *     zero-padded to N_pad = 32 * 2^d (Sec. 3 blocking; Fig. 4 pads 2,250
 *     to 4,096);
 *   - C = SpAMM(A, B, tau) adds the sub-product A_ik B_kj only where
 *     ||A_ik|| ||B_kj|| > tau, tested tier by tier (Eq. 4; the breadth-first
 *     occlusion of Algs. 2-3);
 *   - SP2 builds the spectral projector of a Fockian, the matrix step
 *     function at the n_occ lowest eigenvalues (Sec. 4), by repeated SpAMM
 *     squares.
 *
 * Conventions shared by every entry point:
 *   - Dense matrices are FP64, row-major, with a leading dimension (in
 *     elements) >= n.  A dense pointer may be host memory or device memory
 *     of the current device; the library tells them apart itself.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Device work is
 *     ordered on it.  Calls that write host memory synchronise it first.
 *   - Handles (spamm_matrix, spamm_tasks) are owned by the library and
 *     released with their destroy call; their device memory is freed
 *     stream-ordered on the stream of the call that created them, which
 *     must still exist at destroy time.
 *   - Errors are return codes; nothing is thrown across the ABI.  On a
 *     negative status no output handle is created (it is set to NULL),
 *     caller arrays are left untouched and spamm_last_error() explains.
 *   - Distinct handles may be used from distinct threads; one handle must
 *     not be used by two calls at once.
 */
#ifndef SPAMM_H
#define SPAMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum spamm_status {
    SPAMM_OK = 0,
    SPAMM_NOT_CONVERGED = 1,      /* SP2 stopped at max_iter: p holds the last iterate */
    SPAMM_PENDING = 2,            /* serving: request not finished yet */
    SPAMM_ERR_INVALID_ARG = -1,   /* bad size, pointer, tau, n_occ or option */
    SPAMM_ERR_NONFINITE = -2,     /* input holds NaN or Inf */
    SPAMM_ERR_NOT_SYMMETRIC = -3, /* SP2 input with max|F - F^T| > 1e-12 max|F| */
    SPAMM_ERR_OOM = -4,           /* device allocation failed; no state was changed */
    SPAMM_ERR_DEVICE = -5,        /* a HIP call failed */
    SPAMM_ERR_SHAPE = -6          /* operands of different size or precision */
} spamm_status;

/* Working precision of the stored leaf blocks and of the leaf products.
 * Norms, traces and the SP2 decisions are FP64 in every precision.  The
 * 16-bit forms accumulate in FP32.  FP16 forms need |entries| <= 65504
 * (inputs are not rescaled); a product that leaves that range fails with
 * SPAMM_ERR_NONFINITE. */
typedef enum spamm_precision {
    SPAMM_FP64 = 0,   /* FP64 tiles, FP64 MFMA products */
    SPAMM_FP32 = 1,   /* FP32 tiles, FP32 MFMA products */
    SPAMM_BF16 = 2,   /* BF16 tiles, BF16 MFMA products */
    SPAMM_FP16 = 3,   /* FP16 tiles, FP16 MFMA products */
    SPAMM_BF16X3 = 4, /* x = hi + lo in BF16; hi*hi + hi*lo + lo*hi on BF16 MFMA */
    SPAMM_FP16X3 = 5  /* x = hi + lo/2^11 in FP16; hi*hi + (hi*lo + lo*hi)/2^11 on FP16 MFMA */
} spamm_precision;

#define SPAMM_LEAF 32            /* leaf block edge N_b (Sec. 3) */
#define SPAMM_MAX_DEPTH 15       /* N_pad <= 32 * 2^15 */
#define SP2_MAX_ITER 256         /* upper limit of sp2_options.max_iter */

typedef struct spamm_matrix spamm_matrix;
typedef struct spamm_tasks spamm_tasks;

typedef struct spamm_info {
    int64_t n;          /* logical dimension */
    int64_t n_pad;      /* 32 * 2^depth */
    int32_t nb;         /* leaf blocks per dimension, n_pad / 32 */
    int32_t depth;      /* d: tier of the leaves (root is tier 0) */
    int32_t precision;  /* spamm_precision of the tiles */
    int32_t reserved;
    int64_t n_blocks;   /* stored (non-zero) leaf blocks */
    double frobenius;   /* root norm, ||A||_F (Eqs. 2-3) */
} spamm_info;

/* Statistics of one SpAMM product (filled when the pointer is non-NULL). */
typedef struct spamm_mult_stats {
    int64_t n_exec;          /* executed 32x32x32 leaf products, |E(tau)| */
    int64_t n_cblocks;       /* C blocks with >= 1 executed product (= stored blocks of C) */
    int64_t n_nonzero_pairs; /* #(i,j,k) with A_ik != 0 and B_kj != 0 */
    int64_t n_dense;         /* nb^3 */
    double err_bound;        /* sum of ||A|| ||B|| over the maximal culled octree nodes;
                                bounds ||C~ - AB||_F (sub-multiplicativity, Sec. 2) */
    int32_t cull_restarts;   /* frontier buffers regrown during the culling pass */
    int32_t reserved;
} spamm_mult_stats;

/* sp2_options: leaf precision and stopping rules (the paper runs SP2 to
 * convergence, Sec. 4; the rules below are this library's reading). */
typedef struct sp2_options {
    int32_t precision;   /* spamm_precision; default SPAMM_FP32 */
    int32_t max_iter;    /* 1..SP2_MAX_ITER; default 100 */
    int32_t min_iter;    /* no stop before this many iterations; default 0 */
    int32_t stall_rule;  /* 1: stop when e_n >= e_{n-2} once
                            e_n < stall_floor * sqrt(max(n_occ, 1)); default 1 */
    double tol;          /* stop when e_n = ||X~_n^2 - X_n||_F < tol; default 1e-8 */
    double stall_floor;  /* default 0: max(1e-3, 4 u), u the leaf precision's unit
                            roundoff (FP64 2^-53, FP32 2^-24, BF16 2^-8, FP16 2^-11,
                            BF16X3 2^-16, FP16X3 2^-22) */
    int32_t symmetric;   /* 1 (default): when F is exactly symmetric, every X_n is
                            too, so each square computes only the C blocks (i, j)
                            with i <= j (the products of E(tau) with i <= j; the
                            task set of (j, i) is the same) and stores (j, i) as
                            the transpose; 0: all C blocks */
    int32_t reserved;
} sp2_options;

enum { SP2_STOP_CONVERGED = 0, SP2_STOP_STALLED = 1, SP2_STOP_MAX_ITER = 2 };

typedef struct sp2_stats {
    int32_t iterations;               /* products computed */
    int32_t stop_reason;              /* SP2_STOP_* */
    int32_t symmetric;                /* 1: upper-triangle squares (see sp2_options) */
    int32_t reserved;
    double eps_min, eps_max;          /* Gershgorin bounds of F */
    double trace_final;               /* tr P */
    int64_t n_exec_total;             /* leaf products over all iterations */
    int8_t branch[SP2_MAX_ITER];      /* 1: X <- X^2, 0: X <- 2X - X^2 */
    double trace[SP2_MAX_ITER];       /* t_n = tr X_n */
    double err[SP2_MAX_ITER];         /* e_n = ||X~_n^2 - X_n||_F */
    int64_t n_exec[SP2_MAX_ITER];     /* executed leaf products of iteration n
                                         (upper-triangle C blocks when symmetric) */
    int64_t n_blocks[SP2_MAX_ITER];   /* stored blocks of X_n */
} sp2_stats;

/* Fill `o` with the defaults listed in sp2_options. */
void sp2_options_default(sp2_options* o);

/*
 * spamm_tree_build -- ingest a dense FP64 matrix as a SpAMM quadtree.
 * (Sec. 2, Eqs. 1-3; Sec. 3 leaf blocking; Fig. 4 padding.)
 *
 * a:      n x n FP64, row-major, leading dimension lda >= n; host or device.
 * prec:   working precision of the stored tiles.
 * out:    new handle: the padded matrix as 32 x 32 tiles (only blocks with a
 *         non-zero entry are stored), the block map, and the FP64 norm of
 *         every quadtree node.  Leaf norms are taken from the FP64 input
 *         values before conversion to the working precision.
 * Errors: SPAMM_ERR_INVALID_ARG (n < 1, lda < n, NULL pointers, bad prec,
 *         depth > SPAMM_MAX_DEPTH), SPAMM_ERR_NONFINITE, SPAMM_ERR_OOM,
 *         SPAMM_ERR_DEVICE.
 */
int spamm_tree_build(const double* a, int64_t n, int64_t lda, int32_t prec, void* stream,
                     spamm_matrix** out);

/*
 * spamm_multiply -- C = SpAMM(A, B, tau).  (Eq. 4; Algs. 2-3.)
 *
 * Executes exactly the leaf products with ||A_ik|| ||B_kj|| > tau (strict),
 * found by tier-by-tier occlusion of the (i, j, k) octree, and accumulates
 * each C block over its k in ascending order (deterministic, no atomics).
 * tau is absolute; tau = 0 skips only exact-zero products.
 * a, b:   handles of equal n and precision (SPAMM_ERR_SHAPE otherwise).
 * c:      new handle holding exactly the blocks with >= 1 executed product;
 *         its norm tree is that of the stored product.
 * st:     optional statistics; NULL also skips the passes that only they
 *         need (the non-zero pair count, the culled-product bound of the
 *         top tiers).
 * Errors: SPAMM_ERR_INVALID_ARG (NULL handles, tau < 0 or not finite),
 *         SPAMM_ERR_SHAPE, SPAMM_ERR_OOM, SPAMM_ERR_DEVICE.
 */
int spamm_multiply(const spamm_matrix* a, const spamm_matrix* b, double tau, void* stream,
                   spamm_matrix** c, spamm_mult_stats* st);

/*
 * spamm_cull -- the occlusion pass of spamm_multiply alone (Algs. 2-3):
 * the leaf task list E(tau) grouped by C block.
 * out:    new handle; read it with spamm_tasks_info / spamm_tasks_copy.
 * Errors: as spamm_multiply.
 */
int spamm_cull(const spamm_matrix* a, const spamm_matrix* b, double tau, void* stream,
               spamm_tasks** out);

/* Sizes of a task list: C blocks and leaf products. */
int spamm_tasks_info(const spamm_tasks* t, int64_t* n_cblocks, int64_t* n_tasks);

/*
 * spamm_tasks_copy -- copy a task list to host or device arrays.
 * c_i, c_j: int32[n_cblocks], block row / column of each C block, in Morton
 *           order of (i, j);
 * c_ptr:    int64[n_cblocks + 1], offsets of each C block's products in k;
 * k:        int32[n_tasks], the k of each product, ascending per C block.
 */
int spamm_tasks_copy(const spamm_tasks* t, int32_t* c_i, int32_t* c_j, int64_t* c_ptr,
                     int32_t* k, void* stream);

void spamm_tasks_destroy(spamm_tasks* t); /* NULL-safe */

/*
 * sp2_solve -- spectral projector of symmetric F by SP2 with SpAMM squares.
 * (Sec. 4: the density matrix as the Heaviside step function of the
 * Fockian, built by second-order spectral projection.)
 *
 * Steps: Gershgorin bounds eps_min, eps_max over the n rows;
 * X_0 = (eps_max I_n - F) / (eps_max - eps_min) (padding stays 0); then for
 * n = 0, 1, ...: t_n = tr X_n, C = SpAMM(X_n, X_n, tau),
 * e_n = ||C - X_n||_F, X_{n+1} = C if t_n > n_occ else 2 X_n - C, stopping
 * on e_n < tol, on a stall (stall_rule) or at max_iter.  P = X_{n+1} of the
 * stopping iteration.  Traces, e_n, the branch and the stop test are FP64.
 * With an exactly symmetric F (and opt->symmetric) each square computes the
 * C blocks (i, j) with i <= j and mirrors the rest (see sp2_options).
 * Device work runs on `stream`; the call returns after P is written.
 *
 * f:      n x n FP64 symmetric, row-major, ldf >= n; host or device.
 * n_occ:  0 <= n_occ <= n.
 * opt:    NULL for the defaults.
 * p:      n x n FP64 output, ldp >= n; host or device; written on
 *         SPAMM_OK and SPAMM_NOT_CONVERGED.
 * st:     optional statistics.
 * Returns SPAMM_OK, SPAMM_NOT_CONVERGED (max_iter reached; p is the last
 * iterate), or SPAMM_ERR_INVALID_ARG / _NONFINITE / _NOT_SYMMETRIC / _OOM /
 * _DEVICE.
 */
int sp2_solve(const double* f, int64_t n, int64_t ldf, int64_t n_occ, double tau,
              const sp2_options* opt, void* stream, double* p, int64_t ldp, sp2_stats* st);

/*
 * sp2_initial_guess -- the first SP2 iterate alone (the scaling step of the
 * SP2 scheme; Sec. 4): Gershgorin bounds eps_min, eps_max over the n rows
 * (eps = F_ii -/+ sum_{j != i} |F_ij|), then the tree of
 * X_0 = (eps_max I_n - F) / (eps_max - eps_min), zero in the padding, with
 * leaf norms from the FP64 values of X_0.
 * f:       as in sp2_solve; x0: new handle; eps_min, eps_max: optional.
 * Errors:  as sp2_solve's input checks (INVALID_ARG, NONFINITE,
 *          NOT_SYMMETRIC, OOM, DEVICE).
 */
int sp2_initial_guess(const double* f, int64_t n, int64_t ldf, int32_t prec, void* stream,
                      spamm_matrix** x0, double* eps_min, double* eps_max);

/*
 * sp2_footprint_bytes -- device memory an SP2 solve of order n in precision
 * prec holds at its peak, as an upper bound over the fill-in SpAMM allows:
 * the tiles of X_n and X_{n+1} (up to 3 (ceil(n/32))^2 tiles), both trees'
 * block maps and norm pyramids, a dense FP64 copy of F and of P, the SP2
 * partial sums and a culling workspace sized for the dense task count.
 * Host-only arithmetic; 0 for n < 1 or an unknown precision.
 */
size_t sp2_footprint_bytes(int64_t n, int32_t prec);

/*
 * ---- Serving: many SP2 solves on one device -------------------------------
 *
 * A server owns a worker thread and a stream (default priority) on one
 * device.  Requests are admitted first come, first served, while the sum of
 * sp2_footprint_bytes over the running requests, the results not yet
 * collected and the buffers finished requests left for reuse fits in the
 * budget (those buffers are dropped first when the next request would not
 * fit), a slot is free, and the running requests leave the device room
 * (fill_products).  Each step runs one SP2 iteration of every
 * running request: the leaf products of all requests of one precision go to
 * one batched launch, the occlusion passes and epilogues of the requests are
 * queued behind it, and the step ends with one synchronisation.  Every
 * request computes exactly what sp2_solve computes for it alone (the same
 * kernels on the same task lists, in the same order), bit for bit.
 */
typedef struct spamm_server spamm_server;

typedef struct spamm_server_options {
    int32_t max_active;  /* requests iterated together, 1..1024; default 64 */
    int32_t batch_gemm;  /* 1 (default): one leaf-product launch per precision
                            and step; 0: one launch per request */
    int32_t device;      /* HIP device; -1 (default): the current device */
    int32_t fill_products; /* admit more requests only while the running ones
                              execute fewer leaf products per step than this
                              (default 2^18; 0: no limit) */
} spamm_server_options;

typedef struct spamm_server_info {
    int64_t submitted, completed, failed;  /* requests */
    int64_t queued, active;                /* requests now waiting / running */
    int64_t steps;                         /* lockstep iterations run */
    int64_t gemm_launches;                 /* leaf-product launches */
    int64_t solve_iterations;              /* SP2 iterations of completed requests */
    uint64_t budget_bytes;
    uint64_t used_bytes;      /* footprints of running requests + results held */
    uint64_t cached_bytes;    /* buffers idle workspaces keep for reuse */
    uint64_t peak_used_bytes; /* peak of used + cached (<= budget) */
} spamm_server_info;

void spamm_server_options_default(spamm_server_options* o);

/* o: NULL for the defaults.  hbm_budget_bytes > 0.  Errors: INVALID_ARG,
 * DEVICE, OOM. */
int spamm_server_create(size_t hbm_budget_bytes, const spamm_server_options* o,
                        spamm_server** out);

/*
 * spamm_server_submit -- queue an SP2 solve (arguments as in sp2_solve;
 * opt NULL for the defaults).  A host F is copied during the call; a device
 * F is read when the request starts, so it must stay valid and unchanged
 * until the request has finished (poll/wait no longer returns PENDING).
 * Argument errors return at once (INVALID_ARG, or OOM when the request's
 * footprint exceeds the whole budget); errors found in F (NONFINITE,
 * NOT_SYMMETRIC) and device failures are the request's status at poll time.
 * request_id: the request's id (> 0).
 */
int spamm_server_submit(spamm_server* s, const double* f, int64_t n, int64_t ldf, int64_t n_occ,
                        double tau, const sp2_options* opt, uint64_t* request_id);

/*
 * spamm_server_poll -- SPAMM_PENDING while the request is queued or running.
 * Once it has finished: copies P into p (n x n FP64, ldp >= n, host or
 * device memory of the server's device), fills st (optional), forgets the
 * request and releases its budget, and returns its status as sp2_solve
 * would (SPAMM_OK, SPAMM_NOT_CONVERGED or a negative error; p untouched on
 * an error).  spamm_server_wait blocks until the request has finished.
 * Results held for collection count against the budget: poll finished
 * requests to keep admission going.
 */
int spamm_server_poll(spamm_server* s, uint64_t id, double* p, int64_t ldp, sp2_stats* st);
int spamm_server_wait(spamm_server* s, uint64_t id, double* p, int64_t ldp, sp2_stats* st);

int spamm_server_stats(spamm_server* s, spamm_server_info* out);

/* Stops the worker after its current step; requests not yet collected are
 * discarded.  NULL-safe. */
void spamm_server_destroy(spamm_server* s);

/* Unpad and upcast a handle to a dense n x n FP64 array (host or device). */
int spamm_to_dense(const spamm_matrix* m, double* out, int64_t ld, void* stream);

/* Shape, precision, block count and root norm of a handle. */
int spamm_matrix_info(const spamm_matrix* m, spamm_info* info);

/*
 * spamm_matrix_norms -- copy the FP64 norms of every quadtree tier (Eq. 3):
 * tier t (0 = root .. depth) is a 2^t x 2^t row-major array starting at
 * element (4^t - 1) / 3 of `out`, which holds (4^(depth+1) - 1) / 3 doubles
 * (host or device).
 */
int spamm_matrix_norms(const spamm_matrix* m, double* out, void* stream);

void spamm_matrix_destroy(spamm_matrix* m); /* NULL-safe */

/* Message of the last failed call on this thread ("" if none). */
const char* spamm_last_error(void);

/* Library version string. */
const char* spamm_version(void);

/*
 * Kernel timing.  While enabled, every device phase selected by
 * spamm_profile_phases (all of them unless restricted) is bracketed by
 * HIP events on the stream it runs on; spamm_profile_read synchronises the
 * device and returns the totals per phase since the last reset.  Each
 * bracket costs host time between launches, so a timed run may select only
 * the phases it reports.
 */
enum {
    SPAMM_PHASE_TREE = 0,     /* ingest, Gershgorin, leaf norms, tile write */
    SPAMM_PHASE_PYRAMID = 1,  /* tier norms (Eq. 3) */
    SPAMM_PHASE_CULL = 2,     /* occlusion and task-list compaction */
    SPAMM_PHASE_GEMM = 3,     /* leaf products (+ fused SP2 update) */
    SPAMM_PHASE_EPILOGUE = 4, /* SP2 blocks of X_n without products, reductions */
    SPAMM_PHASE_DENSE = 5,    /* unpad / upcast */
    SPAMM_N_PHASES = 6
};

typedef struct spamm_profile {
    int64_t launches[SPAMM_N_PHASES];
    double ms[SPAMM_N_PHASES];
    int64_t gemm_products;    /* leaf products run by the timed GEMM launches */
} spamm_profile;

int spamm_profile_enable(int on);
/* mask: bit p selects phase p (SPAMM_PHASE_*); 0 or bits >= SPAMM_N_PHASES:
 * SPAMM_ERR_INVALID_ARG.  Default: every phase. */
int spamm_profile_phases(unsigned mask);
int spamm_profile_reset(void);
int spamm_profile_read(spamm_profile* out);

#ifdef __cplusplus
}
#endif

#endif /* SPAMM_H */
