/*
 * FP64 CPU oracle: SpAMM in the recursive task form of the paper's Alg. 1
 * (Sec. 3.1), with OpenMP untied tasks and one lock per C leaf block.
 *
 * TEST INFRASTRUCTURE ONLY.  It is built next to the device library but is
 * never linked into it; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load it.  It shares no code, header or table with the
 * device path.
 *
 * Storage: every matrix is an array of nb x nb dense 32 x 32 leaf blocks,
 * block (i, j) at offset (i * nb + j) * 1024, each block row-major.  The
 * quadtree of Eq. 1 is implicit in this numbering: node (i, j) of tier t
 * covers leaf rows [i 2^(d-t), (i+1) 2^(d-t)) and the same range of columns.
 *
 * Norms: leaf norms are sqrt(sum a^2) over the block (Eq. 2); tier norms are
 * sqrt(sum of the four children's squared norms) (Eq. 3).
 *
 * Recursion (Alg. 1): on tier t < d, each of the eight child triples
 * (i', j', k') is tested with ||A^{t+1}_{i'k'}|| ||B^{t+1}_{k'j'}|| > tau
 * (the children's norms, as Alg. 3 tests them); a passing child is spawned as an
 * untied task and the node waits for all of them.  On tier d the leaf
 * product C_ij += A_ik B_kj runs with three nested loops under the lock of
 * C_ij.  With depth 0 the root is the single leaf and is tested against tau
 * first; for depth >= 1 the root itself is not tested (Alg. 1 tests children
 * only), which changes nothing because norms are monotone up the tree.
 *
 * Also reported: the number of executed leaf products and the sum of
 * ||A|| ||B|| over every tested-and-culled node, an upper bound on the
 * Frobenius error of the product (sub-multiplicativity, Sec. 2).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define LEAF 32
#define LEAF2 (LEAF * LEAF)

typedef struct {
    int depth;
    int nb;
    const double *a, *b;
    double *c;
    double **na, **nbm;       /* per-tier norms, tier t is (2^t)^2 row-major */
    double tau;
    omp_lock_t *locks;
    int64_t n_exec;
    double culled;
} spamm_ctx;

static void leaf_norms(const double *m, int nb, double *out) {
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) {
            const double *blk = m + ((size_t)i * nb + j) * LEAF2;
            double s = 0.0;
            for (int e = 0; e < LEAF2; ++e) s += blk[e] * blk[e];
            out[(size_t)i * nb + j] = sqrt(s);
        }
}

/* tiers[d] = leaf norms; tiers[t] built from tiers[t+1] by Eq. 3. */
static double **norm_tiers(const double *m, int nb, int depth) {
    double **tiers = (double **)calloc((size_t)depth + 1, sizeof(double *));
    if (!tiers) return NULL;
    for (int t = 0; t <= depth; ++t) {
        size_t w = (size_t)1 << t;
        tiers[t] = (double *)malloc(w * w * sizeof(double));
        if (!tiers[t]) return NULL;
    }
    leaf_norms(m, nb, tiers[depth]);
    for (int t = depth - 1; t >= 0; --t) {
        size_t w = (size_t)1 << t, wc = w * 2;
        const double *ch = tiers[t + 1];
        for (size_t i = 0; i < w; ++i)
            for (size_t j = 0; j < w; ++j) {
                double s = 0.0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        double v = ch[(2 * i + a) * wc + (2 * j + b)];
                        s += v * v;
                    }
                tiers[t][i * w + j] = sqrt(s);
            }
    }
    return tiers;
}

static void free_tiers(double **tiers, int depth) {
    if (!tiers) return;
    for (int t = 0; t <= depth; ++t) free(tiers[t]);
    free(tiers);
}

/* Dense leaf product C += A B, three nested loops (Sec. 3). */
static void leaf_product(const double *a, const double *b, double *c) {
    for (int r = 0; r < LEAF; ++r)
        for (int q = 0; q < LEAF; ++q) {
            double av = a[r * LEAF + q];
            for (int s = 0; s < LEAF; ++s) c[r * LEAF + s] += av * b[q * LEAF + s];
        }
}

static void spamm_omp(spamm_ctx *x, int t, int i, int j, int k) {
    if (t < x->depth) {
        size_t w = (size_t)1 << (t + 1);
        const double *na = x->na[t + 1], *nbm = x->nbm[t + 1];
        for (int ci = 2 * i; ci <= 2 * i + 1; ++ci)
            for (int cj = 2 * j; cj <= 2 * j + 1; ++cj)
                for (int ck = 2 * k; ck <= 2 * k + 1; ++ck) {
                    double p = na[ci * w + ck] * nbm[ck * w + cj];
                    if (p > x->tau) {
#pragma omp task untied firstprivate(ci, cj, ck)
                        spamm_omp(x, t + 1, ci, cj, ck);
                    } else {
#pragma omp atomic
                        x->culled += p;
                    }
                }
#pragma omp taskwait
    } else {
        size_t nb = (size_t)x->nb;
        omp_set_lock(&x->locks[i * nb + j]);
        leaf_product(x->a + ((size_t)i * nb + k) * LEAF2, x->b + ((size_t)k * nb + j) * LEAF2,
                     x->c + ((size_t)i * nb + j) * LEAF2);
        omp_unset_lock(&x->locks[i * nb + j]);
#pragma omp atomic
        x->n_exec += 1;
    }
}

/*
 * C = SpAMM(A, B, tau) on blocked FP64 arrays (layout above); C is
 * overwritten.  threads <= 0 uses the OpenMP default.  Returns 0 on success,
 * -1 on bad arguments, -2 on allocation failure.
 */
int oracle_spamm_alg1(int depth, const double *a, const double *b, double tau, double *c,
                      int threads, int64_t *n_exec, double *culled_bound) {
    if (depth < 0 || depth > 12 || !a || !b || !c || !(tau >= 0.0) || isinf(tau)) return -1;
    int nb = 1 << depth;
    size_t nblk = (size_t)nb * nb;
    memset(c, 0, nblk * LEAF2 * sizeof(double));
    spamm_ctx x;
    memset(&x, 0, sizeof(x));
    x.depth = depth;
    x.nb = nb;
    x.a = a;
    x.b = b;
    x.c = c;
    x.tau = tau;
    x.na = norm_tiers(a, nb, depth);
    x.nbm = norm_tiers(b, nb, depth);
    x.locks = (omp_lock_t *)malloc(nblk * sizeof(omp_lock_t));
    if (!x.na || !x.nbm || !x.locks) {
        free_tiers(x.na, depth);
        free_tiers(x.nbm, depth);
        free(x.locks);
        return -2;
    }
    for (size_t e = 0; e < nblk; ++e) omp_init_lock(&x.locks[e]);
    if (depth == 0) {
        double p = x.na[0][0] * x.nbm[0][0];
        if (p > tau) {
            leaf_product(a, b, c);
            x.n_exec = 1;
        } else {
            x.culled = p;
        }
    } else {
        if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel
#pragma omp single
        spamm_omp(&x, 0, 0, 0, 0);
    }
    for (size_t e = 0; e < nblk; ++e) omp_destroy_lock(&x.locks[e]);
    free(x.locks);
    free_tiers(x.na, depth);
    free_tiers(x.nbm, depth);
    if (n_exec) *n_exec = x.n_exec;
    if (culled_bound) *culled_bound = x.culled;
    return 0;
}

/* Threads the OpenMP runtime would use for a parallel region. */
int oracle_max_threads(void) { return omp_get_max_threads(); }
