/*
 * lapref.h - FP64 reference ("oracle") for the solve phase of Hu & Lin,
 * "Solving Graph Laplacians via Multilevel Sparsifiers" (arXiv 2207.07847).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against a plain, slow, obviously correct CPU computation.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Everything is double precision, single-threaded, with sequential sums in
 * the order stated beside each function.
 *
 * Indices are int64_t, values double.  Objects returned through pointers are
 * owned by the caller and released with the matching lr_*_free function.
 */
#ifndef LAPREF_H
#define LAPREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { LR_OK = 0, LR_EINVAL = 1, LR_EDISCONNECTED = 2, LR_ENOMEM = 3,
       LR_ENOCONV = 5, LR_EBREAKDOWN = 6 };

/* Symmetric weighted adjacency in CSR form (no diagonal stored). */
typedef struct {
    int64_t n, nnz;
    int64_t *ptr;   /* n+1 */
    int64_t *col;   /* nnz, ascending within a row */
    double *w;      /* nnz */
} lr_csr;

typedef struct lr_hier lr_hier;      /* aggregation hierarchy */
typedef struct lr_msp lr_msp;        /* factored MSP sparsifier */

/* Graph of Sec. 2.1: build the symmetric CSR of an undirected edge list.
 * Rejects ids out of range, self-loops, non-finite or non-positive weights
 * (LR_EINVAL).  Parallel edges are summed in ascending input order. */
int lr_csr_build(int64_t n, int64_t m, const int64_t *u, const int64_t *v,
                 const double *w, lr_csr **out);
void lr_csr_free(lr_csr *g);
int lr_connected(const lr_csr *g);   /* 1 if one component (BFS) */

/* (L_G x)_i = sum_j w_ij (x_i - x_j), from L_G = B^T W B (Sec. 2.1). */
void lr_lap_apply(const lr_csr *g, const double *x, double *y);

/* Maximal weighted matching aggregation of Sec. 2.2.  order = visit order
 * (NULL = natural).  agg[i] = aggregate of i; matched[i] = 1 if i was paired
 * in the matching pass, 0 if it joined its heaviest neighbour's aggregate
 * afterwards (may be NULL).  Returns the number of aggregates. */
int64_t lr_mwm(const lr_csr *g, const int64_t *order, int64_t *agg,
               int8_t *matched);

/* Coarse graph: Laplacian of P^T L P for the piecewise-constant P built
 * from agg (Sec. 2.2 / Sec. 3.1).  Coarse weight of {A,B} = sum of fine
 * w_ij over i<j with {agg i, agg j} = {A,B}, summed in ascending (i,j). */
int lr_coarsen(const lr_csr *f, const int64_t *agg, int64_t nc, lr_csr **out);

/* Hierarchy to level max (max_levels = 0) or to max_levels levels; stops
 * when the top has <= n_top nodes and never creates a level of < 2 nodes.
 * seed = 0: natural visit order; otherwise a SplitMix64-driven Fisher-Yates
 * permutation seeded with seed + (1-based index of the level aggregated). */
int lr_hier_build(const lr_csr *g, int32_t max_levels, int64_t n_top,
                  uint64_t seed, lr_hier **out);
/* The same with the aggregation chosen: matching 0 = the visit-order
 * matching above (lr_mwm), 1 = the greedy matching by edge weight
 * (lr_greedy_match; seed unused). */
int lr_hier_build_ex(const lr_csr *g, int32_t max_levels, int64_t n_top,
                     uint64_t seed, int32_t matching, lr_hier **out);
/* Greedy matching aggregation: edges in decreasing weight (ties: smaller
 * (i, j) first) join while both ends are free; pair ids by the smaller end;
 * leftovers join their heaviest neighbour's aggregate. */
int64_t lr_greedy_match(const lr_csr *g, int64_t *agg, int8_t *matched);
void lr_hier_free(lr_hier *h);
int32_t lr_hier_nlev(const lr_hier *h);
int64_t lr_hier_nk(const lr_hier *h, int32_t k);             /* k = 0-based */
void lr_hier_agg(const lr_hier *h, int32_t k, int64_t *agg, int8_t *matched);
int64_t lr_hier_level_nnz(const lr_hier *h, int32_t k);
void lr_hier_level_csr(const lr_hier *h, int32_t k, int64_t *ptr,
                       int64_t *col, double *w);
int64_t lr_hier_ntilde(const lr_hier *h);

/* P(mu)^T r  (length n -> n~) and P(mu) y (length n~ -> n), Sec. 2.2. */
void lr_restrict_mu(const lr_hier *h, double mu, const double *r, double *rt);
void lr_prolong_mu(const lr_hier *h, double mu, const double *yt, double *z);

/* MSP sparsifier T~ of Sec. 3.3 as an edge list over the n~ expanded nodes
 * (levels stacked fine to coarse).  Arrays are malloc'ed; free with
 * lr_free. */
int lr_msp_edges(const lr_hier *h, double mu, int64_t *ne, int64_t **eu,
                 int64_t **ev, double **ew);
void lr_free(void *p);

/* Factor L_T~ by Gaussian elimination, aggregates of the finest level first
 * (leftover members before matched ones), level by level, top level last
 * with its last node grounded (Sec. 3.3). */
int lr_msp_factor(const lr_hier *h, double mu, lr_msp **out);
void lr_msp_free(lr_msp *f);
int64_t lr_msp_fill(const lr_msp *f);   /* entries created by elimination */
/* z = P(mu) L_T~^+ P(mu)^T r with the mean of z removed. */
void lr_msp_apply(void *f, const double *r, double *z);
/* grounded solve of L_T~ y~ = b~ in the expanded space (ntilde values) */
void lr_msp_solve_expanded(const lr_msp *f, const double *bt, double *y);

/* Preconditioned CG on L_G x = b (see lr_pcg for the exact steps). */
typedef void (*lr_precond_fn)(void *ctx, const double *r, double *z);
typedef struct {
    int32_t iterations;        /* number of products with L_G (all restarts) */
    int32_t status;            /* LR_OK, LR_ENOCONV, LR_EBREAKDOWN */
    double relres_recursive;   /* ||r_k|| / ||b - mean(b)|| */
    double relres_true;        /* ||b^ - L x|| / ||b^|| after projection */
    int32_t restarts;          /* residual replacements after a converged
                                  recurrence whose true residual was above tol */
    int32_t pad;
} lr_pcg_info;
/* Residual replacements lr_pcg and lr_pcg_noisy allow (Sec. 4 stop rule). */
#define LR_MAX_RESTARTS 3
int lr_pcg(const lr_csr *g, lr_precond_fn M, void *ctx, const double *b,
           double tol, int32_t maxit, double *x, lr_pcg_info *info,
           double *relres_hist);
/* Same, with L p and M r perturbed entrywise by relative noise in
 * [-noise, noise) (SplitMix64 stream from seed): a rounding model used to
 * measure how far iteration counts move under reordered FP64 arithmetic. */
int lr_pcg_noisy(const lr_csr *g, lr_precond_fn M, void *ctx, const double *b,
                 double tol, int32_t maxit, double *x, lr_pcg_info *info,
                 double *relres_hist, double noise, uint64_t seed);
/* Same, with the number of residual replacements given (0: none; the
 * status is then LR_ENOCONV whenever the true residual misses tol). */
int lr_pcg_ex(const lr_csr *g, lr_precond_fn M, void *ctx, const double *b,
              double tol, int32_t maxit, double *x, lr_pcg_info *info,
              double *relres_hist, double noise, uint64_t seed, int32_t max_restarts);

#ifdef __cplusplus
}
#endif
#endif
