/*
 * lap.h - C ABI of the MI355X (gfx950) Laplacian solver: preconditioned
 * conjugate gradients on a weighted graph Laplacian L_G, preconditioned by
 * the multilevel sparsifier preconditioner (MSP, Sec. 3.3) or the
 * positively-weighted expanded graph preconditioner (PEGP, Sec. 3.2) of
 * Hu & Lin, "Solving Graph Laplacians via Multilevel Sparsifiers"
 * (arXiv 2207.07847), or left unpreconditioned.  Both preconditioners are
 * applied through the lifting of Sec. 3.1: M = P(mu) S^+ P(mu)^T, S the
 * sparsifier of the expanded graph (the tree T~ for MSP, H~ for PEGP).
 *
 * Problem (Sec. 1, Sec. 2.1): G = (E, V, w) simply connected with positive
 * weights, L_G = B^T W B symmetric positive semidefinite with null space
 * span{1}.  lap_solve returns the mean-free x with L_G x = b - mean(b).
 *
 * Conventions
 *   - Every function returns a lap_status (0 = LAP_OK); nothing throws or
 *     aborts across this boundary.  lap_status_str names a code.
 *   - Host pointers are read only during the call and stay owned by the
 *     caller.  Device pointers are hipMalloc'ed (or torch) memory on the
 *     current device; the library reads/writes them on the given stream.
 *   - "stream" is a hipStream_t passed as void* (NULL = default stream).
 *   - A hierarchy owns its device memory until lap_free.  It holds one solve
 *     workspace: calls that use the same hierarchy must not overlap in time
 *     (issue them from one host thread; any stream is fine).
 */
#ifndef LAP_H
#define LAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LAP_OK = 0,
    LAP_EINVAL = 1,         /* invalid argument or graph */
    LAP_EDISCONNECTED = 2,  /* graph has more than one component */
    LAP_ENOMEM = 3,         /* host or device allocation failed */
    LAP_EDEVICE = 4,        /* HIP runtime error, or no device */
    LAP_ENOCONV = 5,        /* max_iter reached; x and info still written */
    LAP_EBREAKDOWN = 6,     /* p^T L p <= 0 or a non-finite value */
    LAP_EUNSUPPORTED = 7    /* valid, but a combination the library does not support */
} lap_status;

typedef enum {
    LAP_PREC_MSP = 0,       /* multilevel sparsifier preconditioner, Sec. 3.3 */
    LAP_PREC_PEGP = 1,      /* positively-weighted expanded graph, Sec. 3.2:
                               FP64 single right-hand-side solves only, and
                               expanded graphs of at most 19,456 nodes (the
                               sum of all level sizes) in at most 64 levels */
    LAP_PREC_NONE = 2,      /* plain conjugate gradients */
    LAP_PREC_OFFTREE = 3,   /* the MSP tree T~ with off-tree edges of H~ added
                               back (Sec. 3.3, the sparsifiers after its
                               stretch bound): the ceil(offtree_frac * count)
                               off-tree edges of largest stretch in T~ (w_e
                               times the effective resistance between the
                               ends through T~; ties to the smaller pair),
                               solved like PEGP on that subgraph of H~ (the
                               same limits).  offtree_frac 0 gives the MSP
                               operator, 1 the PEGP one */
    LAP_PREC_SPANNING = 4   /* the same with the other tree of Sec. 3.3's
                               remark: a maximum-weight spanning tree of H~
                               (Kruskal: heaviest edge first, ties to the
                               smaller pair), its off-tree edges ranked by
                               stretch (w_e times the resistance of the tree
                               path between the ends) and the largest
                               ceil(offtree_frac * count) added back, solved
                               like PEGP (the same limits).  offtree_frac 1
                               gives the PEGP operator */
} lap_precond;

typedef enum {
    LAP_FP64 = 0,           /* all arithmetic in double precision */
    LAP_MIXED_FP32_FP64 = 1 /* iterative refinement: FP64 residual b - L x,
                               x, inner products and mean projection; each
                               correction by PCG with FP32 SpMV and FP32
                               preconditioner (FP32 arithmetic, FP64 sums) */
} lap_precision;

/* Flags for lap_params.flags */
#define LAP_FLAG_HOST_ONLY 1u  /* lap_setup builds the host hierarchy only:
                                  export/info calls work, solves return
                                  LAP_EUNSUPPORTED; no device is touched. */
#define LAP_FLAG_MULTI_RHS 2u  /* lap_setup also builds the block solve: calls
                                  with nrhs > 1 advance up to 64 columns
                                  together (see lap_solve) */
#define LAP_FLAG_DEVICE_SETUP 8u /* lap_setup builds the graphs of the
                                  hierarchy on the device: the symmetric
                                  adjacency of the edge list and each coarse
                                  graph P^T L P (Sec. 2.2), by stable radix
                                  sorts of (row, column) keys with each run's
                                  weights summed in the host's order, so the
                                  hierarchy is bit-identical to the host
                                  build.  The matching and the rest of the
                                  setup stay on the host.  Ignored with
                                  LAP_FLAG_HOST_ONLY. */
#define LAP_FLAG_PARALLEL_MATCHING 16u /* aggregate every level by the
                                  locally dominant matching instead of the
                                  visit-order matching of Sec. 2.2: rounds in
                                  which every free vertex points at its
                                  heaviest free neighbour (ties: smaller id)
                                  and mutual pointers pair up, until no free
                                  vertex has a free neighbour.  The result is
                                  the greedy matching by edge weight (ties:
                                  smaller (i, j)), a different hierarchy from
                                  the default: pair ids follow the smaller
                                  end, leftovers join their heaviest
                                  neighbour as in Sec. 2.2.  On the device
                                  with LAP_FLAG_DEVICE_SETUP (a thread per
                                  vertex per round), else on the host;
                                  mwm_seed is not used. */
#define LAP_FLAG_FGMRES 4u     /* lap_solve runs FGMRES on the expanded system
                                  L_G~ x~ = P(mu)^T b^ (Sec. 2.2, the solver of
                                  Sec. 4) instead of PCG: right-preconditioned
                                  by the MSP or PEGP solve, no restart before
                                  LAPGPU_FGMRES_RESTART (default 1000) steps
                                  or an 8 GiB basis; tol applies to the
                                  expanded residual.  FP64, one right-hand
                                  side at a time; LAP_EUNSUPPORTED with
                                  LAP_PREC_NONE or mixed precision.
                                  info.iterations counts products with L_G~,
                                  info.relres_recursive is the expanded
                                  residual estimate.  LAP_OK means the
                                  expanded residual met tol (the stop test
                                  of Sec. 4); info.relres_true reports the
                                  residual of the original system as
                                  measured, which may lie above tol. */

/* Undirected weighted graph, host memory, edges (u[e], v[e], w[e]).
 * Requirements: n >= 2; 0 <= u, v < n; u != v; w finite and > 0.
 * Parallel edges are merged by summing their weights. */
typedef struct {
    int64_t n;
    int64_t m;
    const int64_t *u;
    const int64_t *v;
    const double *w;
} lap_graph;

typedef struct {
    double mu;            /* level weight 0 < mu < 1 of P(mu) (Sec. 2.2) */
    int32_t max_levels;   /* 0 = level max (Sec. 3.2); else at most this many */
    int32_t n_top;        /* coarsen while a level has more nodes (default 2) */
    uint64_t mwm_seed;    /* 0 = natural visit order; else seeded random order */
    int32_t precond;      /* lap_precond */
    int32_t precision;    /* lap_precision */
    int32_t max_iter;     /* iteration cap of lap_solve (default 1000) */
    uint32_t flags;       /* LAP_FLAG_* */
    double offtree_frac;  /* LAP_PREC_OFFTREE, LAP_PREC_SPANNING: fraction in [0, 1] of the
                             off-tree edges added back (default 0.1) */
} lap_params;

typedef struct {
    int32_t iterations;        /* products with L_G performed */
    int32_t refinements;       /* mixed precision: refinement steps; FP64
                                  PCG: residual replacements taken (0..3) */
    double relres_true;        /* ||b^ - L_G x|| / ||b^|| in FP64, b^ = b - mean(b) */
    double relres_recursive;   /* ||r_k|| / ||b^|| of the PCG recurrence */
    double seconds;            /* host wall time of the call */
    int32_t status;            /* lap_status of this right-hand side */
    int32_t pad;
} lap_solve_info;

#define LAP_MAX_LEVELS 64
typedef struct {
    int32_t nlev;                 /* levels, fine (0) to top (nlev-1) */
    int32_t tail_level;           /* first level handled by the one-block tail */
    int64_t sizes[LAP_MAX_LEVELS];/* nodes per level */
    int64_t ntilde;               /* sum of sizes: nodes of the expanded graph */
    int64_t nnz;                  /* stored adjacency entries of L_G (2m) */
    int64_t device_bytes;         /* device memory held by the hierarchy */
    double setup_seconds;         /* host time spent in lap_setup */
    /* Block solve (LAP_FLAG_MULTI_RHS), index 0 FP64, 1 the FP32 inner
     * solve of mixed precision; 0 where absent.  Sizes picked at set-up by
     * timing candidates on the device (the autotuner):
     *   mm_chunk: matrix entries per SpMM work item (longer rows are split);
     *   mm_grid:  workgroups of the SpMM launch;
     *   mm_seg:   children per work item of restriction and prolongation. */
    int32_t mm_chunk[2];
    int32_t mm_grid[2];
    int32_t mm_seg[2];
    double mm_tune_seconds;       /* host time of the autotuner in lap_setup */
    /* 1 if the SpMV of an iteration forms p itself (one kernel, k_spmv_p),
     * 0 if a separate p pass runs first (k_pupd, then k_spmv_q) */
    int32_t spmv_fused;
    /* the fine-node count of the explicit PEGP operator (0: none; PEGP
     * then runs through its factor) */
    int32_t pegp_operator_n;
} lap_hierarchy_desc;

typedef struct lap_hierarchy lap_hierarchy;

/* Defaults: mu 0.8, level max, n_top 2, natural order, MSP, FP64,
 * max_iter 1000, no flags.  Errors: LAP_EINVAL if p is NULL. */
lap_status lap_default_params(lap_params *p);

/* Device allocator for the hierarchies set up after this call (for
 * example a framework's caching allocator, so that a hierarchy lives in the
 * caller's memory pool).  alloc(bytes, ctx) returns device memory of the
 * current device (at least 256-byte aligned) or NULL; free(ptr, ctx)
 * releases a pointer alloc returned.  Both NULL restores hipMalloc /
 * hipFree.  The library calls alloc from lap_setup (and from the first
 * FGMRES solve of a hierarchy, for its basis) and free from lap_free, on the
 * calling thread; a hierarchy keeps the pair it was set up with.  The
 * request server's staging buffers and the set-up graphs built on the
 * device (LAP_FLAG_DEVICE_SETUP) still use hipMallocAsync / hipMalloc.
 * Process-wide; thread-safe.  Errors: LAP_EINVAL when exactly one of
 * alloc, free is NULL.  An alloc that returns NULL makes lap_setup return
 * LAP_ENOMEM. */
typedef void *(*lap_alloc_fn)(size_t bytes, void *ctx);
typedef void (*lap_free_fn)(void *ptr, void *ctx);
lap_status lap_set_allocator(lap_alloc_fn alloc, lap_free_fn free, void *ctx);

/* Host setup (Sec. 2.2, Sec. 3.3) then upload on `stream`.
 *   1. validate and build the symmetric adjacency (parallel edges summed in
 *      input order); reject a disconnected graph (LAP_EDISCONNECTED);
 *   2. aggregate each level by maximal weighted matching (visit order per
 *      mwm_seed; an unaggregated vertex pairs with its heaviest unaggregated
 *      neighbour, ties to the smaller id; leftovers join their heaviest
 *      neighbour's aggregate) and form the coarse graph P^T L P;
 *   3. derive the MSP coefficients: per aggregate the local solve of its
 *      sparsifier block, per level the weight theta_j, the top-level
 *      pseudo-inverse; renumber the levels so aggregates are contiguous;
 *   4. copy everything to the device.
 * On success *out owns the hierarchy.  Errors: LAP_EINVAL (bad graph or
 * params: mu outside (0,1), n_top < 2, unknown precond/precision),
 * LAP_EDISCONNECTED, LAP_ENOMEM, LAP_EDEVICE, LAP_EUNSUPPORTED (top level
 * larger than the on-chip coarse solve allows; PEGP or the off-tree
 * sparsifier with mixed precision, with LAP_FLAG_MULTI_RHS, or with an
 * expanded graph above 19,456 nodes or 64 levels).  LAP_EINVAL also for
 * LAP_PREC_OFFTREE or LAP_PREC_SPANNING with offtree_frac outside [0, 1].
 * PEGP (Sec. 3.2) factors the grounded, level-scaled L_H~ once on the host
 * (sparse LDL^T) and applies it on the device. */
lap_status lap_setup(const lap_graph *g, const lap_params *p, void *stream,
                     lap_hierarchy **out);

/* Preconditioned CG on L_G x = b (Sec. 4 solves the equivalent expanded
 * system; the Theorem of Sec. 3.1 maps it back).  b, x: device arrays of
 * nrhs columns with leading dimension ld >= n (column c at b + c*ld),
 * original vertex order.  x is overwritten with the mean-free solution.
 * info: host array of nrhs entries (may be NULL).
 *
 * FP64 PCG stops when the recursive residual meets ||r_k|| <= tol ||b^||;
 * then the true residual t = b^ - L x of the mean-free x is formed in FP64
 * (Sec. 4 stops on the residual of the original system).  If ||t|| is
 * still above tol ||b^||, PCG restarts from x with r = t - mean(t) (a
 * residual replacement; at most 3, all within max_iter products with L).
 * LAP_OK therefore means info->relres_true <= tol.  info->iterations counts
 * products with L over all restarts, info->refinements the replacements.
 *
 * Returns the worst per-column status: LAP_ENOCONV when max_iter is
 * reached or the true residual misses tol after the last replacement (x
 * and info are still written), LAP_EBREAKDOWN, LAP_EINVAL (tol <= 0,
 * nrhs < 1, ld < n, non-finite b), LAP_EDEVICE.
 *
 * Mixed precision (LAP_MIXED_FP32_FP64): x and r = b^ - L x are kept in
 * FP64; one PCG run with FP32 vectors, FP32 SpMV and FP32 preconditioner
 * (inner products and the mean projection summed in FP64) produces the
 * corrections.  Each time its residual has fallen 10x, a refinement step
 * (reliable update) adds its correction to x, replaces its residual by the
 * FP64 b^ - L x, and continues along the same search direction.  The stop
 * test is on that FP64 residual; info->iterations counts FP32 iterations,
 * info->refinements the refinement steps, info->relres_true the final FP64
 * ||b^ - L x|| / ||b^||. */
lap_status lap_solve(lap_hierarchy *h, const double *b, double *x,
                     int32_t nrhs, int64_t ld, double tol,
                     lap_solve_info *info, void *stream);

/* Precision of later lap_solve calls on h.  A hierarchy set up with
 * LAP_MIXED_FP32_FP64 holds both the FP32 and the FP64 solve and may switch
 * either way; one set up with LAP_FP64 only supports LAP_FP64.  Errors:
 * LAP_EINVAL (NULL, unknown precision), LAP_EUNSUPPORTED (FP32 solve not
 * built, or host-only). */
lap_status lap_set_precision(lap_hierarchy *h, int32_t precision);

/* y = L_G x on the device (original order).  Errors: LAP_EINVAL,
 * LAP_EDEVICE, LAP_EUNSUPPORTED for a host-only hierarchy. */
lap_status lap_apply_laplacian(lap_hierarchy *h, const double *x, double *y,
                               void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as lap_apply_laplacian, y = L_G x on the device in original
 * order, with its work vectors taken from a static device array of the
 * library instead of the hierarchy.  Allocates nothing and calls no
 * allocating routine.  The array holds 64 MiB per device (kept until the
 * process ends): a hierarchy whose solve order differs from the input order
 * (graphs with rows above 64 neighbours or heavy slice padding) needs
 * 16 n bytes of it, so n <= 4,194,304 there; other hierarchies use none.
 * All calls on one device share the array: calls that overlap in time on
 * one device race (issue them in order on one stream, or from one host
 * thread).  The current device must be the hierarchy's.  Errors:
 * LAP_EINVAL (NULL, or the current device is not the hierarchy's),
 * LAP_EUNSUPPORTED (host-only hierarchy, or more scratch than the array
 * holds: lap_last_error states the sizes), LAP_EDEVICE. */
lap_status lap_apply_laplacian_noalloc(lap_hierarchy *h, const double *x, double *y,
                                       void *stream);

/* z = M r - mean, the hierarchy's preconditioner applied through the
 * lifting of Sec. 3.1: M = P(mu) L_T~^+ P(mu)^T for MSP (Sec. 3.3, in the
 * closed form of its tree elimination), M = P(mu) L_H~^+ P(mu)^T for PEGP
 * (Sec. 3.2, by the grounded factor).  r must be mean-free (a residual).
 * Device arrays of n values, original order; r is read, z written.  Uses
 * the hierarchy's solve workspace.  A mixed-precision hierarchy applies
 * its FP32 form.  Errors: LAP_EINVAL (NULL), LAP_EUNSUPPORTED (host-only),
 * LAP_EDEVICE. */
lap_status lap_apply_precond(lap_hierarchy *h, const double *r, double *z,
                             void *stream);

/* Kernel timing for roofline reports.  Runs one untimed and then `reps`
 * timed PCG iterations on `stream`, on the hierarchy's own workspace (its
 * contents are overwritten; the next lap_solve reinitialises it), with a
 * pair of HIP events around the chosen part of every timed iteration, so
 * the part is timed in the cache state of a real solve.  Returns the
 * average milliseconds of the part and the algorithmic HBM bytes it must
 * move (FP64 values, int32 indices, each datum counted once):
 *   LAP_KERNEL_SPMV     p update + q = L p + p^T q, with the previous
 *                       iteration's x step riding along (48 n + 12 nnz
 *                       bytes: z, p_old, x read, p, q, x written, and col,
 *                       w of the matrix; 56 n + 12 nnz where p is formed
 *                       in a pass of its own, for graphs without locality)
 *   LAP_KERNEL_UPDATE   x, r update + level-0 restriction and pair solves
 *   LAP_KERNEL_DOWN0    level-0 prolongation + z, r^T z reductions
 *   LAP_KERNEL_PRECOND  update through down0: the x, r update and the
 *                       whole preconditioner (all levels)
 *   LAP_KERNEL_ITER     one whole PCG iteration
 *   LAP_KERNEL_BLOCK_SPMM  block solve (LAP_FLAG_MULTI_RHS): Q = L P over 64
 *                       columns (2 n 64 v + (4 + v) nnz bytes, v = value size)
 *   LAP_KERNEL_BLOCK_ITER  one whole iteration of the block solve
 *   LAP_KERNEL_PEGP_OP  PEGP hierarchy applied by its explicit operator: the
 *                       matrix-vector product z = M r (8 opn^2 + 20 n bytes:
 *                       the operator's entries as stored, r and its index
 *                       read, z written)
 * Errors: LAP_EINVAL (bad id, reps < 1), LAP_EUNSUPPORTED (host-only or a
 * part the hierarchy does not have), LAP_EBREAKDOWN (the iterations hit a
 * breakdown, so the timing is not representative), LAP_EDEVICE. */
enum { LAP_KERNEL_SPMV = 0, LAP_KERNEL_UPDATE = 1, LAP_KERNEL_DOWN0 = 2,
       LAP_KERNEL_PRECOND = 3, LAP_KERNEL_ITER = 4,
       LAP_KERNEL_BLOCK_SPMM = 5, LAP_KERNEL_BLOCK_ITER = 6, LAP_KERNEL_PEGP_OP = 7 };
lap_status lap_profile_kernel(lap_hierarchy *h, int32_t kernel, int32_t reps,
                              void *stream, double *avg_ms, double *alg_bytes);

/* Extreme eigenvalues of the preconditioned operator M L_G on range(L_G),
 * whose ratio kappa governs PCG's convergence (the theorem of Sec. 3.2
 * bounds it by 1/(1 - rho) when mu is small enough; how to choose mu is
 * left open after it).  Estimated from PCG's own coefficients: up to `steps`
 * FP64 PCG iterations on b with the hierarchy's preconditioner (MSP or
 * PEGP), stopping early at ||r|| <= 1e-10 ||b^||; the step lengths alpha_j
 * and direction updates beta_j give the Lanczos tridiagonal
 *   T_jj = 1/alpha_j + beta_j/alpha_{j-1},  T_j,j+1 = sqrt(beta_{j+1})/alpha_j
 * (Saad, Iterative Methods for Sparse Linear Systems, Sec. 6.7.3), whose
 * extreme eigenvalues (bisection on Sturm counts) approach the operator's
 * from inside.  b: device array of n values, original order (any b with a
 * component on every eigenvector; a random one).  *lmin, *lmax, *taken
 * (steps taken; may be NULL): host outputs.  Uses the solve workspace.
 * Errors: LAP_EINVAL (NULL, steps < 1, non-finite b), LAP_EUNSUPPORTED
 * (host-only, or no preconditioner), LAP_EBREAKDOWN (no step taken),
 * LAP_EDEVICE. */
lap_status lap_estimate_spectrum(lap_hierarchy *h, const double *b, int32_t steps,
                                 double *lmin, double *lmax, int32_t *taken,
                                 void *stream);

/* The mu among mus[0..nmu) with the smallest estimated kappa: for each
 * candidate, a hierarchy set up from g and p with p->mu replaced, the
 * estimate of lap_estimate_spectrum with `steps` steps on b, and the
 * hierarchy freed.  PCG's step count grows as sqrt(kappa), and an MSP
 * application costs the same at every mu.  kappa: host array of nmu
 * entries (may be NULL; HUGE_VAL for a candidate whose setup or estimate
 * failed); *best: the chosen index.  Errors: LAP_EINVAL (NULL, nmu < 1,
 * steps < 1), else the first failing candidate's status when none
 * succeeded. */
lap_status lap_select_mu(const lap_graph *g, const lap_params *p, const double *mus,
                         int32_t nmu, const double *b, int32_t steps, double *kappa,
                         int32_t *best, void *stream);

/* Sizes and memory of a hierarchy.  Errors: LAP_EINVAL on NULL. */
lap_status lap_hierarchy_info(const lap_hierarchy *h, lap_hierarchy_desc *d);

/* The off-tree edges of a LAP_PREC_OFFTREE or LAP_PREC_SPANNING hierarchy
 * (outside T~, or outside the spanning tree): *count receives
 * their number; each array (host, count entries; any may be NULL) receives
 * per edge its ends a < b as expanded indices (level offset, the sum of the
 * sizes of the finer levels, plus the node's id in its level's own
 * numbering, as lap_export_level uses), its weight in H~, its stretch in
 * its tree, and kept = 1 if it was added back.  Errors: LAP_EINVAL (NULL,
 * or not an off-tree hierarchy). */
lap_status lap_export_offtree(const lap_hierarchy *h, int64_t *count, int64_t *a, int64_t *b,
                              double *w, double *stretch, int8_t *kept);

/* Integer outputs of level `level` (0 = fine) for 0 <= level < nlev-1, in
 * the level's own numbering (aggregate ids in pair-creation order):
 * agg[i] = aggregate of node i on level+1, matched[i] = 1 if i was paired
 * by the matching, 0 if it joined as a leftover.  Host arrays of
 * sizes[level] entries; either may be NULL.  Errors: LAP_EINVAL. */
lap_status lap_export_level(const lap_hierarchy *h, int32_t level,
                            int64_t *agg, int8_t *matched);

/* Graph of level `level` (0 <= level < nlev) as symmetric CSR in that
 * level's numbering, neighbours ascending: ptr (sizes[level]+1), col and w
 * (ptr[last] entries).  Pass col = w = NULL to query ptr only.  Host
 * arrays.  Errors: LAP_EINVAL. */
lap_status lap_export_graph(const lap_hierarchy *h, int32_t level,
                            int64_t *ptr, int64_t *col, double *w);

/* ------------------------------------------------------------ serving
 *
 * A request server over resident hierarchies (continuous batching).  Every
 * registered hierarchy (set up with LAP_FLAG_MULTI_RHS) keeps its FP64
 * block solve resident with its own stream: 64 column slots, each running
 * its own PCG (per-column scalars and stop test).  A background thread
 * advances the graphs with work in chunks of iterations and, at every chunk
 * boundary of a graph, hands out the columns that have stopped and admits
 * queued requests into the free slots while the other columns keep
 * iterating; graphs run concurrently on their streams.  A request (1..64
 * right-hand sides of one graph) is admitted when it fits the free slots
 * and its staging memory fits the HBM budget (resident hierarchies count
 * against the budget too).  Each column's result is the same PCG run as a
 * block solve of that column alone: columns never mix.
 */
typedef struct lap_server lap_server;

typedef struct {
    int64_t tag;               /* the caller's tag */
    int32_t graph;             /* graph id of the request */
    int32_t nrhs;
    int32_t status;            /* worst lap_status of the columns */
    int32_t iterations_max;    /* PCG iterations of the slowest column */
    double relres_max;         /* max over columns of ||r|| / ||b^|| (FP64 recursive) */
    double queue_seconds;      /* submit -> admission */
    double total_seconds;      /* submit -> result in the caller's buffer */
} lap_request_result;

/* New server with an HBM budget in bytes (0: no limit).  Errors:
 * LAP_EINVAL, LAP_ENOMEM, LAP_EDEVICE. */
lap_status lap_server_create(int64_t hbm_budget_bytes, lap_server **out);

/* Register h (set up with LAP_FLAG_MULTI_RHS, not host-only) under a new
 * graph id.  The server uses h exclusively until lap_server_destroy; h is
 * freed by the caller afterwards.  Errors: LAP_EINVAL, LAP_EUNSUPPORTED
 * (no block solve), LAP_ENOMEM (budget exceeded), LAP_EDEVICE. */
lap_status lap_server_add(lap_server *srv, lap_hierarchy *h, int32_t *graph_id);

/* Queue a request: nrhs (1..64) right-hand sides of graph `graph`, host
 * array b (column c at b + c*n, original vertex order), solution written
 * to the host array x (same layout, mean-free) before the result is
 * returned by lap_server_poll; both must stay valid until then.  Stop at
 * ||r|| <= tol ||b^|| per column.  Errors: LAP_EINVAL. */
lap_status lap_server_submit(lap_server *srv, int32_t graph, const double *b,
                             double *x, int32_t nrhs, double tol, int64_t tag);

/* Completed requests, at most max, waiting up to wait_ms for the first
 * one (0: no wait); *count receives how many were written to out. */
lap_status lap_server_poll(lap_server *srv, lap_request_result *out,
                           int32_t max, int32_t wait_ms, int32_t *count);

/* Stop the server: requests not yet admitted are dropped, running ones are
 * abandoned once the chunk in flight ends (their results are not
 * delivered), then the server thread ends and the server's staging memory
 * is released (not the hierarchies).  Poll every result first to keep it.
 * NULL is a no-op. */
void lap_server_destroy(lap_server *srv);

/* Release the hierarchy and its device memory (NULL is a no-op). */
void lap_free(lap_hierarchy *h);

/* Static string naming a status. */
const char *lap_status_str(lap_status s);

/* Description of the last HIP runtime failure seen by this thread (the
 * failing call and HIP's error string), "" if none.  Valid until the next
 * library call on the thread. */
const char *lap_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
