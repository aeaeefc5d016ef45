/*
 * lapref.c - FP64 reference ("oracle") for the solve phase of Hu & Lin,
 * "Solving Graph Laplacians via Multilevel Sparsifiers" (arXiv 2207.07847).
 *
 * TEST INFRASTRUCTURE ONLY: plain, sequential, double precision.  It shares
 * no code with the GPU library.  Readings of points the paper leaves open
 * are stated beside the code they govern.
 */
#include "lapref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ graph */

typedef struct {
    int64_t r, c, idx;
    double w;
} entry_t;

static int cmp_entry(const void *a, const void *b)
{
    const entry_t *x = (const entry_t *)a, *y = (const entry_t *)b;
    if (x->r != y->r) return x->r < y->r ? -1 : 1;
    if (x->c != y->c) return x->c < y->c ? -1 : 1;
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

void lr_csr_free(lr_csr *g)
{
    if (!g) return;
    free(g->ptr);
    free(g->col);
    free(g->w);
    free(g);
}

void lr_free(void *p) { free(p); }

/* Section 2.1: G = (E, V, w) with positive weights; L_G = B^T W B.  Each
 * undirected edge contributes to rows u and v; parallel edges are merged by
 * summing their weights in ascending input position, the same order in both
 * rows, so the result is exactly symmetric. */
int lr_csr_build(int64_t n, int64_t m, const int64_t *u, const int64_t *v,
                 const double *w, lr_csr **out)
{
    *out = NULL;
    if (n < 1 || m < 0) return LR_EINVAL;
    for (int64_t e = 0; e < m; ++e) {
        if (u[e] < 0 || u[e] >= n || v[e] < 0 || v[e] >= n) return LR_EINVAL;
        if (u[e] == v[e]) return LR_EINVAL;
        if (!(w[e] > 0.0) || !isfinite(w[e])) return LR_EINVAL;
    }
    entry_t *E = (entry_t *)malloc(sizeof(entry_t) * (size_t)(2 * m + 1));
    if (!E) return LR_ENOMEM;
    for (int64_t e = 0; e < m; ++e) {
        E[2 * e] = (entry_t){u[e], v[e], e, w[e]};
        E[2 * e + 1] = (entry_t){v[e], u[e], e, w[e]};
    }
    qsort(E, (size_t)(2 * m), sizeof(entry_t), cmp_entry);
    int64_t nnz = 0;
    for (int64_t k = 0; k < 2 * m; ++k)
        if (k == 0 || E[k].r != E[k - 1].r || E[k].c != E[k - 1].c) ++nnz;
    lr_csr *g = (lr_csr *)calloc(1, sizeof(lr_csr));
    g->n = n;
    g->nnz = nnz;
    g->ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    g->col = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz + 1));
    g->w = (double *)malloc(sizeof(double) * (size_t)(nnz + 1));
    int64_t t = -1;
    for (int64_t k = 0; k < 2 * m; ++k) {
        if (k == 0 || E[k].r != E[k - 1].r || E[k].c != E[k - 1].c) {
            ++t;
            g->col[t] = E[k].c;
            g->w[t] = E[k].w;
            g->ptr[E[k].r + 1] += 1;
        } else {
            g->w[t] += E[k].w;
        }
    }
    for (int64_t i = 0; i < n; ++i) g->ptr[i + 1] += g->ptr[i];
    free(E);
    *out = g;
    return LR_OK;
}

int lr_connected(const lr_csr *g)
{
    int64_t n = g->n;
    if (n == 0) return 0;
    char *seen = (char *)calloc((size_t)n, 1);
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t head = 0, tail = 0;
    seen[0] = 1;
    queue[tail++] = 0;
    while (head < tail) {
        int64_t i = queue[head++];
        for (int64_t k = g->ptr[i]; k < g->ptr[i + 1]; ++k)
            if (!seen[g->col[k]]) {
                seen[g->col[k]] = 1;
                queue[tail++] = g->col[k];
            }
    }
    free(seen);
    free(queue);
    return tail == n;
}

/* (L_G x)_i = sum over edges (i,j) of w_ij (x_i - x_j): the row of
 * B^T W B x, so constant vectors map to exactly zero. */
void lr_lap_apply(const lr_csr *g, const double *x, double *y)
{
    for (int64_t i = 0; i < g->n; ++i) {
        double s = 0.0;
        for (int64_t k = g->ptr[i]; k < g->ptr[i + 1]; ++k)
            s += g->w[k] * (x[i] - x[g->col[k]]);
        y[i] = s;
    }
}

/* ------------------------------------------------------------ aggregation */

/* Section 2.2: visit vertices in the given order; an unaggregated vertex is
 * matched with its unaggregated neighbour of largest edge weight (ties to the
 * smaller id).  Vertices left over (all neighbours already matched) join the
 * aggregate of their heaviest neighbour (ties to the smaller id).  Aggregate
 * ids are numbered in the order the pairs are formed. */
int64_t lr_mwm(const lr_csr *g, const int64_t *order, int64_t *agg,
               int8_t *matched)
{
    int64_t n = g->n, nc = 0;
    for (int64_t i = 0; i < n; ++i) agg[i] = -1;
    for (int64_t t = 0; t < n; ++t) {
        int64_t v = order ? order[t] : t;
        if (agg[v] >= 0) continue;
        int64_t best = -1;
        double bw = 0.0;
        for (int64_t k = g->ptr[v]; k < g->ptr[v + 1]; ++k) {
            int64_t u = g->col[k];
            if (agg[u] >= 0) continue;
            if (best < 0 || g->w[k] > bw || (g->w[k] == bw && u < best)) {
                best = u;
                bw = g->w[k];
            }
        }
        if (best >= 0) {
            agg[v] = nc;
            agg[best] = nc;
            ++nc;
        }
    }
    if (matched)
        for (int64_t i = 0; i < n; ++i) matched[i] = (int8_t)(agg[i] >= 0);
    for (int64_t v = 0; v < n; ++v) {
        if (agg[v] >= 0) continue;
        int64_t best = -1;
        double bw = 0.0;
        for (int64_t k = g->ptr[v]; k < g->ptr[v + 1]; ++k) {
            int64_t u = g->col[k];
            if (best < 0 || g->w[k] > bw || (g->w[k] == bw && u < best)) {
                best = u;
                bw = g->w[k];
            }
        }
        /* A leftover's neighbours were all matched in the first pass. */
        agg[v] = agg[best];
    }
    return nc;
}

/* The greedy matching by edge weight, the aggregation of a parallel
 * setup (an alternative to the visit-order matching of Sec. 2.2; not the
 * paper's): edges {i, j}, i < j, are taken in decreasing weight, ties to
 * the smaller (i, j) in lexicographic order, and an edge joins the matching
 * when both its ends are still free.  A pair's aggregate id is its rank
 * among the pairs ordered by their smaller end.  Vertices left free (all
 * neighbours matched: the matching is maximal) join the aggregate of their
 * heaviest neighbour, ties to the smaller id, as in Sec. 2.2. */
typedef struct {
    double w;
    int64_t i, j;
} gedge_t;

static int cmp_gedge(const void *p, const void *q)
{
    const gedge_t *x = (const gedge_t *)p, *y = (const gedge_t *)q;
    if (x->w != y->w) return x->w > y->w ? -1 : 1;
    if (x->i != y->i) return x->i < y->i ? -1 : 1;
    if (x->j != y->j) return x->j < y->j ? -1 : 1;
    return 0;
}

int64_t lr_greedy_match(const lr_csr *g, int64_t *agg, int8_t *matched)
{
    int64_t n = g->n, m = 0, nc = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = g->ptr[i]; k < g->ptr[i + 1]; ++k)
            if (g->col[k] > i) ++m;
    gedge_t *E = (gedge_t *)malloc(sizeof(gedge_t) * (size_t)(m + 1));
    int64_t t = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = g->ptr[i]; k < g->ptr[i + 1]; ++k)
            if (g->col[k] > i) {
                E[t].w = g->w[k];
                E[t].i = i;
                E[t].j = g->col[k];
                ++t;
            }
    qsort(E, (size_t)m, sizeof(gedge_t), cmp_gedge);
    int64_t *mate = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) mate[i] = -1;
    for (int64_t e = 0; e < m; ++e)
        if (mate[E[e].i] < 0 && mate[E[e].j] < 0) {
            mate[E[e].i] = E[e].j;
            mate[E[e].j] = E[e].i;
        }
    free(E);
    for (int64_t i = 0; i < n; ++i) agg[i] = -1;
    for (int64_t i = 0; i < n; ++i)
        if (mate[i] > i) {
            agg[i] = nc;
            agg[mate[i]] = nc;
            ++nc;
        }
    if (matched)
        for (int64_t i = 0; i < n; ++i) matched[i] = (int8_t)(mate[i] >= 0);
    for (int64_t v = 0; v < n; ++v) {
        if (mate[v] >= 0) continue;
        int64_t best = -1;
        double bw = 0.0;
        for (int64_t k = g->ptr[v]; k < g->ptr[v + 1]; ++k) {
            int64_t u = g->col[k];
            if (best < 0 || g->w[k] > bw || (g->w[k] == bw && u < best)) {
                best = u;
                bw = g->w[k];
            }
        }
        agg[v] = agg[best];
    }
    free(mate);
    return nc;
}

typedef struct {
    int64_t a, b, i, j;
    double w;
} cedge_t;

static int cmp_cedge(const void *p, const void *q)
{
    const cedge_t *x = (const cedge_t *)p, *y = (const cedge_t *)q;
    if (x->a != y->a) return x->a < y->a ? -1 : 1;
    if (x->b != y->b) return x->b < y->b ? -1 : 1;
    if (x->i != y->i) return x->i < y->i ? -1 : 1;
    if (x->j != y->j) return x->j < y->j ? -1 : 1;
    return 0;
}

/* Coarse graph of P^T L P (P piecewise constant, Sec. 2.2): an edge {A,B}
 * between different aggregates carries the sum of the fine weights w_ij,
 * i<j, with {agg i, agg j} = {A,B}, added in ascending (i,j) order.  Edges
 * inside an aggregate vanish from the coarse Laplacian. */
int lr_coarsen(const lr_csr *f, const int64_t *agg, int64_t nc, lr_csr **out)
{
    int64_t cnt = 0;
    for (int64_t i = 0; i < f->n; ++i)
        for (int64_t k = f->ptr[i]; k < f->ptr[i + 1]; ++k)
            if (f->col[k] > i && agg[f->col[k]] != agg[i]) ++cnt;
    cedge_t *C = (cedge_t *)malloc(sizeof(cedge_t) * (size_t)(cnt + 1));
    int64_t t = 0;
    for (int64_t i = 0; i < f->n; ++i)
        for (int64_t k = f->ptr[i]; k < f->ptr[i + 1]; ++k) {
            int64_t j = f->col[k];
            if (j <= i || agg[j] == agg[i]) continue;
            int64_t A = agg[i] < agg[j] ? agg[i] : agg[j];
            int64_t B = agg[i] < agg[j] ? agg[j] : agg[i];
            C[t++] = (cedge_t){A, B, i, j, f->w[k]};
        }
    qsort(C, (size_t)cnt, sizeof(cedge_t), cmp_cedge);
    int64_t ne = 0;
    int64_t *eu = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cnt + 1));
    int64_t *ev = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cnt + 1));
    double *ew = (double *)malloc(sizeof(double) * (size_t)(cnt + 1));
    for (int64_t k = 0; k < cnt; ++k) {
        if (k > 0 && C[k].a == C[k - 1].a && C[k].b == C[k - 1].b) {
            ew[ne - 1] += C[k].w;
        } else {
            eu[ne] = C[k].a;
            ev[ne] = C[k].b;
            ew[ne] = C[k].w;
            ++ne;
        }
    }
    free(C);
    int rc = lr_csr_build(nc, ne, eu, ev, ew, out);
    free(eu);
    free(ev);
    free(ew);
    return rc;
}

/* -------------------------------------------------------------- hierarchy */

struct lr_hier {
    int32_t nlev;
    int64_t *nk;        /* nodes per level */
    lr_csr **A;         /* graph of each level */
    int64_t **agg;      /* agg[k]: level k node -> level k+1 node */
    int8_t **matched;   /* matched[k][i]: paired in the matching pass */
};

static uint64_t splitmix64(uint64_t *s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static lr_csr *csr_copy(const lr_csr *g)
{
    lr_csr *c = (lr_csr *)calloc(1, sizeof(lr_csr));
    c->n = g->n;
    c->nnz = g->nnz;
    c->ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(g->n + 1));
    c->col = (int64_t *)malloc(sizeof(int64_t) * (size_t)(g->nnz + 1));
    c->w = (double *)malloc(sizeof(double) * (size_t)(g->nnz + 1));
    memcpy(c->ptr, g->ptr, sizeof(int64_t) * (size_t)(g->n + 1));
    memcpy(c->col, g->col, sizeof(int64_t) * (size_t)g->nnz);
    memcpy(c->w, g->w, sizeof(double) * (size_t)g->nnz);
    return c;
}

/* Recursive aggregation of Sec. 2.2 up to "level = max" (two nodes on the
 * top level, Sec. 3.2) or up to a given number of levels (Sec. 4.1,
 * "level = 2").  A coarsening that would leave fewer than two nodes is not
 * performed, so the top level keeps a connected graph of >= 2 nodes. */
int lr_hier_build(const lr_csr *g, int32_t max_levels, int64_t n_top,
                  uint64_t seed, lr_hier **out)
{
    return lr_hier_build_ex(g, max_levels, n_top, seed, 0, out);
}

int lr_hier_build_ex(const lr_csr *g, int32_t max_levels, int64_t n_top,
                     uint64_t seed, int32_t matching, lr_hier **out)
{
    *out = NULL;
    if (!lr_connected(g)) return LR_EDISCONNECTED;
    int cap = 80;
    lr_hier *h = (lr_hier *)calloc(1, sizeof(lr_hier));
    h->nk = (int64_t *)calloc((size_t)cap, sizeof(int64_t));
    h->A = (lr_csr **)calloc((size_t)cap, sizeof(lr_csr *));
    h->agg = (int64_t **)calloc((size_t)cap, sizeof(int64_t *));
    h->matched = (int8_t **)calloc((size_t)cap, sizeof(int8_t *));
    h->A[0] = csr_copy(g);
    h->nk[0] = g->n;
    h->nlev = 1;
    while ((max_levels <= 0 || h->nlev < max_levels) && h->nlev < cap - 1) {
        const lr_csr *f = h->A[h->nlev - 1];
        if (f->n <= n_top) break;
        int64_t *order = NULL;
        if (seed != 0) {
            uint64_t s = seed + (uint64_t)h->nlev;
            order = (int64_t *)malloc(sizeof(int64_t) * (size_t)f->n);
            for (int64_t i = 0; i < f->n; ++i) order[i] = i;
            for (int64_t i = f->n - 1; i > 0; --i) {
                int64_t j = (int64_t)(splitmix64(&s) % (uint64_t)(i + 1));
                int64_t tmp = order[i];
                order[i] = order[j];
                order[j] = tmp;
            }
        }
        int64_t *agg = (int64_t *)malloc(sizeof(int64_t) * (size_t)f->n);
        int8_t *mt = (int8_t *)malloc((size_t)f->n);
        int64_t nc = matching == 1 ? lr_greedy_match(f, agg, mt) : lr_mwm(f, order, agg, mt);
        free(order);
        if (nc < 2 || nc >= f->n) {
            free(agg);
            free(mt);
            break;
        }
        lr_csr *c = NULL;
        int rc = lr_coarsen(f, agg, nc, &c);
        if (rc != LR_OK) {
            free(agg);
            free(mt);
            lr_hier_free(h);
            return rc;
        }
        h->agg[h->nlev - 1] = agg;
        h->matched[h->nlev - 1] = mt;
        h->A[h->nlev] = c;
        h->nk[h->nlev] = nc;
        h->nlev += 1;
    }
    *out = h;
    return LR_OK;
}

void lr_hier_free(lr_hier *h)
{
    if (!h) return;
    for (int32_t k = 0; k < h->nlev; ++k) {
        lr_csr_free(h->A[k]);
        free(h->agg[k]);
        free(h->matched[k]);
    }
    free(h->A);
    free(h->agg);
    free(h->matched);
    free(h->nk);
    free(h);
}

int32_t lr_hier_nlev(const lr_hier *h) { return h->nlev; }
int64_t lr_hier_nk(const lr_hier *h, int32_t k) { return h->nk[k]; }
int64_t lr_hier_level_nnz(const lr_hier *h, int32_t k) { return h->A[k]->nnz; }

void lr_hier_agg(const lr_hier *h, int32_t k, int64_t *agg, int8_t *matched)
{
    memcpy(agg, h->agg[k], sizeof(int64_t) * (size_t)h->nk[k]);
    if (matched) memcpy(matched, h->matched[k], (size_t)h->nk[k]);
}

void lr_hier_level_csr(const lr_hier *h, int32_t k, int64_t *ptr,
                       int64_t *col, double *w)
{
    const lr_csr *g = h->A[k];
    memcpy(ptr, g->ptr, sizeof(int64_t) * (size_t)(g->n + 1));
    memcpy(col, g->col, sizeof(int64_t) * (size_t)g->nnz);
    memcpy(w, g->w, sizeof(double) * (size_t)g->nnz);
}

int64_t lr_hier_ntilde(const lr_hier *h)
{
    int64_t s = 0;
    for (int32_t k = 0; k < h->nlev; ++k) s += h->nk[k];
    return s;
}

/* ----------------------------------------------------- expanded operators */

/* Ancestor of every fine node on every level: anc[k][i] is the level-k node
 * whose aggregate chain contains fine node i, i.e. P^k(i, anc) = 1 in the
 * composite prolongation of Eq. (def:P). */
static int64_t **ancestors(const lr_hier *h)
{
    int64_t n = h->nk[0];
    int64_t **anc = (int64_t **)malloc(sizeof(int64_t *) * (size_t)h->nlev);
    anc[0] = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) anc[0][i] = i;
    for (int32_t k = 1; k < h->nlev; ++k) {
        anc[k] = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
        for (int64_t i = 0; i < n; ++i) anc[k][i] = h->agg[k - 1][anc[k - 1][i]];
    }
    return anc;
}

static void free_anc(const lr_hier *h, int64_t **anc)
{
    for (int32_t k = 0; k < h->nlev; ++k) free(anc[k]);
    free(anc);
}

/* P(mu) = [I, -mu P^2, mu^2 P^3, ..., (-mu)^(l-1) P^l]  (Sec. 2.2).
 * rt = P(mu)^T r: block k holds (-mu)^k (P^(k+1))^T r. */
void lr_restrict_mu(const lr_hier *h, double mu, const double *r, double *rt)
{
    int64_t n = h->nk[0];
    int64_t **anc = ancestors(h);
    int64_t off = 0;
    double s = 1.0;
    for (int32_t k = 0; k < h->nlev; ++k) {
        for (int64_t J = 0; J < h->nk[k]; ++J) rt[off + J] = 0.0;
        for (int64_t i = 0; i < n; ++i) rt[off + anc[k][i]] += r[i];
        for (int64_t J = 0; J < h->nk[k]; ++J) rt[off + J] *= s;
        off += h->nk[k];
        s *= -mu;
    }
    free_anc(h, anc);
}

/* z = P(mu) y: z_i = sum_k (-mu)^k y[level k ancestor of i]. */
void lr_prolong_mu(const lr_hier *h, double mu, const double *yt, double *z)
{
    int64_t n = h->nk[0];
    int64_t **anc = ancestors(h);
    for (int64_t i = 0; i < n; ++i) z[i] = 0.0;
    int64_t off = 0;
    double s = 1.0;
    for (int32_t k = 0; k < h->nlev; ++k) {
        for (int64_t i = 0; i < n; ++i) z[i] += s * yt[off + anc[k][i]];
        off += h->nk[k];
        s *= -mu;
    }
    free_anc(h, anc);
}

/* -------------------------------------------------------------------- MSP */

/* Sec. 3.3: MSP keeps, from the positive subgraph H~, the edges of the top
 * coarse level, the edges between levels and the edges inside the
 * aggregations.  With levels k = 0..l-1 (0-based) the corresponding entries
 * of L_G~ = P(mu)^T L_G P(mu) (Eq. def:L_ell) are
 *   - same level k, i and j in one aggregate:  -mu^(2k) w_ij      (kept);
 *   - node i of level k<l-1 and its own aggregate agg(i) on level k+1:
 *       (-mu)^k (-mu)^(k+1) (L_k P_k^(k+1))(i, agg i) = -mu^(2k+1) ext_k(i)
 *     with ext_k(i) = sum of w_ij over neighbours j outside i's aggregate
 *     (kept, a positive edge, omitted when ext = 0);
 *   - top level: -mu^(2(l-1)) w_ij (kept).
 * Reading: intra-aggregate edges are kept on every level below the top and
 * only parent links between adjacent levels are kept. */
int lr_msp_edges(const lr_hier *h, double mu, int64_t *ne, int64_t **eu,
                 int64_t **ev, double **ew)
{
    int64_t cap = 0;
    for (int32_t k = 0; k < h->nlev; ++k) cap += h->A[k]->nnz / 2 + h->nk[k];
    int64_t *U = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cap + 1));
    int64_t *V = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cap + 1));
    double *W = (double *)malloc(sizeof(double) * (size_t)(cap + 1));
    int64_t t = 0, off = 0;
    int32_t top = h->nlev - 1;
    for (int32_t k = 0; k < h->nlev; ++k) {
        const lr_csr *g = h->A[k];
        double s2k = pow(mu, 2.0 * k);
        double s2k1 = pow(mu, 2.0 * k + 1.0);
        for (int64_t i = 0; i < g->n; ++i) {
            double ext = 0.0;
            for (int64_t q = g->ptr[i]; q < g->ptr[i + 1]; ++q) {
                int64_t j = g->col[q];
                int same = (k == top) || (h->agg[k][i] == h->agg[k][j]);
                if (k < top && h->agg[k][i] != h->agg[k][j]) ext += g->w[q];
                if (j > i && same) {
                    U[t] = off + i;
                    V[t] = off + j;
                    W[t] = s2k * g->w[q];
                    ++t;
                }
            }
            if (k < top && ext > 0.0) {
                U[t] = off + i;
                V[t] = off + g->n + h->agg[k][i];
                W[t] = s2k1 * ext;
                ++t;
            }
        }
        off += g->n;
    }
    *ne = t;
    *eu = U;
    *ev = V;
    *ew = W;
    return LR_OK;
}

/* Sparse symmetric Gaussian elimination of L_T~ (Sec. 3.3: the tree-like
 * MSP is eliminated aggregate by aggregate from the base level).
 * The working matrix keeps, per node, a growable list of off-diagonal
 * entries (neighbour, value); eliminated neighbours are skipped. */
typedef struct {
    int64_t *nb;
    double *val;
    int64_t len, cap;
} row_t;

struct lr_msp {
    const lr_hier *h;
    double mu;
    int64_t nt;          /* n~ */
    int64_t neli;        /* eliminated nodes (n~ - 1) */
    int64_t *order;      /* elimination order, neli entries */
    double *piv;         /* pivot of each eliminated node (by position) */
    int64_t *cptr;       /* column of the factor for each position */
    int64_t *cidx;
    double *cval;
    int64_t ground;      /* grounded node (last top-level node) */
    int64_t fill;
};

static void row_add(row_t *r, int64_t j, double v)
{
    for (int64_t q = 0; q < r->len; ++q)
        if (r->nb[q] == j) {
            r->val[q] += v;
            return;
        }
    if (r->len == r->cap) {
        r->cap = r->cap ? 2 * r->cap : 4;
        r->nb = (int64_t *)realloc(r->nb, sizeof(int64_t) * (size_t)r->cap);
        r->val = (double *)realloc(r->val, sizeof(double) * (size_t)r->cap);
    }
    r->nb[r->len] = j;
    r->val[r->len] = v;
    r->len += 1;
}

static int row_has(const row_t *r, int64_t j)
{
    for (int64_t q = 0; q < r->len; ++q)
        if (r->nb[q] == j) return 1;
    return 0;
}

int lr_msp_factor(const lr_hier *h, double mu, lr_msp **out)
{
    *out = NULL;
    int64_t nt = lr_hier_ntilde(h);
    int64_t ne;
    int64_t *eu, *ev;
    double *ew;
    lr_msp_edges(h, mu, &ne, &eu, &ev, &ew);
    row_t *R = (row_t *)calloc((size_t)nt, sizeof(row_t));
    double *diag = (double *)calloc((size_t)nt, sizeof(double));
    for (int64_t e = 0; e < ne; ++e) {
        /* Laplacian of T~: off-diagonal -w, diagonal = weighted degree. */
        row_add(&R[eu[e]], ev[e], -ew[e]);
        row_add(&R[ev[e]], eu[e], -ew[e]);
        diag[eu[e]] += ew[e];
        diag[ev[e]] += ew[e];
    }
    free(eu);
    free(ev);
    free(ew);

    lr_msp *f = (lr_msp *)calloc(1, sizeof(lr_msp));
    f->h = h;
    f->mu = mu;
    f->nt = nt;
    f->neli = nt - 1;
    f->order = (int64_t *)malloc(sizeof(int64_t) * (size_t)nt);
    /* Order: level by level from the finest; on a level below the top the
     * leftover members of the aggregates go before the matched pairs; the
     * top level comes last and its last node is grounded. */
    int64_t t = 0, off = 0;
    for (int32_t k = 0; k < h->nlev; ++k) {
        if (k < h->nlev - 1) {
            for (int64_t i = 0; i < h->nk[k]; ++i)
                if (!h->matched[k][i]) f->order[t++] = off + i;
            for (int64_t i = 0; i < h->nk[k]; ++i)
                if (h->matched[k][i]) f->order[t++] = off + i;
        } else {
            for (int64_t i = 0; i < h->nk[k]; ++i) f->order[t++] = off + i;
        }
        off += h->nk[k];
    }
    f->ground = f->order[nt - 1];

    char *done = (char *)calloc((size_t)nt, 1);
    f->piv = (double *)malloc(sizeof(double) * (size_t)nt);
    f->cptr = (int64_t *)calloc((size_t)nt + 1, sizeof(int64_t));
    int64_t ccap = 16, clen = 0;
    f->cidx = (int64_t *)malloc(sizeof(int64_t) * (size_t)ccap);
    f->cval = (double *)malloc(sizeof(double) * (size_t)ccap);
    int64_t fill = 0;
    int64_t *nbl = (int64_t *)malloc(sizeof(int64_t) * (size_t)nt);
    double *nbv = (double *)malloc(sizeof(double) * (size_t)nt);
    for (int64_t pos = 0; pos < f->neli; ++pos) {
        int64_t p = f->order[pos];
        double d = diag[p];
        int64_t cnt = 0;
        for (int64_t q = 0; q < R[p].len; ++q) {
            int64_t i = R[p].nb[q];
            if (done[i] || R[p].val[q] == 0.0) continue;
            nbl[cnt] = i;
            nbv[cnt] = R[p].val[q];
            ++cnt;
        }
        f->piv[pos] = d;
        for (int64_t a = 0; a < cnt; ++a) {
            if (clen == ccap) {
                ccap *= 2;
                f->cidx = (int64_t *)realloc(f->cidx, sizeof(int64_t) * (size_t)ccap);
                f->cval = (double *)realloc(f->cval, sizeof(double) * (size_t)ccap);
            }
            f->cidx[clen] = nbl[a];
            f->cval[clen] = nbv[a];
            ++clen;
        }
        f->cptr[pos + 1] = clen;
        /* Schur update: A_ij -= A_ip A_pj / A_pp over remaining neighbours. */
        for (int64_t a = 0; a < cnt; ++a) {
            int64_t i = nbl[a];
            diag[i] -= nbv[a] * nbv[a] / d;
            for (int64_t b = 0; b < cnt; ++b) {
                if (b == a) continue;
                int64_t j = nbl[b];
                if (!row_has(&R[i], j)) ++fill;
                row_add(&R[i], j, -nbv[a] * nbv[b] / d);
            }
        }
        done[p] = 1;
    }
    f->fill = fill / 2;
    free(nbl);
    free(nbv);
    free(done);
    free(diag);
    for (int64_t i = 0; i < nt; ++i) {
        free(R[i].nb);
        free(R[i].val);
    }
    free(R);
    *out = f;
    return LR_OK;
}

void lr_msp_free(lr_msp *f)
{
    if (!f) return;
    free(f->order);
    free(f->piv);
    free(f->cptr);
    free(f->cidx);
    free(f->cval);
    free(f);
}

int64_t lr_msp_fill(const lr_msp *f) { return f->fill; }

/* z = P(mu) y with L_T~ y = P(mu)^T r (grounded solution; any other solution
 * differs by a constant, which P(mu) maps to a constant), mean removed. */
/* y~ = the grounded solve of L_T~ y~ = b~ in the expanded space (Sec. 3.3):
 * elimination with the factor of lr_msp_factor, y~ = 0 on the ground node.
 * This is the preconditioner of the expanded system (Sec. 4); b~ and y~
 * hold ntilde values. */
void lr_msp_solve_expanded(const lr_msp *f, const double *bt, double *y)
{
    int64_t nt = f->nt;
    double *b = (double *)malloc(sizeof(double) * (size_t)nt);
    memcpy(b, bt, sizeof(double) * (size_t)nt);
    for (int64_t pos = 0; pos < f->neli; ++pos) {
        int64_t p = f->order[pos];
        double bp = b[p] / f->piv[pos];
        for (int64_t q = f->cptr[pos]; q < f->cptr[pos + 1]; ++q)
            b[f->cidx[q]] -= f->cval[q] * bp;
    }
    y[f->ground] = 0.0;
    for (int64_t pos = f->neli - 1; pos >= 0; --pos) {
        int64_t p = f->order[pos];
        double s = b[p];
        for (int64_t q = f->cptr[pos]; q < f->cptr[pos + 1]; ++q)
            s -= f->cval[q] * y[f->cidx[q]];
        y[p] = s / f->piv[pos];
    }
    free(b);
}

void lr_msp_apply(void *ctx, const double *r, double *z)
{
    const lr_msp *f = (const lr_msp *)ctx;
    const lr_hier *h = f->h;
    int64_t nt = f->nt, n = h->nk[0];
    double *b = (double *)malloc(sizeof(double) * (size_t)nt);
    double *y = (double *)malloc(sizeof(double) * (size_t)nt);
    lr_restrict_mu(h, f->mu, r, b);
    for (int64_t pos = 0; pos < f->neli; ++pos) {
        int64_t p = f->order[pos];
        double bp = b[p] / f->piv[pos];
        for (int64_t q = f->cptr[pos]; q < f->cptr[pos + 1]; ++q)
            b[f->cidx[q]] -= f->cval[q] * bp;
    }
    y[f->ground] = 0.0;
    for (int64_t pos = f->neli - 1; pos >= 0; --pos) {
        int64_t p = f->order[pos];
        double s = b[p];
        for (int64_t q = f->cptr[pos]; q < f->cptr[pos + 1]; ++q)
            s -= f->cval[q] * y[f->cidx[q]];
        y[p] = s / f->piv[pos];
    }
    lr_prolong_mu(h, f->mu, y, z);
    double mean = 0.0;
    for (int64_t i = 0; i < n; ++i) mean += z[i];
    mean /= (double)n;
    for (int64_t i = 0; i < n; ++i) z[i] -= mean;
    free(b);
    free(y);
}

/* -------------------------------------------------------------------- PCG */

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static void remove_mean(int64_t n, double *a)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i];
    s /= (double)n;
    for (int64_t i = 0; i < n; ++i) a[i] -= s;
}

/* Preconditioned conjugate gradients on the original system (the Theorem of
 * Sec. 3.1 shows it is equivalent to the expanded one):
 *   b^ = b - mean(b); x = 0; r = b^; z = M r - mean; p = z; rho = r.z
 *   repeat: q = L p; pq = p.q (breakdown if pq <= 0 or not finite);
 *           alpha = rho/pq; x += alpha p; r -= alpha q;
 *           stop if ||r|| <= tol ||b^|| (iterations = products with L);
 *           z = M r - mean; rho' = r.z; beta = rho'/rho; p = z + beta p.
 * Sec. 4 stops on the residual of the original system, which the
 * recurrence only tracks: once the recursive residual meets tol, x is made
 * mean-free and the true residual t = b^ - L x is formed.  If ||t|| is
 * still above tol ||b^||, the iteration restarts from x with r = t - mean(t),
 * z = M r - mean, p = z (a residual replacement) and continues under the
 * same stop rule and the same cap on products with L.  After max_restarts
 * replacements a true residual above tol ends the run with LR_ENOCONV.
 *   x -= mean(x); report ||b^ - L x|| / ||b^||.
 * relres_hist (optional, maxit+1 entries) receives ||r_k||/||b^||. */
/* Rounding model for parity bands: with noise > 0 every product L p and
 * every preconditioner output M r is multiplied entrywise by (1 + noise*u),
 * u uniform in [-1, 1) from SplitMix64 seeded with `seed`.  A noise of a few
 * units of round-off models a different summation order; the spread of the
 * iteration count over seeds is the band an independent FP64 implementation
 * of the same method can be expected to fall in. */
static void perturb(int64_t n, double *a, double noise, uint64_t *s)
{
    for (int64_t i = 0; i < n; ++i) {
        double u = (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
        a[i] *= 1.0 + noise * (2.0 * u - 1.0);
    }
}

int lr_pcg(const lr_csr *g, lr_precond_fn M, void *ctx, const double *b,
           double tol, int32_t maxit, double *x, lr_pcg_info *info,
           double *relres_hist)
{
    return lr_pcg_ex(g, M, ctx, b, tol, maxit, x, info, relres_hist, 0.0, 0,
                     LR_MAX_RESTARTS);
}

int lr_pcg_noisy(const lr_csr *g, lr_precond_fn M, void *ctx, const double *b,
                 double tol, int32_t maxit, double *x, lr_pcg_info *info,
                 double *relres_hist, double noise, uint64_t seed)
{
    return lr_pcg_ex(g, M, ctx, b, tol, maxit, x, info, relres_hist, noise, seed,
                     LR_MAX_RESTARTS);
}

/* z = M r - mean (or r - mean without a preconditioner), perturbed by the
 * rounding model when noise > 0; returns r.z. */
static double precondition(int64_t n, lr_precond_fn M, void *ctx, const double *r,
                           double *z, double noise, uint64_t *st)
{
    if (M) M(ctx, r, z);
    else memcpy(z, r, sizeof(double) * (size_t)n);
    if (noise > 0.0) perturb(n, z, noise, st);
    remove_mean(n, z);
    return dot(n, r, z);
}

/* t = b^ - L x after x -= mean(x); returns ||t||. */
static double true_residual(const lr_csr *g, const double *bh, double *x, double *t)
{
    int64_t n = g->n;
    remove_mean(n, x);
    lr_lap_apply(g, x, t);
    for (int64_t i = 0; i < n; ++i) t[i] = bh[i] - t[i];
    return sqrt(dot(n, t, t));
}

int lr_pcg_ex(const lr_csr *g, lr_precond_fn M, void *ctx, const double *b,
              double tol, int32_t maxit, double *x, lr_pcg_info *info,
              double *relres_hist, double noise, uint64_t seed, int32_t max_restarts)
{
    uint64_t st = seed;
    int64_t n = g->n;
    double *bh = (double *)malloc(sizeof(double) * (size_t)n);
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(bh, b, sizeof(double) * (size_t)n);
    remove_mean(n, bh);
    double nb = sqrt(dot(n, bh, bh));
    for (int64_t i = 0; i < n; ++i) {
        x[i] = 0.0;
        r[i] = bh[i];
    }
    int32_t it = 0, restarts = 0;
    int status = LR_ENOCONV;
    double rn = nb;
    if (relres_hist) relres_hist[0] = nb > 0.0 ? 1.0 : 0.0;
    if (nb == 0.0) {
        status = LR_OK;
    } else {
        double rho = precondition(n, M, ctx, r, z, noise, &st);
        memcpy(p, z, sizeof(double) * (size_t)n);
        while (it < maxit) {
            lr_lap_apply(g, p, q);
            if (noise > 0.0) perturb(n, q, noise, &st);
            ++it;
            double pq = dot(n, p, q);
            if (!(pq > 0.0) || !isfinite(pq)) {
                status = LR_EBREAKDOWN;
                break;
            }
            double alpha = rho / pq;
            for (int64_t i = 0; i < n; ++i) {
                x[i] += alpha * p[i];
                r[i] -= alpha * q[i];
            }
            rn = sqrt(dot(n, r, r));
            if (relres_hist) relres_hist[it] = rn / nb;
            if (rn <= tol * nb) {
                /* the recurrence has converged: check the true residual */
                double tn = true_residual(g, bh, x, q);
                if (tn <= tol * nb) {
                    status = LR_OK;
                    break;
                }
                if (restarts == max_restarts) {
                    status = LR_ENOCONV;
                    break;
                }
                ++restarts;
                memcpy(r, q, sizeof(double) * (size_t)n);
                remove_mean(n, r);
                rn = sqrt(dot(n, r, r));
                rho = precondition(n, M, ctx, r, z, noise, &st);
                memcpy(p, z, sizeof(double) * (size_t)n);
                continue;
            }
            double rho2 = precondition(n, M, ctx, r, z, noise, &st);
            double beta = rho2 / rho;
            rho = rho2;
            for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        }
    }
    double tn = true_residual(g, bh, x, q);
    if (info) {
        info->iterations = it;
        info->status = status;
        info->restarts = restarts;
        info->relres_recursive = nb > 0.0 ? rn / nb : 0.0;
        info->relres_true = nb > 0.0 ? tn / nb : 0.0;
    }
    free(bh);
    free(r);
    free(z);
    free(p);
    free(q);
    return status;
}
