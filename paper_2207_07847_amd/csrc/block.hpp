// Device kernels of the multi-right-hand-side solve: kCols independent PCG
// runs advanced together, one per column, so every pass over the matrix and
// the hierarchy serves all columns (the SpMV becomes an SpMM).  Each column
// keeps its own alpha, beta, rho and stop test (no block Krylov space, so
// rank-deficient blocks cannot break down); a converged column is frozen.
//
// Layout: a block vector holds n rows of kCols values, row-major (row i's
// columns contiguous: 256 B in FP32, 512 B in FP64).  One wavefront handles
// one row, aggregate or chunk, lane c being column c, so every vector access
// is one coalesced row.  Work is split into chunks so that rows and
// aggregates with thousands of entries are shared by several wavefronts:
// chunks of a row or aggregate with more than one chunk write partial rows
// that a combine kernel adds.  Included by lap.hip only.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"

namespace lapgpu {

constexpr int kCols = 64;          // columns of a block vector (= wavefront)
constexpr int kMmWaves = 4;        // wavefronts per block of the block kernels
constexpr int kMmChunk = 64;       // matrix entries / children per chunk

// Scalars of the kCols runs.
struct ScalM {
    double rho[kCols], pq[kCols], alpha[kCols], beta[kCols], zbar[kCols];
    double rr[kCols], bn2[kCols], sum[kCols], res2[kCols];
    double tol2[kCols];      // stop when ||r||^2 <= tol2 * ||r_0||^2
    int32_t done[kCols];     // 0 running, 1 converged, 2 max_iter, 3 breakdown,
                             // 4 bad input, 5 not part of this run
    int32_t iter[kCols];     // products with L performed by the column's run
    int32_t fresh[kCols];    // 1: the next rho finish starts the column's run (beta = 0)
    int32_t maxit, admit, all_done, pad;   // admit: the next rho finish serves
                                           // fresh columns only (a column admission)
};

// Column admission and extraction of the serving loop (device copy, set by
// the host before it enqueues the kernels that read it): column c takes a
// new right-hand side from src[c] (input order, FP64) with stop tolerance
// tol2[c], or hands its mean-free solution to dst[c] (input order); null
// pointers leave the column alone.
struct ServeCtl {
    const double* src[kCols];
    double* dst[kCols];
    double tol2[kCols];
};

// Work items: chunk i covers entries (children) [t0[i], t1[i]) of row (or
// aggregate) id[i].  Rows (aggregates) split into several chunks are listed
// in multi: multi[m] = id, their chunks are mfirst[m] .. mfirst[m+1]-1 and
// write partial rows to scratch row mfirst[m] + k.
struct Chunks {
    int32_t nitems;
    const int32_t* id;
    const int32_t* t0;
    const int32_t* t1;
    const int32_t* slot;     // scratch row of the chunk, -1 when the chunk is whole
    int32_t nmulti;
    const int32_t* multi;
    const int32_t* mfirst;
};

// CSR Laplacian in the solve order (rows ascending).
template <class T>
struct Csr {
    int32_t n;
    const int64_t* ptr;
    const int32_t* col;
    const T* w;
};

constexpr int kMmMaxGrid = 1024;   // blocks of a block-vector kernel (bounds the partials)

// Items [i0, i1) of this block: contiguous ranges per block (blocks
// renumbered per XCD), the block's wavefronts taking every kMmWaves-th.
__device__ inline void mm_range(int nitems, int& i0, int& i1) {
    const int G = gridDim.x, b = xcd_block();
    const int per = (nitems + G - 1) / G;
    i0 = min(b * per, nitems);
    i1 = min(i0 + per, nitems);
    i0 += (int)(threadIdx.x >> 6);
}
#define MM_FOR(it, nitems)         \
    int it##_0, it##_1;            \
    mm_range(nitems, it##_0, it##_1); \
    for (int it = it##_0; it < it##_1; it += kMmWaves)

// ------------------------------------------------------------- reductions

// Per-block partial sums of NV per-column values: part[(v*G + b)*kCols + c].
// Each wavefront holds its column value in its lane; the block's
// wavefronts are added in a fixed order.
template <int NV>
__device__ inline void mm_partial(const double (&v)[NV], double* part) {
    __shared__ double red[NV][kMmWaves][kCols];
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < NV; ++i) red[i][wid][lane] = v[i];
    __syncthreads();
    if (wid == 0) {
        const int G = gridDim.x;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double s = 0.0;
            for (int w = 0; w < kMmWaves; ++w) s += red[i][w][lane];
            part[((size_t)i * G + blockIdx.x) * kCols + lane] = s;
        }
    }
}

enum MmFin { kMmPq, kMmRho, kMmSum, kMmBn2, kMmRes2, kMmAdmit };

// One-block finish: 1024 threads = 16 groups x 64 columns; group g adds the
// partials of blocks g, g+16, ... of its column, then the groups are added
// in order.  `part` holds NV values per block per column (G blocks); kMmRho
// also takes the update kernel's ||r||^2 partials and kMmPq the p^T q
// shares of split rows (G2 blocks at part2).
template <int OP>
__global__ __launch_bounds__(1024) void k_mm_finish(int G, int n, const double* __restrict__ part,
                                                    int G2, const double* __restrict__ part2,
                                                    ScalM* S, const ServeCtl* ctl = nullptr) {
    if ((OP == kMmPq || OP == kMmRho) && S->all_done) return;
    constexpr int NV = OP == kMmRho ? 3 : 1;
    constexpr int NG = 16;
    __shared__ double red[NV + 1][NG][kCols];
    const int g = threadIdx.x >> 6, c = threadIdx.x & 63;
    double v[NV + 1];
    for (int i = 0; i < NV; ++i) {
        double s = 0.0;
        for (int b = g; b < G; b += NG) s += part[((size_t)i * G + b) * kCols + c];
        v[i] = s;
    }
    double r2 = 0.0;
    if (OP == kMmRho || OP == kMmPq || OP == kMmRes2)
        for (int b = g; b < G2; b += NG) r2 += part2[(size_t)b * kCols + c];
    v[NV] = r2;
    for (int i = 0; i <= NV; ++i) red[i][g][c] = v[i];
    __syncthreads();
    if (g != 0) return;
    double t[NV + 1];
    for (int i = 0; i <= NV; ++i) {
        double s = 0.0;
        for (int q = 0; q < NG; ++q) s += red[i][q][c];
        t[i] = s;
    }
    const int d = S->done[c];
    if (OP == kMmPq) {
        const double pq = t[0] + t[NV];   // whole rows + rows split over chunks
        if (d == 0) {
            S->pq[c] = pq;
            S->iter[c] += 1;
            if (!(pq > 0.0) || !isfinite(pq)) {
                S->done[c] = 3;
                S->alpha[c] = 0.0;
            } else {
                S->alpha[c] = S->rho[c] / pq;
            }
        } else {
            S->alpha[c] = 0.0;
        }
    } else if (OP == kMmRho) {
        const double zbar = t[0] / (double)n;
        const double rho = t[1] - zbar * t[2];
        const int fresh = S->fresh[c];
        if (d == 0 && (fresh || !S->admit)) {
            S->zbar[c] = zbar;
            S->beta[c] = fresh ? 0.0 : rho / S->rho[c];
            S->fresh[c] = 0;
            S->rho[c] = rho;
            if (!isfinite(rho)) S->done[c] = 3;
            if (G2 > 0) {
                S->rr[c] = t[NV];
                if (!isfinite(t[NV])) S->done[c] = 3;
                else if (t[NV] <= S->tol2[c] * S->bn2[c]) S->done[c] = 1;
                else if (S->iter[c] >= S->maxit) S->done[c] = 2;
            }
        }
        // every column stopped: later kernels of the chunk return at once
        // (group 0 is one wavefront: a vote over its lanes)
        const unsigned long long stopped = __ballot(S->done[c] != 0);
        if (c == 0) {
            S->admit = 0;
            S->all_done = stopped == ~0ull;
        }
    } else if (OP == kMmSum) {
        S->sum[c] = t[0];
    } else if (OP == kMmBn2 || OP == kMmAdmit) {
        // kMmBn2: a new run of every column not marked 5; kMmAdmit: a new
        // run of the columns the serving loop admits, the others untouched
        const bool start = OP == kMmBn2 ? S->done[c] != 5 : ctl->src[c] != nullptr;
        if (start || OP == kMmBn2) {
            S->bn2[c] = t[0];
            S->rr[c] = t[0];
            S->iter[c] = 0;
            S->alpha[c] = S->beta[c] = S->zbar[c] = 0.0;
            S->fresh[c] = 1;
        }
        if (start) {
            if (OP == kMmAdmit) S->tol2[c] = ctl->tol2[c];
            if (!isfinite(t[0])) S->done[c] = 4;
            else if (t[0] == 0.0) S->done[c] = 1;
            else if (S->maxit <= 0) S->done[c] = 2;
            else S->done[c] = 0;
        }
        const unsigned long long stopped = __ballot(S->done[c] != 0);
        if (c == 0) {
            S->admit = OP == kMmAdmit;
            S->all_done = stopped == ~0ull;
        }
    } else if (OP == kMmRes2) {
        S->res2[c] = t[0] + t[NV];        // whole rows + rows split over chunks
    }
}

// ------------------------------------------------------------------ SpMM

// p = zn - zbar + beta p_old for the running columns (solve order).
template <class T>
__global__ __launch_bounds__(kMmWaves * 64) void k_mm_pupd(int n, const T* __restrict__ zn,
                                                           const T* __restrict__ pold,
                                                           T* __restrict__ pnew,
                                                           const ScalM* S) {
    if (S->all_done) return;
    const int c = threadIdx.x & 63;
    // A stopped column keeps its last direction: repeating the update with
    // its final beta would grow p geometrically whenever beta > 1 and
    // overflow while the other columns run on (then alpha = 0 times an
    // infinite p puts NaN into x).  Admission zeroes both directions.
    if (S->done[c] != 0) return;
    const T zb = (T)S->zbar[c], be = (T)S->beta[c];
    MM_FOR(i, n) {
        const size_t o = (size_t)i * kCols + c;
        pnew[o] = (zn[o] - zb) + be * pold[o];
    }
}

// Q = L P over chunks of kMmChunk entries: a whole row writes its row of Q
// and its p^T q share; a chunk of a split row writes a partial row to
// scratch.  The matrix entries of a chunk are the same for all lanes
// (uniform loads); each entry gathers one row of P.
template <class T>
__global__ __launch_bounds__(kMmWaves * 64) void k_mm_spmm(Csr<T> A, Chunks C,
                                                           const T* __restrict__ p,
                                                           T* __restrict__ q,
                                                           T* __restrict__ scr, const ScalM* S,
                                                           double* part) {
    if (S->all_done) return;
    const int c = threadIdx.x & 63;
    double v[1] = {0.0};
    MM_FOR(it, C.nitems) {
        const int row = C.id[it], k0 = C.t0[it], k1 = C.t1[it];
        const T pi = p[(size_t)row * kCols + c];
        T acc = T(0);
        int k = k0;
        // eight entries' gathers in flight per wavefront
        for (; k + 7 < k1; k += 8) {
            int j[8];
            T wv[8], pv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                j[u] = A.col[k + u];
                wv[u] = A.w[k + u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) pv[u] = p[(size_t)j[u] * kCols + c];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += wv[u] * (pi - pv[u]);
        }
        for (; k < k1; ++k) acc += A.w[k] * (pi - p[(size_t)A.col[k] * kCols + c]);
        const int sl = C.slot[it];
        if (sl < 0) {
            q[(size_t)row * kCols + c] = acc;
            v[0] += (double)pi * (double)acc;
        } else {
            scr[(size_t)sl * kCols + c] = acc;
        }
    }
    mm_partial<1>(v, part);
}

// Rows split over several chunks: Q row = sum of its partial rows (in chunk
// order), with its p^T q share.
template <class T>
__global__ __launch_bounds__(kMmWaves * 64) void k_mm_spmm_combine(Chunks C,
                                                                   const T* __restrict__ p,
                                                                   T* __restrict__ q,
                                                                   const T* __restrict__ scr,
                                                                   const ScalM* S, double* part) {
    if (S->all_done) return;
    const int c = threadIdx.x & 63;
    double v[1] = {0.0};
    MM_FOR(m, C.nmulti) {
        const int row = C.multi[m];
        const int s0 = C.mfirst[m], s1 = C.mfirst[m + 1];
        // eight partial rows in flight (a hub's row is split into hundreds)
        constexpr int U = 8;
        T a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = T(0);
        int s = s0;
        for (; s + U <= s1; s += U) {
            T y[U];
#pragma unroll
            for (int u = 0; u < U; ++u) y[u] = scr[(size_t)(s + u) * kCols + c];
#pragma unroll
            for (int u = 0; u < U; ++u) a[u] += y[u];
        }
        for (; s < s1; ++s) a[0] += scr[(size_t)s * kCols + c];
        const T acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
        q[(size_t)row * kCols + c] = acc;
        v[0] += (double)p[(size_t)row * kCols + c] * (double)acc;
    }
    mm_partial<1>(v, part);
}

// ------------------------------------------------------- level-0 update

// X += alpha P (solve order, positional); R -= alpha Q (tree order, Q row
// perm[t]); per-column ||r||^2 partials.  One wavefront per row.
template <class T>
__global__ __launch_bounds__(kMmWaves * 64) void k_mm_update(int n,
                                                             const int32_t* __restrict__ perm,
                                                             T* __restrict__ x, T* __restrict__ r,
                                                             const T* __restrict__ p,
                                                             const T* __restrict__ q,
                                                             const ScalM* S, double* part) {
    if (S->all_done) return;
    const int c = threadIdx.x & 63;
    const T a = (T)S->alpha[c];
    double v[1] = {0.0};
    MM_FOR(t, n) {
        const size_t o = (size_t)t * kCols + c;
        x[o] += a * p[o];
        const T rt = r[o] - a * q[(size_t)(perm ? perm[t] : t) * kCols + c];
        r[o] = rt;
        v[0] += (double)rt * rt;
    }
    mm_partial<1>(v, part);
}

// ------------------------------------------------------------ level sweeps

// Up-sweep chunk: sums of a chunk of aggregate J's children, {sum, g_a,
// g_b} per column (a whole aggregate solves its pair block directly).
template <class T>
__global__ __launch_bounds__(kMmWaves * 64) void k_mm_up(LevelDev<T> s, Chunks C,
                                                         const T* __restrict__ rk,
                                                         T* __restrict__ rk1,
                                                         T* __restrict__ scr, const ScalM* S) {
    if (S->all_done) return;
    const int c = threadIdx.x & 63;
    MM_FOR(it, C.nitems) {
    const int J = C.id[it], c0 = C.t0[it], c1 = C.t1[it];
    const int b0 = s.cptr[J];
    T sum = T(0), ga = T(0), gb = T(0);
    int t = c0;
    // the matched pair leads the children; then the leftovers, eight rows
    // and their coefficients in flight at a time (a hub's chunk is long)
    if (t == b0 && t < c1) {
        const T rv = rk[(size_t)t * kCols + c];
        sum += rv;
        ga += rv;
        ++t;
    }
    if (t == b0 + 1 && t < c1) {
        const T rv = rk[(size_t)t * kCols + c];
        sum += rv;
        gb += rv;
        ++t;
    }
    constexpr int U = 8;
    for (; t + U <= c1; t += U) {
        T rv[U], a1[U], a2[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int li = t + u - 2 * J - 2;
            rv[u] = rk[(size_t)(t + u) * kCols + c];
            a1[u] = s.l1[li];
            a2[u] = s.l2[li];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            sum += rv[u];
            ga += a1[u] * rv[u];
            gb += a2[u] * rv[u];
        }
    }
    for (; t < c1; ++t) {
        const T rv = rk[(size_t)t * kCols + c];
        const int li = t - 2 * J - 2;
        sum += rv;
        ga += s.l1[li] * rv;
        gb += s.l2[li] * rv;
    }
    const int sl = C.slot[it];
    if (sl < 0) {
        const T saa = s.saa[J], sab = s.sab[J], sbb = s.sbb[J];
        s.ea[(size_t)J * kCols + c] = saa * ga + sab * gb;
        s.eb[(size_t)J * kCols + c] = sab * ga + sbb * gb;
        rk1[(size_t)J * kCols + c] = sum;
    } else {
        scr[(size_t)(3 * sl) * kCols + c] = sum;
        scr[(size_t)(3 * sl + 1) * kCols + c] = ga;
        scr[(size_t)(3 * sl + 2) * kCols + c] = gb;
    }
    }
}

// Aggregates split over several chunks: add the chunk sums, solve the pair.
template <class T>
__global__ __launch_bounds__(kMmWaves * 64) void k_mm_up_combine(LevelDev<T> s, Chunks C,
                                                                 T* __restrict__ rk1,
                                                                 const T* __restrict__ scr,
                                                                 const ScalM* S) {
    if (S->all_done) return;
    const int c = threadIdx.x & 63;
    MM_FOR(m, C.nmulti) {
        const int J = C.multi[m];
        T sum = T(0), ga = T(0), gb = T(0);
        const int q1 = C.mfirst[m + 1];
        int q = C.mfirst[m];
        // the chunks' sums in order, four chunks' loads in flight
        constexpr int U = 4;
        for (; q + U <= q1; q += U) {
            T y[3 * U];
#pragma unroll
            for (int i = 0; i < 3 * U; ++i) y[i] = scr[(size_t)(3 * q + i) * kCols + c];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                sum += y[3 * u];
                ga += y[3 * u + 1];
                gb += y[3 * u + 2];
            }
        }
        for (; q < q1; ++q) {
            sum += scr[(size_t)(3 * q) * kCols + c];
            ga += scr[(size_t)(3 * q + 1) * kCols + c];
            gb += scr[(size_t)(3 * q + 2) * kCols + c];
        }
        const T saa = s.saa[J], sab = s.sab[J], sbb = s.sbb[J];
        s.ea[(size_t)J * kCols + c] = saa * ga + sab * gb;
        s.eb[(size_t)J * kCols + c] = sab * ga + sbb * gb;
        rk1[(size_t)J * kCols + c] = sum;
    }
}

// Down-sweep chunk: corrections of a chunk of aggregate J's children.
template <class T>
__global__ __launch_bounds__(kMmWaves * 64) void k_mm_down(LevelDev<T> s, Chunks C,
                                                           const T* __restrict__ rk,
                                                           T* __restrict__ yk,
                                                           const T* __restrict__ yk1,
                                                           const ScalM* S) {
    if (S->all_done) return;
    const int c = threadIdx.x & 63;
    MM_FOR(it, C.nitems) {
    const int J = C.id[it], c0 = C.t0[it], c1 = C.t1[it];
    const int b0 = s.cptr[J];
    const T yJ = yk1[(size_t)J * kCols + c];
    const T ea = s.ea[(size_t)J * kCols + c], eb = s.eb[(size_t)J * kCols + c];
    int t = c0;
    // the pair first, then the leftovers eight at a time (loads in flight)
    if (t == b0 && t < c1) {
        yk[(size_t)t * kCols + c] = ea + yJ;
        ++t;
    }
    if (t == b0 + 1 && t < c1) {
        yk[(size_t)t * kCols + c] = eb + yJ;
        ++t;
    }
    constexpr int U = 8;
    for (; t + U <= c1; t += U) {
        T rv[U], a0[U], a1[U], a2[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int li = t + u - 2 * J - 2;
            rv[u] = rk[(size_t)(t + u) * kCols + c];
            a0[u] = s.l0[li];
            a1[u] = s.l1[li];
            a2[u] = s.l2[li];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            yk[(size_t)(t + u) * kCols + c] = a0[u] * rv[u] + a1[u] * ea + a2[u] * eb + yJ;
    }
    for (; t < c1; ++t) {
        const int li = t - 2 * J - 2;
        const size_t o = (size_t)t * kCols + c;
        yk[o] = s.l0[li] * rk[o] + s.l1[li] * ea + s.l2[li] * eb + yJ;
    }
    }
}

// Top level: y = theta_top pinv(L_top) r, nt <= kTopMax rows, one block.
template <class T>
__global__ __launch_bounds__(kMmWaves * 64) void k_mm_top(int nt, const T* __restrict__ tp,
                                                          const T* __restrict__ r,
                                                          T* __restrict__ y, const ScalM* S) {
    if (S->all_done) return;
    const int wid = threadIdx.x >> 6, c = threadIdx.x & 63;
    for (int i = wid; i < nt; i += kMmWaves) {
        T acc = T(0);
        for (int j = 0; j < nt; ++j) acc += tp[i * nt + j] * r[(size_t)j * kCols + c];
        y[(size_t)i * kCols + c] = acc;
    }
}

// Level 0 after the down-sweep: z (tree order, already in y_0) copied to
// the solve order for the next SpMM; per-column sums of z, r z and r.
template <class T>
__global__ __launch_bounds__(kMmWaves * 64) void k_mm_zout(int n, const int32_t* __restrict__ perm,
                                                           const T* __restrict__ r,
                                                           const T* __restrict__ z,
                                                           T* __restrict__ zn, const ScalM* S,
                                                           double* part) {
    if (S->all_done) return;
    const int c = threadIdx.x & 63;
    double v[3] = {0.0, 0.0, 0.0};
    MM_FOR(t, n) {
        const size_t o = (size_t)t * kCols + c;
        const T zt = z[o], rt = r[o];
        zn[(size_t)(perm ? perm[t] : t) * kCols + c] = zt;
        v[0] += zt;
        v[1] += (double)rt * zt;
        v[2] += rt;
    }
    mm_partial<3>(v, part);
}

// Plain CG: z = r.
template <class T>
__global__ __launch_bounds__(kMmWaves * 64) void k_mm_copy(int n, const T* __restrict__ r,
                                                           T* __restrict__ z, const ScalM* S) {
    if (S->all_done) return;
    const int c = threadIdx.x & 63;
    MM_FOR(t, n) z[(size_t)t * kCols + c] = r[(size_t)t * kCols + c];
}

// ------------------------------------------------ set-up, outer loop, exit

// Per-column sums of a block vector (FP64).
__global__ __launch_bounds__(kMmWaves * 64) void k_mm_colsum(int n, const double* __restrict__ a,
                                                             double* part) {
    const int c = threadIdx.x & 63;
    double v[1] = {0.0};
    MM_FOR(t, n) v[0] += a[(size_t)t * kCols + c];
    mm_partial<1>(v, part);
}

// Per-column sums of the caller's columns (column c at b + c*ld, input
// order); columns >= nrhs are zero.
__global__ __launch_bounds__(kMmWaves * 64) void k_mm_colsum_in(int n, const double* __restrict__ b,
                                                                int64_t ld, int nrhs,
                                                                double* part) {
    const int c = threadIdx.x & 63;
    double v[1] = {0.0};
    if (c < nrhs) {
        MM_FOR(t, n) v[0] += b[(size_t)c * ld + t];
    }
    mm_partial<1>(v, part);
}

// bh = b - mean (solve order, interleaved; row s is input vertex sperm[s]);
// x = 0; r = bh; partial ||bh||^2 per column.
__global__ __launch_bounds__(kMmWaves * 64) void k_mm_begin(int n, const int32_t* __restrict__ sperm,
                                                            const double* __restrict__ b,
                                                            int64_t ld, int nrhs,
                                                            double* __restrict__ bh,
                                                            double* __restrict__ x,
                                                            double* __restrict__ r,
                                                            const ScalM* S, double* part) {
    const int c = threadIdx.x & 63;
    const double mean = S->sum[c] / (double)n;
    double v[1] = {0.0};
    MM_FOR(t, n) {
        const int src = sperm ? sperm[t] : t;
        const double bt = c < nrhs ? b[(size_t)c * ld + src] - mean : 0.0;
        const size_t o = (size_t)t * kCols + c;
        bh[o] = bt;
        x[o] = 0.0;
        r[o] = bt;
        v[0] += bt * bt;
    }
    mm_partial<1>(v, part);
}

// Inner PCG start for the right-hand sides rhs (solve order, FP64): r =
// rhs - mean (tree order, type T; tree row t reads solve row perm[t]), x =
// p0 = p1 = 0; partial ||r||^2 per column.
template <class T>
__global__ __launch_bounds__(kMmWaves * 64) void k_mm_init(int n, const int32_t* __restrict__ perm,
                                                           const double* __restrict__ rhs,
                                                           T* __restrict__ r, T* __restrict__ x,
                                                           T* __restrict__ p0, T* __restrict__ p1,
                                                           const ScalM* S, double* part) {
    const int c = threadIdx.x & 63;
    const double mean = S->sum[c] / (double)n;
    double v[1] = {0.0};
    MM_FOR(t, n) {
        const size_t o = (size_t)t * kCols + c;
        const double bt = rhs[o] - mean;
        r[o] = (T)(rhs[(size_t)(perm ? perm[t] : t) * kCols + c] - mean);
        x[o] = T(0);
        p0[o] = T(0);
        p1[o] = T(0);
        v[0] += bt * bt;
    }
    mm_partial<1>(v, part);
}

// x64 += d (columns still refining).
template <class T>
__global__ __launch_bounds__(kMmWaves * 64) void k_mm_addcorr(int n, double* __restrict__ x,
                                                              const T* __restrict__ d) {
    const int c = threadIdx.x & 63;
    MM_FOR(t, n) x[(size_t)t * kCols + c] += (double)d[(size_t)t * kCols + c];
}

// r = bh - L x (FP64, solve order) over chunks; split rows combined below;
// per-column ||r||^2 partial of whole rows.
__global__ __launch_bounds__(kMmWaves * 64) void k_mm_resid(Csr<double> A, Chunks C,
                                                            const double* __restrict__ x,
                                                            const double* __restrict__ bh,
                                                            double* __restrict__ r,
                                                            double* __restrict__ scr,
                                                            double* part) {
    const int c = threadIdx.x & 63;
    double v[1] = {0.0};
    MM_FOR(it, C.nitems) {
        const int row = C.id[it], k0 = C.t0[it], k1 = C.t1[it];
        const double xi = x[(size_t)row * kCols + c];
        double acc = 0.0;
        for (int k = k0; k < k1; ++k) acc += A.w[k] * (xi - x[(size_t)A.col[k] * kCols + c]);
        const int sl = C.slot[it];
        if (sl < 0) {
            const double d = bh[(size_t)row * kCols + c] - acc;
            r[(size_t)row * kCols + c] = d;
            v[0] += d * d;
        } else {
            scr[(size_t)sl * kCols + c] = acc;
        }
    }
    mm_partial<1>(v, part);
}

__global__ __launch_bounds__(kMmWaves * 64) void k_mm_resid_combine(Chunks C,
                                                                    const double* __restrict__ bh,
                                                                    double* __restrict__ r,
                                                                    const double* __restrict__ scr,
                                                                    double* part) {
    const int c = threadIdx.x & 63;
    double v[1] = {0.0};
    MM_FOR(m, C.nmulti) {
        const int row = C.multi[m];
        double acc = 0.0;
        for (int s = C.mfirst[m]; s < C.mfirst[m + 1]; ++s) acc += scr[(size_t)s * kCols + c];
        const double d = bh[(size_t)row * kCols + c] - acc;
        r[(size_t)row * kCols + c] = d;
        v[0] += d * d;
    }
    mm_partial<1>(v, part);
}

// x out: column c of the caller (input order) = x - mean for c < nrhs.
__global__ __launch_bounds__(kMmWaves * 64) void k_mm_out(int n, const int32_t* __restrict__ sperm,
                                                          const double* __restrict__ x,
                                                          double* __restrict__ xc,
                                                          double* __restrict__ dst, int64_t ld,
                                                          int nrhs, const ScalM* S) {
    const int c = threadIdx.x & 63;
    const double mean = S->sum[c] / (double)n;
    MM_FOR(t, n) {
        const size_t o = (size_t)t * kCols + c;
        const double v = x[o] - mean;
        xc[o] = v;
        if (c < nrhs) dst[(size_t)c * ld + (sperm ? sperm[t] : t)] = v;
    }
}

// ------------------------------------------------------------- serving

// Per-column sums of the admitted right-hand sides (ctl->src, input order).
__global__ __launch_bounds__(kMmWaves * 64) void k_srv_colsum(int n, const ServeCtl* ctl,
                                                              double* part) {
    const int c = threadIdx.x & 63;
    const double* src = ctl->src[c];
    double v[1] = {0.0};
    if (src) {
        MM_FOR(t, n) v[0] += src[t];
    }
    mm_partial<1>(v, part);
}

// Admitted column c: r = src - mean in tree order (tree row t is input
// vertex perm0[t]), x = p0 = p1 = 0 (solve order); partial ||r||^2.
template <class T>
__global__ __launch_bounds__(kMmWaves * 64) void k_srv_admit(int n, const int32_t* __restrict__ perm0,
                                                             const ServeCtl* ctl,
                                                             T* __restrict__ r, T* __restrict__ x,
                                                             T* __restrict__ p0, T* __restrict__ p1,
                                                             const ScalM* S, double* part) {
    const int c = threadIdx.x & 63;
    const double* src = ctl->src[c];
    double v[1] = {0.0};
    if (src) {
        const double mean = S->sum[c] / (double)n;
        MM_FOR(t, n) {
            const size_t o = (size_t)t * kCols + c;
            const double bt = src[perm0[t]] - mean;
            r[o] = (T)bt;
            x[o] = T(0);
            p0[o] = T(0);
            p1[o] = T(0);
            v[0] += bt * bt;
        }
    }
    mm_partial<1>(v, part);
}

// Extracted column c: dst = x - mean(x) in input order (solve row s is
// input vertex sperm[s]; sperm null: the same).  Column sums from S->sum.
template <class T>
__global__ __launch_bounds__(kMmWaves * 64) void k_srv_extract(int n, const int32_t* __restrict__ sperm,
                                                               const ServeCtl* ctl,
                                                               const T* __restrict__ x,
                                                               const ScalM* S) {
    const int c = threadIdx.x & 63;
    double* dst = ctl->dst[c];
    if (!dst) return;
    const double mean = S->sum[c] / (double)n;
    MM_FOR(t, n) dst[sperm ? sperm[t] : t] = (double)x[(size_t)t * kCols + c] - mean;
}

// Per-column sums of a block vector of type T.
template <class T>
__global__ __launch_bounds__(kMmWaves * 64) void k_srv_xsum(int n, const T* __restrict__ x,
                                                            double* part) {
    const int c = threadIdx.x & 63;
    double v[1] = {0.0};
    MM_FOR(t, n) v[0] += (double)x[(size_t)t * kCols + c];
    mm_partial<1>(v, part);
}

}  // namespace lapgpu
