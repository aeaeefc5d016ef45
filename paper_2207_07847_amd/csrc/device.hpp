// Device kernels of the solve (gfx950).  Included by lap.hip only.
//
// The kernels are templates on the value type T of vectors, matrix weights
// and preconditioner coefficients: double for the FP64 solve, float for the
// inner solve of mixed precision.  Every reduction (inner products, sums for
// the mean projection, norms) is carried in double whatever T is.
//
// Vector orders.  The SpMV gathers neighbour values, so the vectors it reads
// and writes (x, p, q and a copy of z) stay in the graph's own vertex order,
// where neighbours of a mesh or grid row are contiguous across a wavefront.
// The preconditioner works in the tree order of the hierarchy (children of
// every aggregate contiguous), so r, z and all coarse-level vectors use it.
// Level 0 converts between the two: the restriction reads q through the
// permutation and the prolongation writes z back through it.
//
// One PCG iteration is this kernel sequence (all on one stream):
//   spmv_p      p = z - zbar + beta p_old;  q = L p;  partial p^T q
//   finish      alpha = rho / p^T q
//   update_up0  x += alpha p;  r -= alpha q;  partial ||r||^2; restriction of
//               r to level 1 fused with the local solves of level-0 aggregates
//   up / group  restriction + local solves of the middle levels
//   tail        one workgroup in LDS: the small levels and the top solve
//   down/group  prolongation + local corrections of the middle levels
//   down0       z on level 0 (both orders); partial sum z, r^T z, sum r
//   finish      zbar, rho, beta, convergence
// Every reduction ends in a one-block finish kernel that adds the per-block
// partials in a fixed order (bitwise reproducible).  Every kernel returns at
// once when the device flag `done` is set, so chunks of iterations captured
// in a hipGraph are replayed without a host round trip per iteration.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.hpp"

namespace lapgpu {

// ------------------------------------------------------------ reductions

template <class V>
__device__ inline V wave_sum1(V v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int N>
__device__ inline void wave_sum(double (&v)[N]) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], off, 64);
}

// Block sum in a fixed order; the result is valid in thread 0.
template <int N, int NT>
__device__ inline void block_sum(double (&v)[N], double* lds) {
    constexpr int NW = NT / 64;
    wave_sum<N>(v);
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < N; ++i) lds[i * NW + wid] = v[i];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double s = 0.0;
            for (int w = 0; w < NW; ++w) s += lds[i * NW + w];
            v[i] = s;
        }
}

// Each block stores its partial sums (value i of block b at part[i*G + b]);
// a one-block finish kernel adds them in block order after the producing
// kernel has completed.  No device-scope fence is needed in the producer:
// the kernel boundary orders the partials before the finish.
template <int N>
__device__ inline void block_partial(double (&v)[N], double* part) {
    __shared__ double lds[N * (kBlock / 64)];
    block_sum<N, kBlock>(v, lds);
    if (threadIdx.x == 0) {
        const int G = gridDim.x;
#pragma unroll
        for (int i = 0; i < N; ++i) part[i * G + blockIdx.x] = v[i];
    }
}

enum FinOp { kFinPq, kFinRr, kFinRho, kFinBsum, kFinBn2, kFinXsum, kFinRes2 };

// Sums the partials of a producer grid of G blocks in a fixed order and
// applies the scalar step of the solver that needs the total.  kFinRho also
// receives the ||r||^2 partials of the update kernel (G2 blocks at part2)
// when G2 > 0 and takes the convergence decision there: the preconditioner
// pass between the update and this point is then wasted only on the final
// iteration, and one launch per iteration is saved.
template <int OP>
__global__ __launch_bounds__(kFinThreads) void k_finish(int G, int n,
                                                        const double* __restrict__ part, int G2,
                                                        const double* __restrict__ part2,
                                                        Scal* S) {
    constexpr int N = (OP == kFinRho) ? 4 : 1;
    constexpr bool loop = OP == kFinPq || OP == kFinRr || OP == kFinRho;
    // the state read below, and the stop flag, are loaded together with the
    // partials: one memory latency for all of them
    const int done = S->done, iter = S->iter, maxit = S->maxit, first = S->first;
    const double rho0 = S->rho, tol2 = S->tol2, bn2 = S->bn2;
    __shared__ double lds[N * (kFinThreads / 64)];
    double v[N];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = 0.0;
    constexpr int nv = (OP == kFinRho) ? 3 : 1;
    // up to kFinUnroll partials of every array per thread, all loads issued
    // before the adds (one memory latency instead of one per partial)
    constexpr int U = kFinUnroll;
    const int tid = threadIdx.x;
    if (G <= U * kFinThreads && G2 <= U * kFinThreads) {
        double a[N][U];
#pragma unroll
        for (int i = 0; i < nv; ++i)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int b = tid + u * kFinThreads;
                a[i][u] = b < G ? part[i * G + b] : 0.0;
            }
        if (OP == kFinRho)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int b = tid + u * kFinThreads;
                a[N - 1][u] = b < G2 ? part2[b] : 0.0;
            }
        // (starting the sum from the first partial rather than from 0.0
        // keeps the compiler from waiting on that load before issuing the
        // others)
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double t = a[i][0];
#pragma unroll
            for (int u = 1; u < U; ++u) t += a[i][u];
            v[i] = t;
        }
    } else {
        for (int i = 0; i < nv; ++i)
            for (int b = tid; b < G; b += kFinThreads) v[i] += part[i * G + b];
        if (OP == kFinRho)
            for (int b = tid; b < G2; b += kFinThreads) v[N - 1] += part2[b];
    }
    if (loop && done) return;
    block_sum<N, kFinThreads>(v, lds);
    if (threadIdx.x != 0) return;
    if (OP == kFinPq) {
        const double pq = v[0];
        S->pq = pq;
        S->iter = iter + 1;
        if (!(pq > 0.0) || !isfinite(pq)) {
            S->done = 3;
            S->alpha = 0.0;  // the step is not taken (x gets no alpha p)
        } else {
            S->alpha = rho0 / pq;
        }
    } else if (OP == kFinRr) {
        S->rr = v[0];
        if (!isfinite(v[0])) S->done = 3;
        else if (v[0] <= tol2 * bn2) S->done = 1;
        else if (iter >= maxit) S->done = 2;
    } else if (OP == kFinRho) {
        const double zbar = v[0] / (double)n;
        const double rho = v[1] - zbar * v[2];
        S->zbar = zbar;
        if (!isfinite(rho)) S->done = 3;
        S->beta = first ? 0.0 : rho / rho0;
        S->first = 0;
        S->rho = rho;
        if (G2 > 0) {
            S->rr = v[3];
            if (!isfinite(v[3])) S->done = 3;
            else if (v[3] <= tol2 * bn2) S->done = 1;
            else if (iter >= maxit) S->done = 2;
        }
    } else if (OP == kFinBsum) {
        S->bsum = v[0];
    } else if (OP == kFinBn2) {
        S->bn2 = v[0];
        S->iter = 0;
        S->first = 1;
        S->alpha = 0.0;
        S->beta = 0.0;
        S->zbar = 0.0;
        S->rr = v[0];
        if (!isfinite(v[0])) S->done = 4;
        else if (v[0] == 0.0) S->done = 1;
        else if (maxit <= 0) S->done = 2;
        else S->done = 0;
    } else if (OP == kFinXsum) {
        S->xsum = v[0];
    } else if (OP == kFinRes2) {
        S->res2 = v[0];
    }
}

// Blocks are dispatched to the eight XCDs in turn (block b runs on XCD
// b mod 8).  The streaming kernels renumber their blocks so that every XCD
// owns one contiguous range of the work: neighbouring rows and aggregates,
// and the vertices their values are gathered from, then share one L2.
__device__ inline int xcd_map(int b, int G) {
    const int x = b & 7, q = G >> 3, rem = G & 7;
    return x * q + (x < rem ? x : rem) + (b >> 3);
}
__device__ inline int xcd_block() { return xcd_map(blockIdx.x, gridDim.x); }

// SpMV grids: the heavy-row blocks come first, in dispatch order over all
// XCDs (they are the longest); the sliced rows follow, renumbered so every
// XCD owns one contiguous range of slices.  Returns the slice block, or -1
// - (heavy block) for a heavy block.
__device__ inline int spmv_block(int nhb) {
    const int b = blockIdx.x;
    if (b < nhb) return -1 - b;
    return xcd_map(b - nhb, gridDim.x - nhb);
}

// Data read once per iteration and not again before the next (the matrix,
// the pair coefficients, the packed coefficients of level groups) is loaded
// non-temporally, so it does not evict the vectors the next kernels re-read.
template <class V>
__device__ inline V ld_nt(const V* p) { return __builtin_nontemporal_load(p); }

// -------------------------------------------------------- Laplacian rows

// One light row of sliced ELL: sum over its slots of w * diff(j), where
// diff(j) is the row's value minus the neighbour's, (L v)_i = sum_j
// w_ij (v_i - v_j) (the Laplacian of Sec. 2.1 with no stored diagonal).
// Slots are taken eight at a time: their column indices and weights are
// loaded first, then the eight neighbour values, so a row costs two memory
// latencies per eight entries instead of two per entry.  The width is the
// same for the whole slice (a wavefront), so the bounds tests are uniform.
template <class T, class F>
__device__ inline T light_row(const Sell<T>& A, int slot, F diff) {
    constexpr int U = 8;
    const int sl = slot >> 6;
    const int base = A.off[sl] + (slot & 63);
    const int W = A.width[sl];
    T acc = T(0);
    for (int k = 0; k < W; k += U) {
        int j[U];
        T w[U], d[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k + u < W) {
                // the matrix streams through once per product: non-temporal,
                // so it does not evict the vectors the next kernels re-read
                j[u] = ld_nt(A.col + base + (k + u) * 64);
                w[u] = ld_nt(A.w + base + (k + u) * 64);
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k + u < W) d[u] = diff(j[u]);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k + u < W) acc += w[u] * d[u];
    }
    return acc;
}

// The same sum for heavy row h, entries strided over `nt` threads from
// thread `t`; each thread returns its share.
template <class T, class F>
__device__ inline T heavy_share(const Sell<T>& A, int h, int t, int nt, F diff) {
    T acc = T(0);
    for (int q = A.hptr[h] + t; q < A.hptr[h + 1]; q += nt)
        acc += ld_nt(A.hw + q) * diff(ld_nt(A.hcol + q));
    return acc;
}

// Heavy block hb: calls fin(row, sum) once per heavy row, from one thread,
// after the row's sum is complete.  One wavefront per row, or the whole
// block for a single row above kHeavyBlockDeg.  `mk(row)` returns the
// neighbour-difference functor of that row.
template <class T, class Mk, class Fin>
__device__ inline void heavy_block(const Sell<T>& A, int hb, Mk mk, Fin fin) {
    __shared__ T red[kBlock / 64];
    const int h0 = A.hblk[hb], h1 = A.hblk[hb + 1];
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (h1 - h0 == 1 && A.hptr[h0 + 1] - A.hptr[h0] > kHeavyBlockDeg) {
        const int row = A.hrow[h0];
        T acc = wave_sum1(heavy_share(A, h0, (int)threadIdx.x, kBlock, mk(row)));
        if (lane == 0) red[wid] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            T tot = red[0];
            for (int w = 1; w < kBlock / 64; ++w) tot += red[w];
            fin(row, tot);
        }
    } else if (h0 + wid < h1) {
        const int h = h0 + wid, row = A.hrow[h];
        const T acc = wave_sum1(heavy_share(A, h, lane, 64, mk(row)));
        if (lane == 0) fin(row, acc);
    }
}

// ------------------------------------------------------ fine-level kernels

// Solve order: p = zn - zbar + beta p_old; q = L p; partial p^T q.  The
// neighbours' p are formed on the fly from zn and p_old, as differences
// (z_i - z_j) + beta (p_i - p_j) in which zbar cancels (nlb: slice blocks;
// the grid holds those and the heavy blocks, see spmv_block).
template <class T>
__global__ __launch_bounds__(kBlock) void k_spmv_p(int nlb, Sell<T> A, const T* __restrict__ zn,
                                                   const T* __restrict__ pold,
                                                   T* __restrict__ pnew, T* __restrict__ q,
                                                   T* __restrict__ x, Scal* S, double* part) {
    // the stop flag is loaded with the scalars the kernel needs (one
    // memory latency before the first data loads, not two)
    const int done = S->done;
    const T beta = (T)S->beta, zbar = (T)S->zbar, alpha = (T)S->alpha;
    if (done) return;
    const int lb = spmv_block(A.nheavyblk);
    double v[1] = {0.0};
    if (lb >= 0) {
        const int slot = lb * kBlock + threadIdx.x;
        if (slot < A.nlight) {
            const int row = A.row ? A.row[slot] : slot;
            const T zi = zn[row], poi = pold[row];
            const T pi = (zi - zbar) + beta * poi;
            const T acc = light_row(A, slot, [&](int j) {
                return (zi - zn[j]) + beta * (poi - pold[j]);
            });
            pnew[row] = pi;
            q[row] = acc;
            x[row] += alpha * poi;
            v[0] = (double)pi * (double)acc;
        }
    } else {
        heavy_block(
            A, -1 - lb,
            [&](int row) {
                const T zi = zn[row], poi = pold[row];
                return [=](int j) { return (zi - zn[j]) + beta * (poi - pold[j]); };
            },
            [&](int row, T acc) {
                const T po = pold[row];
                const T pi = (zn[row] - zbar) + beta * po;
                pnew[row] = pi;
                q[row] = acc;
                x[row] += alpha * po;
                v[0] = (double)pi * (double)acc;
            });
    }
    block_partial<1>(v, part);
}

// One entry of the new search direction, p = (zn - zbar) + beta p_old, as
// one fused multiply-add, so that every kernel that forms it gets the same
// bits.
template <class T>
__device__ inline T p_next(T zn, T zbar, T beta, T po) {
    if constexpr (std::is_same<T, double>::value) return __builtin_fma(beta, po, zn - zbar);
    else return __builtin_fmaf(beta, po, zn - zbar);
}

// p = zn - zbar + beta p_old (solve order), for the SpMV below, and the
// previous step x += alpha p_old.  The blocks past the first ceil(n/kBlock)
// also form the compact copy of p's hot columns, ph[k] = p[hot[k]], from
// the same inputs (p_old is not written here, so the two agree bit for bit).
template <class T>
__global__ __launch_bounds__(kBlock) void k_pupd(int n, const T* __restrict__ zn,
                                                 const T* __restrict__ pold, T* __restrict__ pnew,
                                                 T* __restrict__ x, const Scal* S, int nhot,
                                                 const int32_t* __restrict__ hot,
                                                 T* __restrict__ ph) {
    const int done = S->done;
    const T beta = (T)S->beta, zbar = (T)S->zbar, alpha = (T)S->alpha;
    if (done) return;
    const int b = xcd_block(), nbm = (n + kBlock - 1) / kBlock;
    if (b < nbm) {
        const int t = b * kBlock + threadIdx.x;
        if (t < n) {
            const T po = pold[t];
            pnew[t] = p_next(zn[t], zbar, beta, po);
            x[t] += alpha * po;
        }
    } else {
        const int k = (b - nbm) * kBlock + threadIdx.x;
        if (k < nhot) {
            const int c = hot[k];
            ph[k] = p_next(zn[c], zbar, beta, pold[c]);
        }
    }
}

// The step of the last iteration of a run, x += alpha p_last: each product
// adds the previous iteration's step (it reads that p anyway), so a run that
// stops still owes its last one.  With pcopy, p_last is also copied there
// (a run that continues from a chunk boundary reads its p_old from p[0]).
// Runs after the stop flag is set, so it does not test it.
template <class T>
__global__ __launch_bounds__(kBlock) void k_last_step(int n, T* __restrict__ x,
                                                      const T* __restrict__ plast,
                                                      T* __restrict__ pcopy, const Scal* S) {
    const T alpha = (T)S->alpha;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < n) {
        const T p = plast[t];
        x[t] += alpha * p;
        if (pcopy) pcopy[t] = p;
    }
}

// q = L p with p already formed (one gathered vector per neighbour instead
// of two: the choice for graphs whose gathers are scattered); partial p^T q.
//
// With hot columns (ph non-null), A's column arrays name a hot column c as
// ~rank(c) and its value is read from the compact copy ph[rank]: the most
// referenced columns of a graph without locality then share cache lines,
// which stay in the L2 of every XCD, instead of one line each.
template <class T>
__device__ inline T gather_hot(const T* __restrict__ p, const T* __restrict__ ph, int j) {
    return j >= 0 ? p[j] : ph[~j];
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_spmv_q(int nlb, Sell<T> A, const T* __restrict__ p,
                                                   const T* __restrict__ ph,
                                                   T* __restrict__ q, Scal* S, double* part) {
    if (S->done) return;
    const int lb = spmv_block(A.nheavyblk);
    double v[1] = {0.0};
    if (lb >= 0) {
        const int slot = lb * kBlock + threadIdx.x;
        if (slot < A.nlight) {
            const int row = A.row ? A.row[slot] : slot;
            const T pi = p[row];
            const T acc = light_row(A, slot, [&](int j) { return pi - gather_hot(p, ph, j); });
            q[row] = acc;
            v[0] = (double)pi * (double)acc;
        }
    } else {
        heavy_block(
            A, -1 - lb,
            [&](int row) {
                const T pi = p[row];
                return [=](int j) { return pi - gather_hot(p, ph, j); };
            },
            [&](int row, T acc) {
                q[row] = acc;
                v[0] = (double)p[row] * (double)acc;
            });
    }
    block_partial<1>(v, part);
}

// y = L x (solve order, FP64).
__global__ __launch_bounds__(kBlock) void k_spmv_plain(int nlb, Sell<double> A,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ y) {
    const int lb = spmv_block(A.nheavyblk);
    if (lb >= 0) {
        const int slot = lb * kBlock + threadIdx.x;
        if (slot >= A.nlight) return;
        const int row = A.row ? A.row[slot] : slot;
        const double xi = x[row];
        y[row] = light_row(A, slot, [&](int j) { return xi - x[j]; });
    } else {
        heavy_block(
            A, -1 - lb,
            [&](int row) {
                const double xi = x[row];
                return [=](int j) { return xi - x[j]; };
            },
            [&](int row, double acc) { y[row] = acc; });
    }
}

// r = bh - L x (solve order, FP64; r may be null); partial ||bh - L x||^2.
__global__ __launch_bounds__(kBlock) void k_resid(int nlb, Sell<double> A,
                                                  const double* __restrict__ x,
                                                  const double* __restrict__ bh,
                                                  double* __restrict__ r, double* part) {
    const int lb = spmv_block(A.nheavyblk);
    double v[1] = {0.0};
    if (lb >= 0) {
        const int slot = lb * kBlock + threadIdx.x;
        if (slot < A.nlight) {
            const int row = A.row ? A.row[slot] : slot;
            const double xi = x[row];
            const double d = bh[row] - light_row(A, slot, [&](int j) { return xi - x[j]; });
            if (r) r[row] = d;
            v[0] = d * d;
        }
    } else {
        heavy_block(
            A, -1 - lb,
            [&](int row) {
                const double xi = x[row];
                return [=](int j) { return xi - x[j]; };
            },
            [&](int row, double acc) {
                const double d = bh[row] - acc;
                if (r) r[row] = d;
                v[0] = d * d;
            });
    }
    block_partial<1>(v, part);
}

// --------------------------------------------------- aggregate primitives

// Restriction of level-k values onto aggregate J plus the pair solve of the
// aggregate's sparsifier block: g = C^T r, eta = theta S^-1 g.  The
// children's values are read from rs[t - toff].
template <class T>
__device__ inline void agg_up(const LevelDev<T>& s, const T* rs, int toff, T* __restrict__ rk1,
                              int J) {
    const int b0 = s.cptr[J], b1 = s.cptr[J + 1];
    const T ra = rs[b0 - toff], rb = rs[b0 + 1 - toff];
    T sum = ra + rb, ga = ra, gb = rb;
    for (int t = b0 + 2; t < b1; ++t) {
        const int li = t - 2 * J - 2;
        const T rv = rs[t - toff];
        sum += rv;
        ga += s.l1[li] * rv;
        gb += s.l2[li] * rv;
    }
    const T saa = s.saa[J], sab = s.sab[J], sbb = s.sbb[J];
    s.ea[J] = saa * ga + sab * gb;
    s.eb[J] = sab * ga + sbb * gb;
    rk1[J] = sum;
}

// Restriction and pair solve of aggregate J by one wavefront (aggregates
// with more than kWaveAgg children): lanes stride over the leftovers, the
// sums are reduced across the wavefront, lane 0 writes.
template <class T>
__device__ inline void agg_up_wave(const LevelDev<T>& s, const T* rs, int toff,
                                   T* __restrict__ rk1, int J, int lane) {
    const int b0 = s.cptr[J], b1 = s.cptr[J + 1];
    T sum = T(0), ga = T(0), gb = T(0);
    for (int t = b0 + 2 + lane; t < b1; t += 64) {
        const int li = t - 2 * J - 2;
        const T rv = rs[t - toff];
        sum += rv;
        ga += s.l1[li] * rv;
        gb += s.l2[li] * rv;
    }
    sum = wave_sum1(sum);
    ga = wave_sum1(ga);
    gb = wave_sum1(gb);
    if (lane == 0) {
        const T ra = rs[b0 - toff], rb = rs[b0 + 1 - toff];
        sum += ra + rb;
        ga += ra;
        gb += rb;
        const T saa = s.saa[J], sab = s.sab[J], sbb = s.sbb[J];
        s.ea[J] = saa * ga + sab * gb;
        s.eb[J] = sab * ga + sbb * gb;
        rk1[J] = sum;
    }
}

// Per-aggregate part of a staged up-sweep block: small aggregates a thread
// each, the large ones (listed in LDS) a wavefront each.
template <class T>
__device__ inline void up_aggregates(const LevelDev<T>& s, const T* rs, int t0, T* __restrict__ rk1,
                                     int J0, int J1, int* nbig, int* big) {
    for (int J = J0 + threadIdx.x; J < J1; J += kBlock) {
        if (s.cptr[J + 1] - s.cptr[J] > kWaveAgg) big[atomicAdd(nbig, 1)] = J;
        else agg_up(s, rs, t0, rk1, J);
    }
    __syncthreads();
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = wid; i < *nbig; i += kBlock / 64) agg_up_wave(s, rs, t0, rk1, big[i], lane);
}

// Contributions of child t of aggregate J (first child b0) to the
// restriction sums v = {sum, g_a, g_b} (double: a block-wide reduction
// over a large aggregate follows).
template <class T>
__device__ inline void child_up(const LevelDev<T>& s, int J, int b0, int t, T rv, double* v) {
    v[0] += rv;
    if (t == b0) v[1] += rv;
    else if (t == b0 + 1) v[2] += rv;
    else {
        const int li = t - 2 * J - 2;
        v[1] += (double)s.l1[li] * rv;
        v[2] += (double)s.l2[li] * rv;
    }
}

// Pair solve of aggregate J from the completed sums v.
template <class T>
__device__ inline void agg_solve(const LevelDev<T>& s, int J, const double* v,
                                 T* __restrict__ rk1) {
    const T ga = (T)v[1], gb = (T)v[2];
    const T saa = s.saa[J], sab = s.sab[J], sbb = s.sbb[J];
    s.ea[J] = saa * ga + sab * gb;
    s.eb[J] = sab * ga + sbb * gb;
    rk1[J] = (T)v[0];
}

// Correction of child t of aggregate J (first child b0).
template <class T>
__device__ inline T child_down(const LevelDev<T>& s, int J, int b0, int t, T rt, T yJ, T ea,
                               T eb) {
    if (t == b0) return ea + yJ;
    if (t == b0 + 1) return eb + yJ;
    const int li = t - 2 * J - 2;
    return s.l0[li] * rt + s.l1[li] * ea + s.l2[li] * eb + yJ;
}

// Down-sweep bookkeeping of one block in LDS: the aggregate of every
// staged child and the aggregate's values.
template <class T>
struct DownBlock {
    int32_t own[kCapP];
    int32_t b0[kAggPerBlock];
    T yJ[kAggPerBlock], ea[kAggPerBlock], eb[kAggPerBlock];
};

// Phase one of a down-sweep block: per aggregate, its values and the owner
// marks of its children.  Returns false for a block holding one aggregate
// too large to stage (every thread then handles it directly).
template <class T>
__device__ inline bool down_stage(const LevelDev<T>& s, const T* __restrict__ yk1, int J0, int J1,
                                  int t0, int len, DownBlock<T>& D) {
    if (len > kCapP) return false;
    for (int j = threadIdx.x; j < J1 - J0; j += kBlock) {
        const int J = J0 + j;
        const int b0 = s.cptr[J], b1 = s.cptr[J + 1];
        D.b0[j] = b0;
        D.yJ[j] = yk1[J];
        D.ea[j] = s.ea[J];
        D.eb[j] = s.eb[J];
        for (int t = b0; t < b1; ++t) D.own[t - t0] = j;
    }
    __syncthreads();
    return true;
}

// r -= alpha q (tree order, q read through the permutation); partial
// ||r||^2; restriction of r to level 1 fused with the local solves of the
// level-0 aggregates.  (x += alpha p is taken by the next product, which
// reads p anyway.)  The element-wise part runs over the block's children
// with coalesced accesses and leaves the new residuals in LDS for the
// per-aggregate part.
template <class T>
__global__ __launch_bounds__(kBlock) void k_update_up0(LevelDev<T> s0,
                                                       const int32_t* __restrict__ perm,
                                                       T* __restrict__ r,
                                                       const T* __restrict__ q,
                                                       T* __restrict__ r1, Scal* S, double* part,
                                                       int do_update) {
    __shared__ T rs[kCapP];
    __shared__ double red[4 * (kBlock / 64)];
    __shared__ int nbig, big[kAggPerBlock];
    const int done = S->done;
    const T alpha = (T)S->alpha;
    const int b = xcd_block();
    const int J0 = s0.bst[b], J1 = s0.bst[b + 1];
    if (done) return;
    const int t0 = s0.cptr[J0], len = s0.cptr[J1] - t0;
    double rr = 0.0;
    if (len <= kCapP) {
        if (threadIdx.x == 0) nbig = 0;
        for (int i = threadIdx.x; i < len; i += kBlock) {
            const int t = t0 + i;
            T rt = r[t];
            if (do_update) {
                rt -= alpha * q[perm ? perm[t] : t];
                r[t] = rt;
                rr += (double)rt * rt;
            }
            rs[i] = rt;
        }
        __syncthreads();
        up_aggregates(s0, rs, t0, r1, J0, J1, &nbig, big);
        if (!do_update) return;
        double v[1] = {rr};
        block_partial<1>(v, part);
        return;
    }
    // one aggregate with more children than LDS holds
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < len; i += kBlock) {
        const int t = t0 + i;
        T rt = r[t];
        if (do_update) {
            rt -= alpha * q[perm ? perm[t] : t];
            r[t] = rt;
            v[3] += (double)rt * rt;
        }
        child_up(s0, J0, t0, t, rt, v);
    }
    block_sum<4, kBlock>(v, red);
    if (threadIdx.x == 0) {
        agg_solve(s0, J0, v, r1);
        if (do_update) part[blockIdx.x] = v[3];
    }
}

// z on the fine level, written through the permutation in input order for
// the next SpMV; partial sums of z, r z and r (tree order).
template <class T>
__global__ __launch_bounds__(kBlock) void k_down0(LevelDev<T> s0, const int32_t* __restrict__ perm,
                                                  const T* __restrict__ r, T* __restrict__ zn,
                                                  const T* __restrict__ y1, Scal* S,
                                                  double* part) {
    __shared__ DownBlock<T> D;
    const int done = S->done;
    const int b = xcd_block();
    const int J0 = s0.bst[b], J1 = s0.bst[b + 1];
    if (done) return;
    const int t0 = s0.cptr[J0], len = s0.cptr[J1] - t0;
    double v[3] = {0.0, 0.0, 0.0};
    if (down_stage(s0, y1, J0, J1, t0, len, D)) {
        for (int i = threadIdx.x; i < len; i += kBlock) {
            const int t = t0 + i, j = D.own[i];
            const T rt = r[t];
            const T zt = child_down(s0, J0 + j, D.b0[j], t, rt, D.yJ[j], D.ea[j], D.eb[j]);
            zn[perm ? perm[t] : t] = zt;
            v[0] += zt;
            v[1] += (double)rt * zt;
            v[2] += rt;
        }
    } else {
        const T yJ = y1[J0], ea = s0.ea[J0], eb = s0.eb[J0];
        for (int i = threadIdx.x; i < len; i += kBlock) {
            const int t = t0 + i;
            const T rt = r[t];
            const T zt = child_down(s0, J0, t0, t, rt, yJ, ea, eb);
            zn[perm ? perm[t] : t] = zt;
            v[0] += zt;
            v[1] += (double)rt * zt;
            v[2] += rt;
        }
    }
    block_partial<3>(v, part);
}

// Levels 0 and 1 together.  Block b owns the level-2 nodes [A0, A1) of a
// partition aligned to level-1 aggregates (Blk01): their
// level-1 children [J0, J1) and level-0 grandchildren [t0, t1) are
// contiguous and staged in LDS, so one launch does the update, the level-0
// restriction and the level-1 restriction (and the down kernel both
// prolongations).  Used when every block fits (kAggPerBlock level-1 nodes,
// kCapP level-0 positions).
template <class T>
__global__ __launch_bounds__(kBlock) void k_update_up01(LevelDev<T> s0, LevelDev<T> s1,
                                                        const Blk01* __restrict__ blk,
                                                        const int32_t* __restrict__ perm,
                                                        T* __restrict__ r,
                                                        const T* __restrict__ q,
                                                        T* __restrict__ r2, Scal* S, double* part,
                                                        int do_update) {
    __shared__ T rs[kCapP];
    __shared__ T r1s[kAggPerBlock];
    __shared__ int nbig, big[kAggPerBlock];
    const int done = S->done;
    const T alpha = (T)S->alpha;
    const Blk01 bd = blk[xcd_block()];
    if (done) return;
    const int A0 = bd.A0, A1 = bd.A1, J0 = bd.J0, J1 = bd.J1, t0 = bd.t0, len = bd.t1 - bd.t0;
    double rr = 0.0;
    if (threadIdx.x == 0) nbig = 0;
    for (int i = threadIdx.x; i < len; i += kBlock) {
        const int t = t0 + i;
        T rt = r[t];
        if (do_update) {
            rt -= alpha * q[perm ? perm[t] : t];
            r[t] = rt;
            rr += (double)rt * rt;
        }
        rs[i] = rt;
    }
    __syncthreads();
    // level 0 -> 1: restricted values to LDS (and to r1 for the down-sweep)
    for (int J = J0 + threadIdx.x; J < J1; J += kBlock) {
        if (s0.cptr[J + 1] - s0.cptr[J] > kWaveAgg) big[atomicAdd(&nbig, 1)] = J;
        else agg_up(s0, rs, t0, s1.r, J);
    }
    __syncthreads();
    {
        const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
        for (int i = wid; i < nbig; i += kBlock / 64) agg_up_wave(s0, rs, t0, s1.r, big[i], lane);
    }
    __syncthreads();
    for (int J = J0 + threadIdx.x; J < J1; J += kBlock) r1s[J - J0] = s1.r[J];
    if (threadIdx.x == 0) nbig = 0;
    __syncthreads();
    // level 1 -> 2
    up_aggregates(s1, r1s, J0, r2, A0, A1, &nbig, big);
    if (!do_update) return;
    double v[1] = {rr};
    block_partial<1>(v, part);
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_down01(LevelDev<T> s0, LevelDev<T> s1,
                                                   const Blk01* __restrict__ blk,
                                                   const int32_t* __restrict__ perm,
                                                   const T* __restrict__ r, T* __restrict__ zn,
                                                   const T* __restrict__ y2, Scal* S,
                                                   double* part) {
    static_assert(kAggPerBlock <= kBlock && kCapP % kBlock == 0, "one level-1 node per thread");
    constexpr int R = kCapP / kBlock;
    __shared__ DownBlock<T> D;
    __shared__ T y1s[kAggPerBlock];
    const int done = S->done;
    const Blk01 bd = blk[xcd_block()];
    if (done) return;
    const int A0 = bd.A0, A1 = bd.A1, J0 = bd.J0, J1 = bd.J1, t0 = bd.t0, len = bd.t1 - bd.t0;
    const int tid = threadIdx.x;
    // The loads of each level-1 node's children range and pair corrections
    // do not depend on the level-2 -> 1 step: issued first, they overlap it.
    const bool has1 = tid < J1 - J0;
    int c0 = 0, c1 = 0;
    T ea0 = T(0), eb0 = T(0);
    if (has1) {
        c0 = s0.cptr[J0 + tid];
        c1 = s0.cptr[J0 + tid + 1];
        ea0 = s0.ea[J0 + tid];
        eb0 = s0.eb[J0 + tid];
    }
    // level 2 -> 1 into LDS
    for (int A = A0 + tid; A < A1; A += kBlock) {
        const int a0 = s1.cptr[A], a1 = s1.cptr[A + 1];
        const T yA = y2[A], ea = s1.ea[A], eb = s1.eb[A];
        for (int J = a0; J < a1; ++J) y1s[J - J0] = child_down(s1, A, a0, J, s1.r[J], yA, ea, eb);
    }
    __syncthreads();
    // level 1 -> 0, z with its reductions
    if (has1) {
        D.b0[tid] = c0;
        D.yJ[tid] = y1s[tid];
        D.ea[tid] = ea0;
        D.eb[tid] = eb0;
        for (int t = c0; t < c1; ++t) D.own[t - t0] = tid;
    }
    __syncthreads();
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const int i = tid + u * kBlock;
        if (i < len) {
            const int t = t0 + i, j = D.own[i];
            const T rt = r[t];
            const T zt = child_down(s0, J0 + j, D.b0[j], t, rt, D.yJ[j], D.ea[j], D.eb[j]);
            zn[perm ? perm[t] : t] = zt;
            v[0] += zt;
            v[1] += (double)rt * zt;
            v[2] += rt;
        }
    }
    block_partial<3>(v, part);
}

// Without a hierarchy below the fine level: the r update only.
template <class T>
__global__ __launch_bounds__(kBlock) void k_update_none(int n, const int32_t* __restrict__ perm,
                                                        T* __restrict__ r,
                                                        const T* __restrict__ q, Scal* S,
                                                        double* part) {
    if (S->done) return;
    const T alpha = (T)S->alpha;
    const int t = xcd_block() * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (t < n) {
        const T rt = r[t] - alpha * q[perm ? perm[t] : t];
        r[t] = rt;
        v[0] = (double)rt * rt;
    }
    block_partial<1>(v, part);
}

// Plain CG: z = r (both orders) with the down0 reductions.
template <class T>
__global__ __launch_bounds__(kBlock) void k_prec_none(int n, const int32_t* __restrict__ perm,
                                                      const T* __restrict__ r, T* __restrict__ z,
                                                      T* __restrict__ zn, Scal* S, double* part) {
    if (S->done) return;
    const int t = xcd_block() * kBlock + threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    if (t < n) {
        const T rt = r[t];
        z[t] = rt;
        zn[perm ? perm[t] : t] = rt;
        v[0] = rt;
        v[1] = (double)rt * rt;
        v[2] = rt;
    }
    block_partial<3>(v, part);
}

// One-level hierarchy (the fine level is the top, at most kTopMax nodes):
// the MSP is theta_0 pinv(L) = pinv(L), applied by one workgroup, which also
// does the finish step of the down0 reductions itself.
template <class T>
__global__ __launch_bounds__(kBlock) void k_top_only(int n, const int32_t* __restrict__ perm,
                                                     const T* __restrict__ tp,
                                                     const T* __restrict__ r, T* __restrict__ z,
                                                     T* __restrict__ zn, Scal* S) {
    if (S->done) return;
    __shared__ double lds[3 * (kBlock / 64)];
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += kBlock) {
        T acc = T(0);
        for (int j = 0; j < n; ++j) acc += tp[i * n + j] * r[j];
        z[i] = acc;
        zn[perm ? perm[i] : i] = acc;
        v[0] += acc;
        v[1] += (double)r[i] * acc;
        v[2] += r[i];
    }
    block_sum<3, kBlock>(v, lds);
    if (threadIdx.x == 0) {
        const double zbar = v[0] / (double)n;
        const double rho = v[1] - zbar * v[2];
        S->zbar = zbar;
        if (!isfinite(rho)) S->done = 3;
        S->beta = S->first ? 0.0 : rho / S->rho;
        S->first = 0;
        S->rho = rho;
    }
}

// ------------------------------------------------------ per-level kernels

template <class T>
__global__ __launch_bounds__(kBlock) void k_up(LevelDev<T> s, const T* __restrict__ rk,
                                               T* __restrict__ rk1, const Scal* S) {
    __shared__ T rs[kCapP];
    __shared__ double red[3 * (kBlock / 64)];
    __shared__ int nbig, big[kAggPerBlock];
    const int done = S->done;
    const int b = xcd_block();
    const int J0 = s.bst[b], J1 = s.bst[b + 1];
    if (done) return;
    const int t0 = s.cptr[J0], len = s.cptr[J1] - t0;
    if (len <= kCapP) {
        if (threadIdx.x == 0) nbig = 0;
        for (int i = threadIdx.x; i < len; i += kBlock) rs[i] = rk[t0 + i];
        __syncthreads();
        up_aggregates(s, rs, t0, rk1, J0, J1, &nbig, big);
        return;
    }
    double v[3] = {0.0, 0.0, 0.0};
    for (int t = t0 + threadIdx.x; t < t0 + len; t += kBlock) child_up(s, J0, t0, t, rk[t], v);
    block_sum<3, kBlock>(v, red);
    if (threadIdx.x == 0) agg_solve(s, J0, v, rk1);
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_down(LevelDev<T> s, const T* __restrict__ rk,
                                                 T* __restrict__ yk, const T* __restrict__ yk1,
                                                 const Scal* S) {
    __shared__ DownBlock<T> D;
    const int done = S->done;
    const int b = xcd_block();
    const int J0 = s.bst[b], J1 = s.bst[b + 1];
    if (done) return;
    const int t0 = s.cptr[J0], len = s.cptr[J1] - t0;
    if (down_stage(s, yk1, J0, J1, t0, len, D)) {
        for (int i = threadIdx.x; i < len; i += kBlock) {
            const int t = t0 + i, j = D.own[i];
            yk[t] = child_down(s, J0 + j, D.b0[j], t, rk[t], D.yJ[j], D.ea[j], D.eb[j]);
        }
    } else {
        const T yJ = yk1[J0], ea = s.ea[J0], eb = s.eb[J0];
        for (int t = t0 + threadIdx.x; t < t0 + len; t += kBlock)
            yk[t] = child_down(s, J0, t0, t, rk[t], yJ, ea, eb);
    }
}

// ------------------------------------------------------- grouped levels

// Flat copy global -> LDS with eight loads in flight per thread (NT:
// non-temporal loads, for data read once per iteration).
template <class T, bool NT = false>
__device__ inline void stage_copy(T* __restrict__ dst, const T* __restrict__ src, int len) {
    constexpr int U = 8, B = kGrpThreads;
    int i = threadIdx.x;
    for (; i + (U - 1) * B < len; i += U * B) {
        T t[U];
#pragma unroll
        for (int u = 0; u < U; ++u) t[u] = NT ? ld_nt(src + i + u * B) : src[i + u * B];
#pragma unroll
        for (int u = 0; u < U; ++u) dst[i + u * B] = t[u];
    }
    for (; i < len; i += B) dst[i] = NT ? ld_nt(src + i) : src[i];
}

// Staging of up to four global ranges into LDS at once: segment k copies
// len[k] values from src[k] to dst[k] (the first nnt segments with
// non-temporal loads).  The ranges are walked as one concatenated index
// space, U loads in flight per thread, so every load of every segment is
// issued before the first LDS write waits for data: one memory latency
// instead of one per range.
template <class T, int U, int NTH>
struct StageSet {
    const T* src[4];
    T* dst[4];
    int end[4];  // running ends of the segments in the concatenated space
    int nnt;
};
template <class T, int U, int NTH>
__device__ inline void stage_set(const StageSet<T, U, NTH>& S) {
    // segment selection by comparisons and selects only: an array indexed
    // at run time would be placed in scratch memory
    const int e0 = S.end[0], e1 = S.end[1], e2 = S.end[2], total = S.end[3];
    const int nnt = S.nnt;
    for (int base = threadIdx.x; base < total; base += U * NTH) {
        T t[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * NTH;
            if (i < total) {
                const int k = i < e0 ? 0 : i < e1 ? 1 : i < e2 ? 2 : 3;
                const T* p = k == 0 ? S.src[0] + i
                           : k == 1 ? S.src[1] + (i - e0)
                           : k == 2 ? S.src[2] + (i - e1)
                                    : S.src[3] + (i - e2);
                t[u] = k < nnt ? ld_nt(p) : *p;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * NTH;
            if (i < total) {
                T* d = i < e0 ? S.dst[0] + i
                     : i < e1 ? S.dst[1] + (i - e0)
                     : i < e2 ? S.dst[2] + (i - e1)
                              : S.dst[3] + (i - e2);
                *d = t[u];
            }
        }
    }
}

// Per-block bookkeeping of a group (level ranges and LDS layout) lives in
// LDS: it is indexed by the level inside loops, and a runtime-indexed
// private array would be placed in scratch memory.
struct GrpBlock {
    int32_t st[kMaxGroupLevels + 1];
    int32_t cnt[kMaxGroupLevels + 1];
    int32_t off[2];  // pack and scratch offsets of the block
    GrpLayout L;
};

// The block's level ranges and its pack and scratch offsets are loaded by
// the lanes of wavefront 0 in one load instruction (lane j <= m: first node
// of level j; lane m+1+j: its end; lanes 62, 63: pack and scratch offsets),
// together with the stop flag; false: the solve has stopped.  (Everything
// lands in GrpBlock: static LDS stays small, and with it the occupancy.)
template <class T>
__device__ inline bool grp_setup(const GroupDev<T>& G, int m, GrpBlock& B,
                                 const int32_t* pack_off, const Scal* S) {
    static_assert(kGrpThreads > 64 && 2 * kMaxGroupLevels + 1 < 62, "setup lanes");
    const int done = S->done;
    const int b = blockIdx.x, nb1 = G.nblocks + 1, tid = threadIdx.x;
    if (tid < 64) {
        const int32_t* src = G.D;
        int32_t* dst = nullptr;
        if (tid <= m) {
            src = G.D + tid * nb1 + b;
            dst = B.st + tid;
        } else if (tid <= 2 * m + 1) {
            src = G.D + (tid - m - 1) * nb1 + b + 1;
            dst = B.cnt + (tid - m - 1);
        } else if (tid >= 62) {
            src = (tid == 62 ? pack_off : G.xoff) + b;
            dst = B.off + (tid - 62);
        }
        const int32_t v = *src;
        if (dst) *dst = v;
    }
    if (done) return false;
    __syncthreads();
    if (tid == 0) {
        for (int j = 0; j <= m; ++j) B.cnt[j] -= B.st[j];
        grp_layout(m, B.cnt, (int)(sizeof(T) / sizeof(int32_t)), B.L);
    }
    __syncthreads();
    return true;
}

// Up-sweep of a level group [k0, k1): level-k0 residuals in, level-k1
// residuals out; intermediate residuals and pair corrections go to the
// block's scratch chunk for the down-sweep.
template <class T>
__global__ __launch_bounds__(kGrpThreads) void k_up_grp(GroupDev<T> G, const Scal* S) {
    extern __shared__ __align__(16) unsigned char smem[];
    T* sm = reinterpret_cast<T*>(smem);
    const int m = G.k1 - G.k0, tid = threadIdx.x, nth = blockDim.x;
    __shared__ GrpBlock B;
    if (!grp_setup(G, m, B, G.uoff, S)) return;
    const int32_t* off = B.off;
    const int32_t* st = B.st;
    const int32_t* cnt = B.cnt;
    const GrpLayout& L = B.L;
    {
        StageSet<T, 16, kGrpThreads> ss;
        ss.src[0] = G.upack + off[0];
        ss.dst[0] = sm;
        ss.end[0] = L.ulen;
        ss.src[1] = G.r_in + st[0];
        ss.dst[1] = sm + L.ur[0];
        ss.end[1] = ss.end[2] = ss.end[3] = L.ulen + cnt[0];
        ss.src[2] = ss.src[3] = ss.src[1];
        ss.dst[2] = ss.dst[3] = ss.dst[1];
        ss.nnt = 1;
        stage_set(ss);
    }
    __syncthreads();
    T* scr = G.scr + off[1];
    for (int j = 0; j < m; ++j) {
        const int na = cnt[j + 1], nl = cnt[j] - 2 * na;
        const int* cp = reinterpret_cast<const int*>(sm + L.ucp[j]);
        const T* sa = sm + L.us[j];
        const T* l1 = sm + L.ul[j];
        const T* l2 = l1 + nl;
        const T* rk = sm + L.ur[j];
        T* rk1 = sm + L.ur[j + 1];
        T* eo = scr + L.xe[j];
        T* ro = (j + 1 < m) ? scr + L.xr[j + 1] : G.r_top + st[m];
        for (int J = tid; J < na; J += nth) {
            const int b0 = cp[J], b1 = cp[J + 1];
            const T ra = rk[b0], rb = rk[b0 + 1];
            T sum = ra + rb, ga = ra, gb = rb;
            for (int c = b0 + 2; c < b1; ++c) {
                const int li = c - 2 * J - 2;
                const T rv = rk[c];
                sum += rv;
                ga += l1[li] * rv;
                gb += l2[li] * rv;
            }
            const T saa = sa[J], sab = sa[na + J], sbb = sa[2 * na + J];
            eo[J] = saa * ga + sab * gb;
            eo[na + J] = sab * ga + sbb * gb;
            rk1[J] = sum;
            ro[J] = sum;
        }
        __syncthreads();
    }
}

// Down-sweep of a level group: level-k1 corrections in, level-k0 out.
template <class T>
__global__ __launch_bounds__(kGrpThreads) void k_down_grp(GroupDev<T> G, const Scal* S) {
    extern __shared__ __align__(16) unsigned char smem[];
    T* sm = reinterpret_cast<T*>(smem);
    const int m = G.k1 - G.k0, tid = threadIdx.x, nth = blockDim.x;
    __shared__ GrpBlock B;
    if (!grp_setup(G, m, B, G.doff, S)) return;
    const int32_t* off = B.off;
    const int32_t* st = B.st;
    const int32_t* cnt = B.cnt;
    const GrpLayout& L = B.L;
    {
        StageSet<T, 16, kGrpThreads> ss;
        ss.src[0] = G.dpack + off[0];
        ss.dst[0] = sm;
        ss.end[0] = L.dlen;
        ss.src[1] = G.scr + off[1];
        ss.dst[1] = sm + L.dx;
        ss.end[1] = ss.end[0] + L.xlen;
        ss.src[2] = G.r_in + st[0];
        ss.dst[2] = sm + L.dr0;
        ss.end[2] = ss.end[1] + cnt[0];
        ss.src[3] = G.y_top + st[m];
        ss.dst[3] = sm + L.dy[m];
        ss.end[3] = ss.end[2] + cnt[m];
        ss.nnt = 1;
        stage_set(ss);
    }
    __syncthreads();
    for (int j = m - 1; j >= 0; --j) {
        const int na = cnt[j + 1], nl = cnt[j] - 2 * na;
        const int* cp = reinterpret_cast<const int*>(sm + L.dcp[j]);
        const T* l0 = sm + L.dl[j];
        const T* l1 = l0 + nl;
        const T* l2 = l1 + nl;
        const T* rk = j == 0 ? sm + L.dr0 : sm + L.dx + L.xr[j];
        const T* e = sm + L.dx + L.xe[j];
        T* yk = sm + L.dy[j];
        const T* yk1 = sm + L.dy[j + 1];
        for (int J = tid; J < na; J += nth) {
            const int b0 = cp[J], b1 = cp[J + 1];
            const T yJ = yk1[J], ea = e[J], eb = e[na + J];
            yk[b0] = ea + yJ;
            yk[b0 + 1] = eb + yJ;
            for (int c = b0 + 2; c < b1; ++c) {
                const int li = c - 2 * J - 2;
                yk[c] = l0[li] * rk[c] + l1[li] * ea + l2[li] * eb + yJ;
            }
        }
        __syncthreads();
    }
    const T* y0 = sm + L.dy[0];
    T* out = G.y_out + st[0];
    for (int t = tid; t < cnt[0]; t += nth) out[t] = y0[t];
}

// ------------------------------------------------------------ coarse tail

// Levels kt .. top in one workgroup, entirely in LDS: the coefficients of
// those levels are staged from one packed device buffer with a coalesced
// copy, then restriction + local solves run upwards, theta_top pinv(L_top)
// on the top, prolongation + corrections back down to level kt.  An
// aggregate with many children (a hub of a power-law graph) is reduced by
// the whole workgroup after the others of its level.
template <class T>
__global__ __launch_bounds__(kTailThreads) void k_tail(const TailDesc* __restrict__ Dg, TailArgs ta,
                                                       const T* __restrict__ pack,
                                                       const T* __restrict__ r_kt,
                                                       T* __restrict__ y_kt, const Scal* S) {
    extern __shared__ __align__(16) unsigned char smem[];
    T* sm = reinterpret_cast<T*>(smem);
    __shared__ double red[3 * (kTailThreads / 64)];
    // the descriptor is read at every level: one copy into LDS up front
    // instead of a dependent global load per step
    __shared__ TailDesc Dl;
    const TailDesc* D = &Dl;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int npack = ta.npack, nsteps = ta.nsteps;
    // the stop flag is tested after the staging loads are issued, so its
    // latency overlaps theirs (a stopped solve stages for nothing)
    const int done = S->done;
    {
        constexpr int W = (int)(sizeof(TailDesc) / sizeof(int32_t));
        static_assert(W <= kTailThreads, "one word per thread");
        const int32_t w = reinterpret_cast<const int32_t*>(Dg)[tid < W ? tid : W - 1];
        StageSet<T, 16, kTailThreads> ss;
        ss.src[0] = pack;
        ss.dst[0] = sm;
        ss.end[0] = npack;
        ss.src[1] = ss.src[2] = ss.src[3] = r_kt;
        ss.dst[1] = ss.dst[2] = ss.dst[3] = sm + ta.r0;
        ss.end[1] = ss.end[2] = ss.end[3] = npack + ta.n0;
        ss.nnt = 0;
        stage_set(ss);
        if (tid < W) reinterpret_cast<int32_t*>(&Dl)[tid] = w;
    }
    if (done) return;
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
        const TailStep t = D->st[s];
        const int* cp = reinterpret_cast<const int*>(sm + t.cptr);
        const T* rk = sm + D->r[s];
        T* rk1 = sm + D->r[s + 1];
        for (int J = tid; J < t.nc; J += nth) {
            const int b0 = cp[J], b1 = cp[J + 1];
            if (b1 - b0 > kTailBig) continue;
            const T ra = rk[b0], rb = rk[b0 + 1];
            T sum = ra + rb, ga = ra, gb = rb;
            for (int c = b0 + 2; c < b1; ++c) {
                const int li = c - 2 * J - 2;
                const T rv = rk[c];
                sum += rv;
                ga += sm[t.l1 + li] * rv;
                gb += sm[t.l2 + li] * rv;
            }
            const T saa = sm[t.saa + J], sab = sm[t.sab + J], sbb = sm[t.sbb + J];
            sm[t.ea + J] = saa * ga + sab * gb;
            sm[t.eb + J] = sab * ga + sbb * gb;
            rk1[J] = sum;
        }
        for (int bi = 0; bi < t.nbig; ++bi) {
            const int J = reinterpret_cast<const int*>(sm + t.big)[bi];
            const int b0 = cp[J], b1 = cp[J + 1];
            double v[3] = {0.0, 0.0, 0.0};
            for (int c = b0 + tid; c < b1; c += nth) {
                const T rv = rk[c];
                v[0] += rv;
                if (c == b0) v[1] += rv;
                else if (c == b0 + 1) v[2] += rv;
                else {
                    const int li = c - 2 * J - 2;
                    v[1] += (double)sm[t.l1 + li] * rv;
                    v[2] += (double)sm[t.l2 + li] * rv;
                }
            }
            block_sum<3, kTailThreads>(v, red);
            if (tid == 0) {
                const T ga = (T)v[1], gb = (T)v[2];
                const T saa = sm[t.saa + J], sab = sm[t.sab + J], sbb = sm[t.sbb + J];
                sm[t.ea + J] = saa * ga + sab * gb;
                sm[t.eb + J] = sab * ga + sbb * gb;
                rk1[J] = (T)v[0];
            }
            __syncthreads();
        }
        __syncthreads();
    }
    {
        const int nt = D->nt;
        const T* rT = sm + D->r[nsteps];
        T* yT = sm + D->y[nsteps];
        const T* tp = sm + D->pinv;
        for (int i = tid; i < nt; i += nth) {
            T acc = T(0);
            for (int j = 0; j < nt; ++j) acc += tp[i * nt + j] * rT[j];
            yT[i] = acc;
        }
        __syncthreads();
    }
    for (int s = nsteps - 1; s >= 0; --s) {
        const TailStep t = D->st[s];
        const int* cp = reinterpret_cast<const int*>(sm + t.cptr);
        const T* rk = sm + D->r[s];
        T* yk = sm + D->y[s];
        const T* yk1 = sm + D->y[s + 1];
        for (int J = tid; J < t.nc; J += nth) {
            const int b0 = cp[J], b1 = cp[J + 1];
            if (b1 - b0 > kTailBig) continue;
            const T yJ = yk1[J], ea = sm[t.ea + J], eb = sm[t.eb + J];
            yk[b0] = ea + yJ;
            yk[b0 + 1] = eb + yJ;
            for (int c = b0 + 2; c < b1; ++c) {
                const int li = c - 2 * J - 2;
                yk[c] = sm[t.l0 + li] * rk[c] + sm[t.l1 + li] * ea + sm[t.l2 + li] * eb + yJ;
            }
        }
        for (int bi = 0; bi < t.nbig; ++bi) {
            const int J = reinterpret_cast<const int*>(sm + t.big)[bi];
            const int b0 = cp[J], b1 = cp[J + 1];
            const T yJ = yk1[J], ea = sm[t.ea + J], eb = sm[t.eb + J];
            for (int c = b0 + tid; c < b1; c += nth) {
                if (c == b0) yk[c] = ea + yJ;
                else if (c == b0 + 1) yk[c] = eb + yJ;
                else {
                    const int li = c - 2 * J - 2;
                    yk[c] = sm[t.l0 + li] * rk[c] + sm[t.l1 + li] * ea + sm[t.l2 + li] * eb + yJ;
                }
            }
        }
        __syncthreads();
    }
    {
        const int n0 = nsteps > 0 ? D->st[0].nk : D->nt;
        const T* y0 = sm + D->y[0];
        for (int i = tid; i < n0; i += nth) y_kt[i] = y0[i];
    }
}

// ------------------------------------------ FGMRES on the expanded system
//
// Expanded vectors (Sec. 2.2) hold the levels one after the other, each in
// its tree numbering: level 0 has n values, level k+1 follows level k.
// P(mu)^T y has level 0 = y and level k+1 = -mu times the sums of level k
// over each aggregate's children.

// Level 0 of P(mu)^T y: y (solve order) into tree order.
__global__ __launch_bounds__(kBlock) void k_fg_level0(int n, const int32_t* __restrict__ t2s,
                                                      const double* __restrict__ y,
                                                      double* __restrict__ w) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < n) w[t] = y[t2s ? t2s[t] : t];
}

// Level k+1 from level k: out[J] = scale * sum over children c of J of in[c].
__global__ __launch_bounds__(kBlock) void k_fg_restrict(int nc, const int32_t* __restrict__ cptr,
                                                        const double* __restrict__ in,
                                                        double* __restrict__ out,
                                                        double scale) {
    const int J = blockIdx.x * kBlock + threadIdx.x;
    if (J >= nc) return;
    double s = 0.0;
    for (int c = cptr[J]; c < cptr[J + 1]; ++c) s += in[c];
    out[J] = scale * s;
}

// Partial dot products of w with k basis vectors: block (x, i) adds the
// rows x*kBlock + tid + j*gridDim.x*kBlock of V_i . w into part[i*G + x].
__global__ __launch_bounds__(kBlock) void k_fg_mdot(int64_t nt, const double* __restrict__ V,
                                                    int64_t ldv, const double* __restrict__ w,
                                                    double* __restrict__ part) {
    __shared__ double lds[kBlock / 64];
    const int i = blockIdx.y, G = gridDim.x;
    const double* v = V + (int64_t)i * ldv;
    double acc[1] = {0.0};
    for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < nt; r += (int64_t)G * kBlock)
        acc[0] += v[r] * w[r];
    block_sum<1, kBlock>(acc, lds);
    if (threadIdx.x == 0) part[(int64_t)i * G + blockIdx.x] = acc[0];
}

// out[i] = sum of the G partials of dot i, in block order (block i).
__global__ __launch_bounds__(kBlock) void k_fg_dot_finish(int G, const double* __restrict__ part,
                                                          double* __restrict__ out) {
    __shared__ double lds[kBlock / 64];
    const int i = blockIdx.x;
    double acc[1] = {0.0};
    for (int b = threadIdx.x; b < G; b += kBlock) acc[0] += part[(int64_t)i * G + b];
    block_sum<1, kBlock>(acc, lds);
    if (threadIdx.x == 0) out[i] = acc[0];
}

// w += sign * sum_i h[i] V_i (k vectors, coefficients on the device).
__global__ __launch_bounds__(kBlock) void k_fg_maxpy(int64_t nt, int k,
                                                     const double* __restrict__ V, int64_t ldv,
                                                     const double* __restrict__ h, double sign,
                                                     double* __restrict__ w) {
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r >= nt) return;
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += h[i] * V[(int64_t)i * ldv + r];
    w[r] += sign * s;
}

// y = a * x + c * y (c = 0: y = a * x, whatever y held)
__global__ __launch_bounds__(kBlock) void k_fg_axpby(int64_t nt, double a,
                                                     const double* __restrict__ x, double c,
                                                     double* __restrict__ y) {
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r < nt) y[r] = c == 0.0 ? a * x[r] : a * x[r] + c * y[r];
}

// ------------------------------------------------- solve set-up and finish

__global__ __launch_bounds__(kBlock) void k_sum(int n, const double* __restrict__ a,
                                                double* part) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    double v[1] = {t < n ? a[t] : 0.0};
    block_partial<1>(v, part);
}

// PCG start for the right-hand side rhs (solve order, FP64): r = rhs -
// mean(rhs) in tree order (tree position t reads solve position perm[t],
// perm null: the same position), x = p0 = p1 = 0; partial ||r||^2.
template <class T>
__global__ __launch_bounds__(kBlock) void k_init(int n, const int32_t* __restrict__ perm,
                                                 const double* __restrict__ rhs,
                                                 T* __restrict__ r, T* __restrict__ x,
                                                 T* __restrict__ p0, T* __restrict__ p1,
                                                 const Scal* S, double* part) {
    const double mean = S->bsum / (double)n;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (t < n) {
        const double bt = rhs[t] - mean;
        r[t] = (T)(rhs[perm ? perm[t] : t] - mean);
        x[t] = T(0);
        p0[t] = T(0);
        p1[t] = T(0);
        v[0] = bt * bt;
    }
    block_partial<1>(v, part);
}

// Solve start: bh = b - mean(b) in solve order (solve position s holds input
// vertex sperm[s]; sperm null: the same); x = 0 and r = bh when given;
// partial ||bh||^2.
__global__ __launch_bounds__(kBlock) void k_init_outer(int n, const int32_t* __restrict__ sperm,
                                                       const double* __restrict__ b,
                                                       double* __restrict__ bh,
                                                       double* __restrict__ x,
                                                       double* __restrict__ r, const Scal* S,
                                                       double* part) {
    const double mean = S->bsum / (double)n;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (t < n) {
        const double bt = b[sperm ? sperm[t] : t] - mean;
        bh[t] = bt;
        if (x) x[t] = 0.0;
        if (r) r[t] = bt;
        v[0] = bt * bt;
    }
    block_partial<1>(v, part);
}

// ------------------------------------------------------------------ PEGP

// sum over k = k0 + first, k0 + first + S, ... < k1 of val[k] * f[col[k]],
// in rounds of eight entries whose loads are all issued before the first
// product (the last round's missing entries are masked off)
template <int S>
__device__ inline double sparse_dot(const double* __restrict__ val,
                                    const int32_t* __restrict__ col, int k0, int k1, int first,
                                    const double* f) {
    constexpr int U = 8;
    double acc = 0.0;
    for (int k = k0 + first; k < k1; k += U * S) {
        double a[U];
        int c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = k + u * S < k1;
            a[u] = ok ? val[k + u * S] : 0.0;
            c[u] = ok ? col[k + u * S] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k + u * S < k1) acc += a[u] * f[c[u]];
    }
    return acc;
}

// The levels of a level-scheduled triangular solve on the LDS vector f, as
// packed by the host: level l's descriptor deals the rows [r0, r0 + nr) of
// the level list to groups of 2^g lanes over P passes of NT threads; thread
// t's u-th entry of pass p is at base + (p U + u) NT + t (columns as LDS
// byte offsets, node * 8).  Each row r gets
// f[rows[r]] -= sum of its entries' values times f at their nodes (no row of
// a level reads another's node).  The first kPegpPre entries of pass 0 of
// the next level are loaded into registers while the current level runs:
// its loads depend on nothing the level computes.  The descriptors are read
// from an LDS copy when there is room for one (an LDS read does not wait for
// the vector loads in flight, as a global one would).
constexpr int kPegpPre = 8;

struct PegpLvl {
    int base, nt, u, np, g, r0, nr;
};

template <class DT>
__device__ __forceinline__ PegpLvl pegp_desc(DT* desc, int l) {
    const int4 d = desc[l];
    return PegpLvl{d.x, d.y & 0xfff, d.y >> 16, d.z & 0xffff, (d.y >> 12) & 0xf, d.w, d.z >> 16};
}

struct PegpPreRow {
    int node;
    double a[kPegpPre];
    int c[kPegpPre];
};

// Pass 0's first entries of thread t (threads past NT load thread NT-1's,
// rounds past U load round U-1's: no load is masked, so none is waited for
// on its own; those values are not used).
// (the round's offset is uniform: it goes into the scalar base of each
// load, which then takes the same per-thread offset)
__device__ __forceinline__ void pegp_fetch(PegpPreRow& s, const PegpLvl& D,
                                           const int32_t* __restrict__ rows,
                                           const double* __restrict__ val,
                                           const int32_t* __restrict__ col, int t) {
    const int tt = min(t, D.nt - 1);
    s.node = rows[D.r0 + (tt >> D.g)];
#pragma unroll
    for (int u = 0; u < kPegpPre; ++u) {
        const size_t off = (size_t)D.base + (size_t)min(u, D.u - 1) * D.nt;
        s.a[u] = (val + off)[tt];
        s.c[u] = (col + off)[tt];
    }
}

// f at an LDS byte offset (the packed columns hold node * 8)
__device__ __forceinline__ double pegp_at(const double* f, int byte_off) {
    return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(f) + byte_off);
}

// v moved by the DPP control CTRL (rows in ROWMASK written, lanes with no
// source read 0; the other rows get 0)
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWMASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, ROWMASK, 0xf, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                            (unsigned)lo));
}

// Sum of each aligned group of 2^g lanes (g <= 6), valid in the group's last
// lane (q = lane within the group): an inclusive scan inside each 16-lane
// row by row shifts (masked at the group's start), then the row totals
// carried up by row broadcasts.  Register moves only, no LDS permutes.
__device__ __forceinline__ double pegp_group_sum(double v, int g, int q) {
    constexpr int kShr = 0x110, kBcast15 = 0x142, kBcast31 = 0x143;
    if (g >= 1) { const double t = dpp_f64<kShr + 1, 0xf>(v); v += q >= 1 ? t : 0.0; }
    if (g >= 2) { const double t = dpp_f64<kShr + 2, 0xf>(v); v += q >= 2 ? t : 0.0; }
    if (g >= 3) { const double t = dpp_f64<kShr + 4, 0xf>(v); v += q >= 4 ? t : 0.0; }
    if (g >= 4) { const double t = dpp_f64<kShr + 8, 0xf>(v); v += q >= 8 ? t : 0.0; }
    if (g >= 5) v += dpp_f64<kBcast15, 0xa>(v);
    if (g >= 6) v += dpp_f64<kBcast31, 0xc>(v);
    return v;
}

__device__ __forceinline__ void pegp_level(double* f, const PegpLvl& D, const PegpPreRow& s,
                                           const int32_t* __restrict__ rows,
                                           const double* __restrict__ val,
                                           const int32_t* __restrict__ col, int t) {
    if (t < D.nt) {
        const int q = t & ((1 << D.g) - 1);
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < kPegpPre; ++u) acc += (u < D.u ? s.a[u] : 0.0) * pegp_at(f, s.c[u]);
        for (int u = kPegpPre; u < D.u; ++u) {
            const int i = D.base + u * D.nt + t;
            acc += val[i] * pegp_at(f, col[i]);
        }
        acc = pegp_group_sum(acc, D.g, q);
        if (q == (1 << D.g) - 1) f[s.node] -= acc;
        // further passes (levels wider than the workgroup's groups)
        for (int p = 1; p < D.np; ++p) {
            const int rr = p * (kPegpThreads >> D.g) + (t >> D.g);
            if (rr < D.nr) {
                double a2 = 0.0;
                for (int u = 0; u < D.u; ++u) {
                    const int i = D.base + (p * D.u + u) * D.nt + t;
                    a2 += val[i] * pegp_at(f, col[i]);
                }
                a2 = pegp_group_sum(a2, D.g, q);
                if (q == (1 << D.g) - 1) f[rows[D.r0 + rr]] -= a2;
            }
        }
    }
    __syncthreads();
}

// The descriptor table copied to LDS at `lds` (16-byte aligned, after the
// vector); the caller's first barrier orders the copy before its reads.
__device__ __forceinline__ void pegp_desc_copy(const int32_t* __restrict__ g, int nl, int4* lds) {
    const int4* src = reinterpret_cast<const int4*>(g);
    for (int l = threadIdx.x; l < nl; l += kPegpThreads) lds[l] = src[l];
}

// (DT: const int4 in LDS, or in global memory when the table does not fit;
// the pointer's address space is known, so that LDS reads stay LDS reads)
template <class DT>
__device__ __forceinline__ void pegp_levels(double* f, DT* desc,
                                            const int32_t* __restrict__ rows,
                                            const double* __restrict__ val,
                                            const int32_t* __restrict__ col, int nl) {
    if (nl <= 0) return;
    const int t = threadIdx.x;
    // two buffers taken in turn (no copy from one to the other, which would
    // wait for the loads in flight); the last level fetches itself again
    // rather than branch
    PegpLvl DA = pegp_desc(desc, 0), DB;
    PegpPreRow A, B;
    pegp_fetch(A, DA, rows, val, col, t);
    for (int l = 0;;) {
        DB = pegp_desc(desc, min(l + 1, nl - 1));
        pegp_fetch(B, DB, rows, val, col, t);
        pegp_level(f, DA, A, rows, val, col, t);
        if (++l == nl) break;
        DA = pegp_desc(desc, min(l + 1, nl - 1));
        pegp_fetch(A, DA, rows, val, col, t);
        pegp_level(f, DB, B, rows, val, col, t);
        if (++l == nl) break;
    }
}

// z = P(mu) S^-1 D P(mu)^T r with S = D L_H~ D grounded (Sec. 3.1-3.2),
// then mean removed.  S = L D L^T is factored on the host; an apply runs
// restriction sums up the tree, signs (-1)^k (D P(mu)^T is (-1)^k times the
// plain sums on level k), the forward solve, the diagonal, the backward
// solve, the signs again and prolongation down the tree.  The level-scheduled
// parts run in one workgroup on an LDS copy of the expanded vector; the
// dense tail of the factor (the last-eliminated nodes) is applied between
// them by kernels over the whole device:
//   k_pegp_fwd        restriction, signs, forward levels -> fg
//   k_pegp_tail_rhs   y = f_tail - (tail rows' entries on the others) f
//   k_pegp_tail_fwd   y = L_tt^-1 y, a kernel per superblock of the tail
//   k_pegp_tail_bwd   y = L_tt^-T D_t^-1 y, the same
//   k_pegp_tail_back  the other rows' entries on the tail times y
//   k_pegp_bwd        diagonal, backward levels, signs, prolongation, z
//                     and the rho / zbar / beta reductions

__global__ __launch_bounds__(kPegpThreads) void k_pegp_fwd(PegpDev P,
                                                           const double* __restrict__ r,
                                                           const Scal* S) {
    if (S->done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    double* f = reinterpret_cast<double*>(smem);
    const int tid = threadIdx.x, nth = kPegpThreads;
    const int n0 = P.off[1] - P.off[0], T = P.nlev - 1;
    int4* dl = reinterpret_cast<int4*>(smem + ((size_t)P.nt * sizeof(double) + 15) / 16 * 16);
    if (P.desc_lds) pegp_desc_copy(P.fdesc, P.nflev, dl);
    for (int t = tid; t < n0; t += nth) f[t] = r[t];
    __syncthreads();
    for (int k = 0; k < T; ++k) {
        const int nc = P.off[k + 2] - P.off[k + 1];
        const int32_t* cp = P.cptr[k];
        const double* fk = f + P.off[k];
        double* fk1 = f + P.off[k + 1];
        for (int J = tid; J < nc; J += nth) {
            double s = 0.0;
            for (int t = cp[J]; t < cp[J + 1]; ++t) s += fk[t];
            fk1[J] = s;
        }
        __syncthreads();
    }
    for (int k = 1; k <= T; k += 2)
        for (int e = P.off[k] + tid; e < P.off[k + 1]; e += nth) f[e] = -f[e];
    __syncthreads();
    if (tid == 0) f[P.ground] = 0.0;
    __syncthreads();
    if (P.desc_lds)
        pegp_levels(f, (const int4*)dl, P.frow, P.fpval, P.fpcol, P.nflev);
    else
        pegp_levels(f, reinterpret_cast<const int4*>(P.fdesc), P.frow, P.fpval, P.fpcol, P.nflev);
    for (int e = tid; e < P.nt; e += nth) P.fg[e] = f[e];
}

// y[p] = f[drow[p]] - sum over tail row p's entries on the other nodes, a
// wavefront per tail row.
__global__ __launch_bounds__(kBlock) void k_pegp_tail_rhs(PegpDev P, const Scal* S) {
    if (S->done) return;
    const int p = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (p >= P.nd) return;
    double acc = sparse_dot<64>(P.dcval, P.dccol, P.dcptr[p], P.dcptr[p + 1], lane, P.fg);
    acc = wave_sum1(acc);
    if (lane == 0) P.ty[p] = P.fg[P.drow[p]] - acc;
}

// The dense tail solves, y = L_tt^-1 y, y = D_t^-1 y and y = L_tt^-T y in
// place on the tail vector, by superblocks of kTailS rows with a kernel per
// superblock (the kernels' order on the stream carries the dependencies).
// A superblock is kTailW blocks of kTailB rows.  In the kernel for
// superblock b, the first kTailW wavefronts of workgroup 0 each take one
// block of the next superblock, a lane per row holding its row of that
// block's diagonal block in registers (coalesced loads of the factor's
// other orientation), and bring it up to date with superblock b's values;
// then, block after block, one wavefront solves its unit triangle with a
// broadcast chain, passes the values on through LDS, and the wavefronts of
// the blocks after it apply them (their loads issued before the wait).  The
// other workgroups apply superblock b's values to all rows past the next
// superblock, a wavefront per row.  The tail is padded to whole superblocks
// (zero factor, unit diagonal, zero values), so no load needs a bound.
constexpr int kTailB = 64;
constexpr int kTailW = 3;
constexpr int kTailS = kTailB * kTailW;
static_assert(kTailW * 64 <= kBlock, "a wavefront of workgroup 0 per block");

// v broadcast from lane j (j uniform)
__device__ inline double lane_bcast(double v, int j) {
    const unsigned long long u = __double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, j);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), j);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// sum over j < kTailB of a[j * stride] * x_j, where lane j holds x_j in xv;
// the loads issued in two batches of half a block each
__device__ inline double tail_dot(const double* __restrict__ a, int stride, double xv) {
    constexpr int H = kTailB / 2;
    double acc = 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        double v[H];
#pragma unroll
        for (int j = 0; j < H; ++j) v[j] = a[(size_t)(h * H + j) * stride];
#pragma unroll
        for (int j = 0; j < H; ++j) acc += v[j] * lane_bcast(xv, h * H + j);
    }
    return acc;
}

// forward, superblock b solved (b = -1: none yet); solves superblock b + 1
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_pegp_tail_fwd(PegpDev P, int b, const Scal* S) {
    if (S->done) return;
    const int nd = P.ndp, b0 = b * kTailS, b1 = (b + 1) * kTailS;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    constexpr int NW = kBlock / 64;
    double* y = P.ty;
    if (blockIdx.x == 0) {
        __shared__ double xs[kTailS];
        const bool act = wid < kTailW;
        const int r0 = b1 + (act ? wid : 0) * kTailB, row = r0 + lane;
        // L[j] = L_tt[row][r0 + j], used for j < lane
        double L[kTailB], yi = 0.0;
        if (act) {
#pragma unroll
            for (int j = 0; j < kTailB; ++j) L[j] = P.dlc[(size_t)(r0 + j) * nd + row];
            yi = y[row];
            if (b >= 0) {
#pragma unroll
                for (int q = 0; q < kTailW; ++q) {
                    const int c = b0 + q * kTailB;
                    yi -= tail_dot(P.dlc + (size_t)c * nd + row, nd, y[c + lane]);
                }
            }
        }
#pragma unroll
        for (int m = 0; m < kTailW; ++m) {
            // stage m: wavefront m solves its block, the later ones apply it
            const bool cross = act && wid > m;
            double C[kTailB];
            if (cross) {
#pragma unroll
                for (int j = 0; j < kTailB; ++j)
                    C[j] = P.dlc[(size_t)(b1 + m * kTailB + j) * nd + row];
            }
            if (wid == m) {
#pragma unroll
                for (int j = 0; j + 1 < kTailB; ++j) {
                    const double xj = lane_bcast(yi, j);
                    if (lane > j) yi -= L[j] * xj;
                }
                y[row] = yi;
                xs[m * kTailB + lane] = yi;
            }
            if (m + 1 < kTailW) __syncthreads();
            if (cross) {
                const double xv = xs[m * kTailB + lane];
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < kTailB; ++j) acc += C[j] * lane_bcast(xv, j);
                yi -= acc;
            }
        }
        return;
    }
    const int r = b1 + kTailS + (blockIdx.x - 1) * NW + wid;
    if (b < 0 || r >= nd) return;
    double a[kTailW];
#pragma unroll
    for (int q = 0; q < kTailW; ++q) {
        const int c = b0 + q * kTailB + lane;
        a[q] = wave_sum1(P.dlr[(size_t)r * nd + c] * y[c]);
    }
    if (lane == 0) {
        double v = y[r];
#pragma unroll
        for (int q = 0; q < kTailW; ++q) v -= a[q];
        y[r] = v;
    }
}

// backward, superblock b solved (b = nblk: none yet; then the diagonal
// D_t^-1 is applied to every tail row first); solves superblock b - 1, its
// last block first
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_pegp_tail_bwd(PegpDev P, int b, int nblk,
                                                          const Scal* S) {
    if (S->done) return;
    const int nd = P.ndp, c0 = (b - 1) * kTailS, b0 = b * kTailS;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    constexpr int NW = kBlock / 64;
    double* y = P.ty;
    if (blockIdx.x == 0) {
        __shared__ double xs[kTailS];
        const bool act = wid < kTailW;
        const int r0 = c0 + (act ? wid : 0) * kTailB, row = r0 + lane;
        // L[j] = L_tt[r0 + j][row], used for j > lane
        double L[kTailB], yi = 0.0;
        if (act) {
#pragma unroll
            for (int j = 0; j < kTailB; ++j) L[j] = P.dlr[(size_t)(r0 + j) * nd + row];
            yi = y[row];
            if (b == nblk) {
                yi /= P.dd[row];
            } else {
#pragma unroll
                for (int q = 0; q < kTailW; ++q) {
                    const int c = b0 + q * kTailB;
                    yi -= tail_dot(P.dlr + (size_t)c * nd + row, nd, y[c + lane]);
                }
            }
        }
#pragma unroll
        for (int m = 0; m < kTailW; ++m) {
            // stage m: wavefront ws solves its block, the earlier ones apply it
            const int ws = kTailW - 1 - m;
            const bool cross = act && wid < ws;
            double C[kTailB];
            if (cross) {
#pragma unroll
                for (int j = 0; j < kTailB; ++j)
                    C[j] = P.dlr[(size_t)(c0 + ws * kTailB + j) * nd + row];
            }
            if (wid == ws) {
#pragma unroll
                for (int j = kTailB - 1; j > 0; --j) {
                    const double xj = lane_bcast(yi, j);
                    if (lane < j) yi -= L[j] * xj;
                }
                y[row] = yi;
                xs[ws * kTailB + lane] = yi;
            }
            if (m + 1 < kTailW) __syncthreads();
            if (cross) {
                const double xv = xs[ws * kTailB + lane];
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < kTailB; ++j) acc += C[j] * lane_bcast(xv, j);
                yi -= acc;
            }
        }
        return;
    }
    if (b == nblk) {
        const int r = (blockIdx.x - 1) * kBlock + tid;
        if (r < c0) y[r] /= P.dd[r];
        return;
    }
    const int r = (blockIdx.x - 1) * NW + wid;
    if (r >= c0) return;
    double a[kTailW];
#pragma unroll
    for (int q = 0; q < kTailW; ++q) {
        const int c = b0 + q * kTailB + lane;
        a[q] = wave_sum1(P.dlc[(size_t)r * nd + c] * y[c]);
    }
    if (lane == 0) {
        double v = y[r];
#pragma unroll
        for (int q = 0; q < kTailW; ++q) v -= a[q];
        y[r] = v;
    }
}

// cpl[i] = sum over row bcrow[i]'s entries on the tail of l * y_tail, a
// wavefront per row.
__global__ __launch_bounds__(kBlock) void k_pegp_tail_back(PegpDev P, const Scal* S) {
    if (S->done) return;
    const int i = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= P.nbc) return;
    double acc = sparse_dot<64>(P.bcval, P.bccol, P.bcptr[i], P.bcptr[i + 1], lane, P.ty);
    acc = wave_sum1(acc);
    if (lane == 0) P.cpl[i] = acc;
}

// Writes z (tree order) and zn (solve order, tree position t at perm[t]) and
// does the finish step of the rho / zbar / beta reductions itself.
__global__ __launch_bounds__(kPegpThreads) void k_pegp_bwd(PegpDev P,
                                                           const int32_t* __restrict__ perm,
                                                           const double* __restrict__ r,
                                                           double* __restrict__ z,
                                                           double* __restrict__ zn, Scal* S) {
    if (S->done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    double* f = reinterpret_cast<double*>(smem);
    __shared__ double red[3 * (kPegpThreads / 64)];
    const int tid = threadIdx.x, nth = kPegpThreads;
    const int n0 = P.off[1] - P.off[0], T = P.nlev - 1;
    int4* dl = reinterpret_cast<int4*>(smem + ((size_t)P.nt * sizeof(double) + 15) / 16 * 16);
    if (P.desc_lds) pegp_desc_copy(P.bdesc, P.nblev, dl);
    for (int e = tid; e < P.nt; e += nth) f[e] = e != P.ground ? P.fg[e] / P.diag[e] : 0.0;
    __syncthreads();
    // the tail's values, and its contributions to the other rows
    for (int p = tid; p < P.nd; p += nth) f[P.drow[p]] = P.ty[p];
    for (int i = tid; i < P.nbc; i += nth) f[P.bcrow[i]] -= P.cpl[i];
    __syncthreads();
    if (P.desc_lds)
        pegp_levels(f, (const int4*)dl, P.brow, P.bpval, P.bpcol, P.nblev);
    else
        pegp_levels(f, reinterpret_cast<const int4*>(P.bdesc), P.brow, P.bpval, P.bpcol, P.nblev);
    for (int k = 1; k <= T; k += 2)
        for (int e = P.off[k] + tid; e < P.off[k + 1]; e += nth) f[e] = -f[e];
    __syncthreads();
    for (int k = T - 1; k >= 0; --k) {
        const int nc = P.off[k + 2] - P.off[k + 1];
        const int32_t* cp = P.cptr[k];
        double* fk = f + P.off[k];
        const double* fk1 = f + P.off[k + 1];
        for (int J = tid; J < nc; J += nth) {
            const double y = fk1[J];
            for (int t = cp[J]; t < cp[J + 1]; ++t) fk[t] += y;
        }
        __syncthreads();
    }
    double v[3] = {0.0, 0.0, 0.0};
    for (int t = tid; t < n0; t += nth) {
        const double zt = f[t], rt = r[t];
        z[t] = zt;
        zn[perm ? perm[t] : t] = zt;
        v[0] += zt;
        v[1] += rt * zt;
        v[2] += rt;
    }
    block_sum<3, kPegpThreads>(v, red);
    if (tid == 0) {
        const double zbar = v[0] / (double)n0;
        const double rho = v[1] - zbar * v[2];
        S->zbar = zbar;
        if (!isfinite(rho)) S->done = 3;
        S->beta = S->first ? 0.0 : rho / S->rho;
        S->first = 0;
        S->rho = rho;
    }
}

// PEGP by its explicit operator: z = M r on the fine level (tree order),
// M = P(mu) L_H~^+ P(mu)^T formed at set-up (PegpPlan::op).  A dense
// matrix-vector product bound by the stream of M: r is staged in LDS, each
// wavefront takes one row, every lane two adjacent columns per load
// (coalesced 1 KB per wavefront load), eight loads in flight per lane.  z
// goes to zn through the permutation; the partial sums of z, r z and r of
// the workgroup's rows go to part for the finish kernel.
__global__ __launch_bounds__(kBlock) void k_pegp_op(PegpDev P, const int32_t* __restrict__ perm,
                                                    const double* __restrict__ r,
                                                    double* __restrict__ zn, const Scal* S,
                                                    double* part) {
    static_assert(kPegpOpRows == kBlock / 64, "one row per wavefront");
    extern __shared__ __align__(16) unsigned char smem[];
    double* rs = reinterpret_cast<double*>(smem);
    const int n = P.opn, ld = P.opld, tid = threadIdx.x;
    const int done = S->done;
    for (int j = tid; j < ld; j += kBlock) rs[j] = j < n ? r[j] : 0.0;
    if (done) return;
    __syncthreads();
    const int lane = tid & 63;
    const int i = blockIdx.x * kPegpOpRows + (tid >> 6);
    double v[3] = {0.0, 0.0, 0.0};
    if (i < n) {
        const double2* row = reinterpret_cast<const double2*>(P.op + (size_t)i * ld);
        const double2* rs2 = reinterpret_cast<const double2*>(rs);
        constexpr int U = 8;
        const int nc2 = ld / 2;  // a multiple of 64: every lane takes the same steps
        double a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = 0.0;
        int c = lane;
        for (; c + (U - 1) * 64 < nc2; c += U * 64) {
            double2 m[U];
#pragma unroll
            for (int u = 0; u < U; ++u) m[u] = row[c + u * 64];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double2 x = rs2[c + u * 64];
                a[u] += m[u].x * x.x + m[u].y * x.y;
            }
        }
        for (; c < nc2; c += 64) {
            const double2 m = row[c], x = rs2[c];
            a[0] += m.x * x.x + m.y * x.y;
        }
        const double zi =
            wave_sum1(((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7])));
        if (lane == 0) {
            const double ri = rs[i];
            zn[perm ? perm[i] : i] = zi;
            v[0] = zi;
            v[1] = ri * zi;
            v[2] = ri;
        }
    }
    block_partial<3>(v, part);
}

// A fixed non-constant vector (kCols columns per row when cols > 1), the
// start of timing runs: v = ((i * 2654435761) mod 1024) / 1024 - 1/2.
__global__ __launch_bounds__(kBlock) void k_pattern(int64_t count, double* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < count) dst[i] = (double)((uint64_t)(i * 2654435761ull) & 1023u) / 1024.0 - 0.5;
}

// x += d and d = 0 (FP64 += FP32 correction, solve order): the correction
// accumulated by the FP32 run since the last reliable update moves into x.
__global__ __launch_bounds__(kBlock) void k_move_corr(int n, double* __restrict__ x,
                                                      float* __restrict__ d) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < n) {
        x[t] += (double)d[t];
        d[t] = 0.0f;
    }
}

// r (tree order, FP32) = r64 (solve order, FP64) rounded; tree position t
// is solve position perm[t] (perm null: the same).
__global__ __launch_bounds__(kBlock) void k_residual_in(int n, const int32_t* __restrict__ perm,
                                                        const double* __restrict__ r64,
                                                        float* __restrict__ r) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < n) r[t] = (float)r64[perm ? perm[t] : t];
}

// x += d (FP64 += FP32 correction, solve order).
__global__ __launch_bounds__(kBlock) void k_add_corr(int n, double* __restrict__ x,
                                                     const float* __restrict__ d) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < n) x[t] += (double)d[t];
}

// xc = x - mean(x) (solve order) and the caller's copy of it in input
// order.
__global__ __launch_bounds__(kBlock) void k_center_out(int n, const int32_t* __restrict__ sperm,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ xc,
                                                       double* __restrict__ dst, const Scal* S) {
    const double mean = S->xsum / (double)n;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < n) {
        const double v = x[t] - mean;
        xc[t] = v;
        dst[sperm ? sperm[t] : t] = v;
    }
}

// dst[t] = src[perm[t]] (a gather: input order -> tree or solve order).
template <class T>
__global__ __launch_bounds__(kBlock) void k_gather(int n, const int32_t* __restrict__ perm,
                                                   const double* __restrict__ src,
                                                   T* __restrict__ dst) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < n) dst[t] = (T)src[perm[t]];
}

// dst[sperm[t]] = src[t] - zbar (solve order -> input order; zbar from S,
// or 0 when S is null).
template <class T>
__global__ __launch_bounds__(kBlock) void k_shift_out(int n, const int32_t* __restrict__ sperm,
                                                      const T* __restrict__ src,
                                                      double* __restrict__ dst, const Scal* S) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < n) dst[sperm ? sperm[t] : t] = (double)src[t] - (S ? S->zbar : 0.0);
}

}  // namespace lapgpu
