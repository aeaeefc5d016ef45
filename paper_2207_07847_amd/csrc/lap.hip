// MI355X (gfx950) solve path of the MSP-preconditioned Laplacian solver and
// its C ABI (include/lap.h).
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
//   finish      convergence flag
//   up / group  restriction + local solves of the middle levels
//   tail        one workgroup in LDS: the small levels and the top solve
//   down/group  prolongation + local corrections of the middle levels
//   down0       z on level 0 (both orders); partial sum z, r^T z, sum r
//   finish      zbar, rho, beta
// Every reduction ends in a one-block finish kernel that adds the per-block
// partials in a fixed order (bitwise reproducible).  Every kernel returns at
// once when the device flag `done` is set, so chunks of iterations captured
// in a hipGraph are replayed without a host round trip per iteration.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "kernels.hpp"
#include "lap.h"
#include "setup.hpp"

namespace lapgpu {

// ------------------------------------------------------------ reductions

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
    if (loop && S->done) return;
    __shared__ double lds[N * (kFinThreads / 64)];
    double v[N];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = 0.0;
    const int nv = (OP == kFinRho) ? 3 : 1;
    for (int i = 0; i < nv; ++i) {
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        int b = threadIdx.x;
        for (; b + 3 * kFinThreads < G; b += 4 * kFinThreads) {
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] += part[i * G + b + u * kFinThreads];
        }
        for (; b < G; b += kFinThreads) a[0] += part[i * G + b];
        v[i] = (a[0] + a[1]) + (a[2] + a[3]);
    }
    if (OP == kFinRho)
        for (int b = threadIdx.x; b < G2; b += kFinThreads) v[N - 1] += part2[b];
    block_sum<N, kFinThreads>(v, lds);
    if (threadIdx.x != 0) return;
    if (OP == kFinPq) {
        const double pq = v[0];
        S->pq = pq;
        S->iter += 1;
        if (!(pq > 0.0) || !isfinite(pq)) S->done = 3;
        else S->alpha = S->rho / pq;
    } else if (OP == kFinRr) {
        S->rr = v[0];
        if (!isfinite(v[0])) S->done = 3;
        else if (v[0] <= S->tol2 * S->bn2) S->done = 1;
        else if (S->iter >= S->maxit) S->done = 2;
    } else if (OP == kFinRho) {
        const double zbar = v[0] / (double)n;
        const double rho = v[1] - zbar * v[2];
        S->zbar = zbar;
        if (!isfinite(rho)) S->done = 3;
        S->beta = S->first ? 0.0 : rho / S->rho;
        S->first = 0;
        S->rho = rho;
        if (G2 > 0) {
            S->rr = v[3];
            if (!isfinite(v[3])) S->done = 3;
            else if (v[3] <= S->tol2 * S->bn2) S->done = 1;
            else if (S->iter >= S->maxit) S->done = 2;
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
        else if (S->maxit <= 0) S->done = 2;
        else S->done = 0;
    } else if (OP == kFinXsum) {
        S->xsum = v[0];
    } else if (OP == kFinRes2) {
        S->res2 = v[0];
    }
}

// --------------------------------------------------- aggregate primitives

// Blocks are dispatched to the eight XCDs in turn (block b runs on XCD
// b mod 8).  Level kernels renumber their blocks so that every XCD owns one
// contiguous range of the partition: neighbouring aggregates, and the
// vertices their values are gathered from, then share one L2.
__device__ inline int xcd_block() {
    const int b = blockIdx.x, G = gridDim.x;
    const int x = b & 7, q = G >> 3, rem = G & 7;
    return x * q + (x < rem ? x : rem) + (b >> 3);
}

// Restriction of level-k values onto aggregate J plus the pair solve of the
// aggregate's sparsifier block: g = C^T r, eta = theta S^-1 g.  The
// children's values are read from rs[t - toff].
__device__ inline void agg_up(const LevelDev& s, const double* rs, int toff,
                              double* __restrict__ rk1, int J) {
    const int b0 = s.cptr[J], b1 = s.cptr[J + 1];
    const double ra = rs[b0 - toff], rb = rs[b0 + 1 - toff];
    double sum = ra + rb, ga = ra, gb = rb;
    for (int t = b0 + 2; t < b1; ++t) {
        const int li = t - 2 * J - 2;
        const double rv = rs[t - toff];
        sum += rv;
        ga += s.l1[li] * rv;
        gb += s.l2[li] * rv;
    }
    const double saa = s.saa[J], sab = s.sab[J], sbb = s.sbb[J];
    s.ea[J] = saa * ga + sab * gb;
    s.eb[J] = sab * ga + sbb * gb;
    rk1[J] = sum;
}

// Contributions of child t of aggregate J (first child b0) to the
// restriction sums v = {sum, g_a, g_b}.
__device__ inline void child_up(const LevelDev& s, int J, int b0, int t, double rv,
                                double* v) {
    v[0] += rv;
    if (t == b0) v[1] += rv;
    else if (t == b0 + 1) v[2] += rv;
    else {
        const int li = t - 2 * J - 2;
        v[1] += s.l1[li] * rv;
        v[2] += s.l2[li] * rv;
    }
}

// Pair solve of aggregate J from the completed sums v (thread 0 of a block
// that reduced them).
__device__ inline void agg_solve(const LevelDev& s, int J, const double* v,
                                 double* __restrict__ rk1) {
    const double saa = s.saa[J], sab = s.sab[J], sbb = s.sbb[J];
    s.ea[J] = saa * v[1] + sab * v[2];
    s.eb[J] = sab * v[1] + sbb * v[2];
    rk1[J] = v[0];
}

// Correction of child t of aggregate J (first child b0).
__device__ inline double child_down(const LevelDev& s, int J, int b0, int t, double rt,
                                    double yJ, double ea, double eb) {
    if (t == b0) return ea + yJ;
    if (t == b0 + 1) return eb + yJ;
    const int li = t - 2 * J - 2;
    return s.l0[li] * rt + s.l1[li] * ea + s.l2[li] * eb + yJ;
}

// Down-sweep bookkeeping of one block in LDS: the aggregate of every
// staged child and the aggregate's values.
struct DownBlock {
    int32_t own[kCapP];
    int32_t b0[kAggPerBlock];
    double yJ[kAggPerBlock], ea[kAggPerBlock], eb[kAggPerBlock];
};

// Phase one of a down-sweep block: per aggregate, its values and the owner
// marks of its children.  Returns false for a block holding one aggregate
// too large to stage (every thread then handles it directly).
__device__ inline bool down_stage(const LevelDev& s, const double* __restrict__ yk1, int J0,
                                  int J1, int t0, int len, DownBlock& D) {
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

// ------------------------------------------------------ fine-level kernels

// Input order: p = zn - zbar + beta p_old; q = L p with
// (L p)_i = sum_j w_ij (p_i - p_j); partial p^T q.
__global__ __launch_bounds__(kBlock) void k_spmv_p(int n, Sell A, const double* __restrict__ zn,
                                                   const double* __restrict__ pold,
                                                   double* __restrict__ pnew,
                                                   double* __restrict__ q, Scal* S,
                                                   double* part) {
    if (S->done) return;
    const double beta = S->beta, zbar = S->zbar;
    const int row = xcd_block() * kBlock + threadIdx.x;
    double pi = 0.0, acc = 0.0;
    if (row < n) {
        const double zi = zn[row], poi = pold[row];
        pi = (zi - zbar) + beta * poi;
        const int sl = row >> 6;
        const int base = A.off[sl] + (row & 63);
        const int W = A.width[sl];
        for (int k = 0; k < W; ++k) {
            const int j = A.col[base + k * 64];
            const double w = A.w[base + k * 64];
            acc += w * ((zi - zn[j]) + beta * (poi - pold[j]));
        }
        pnew[row] = pi;
        q[row] = acc;
    }
    double v[1] = {pi * acc};
    block_partial<1>(v, part);
}

// x += alpha p (input order); r -= alpha q (tree order, q read through the
// permutation); partial ||r||^2; restriction of r to level 1 fused with the
// local solves of the level-0 aggregates.  The children ranges of all
// aggregates partition [0, n), so the same ranges index x and p.  The
// element-wise part runs over the block's children with coalesced accesses
// and leaves the new residuals in LDS for the per-aggregate part.
__global__ __launch_bounds__(kBlock) void k_update_up0(LevelDev s0, const int32_t* __restrict__ perm,
                                                       double* __restrict__ x,
                                                       double* __restrict__ r,
                                                       const double* __restrict__ p,
                                                       const double* __restrict__ q,
                                                       double* __restrict__ r1, Scal* S,
                                                       double* part, int do_update) {
    if (S->done) return;
    __shared__ double rs[kCapP];
    __shared__ double red[4 * (kBlock / 64)];
    const double alpha = S->alpha;
    const int b = xcd_block();
    const int J0 = s0.bst[b], J1 = s0.bst[b + 1];
    const int t0 = s0.cptr[J0], len = s0.cptr[J1] - t0;
    double rr = 0.0;
    if (len <= kCapP) {
        for (int i = threadIdx.x; i < len; i += kBlock) {
            const int t = t0 + i;
            double rt = r[t];
            if (do_update) {
                x[t] += alpha * p[t];
                rt -= alpha * q[perm[t]];
                r[t] = rt;
                rr += rt * rt;
            }
            rs[i] = rt;
        }
        __syncthreads();
        for (int J = J0 + threadIdx.x; J < J1; J += kBlock) agg_up(s0, rs, t0, r1, J);
        if (!do_update) return;
        double v[1] = {rr};
        block_partial<1>(v, part);
        return;
    }
    // one aggregate with more children than LDS holds
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < len; i += kBlock) {
        const int t = t0 + i;
        double rt = r[t];
        if (do_update) {
            x[t] += alpha * p[t];
            rt -= alpha * q[perm[t]];
            r[t] = rt;
            v[3] += rt * rt;
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
__global__ __launch_bounds__(kBlock) void k_down0(LevelDev s0, const int32_t* __restrict__ perm,
                                                  const double* __restrict__ r,
                                                  double* __restrict__ zn,
                                                  const double* __restrict__ y1, Scal* S,
                                                  double* part) {
    if (S->done) return;
    __shared__ DownBlock D;
    const int b = xcd_block();
    const int J0 = s0.bst[b], J1 = s0.bst[b + 1];
    const int t0 = s0.cptr[J0], len = s0.cptr[J1] - t0;
    double v[3] = {0.0, 0.0, 0.0};
    if (down_stage(s0, y1, J0, J1, t0, len, D)) {
        for (int i = threadIdx.x; i < len; i += kBlock) {
            const int t = t0 + i, j = D.own[i];
            const double rt = r[t];
            const double zt = child_down(s0, J0 + j, D.b0[j], t, rt, D.yJ[j], D.ea[j], D.eb[j]);
            zn[perm[t]] = zt;
            v[0] += zt;
            v[1] += rt * zt;
            v[2] += rt;
        }
    } else {
        const double yJ = y1[J0], ea = s0.ea[J0], eb = s0.eb[J0];
        for (int i = threadIdx.x; i < len; i += kBlock) {
            const int t = t0 + i;
            const double rt = r[t];
            const double zt = child_down(s0, J0, t0, t, rt, yJ, ea, eb);
            zn[perm[t]] = zt;
            v[0] += zt;
            v[1] += rt * zt;
            v[2] += rt;
        }
    }
    block_partial<3>(v, part);
}

// Without a hierarchy below the fine level: x and r update only.
__global__ __launch_bounds__(kBlock) void k_update_none(int n, const int32_t* __restrict__ perm,
                                                        double* __restrict__ x,
                                                        double* __restrict__ r,
                                                        const double* __restrict__ p,
                                                        const double* __restrict__ q, Scal* S,
                                                        double* part) {
    if (S->done) return;
    const double alpha = S->alpha;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    double rr = 0.0;
    if (t < n) {
        x[t] += alpha * p[t];
        const double rt = r[t] - alpha * q[perm[t]];
        r[t] = rt;
        rr = rt * rt;
    }
    double v[1] = {rr};
    block_partial<1>(v, part);
}

// Plain CG: z = r (both orders) with the down0 reductions.
__global__ __launch_bounds__(kBlock) void k_prec_none(int n, const int32_t* __restrict__ perm,
                                                      const double* __restrict__ r,
                                                      double* __restrict__ z,
                                                      double* __restrict__ zn, Scal* S,
                                                      double* part) {
    if (S->done) return;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    if (t < n) {
        const double rt = r[t];
        z[t] = rt;
        zn[perm[t]] = rt;
        v[0] = rt;
        v[1] = rt * rt;
        v[2] = rt;
    }
    block_partial<3>(v, part);
}

// One-level hierarchy (the fine level is the top, at most kTopMax nodes):
// the MSP is theta_0 pinv(L) = pinv(L), applied by one workgroup, which also
// does the finish step of the down0 reductions itself.
__global__ __launch_bounds__(kBlock) void k_top_only(int n, const int32_t* __restrict__ perm,
                                                     const double* __restrict__ tp,
                                                     const double* __restrict__ r,
                                                     double* __restrict__ z,
                                                     double* __restrict__ zn, Scal* S) {
    if (S->done) return;
    __shared__ double lds[3 * (kBlock / 64)];
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += kBlock) {
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += tp[i * n + j] * r[j];
        z[i] = acc;
        zn[perm[i]] = acc;
        v[0] += acc;
        v[1] += r[i] * acc;
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

__global__ __launch_bounds__(kBlock) void k_up(LevelDev s, const double* __restrict__ rk,
                                               double* __restrict__ rk1, const Scal* S) {
    if (S->done) return;
    __shared__ double rs[kCapP];
    __shared__ double red[3 * (kBlock / 64)];
    const int b = xcd_block();
    const int J0 = s.bst[b], J1 = s.bst[b + 1];
    const int t0 = s.cptr[J0], len = s.cptr[J1] - t0;
    if (len <= kCapP) {
        for (int i = threadIdx.x; i < len; i += kBlock) rs[i] = rk[t0 + i];
        __syncthreads();
        for (int J = J0 + threadIdx.x; J < J1; J += kBlock) agg_up(s, rs, t0, rk1, J);
        return;
    }
    double v[3] = {0.0, 0.0, 0.0};
    for (int t = t0 + threadIdx.x; t < t0 + len; t += kBlock) child_up(s, J0, t0, t, rk[t], v);
    block_sum<3, kBlock>(v, red);
    if (threadIdx.x == 0) agg_solve(s, J0, v, rk1);
}

__global__ __launch_bounds__(kBlock) void k_down(LevelDev s, const double* __restrict__ rk,
                                                 double* __restrict__ yk,
                                                 const double* __restrict__ yk1, const Scal* S) {
    if (S->done) return;
    __shared__ DownBlock D;
    const int b = xcd_block();
    const int J0 = s.bst[b], J1 = s.bst[b + 1];
    const int t0 = s.cptr[J0], len = s.cptr[J1] - t0;
    if (down_stage(s, yk1, J0, J1, t0, len, D)) {
        for (int i = threadIdx.x; i < len; i += kBlock) {
            const int t = t0 + i, j = D.own[i];
            yk[t] = child_down(s, J0 + j, D.b0[j], t, rk[t], D.yJ[j], D.ea[j], D.eb[j]);
        }
    } else {
        const double yJ = yk1[J0], ea = s.ea[J0], eb = s.eb[J0];
        for (int t = t0 + threadIdx.x; t < t0 + len; t += kBlock)
            yk[t] = child_down(s, J0, t0, t, rk[t], yJ, ea, eb);
    }
}

// ------------------------------------------------------- grouped levels

// Flat copy global -> LDS with eight loads in flight per thread.
__device__ inline void stage_copy(double* __restrict__ dst, const double* __restrict__ src,
                                  int len) {
    constexpr int U = 8, B = kGrpThreads;
    int i = threadIdx.x;
    for (; i + (U - 1) * B < len; i += U * B) {
        double t[U];
#pragma unroll
        for (int u = 0; u < U; ++u) t[u] = src[i + u * B];
#pragma unroll
        for (int u = 0; u < U; ++u) dst[i + u * B] = t[u];
    }
    for (; i < len; i += B) dst[i] = src[i];
}

// Per-block bookkeeping of a group (level ranges and LDS layout) lives in
// LDS: it is indexed by the level inside loops, and a runtime-indexed
// private array would be placed in scratch memory.
struct GrpBlock {
    int32_t st[kMaxGroupLevels + 1];
    int32_t cnt[kMaxGroupLevels + 1];
    GrpLayout L;
};

__device__ inline void grp_setup(const GroupDev& G, int m, GrpBlock& B) {
    if (threadIdx.x == 0) {
        const int b = blockIdx.x, nb1 = G.nblocks + 1;
        for (int j = 0; j <= m; ++j) {
            B.st[j] = G.D[j * nb1 + b];
            B.cnt[j] = G.D[j * nb1 + b + 1] - B.st[j];
        }
        grp_layout(m, B.cnt, B.L);
    }
    __syncthreads();
}

// Up-sweep of a level group [k0, k1): level-k0 residuals in, level-k1
// residuals out; intermediate residuals and pair corrections go to the
// block's scratch chunk for the down-sweep.
__global__ __launch_bounds__(kGrpThreads) void k_up_grp(GroupDev G, const Scal* S) {
    if (S->done) return;
    extern __shared__ double sm[];
    const int m = G.k1 - G.k0, tid = threadIdx.x, nth = blockDim.x;
    __shared__ GrpBlock B;
    grp_setup(G, m, B);
    const int32_t* st = B.st;
    const int32_t* cnt = B.cnt;
    const GrpLayout& L = B.L;
    stage_copy(sm, G.upack + G.uoff[blockIdx.x], L.ulen);
    stage_copy(sm + L.ur[0], G.r_in + st[0], cnt[0]);
    __syncthreads();
    double* scr = G.scr + G.xoff[blockIdx.x];
    for (int j = 0; j < m; ++j) {
        const int na = cnt[j + 1], nl = cnt[j] - 2 * na;
        const int* cp = reinterpret_cast<const int*>(sm + L.ucp[j]);
        const double* sa = sm + L.us[j];
        const double* l1 = sm + L.ul[j];
        const double* l2 = l1 + nl;
        const double* rk = sm + L.ur[j];
        double* rk1 = sm + L.ur[j + 1];
        double* eo = scr + L.xe[j];
        double* ro = (j + 1 < m) ? scr + L.xr[j + 1] : G.r_top + st[m];
        for (int J = tid; J < na; J += nth) {
            const int b0 = cp[J], b1 = cp[J + 1];
            const double ra = rk[b0], rb = rk[b0 + 1];
            double sum = ra + rb, ga = ra, gb = rb;
            for (int c = b0 + 2; c < b1; ++c) {
                const int li = c - 2 * J - 2;
                const double rv = rk[c];
                sum += rv;
                ga += l1[li] * rv;
                gb += l2[li] * rv;
            }
            const double saa = sa[J], sab = sa[na + J], sbb = sa[2 * na + J];
            eo[J] = saa * ga + sab * gb;
            eo[na + J] = sab * ga + sbb * gb;
            rk1[J] = sum;
            ro[J] = sum;
        }
        __syncthreads();
    }
}

// Down-sweep of a level group: level-k1 corrections in, level-k0 out.
__global__ __launch_bounds__(kGrpThreads) void k_down_grp(GroupDev G, const Scal* S) {
    if (S->done) return;
    extern __shared__ double sm[];
    const int m = G.k1 - G.k0, tid = threadIdx.x, nth = blockDim.x;
    __shared__ GrpBlock B;
    grp_setup(G, m, B);
    const int32_t* st = B.st;
    const int32_t* cnt = B.cnt;
    const GrpLayout& L = B.L;
    stage_copy(sm, G.dpack + G.doff[blockIdx.x], L.dlen);
    stage_copy(sm + L.dx, G.scr + G.xoff[blockIdx.x], L.xlen);
    stage_copy(sm + L.dr0, G.r_in + st[0], cnt[0]);
    stage_copy(sm + L.dy[m], G.y_top + st[m], cnt[m]);
    __syncthreads();
    for (int j = m - 1; j >= 0; --j) {
        const int na = cnt[j + 1], nl = cnt[j] - 2 * na;
        const int* cp = reinterpret_cast<const int*>(sm + L.dcp[j]);
        const double* l0 = sm + L.dl[j];
        const double* l1 = l0 + nl;
        const double* l2 = l1 + nl;
        const double* rk = j == 0 ? sm + L.dr0 : sm + L.dx + L.xr[j];
        const double* e = sm + L.dx + L.xe[j];
        double* yk = sm + L.dy[j];
        const double* yk1 = sm + L.dy[j + 1];
        for (int J = tid; J < na; J += nth) {
            const int b0 = cp[J], b1 = cp[J + 1];
            const double yJ = yk1[J], ea = e[J], eb = e[na + J];
            yk[b0] = ea + yJ;
            yk[b0 + 1] = eb + yJ;
            for (int c = b0 + 2; c < b1; ++c) {
                const int li = c - 2 * J - 2;
                yk[c] = l0[li] * rk[c] + l1[li] * ea + l2[li] * eb + yJ;
            }
        }
        __syncthreads();
    }
    const double* y0 = sm + L.dy[0];
    double* out = G.y_out + st[0];
    for (int t = tid; t < cnt[0]; t += nth) out[t] = y0[t];
}

// ------------------------------------------------------------ coarse tail

// Levels kt .. top in one workgroup, entirely in LDS: the coefficients of
// those levels are staged from one packed device buffer with a coalesced
// copy, then restriction + local solves run upwards, theta_top pinv(L_top)
// on the top, prolongation + corrections back down to level kt.
__global__ __launch_bounds__(kTailThreads) void k_tail(const TailDesc* __restrict__ D,
                                                       const double* __restrict__ pack,
                                                       const double* __restrict__ r_kt,
                                                       double* __restrict__ y_kt, const Scal* S) {
    if (S->done) return;
    extern __shared__ double sm[];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int npack = D->pack, nsteps = D->nsteps;
    for (int i = tid; i < npack; i += nth) sm[i] = pack[i];
    {
        const int n0 = nsteps > 0 ? D->st[0].nk : D->nt;
        double* r0 = sm + D->r[0];
        for (int i = tid; i < n0; i += nth) r0[i] = r_kt[i];
    }
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
        const TailStep t = D->st[s];
        const int* cp = reinterpret_cast<const int*>(sm + t.cptr);
        const double* rk = sm + D->r[s];
        double* rk1 = sm + D->r[s + 1];
        for (int J = tid; J < t.nc; J += nth) {
            const int b0 = cp[J], b1 = cp[J + 1];
            const double ra = rk[b0], rb = rk[b0 + 1];
            double sum = ra + rb, ga = ra, gb = rb;
            for (int c = b0 + 2; c < b1; ++c) {
                const int li = c - 2 * J - 2;
                const double rv = rk[c];
                sum += rv;
                ga += sm[t.l1 + li] * rv;
                gb += sm[t.l2 + li] * rv;
            }
            const double saa = sm[t.saa + J], sab = sm[t.sab + J], sbb = sm[t.sbb + J];
            sm[t.ea + J] = saa * ga + sab * gb;
            sm[t.eb + J] = sab * ga + sbb * gb;
            rk1[J] = sum;
        }
        __syncthreads();
    }
    {
        const int nt = D->nt;
        const double* rT = sm + D->r[nsteps];
        double* yT = sm + D->y[nsteps];
        const double* tp = sm + D->pinv;
        for (int i = tid; i < nt; i += nth) {
            double acc = 0.0;
            for (int j = 0; j < nt; ++j) acc += tp[i * nt + j] * rT[j];
            yT[i] = acc;
        }
        __syncthreads();
    }
    for (int s = nsteps - 1; s >= 0; --s) {
        const TailStep t = D->st[s];
        const int* cp = reinterpret_cast<const int*>(sm + t.cptr);
        const double* rk = sm + D->r[s];
        double* yk = sm + D->y[s];
        const double* yk1 = sm + D->y[s + 1];
        for (int J = tid; J < t.nc; J += nth) {
            const int b0 = cp[J], b1 = cp[J + 1];
            const double yJ = yk1[J], ea = sm[t.ea + J], eb = sm[t.eb + J];
            yk[b0] = ea + yJ;
            yk[b0 + 1] = eb + yJ;
            for (int c = b0 + 2; c < b1; ++c) {
                const int li = c - 2 * J - 2;
                yk[c] = sm[t.l0 + li] * rk[c] + sm[t.l1 + li] * ea + sm[t.l2 + li] * eb + yJ;
            }
        }
        __syncthreads();
    }
    {
        const int n0 = nsteps > 0 ? D->st[0].nk : D->nt;
        const double* y0 = sm + D->y[0];
        for (int i = tid; i < n0; i += nth) y_kt[i] = y0[i];
    }
}

// ------------------------------------------------- solve set-up and finish

__global__ __launch_bounds__(kBlock) void k_sum(int n, const double* __restrict__ a,
                                                double* part) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    double v[1] = {t < n ? a[t] : 0.0};
    block_partial<1>(v, part);
}

// b^ = b - mean(b) (input order); r = b^ in tree order; x = p0 = p1 = 0;
// partial ||b^||^2.
__global__ __launch_bounds__(kBlock) void k_init(int n, const int32_t* __restrict__ perm,
                                                 const double* __restrict__ b,
                                                 double* __restrict__ bh, double* __restrict__ r,
                                                 double* __restrict__ x, double* __restrict__ p0,
                                                 double* __restrict__ p1, const Scal* S,
                                                 double* part) {
    const double mean = S->bsum / (double)n;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (t < n) {
        const double bt = b[t] - mean;
        bh[t] = bt;
        r[t] = b[perm[t]] - mean;
        x[t] = 0.0;
        p0[t] = 0.0;
        p1[t] = 0.0;
        v[0] = bt * bt;
    }
    block_partial<1>(v, part);
}

// xc = x - mean(x) and the caller's copy of it (input order).
__global__ __launch_bounds__(kBlock) void k_center_out(int n, const double* __restrict__ x,
                                                       double* __restrict__ xc,
                                                       double* __restrict__ dst, const Scal* S) {
    const double mean = S->xsum / (double)n;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < n) {
        const double v = x[t] - mean;
        xc[t] = v;
        dst[t] = v;
    }
}

// partial ||b^ - L x||^2 (input order).
__global__ __launch_bounds__(kBlock) void k_resid(int n, Sell A, const double* __restrict__ x,
                                                  const double* __restrict__ bh, double* part) {
    const int row = blockIdx.x * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (row < n) {
        const double xi = x[row];
        const int sl = row >> 6;
        const int base = A.off[sl] + (row & 63);
        const int W = A.width[sl];
        double acc = 0.0;
        for (int k = 0; k < W; ++k) acc += A.w[base + k * 64] * (xi - x[A.col[base + k * 64]]);
        const double d = bh[row] - acc;
        v[0] = d * d;
    }
    block_partial<1>(v, part);
}

// y = L x (input order).
__global__ __launch_bounds__(kBlock) void k_spmv_plain(int n, Sell A, const double* __restrict__ x,
                                                       double* __restrict__ y) {
    const int row = blockIdx.x * kBlock + threadIdx.x;
    if (row >= n) return;
    const double xi = x[row];
    const int sl = row >> 6;
    const int base = A.off[sl] + (row & 63);
    const int W = A.width[sl];
    double acc = 0.0;
    for (int k = 0; k < W; ++k) acc += A.w[base + k * 64] * (xi - x[A.col[base + k * 64]]);
    y[row] = acc;
}

// dst[t] = src[perm[t]] (input order -> tree order).
__global__ __launch_bounds__(kBlock) void k_gather(int n, const int32_t* __restrict__ perm,
                                                   const double* __restrict__ src,
                                                   double* __restrict__ dst) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < n) dst[t] = src[perm[t]];
}

// dst = src - zbar (input order).
__global__ __launch_bounds__(kBlock) void k_shift_out(int n, const double* __restrict__ src,
                                                      double* __restrict__ dst, const Scal* S) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < n) dst[t] = src[t] - S->zbar;
}

}  // namespace lapgpu

// ====================================================================== host

using namespace lapgpu;

namespace {

inline int nblk(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

struct HipErr {};
thread_local char g_last_error[256] = "";

void record_error(const char* what, hipError_t e, int line) {
    std::snprintf(g_last_error, sizeof(g_last_error), "lap.hip:%d %s -> %s (%d)", line, what,
                  hipGetErrorString(e), (int)e);
    if (std::getenv("LAPGPU_DEBUG")) std::fprintf(stderr, "[lapgpu] %s\n", g_last_error);
}

#define HIPCHK(expr)                                      \
    do {                                                  \
        const hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) {                           \
            record_error(#expr, e_, __LINE__);            \
            throw HipErr();                               \
        }                                                 \
    } while (0)

int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    return v ? std::atoi(v) : dflt;
}

constexpr size_t kTailLdsBytes = 152 * 1024;
constexpr int kGrpLdsDoubles = 8192;    // 64 KB per group block

// Block partition of one aggregation step for the level kernels: runs of
// at most kAggPerBlock consecutive aggregates whose children fit kCapP; an
// aggregate with more children than kCapP forms a block of its own.
std::vector<int32_t> block_partition(const std::vector<int32_t>& cptr) {
    const int32_t nc = (int32_t)cptr.size() - 1;
    std::vector<int32_t> bst{0};
    int32_t J0 = 0;
    while (J0 < nc) {
        int32_t J1 = J0 + 1;
        if (cptr[J1] - cptr[J0] <= kCapP)
            while (J1 < nc && J1 - J0 < kAggPerBlock && cptr[J1 + 1] - cptr[J0] <= kCapP) ++J1;
        bst.push_back(J1);
        J0 = J1;
    }
    return bst;
}

// Doubles of LDS the tail needs when it starts at level kt.
size_t tail_lds_doubles(const HostPlan& P, int kt) {
    const int T = P.nlev() - 1;
    size_t d = 0;
    for (int k = kt; k < T; ++k) {
        const size_t nk = P.lv[k].g.n, nc = P.lv[k + 1].g.n, nl = nk - 2 * nc;
        d += (nc + 2) / 2 + 3 * nc + 3 * nl + 2 * nc;   // cptr, pair, leftover, eta
    }
    for (int k = kt; k <= T; ++k) d += 2 * P.lv[k].g.n;     // r, y
    d += P.lv[T].g.n * P.lv[T].g.n;                        // top pseudo-inverse
    return d;
}

// Pack the tail coefficients of levels kt..T into one buffer and lay out
// the LDS work space after it.
void build_tail(const HostPlan& P, int kt, TailDesc& D, std::vector<double>& pack) {
    const int T = P.nlev() - 1;
    D.nsteps = T - kt;
    D.nt = (int32_t)P.lv[T].g.n;
    auto put = [&](const double* src, size_t cnt) {
        const int32_t off = (int32_t)pack.size();
        pack.insert(pack.end(), src, src + cnt);
        return off;
    };
    for (int s = 0; s < D.nsteps; ++s) {
        const int k = kt + s;
        const StepCoef& c = P.step[k];
        TailStep& t = D.st[s];
        t.nk = (int32_t)P.lv[k].g.n;
        t.nc = (int32_t)P.lv[k + 1].g.n;
        t.nl = t.nk - 2 * t.nc;
        t.cptr = (int32_t)pack.size();
        const size_t cslots = (c.cptr.size() + 1) / 2;
        pack.resize(pack.size() + cslots, 0.0);
        std::memcpy(pack.data() + t.cptr, c.cptr.data(), c.cptr.size() * sizeof(int32_t));
        t.saa = put(c.saa.data(), c.saa.size());
        t.sab = put(c.sab.data(), c.sab.size());
        t.sbb = put(c.sbb.data(), c.sbb.size());
        t.l0 = put(c.l0.data(), c.l0.size());
        t.l1 = put(c.l1.data(), c.l1.size());
        t.l2 = put(c.l2.data(), c.l2.size());
    }
    D.pinv = put(P.top_pinv.data(), P.top_pinv.size());
    D.pack = (int32_t)pack.size();
    int32_t w = D.pack;
    for (int s = 0; s <= D.nsteps; ++s) {
        const int32_t nk = (int32_t)P.lv[kt + s].g.n;
        D.r[s] = w; w += nk;
        D.y[s] = w; w += nk;
    }
    for (int s = 0; s < D.nsteps; ++s) {
        D.st[s].ea = w; w += D.st[s].nc;
        D.st[s].eb = w; w += D.st[s].nc;
    }
    D.total = w;
}

// Partition the level-k1 nodes into blocks of whole subtrees for the group
// [k0, k1): each block's level-k0 range holds at most `cap` nodes and its
// LDS layouts (up and down) fit kGrpLdsDoubles.  Fails if one subtree alone
// does not fit.
bool plan_group(const HostPlan& P, int k0, int k1, int cap, std::vector<int32_t>& D,
                int& nblocks, size_t& lds_up, size_t& lds_down) {
    const int m = k1 - k0;
    const int64_t nroot = P.lv[k1].g.n;
    std::vector<std::vector<int32_t>> first(m + 1, std::vector<int32_t>(nroot + 1));
    for (int64_t R = 0; R <= nroot; ++R) first[m][R] = (int32_t)R;
    for (int j = m - 1; j >= 0; --j) {
        const std::vector<int32_t>& cptr = P.step[k0 + j].cptr;
        for (int64_t R = 0; R <= nroot; ++R) first[j][R] = cptr[first[j + 1][R]];
    }
    int32_t cnt[kMaxGroupLevels + 1];
    GrpLayout lay;
    auto fits = [&](int64_t A, int64_t B) {
        for (int j = 0; j <= m; ++j) cnt[j] = first[j][B] - first[j][A];
        grp_layout(m, cnt, lay);
        return cnt[0] <= cap && lay.utotal <= kGrpLdsDoubles && lay.dtotal <= kGrpLdsDoubles;
    };
    std::vector<int64_t> cuts{0};
    int32_t up = 0, dn = 0;
    while (cuts.back() < nroot) {
        const int64_t A = cuts.back();
        if (!fits(A, A + 1)) return false;
        int64_t lo = A + 1, hi = nroot;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if (fits(A, mid)) lo = mid;
            else hi = mid - 1;
        }
        fits(A, lo);
        up = std::max(up, lay.utotal);
        dn = std::max(dn, lay.dtotal);
        cuts.push_back(lo);
    }
    nblocks = (int)cuts.size() - 1;
    D.assign((size_t)(m + 1) * (nblocks + 1), 0);
    for (int j = 0; j <= m; ++j)
        for (int b = 0; b <= nblocks; ++b) D[(size_t)j * (nblocks + 1) + b] = first[j][cuts[b]];
    lds_up = (size_t)up * sizeof(double);
    lds_down = (size_t)dn * sizeof(double);
    return true;
}

// Pack one group's per-block coefficients in the order of grp_layout.
void pack_group(const HostPlan& P, int k0, int k1, int nblocks, const std::vector<int32_t>& D,
                std::vector<int32_t>& uoff, std::vector<int32_t>& doff,
                std::vector<int32_t>& xoff, std::vector<double>& up, std::vector<double>& dn) {
    const int m = k1 - k0, nb1 = nblocks + 1;
    uoff.assign(nb1, 0);
    doff.assign(nb1, 0);
    xoff.assign(nb1, 0);
    up.clear();
    dn.clear();
    int32_t cnt[kMaxGroupLevels + 1], st[kMaxGroupLevels + 1];
    GrpLayout L;
    for (int b = 0; b < nblocks; ++b) {
        for (int j = 0; j <= m; ++j) {
            st[j] = D[(size_t)j * nb1 + b];
            cnt[j] = D[(size_t)j * nb1 + b + 1] - st[j];
        }
        grp_layout(m, cnt, L);
        const size_t ub = up.size(), db = dn.size();
        up.resize(ub + L.ulen, 0.0);
        dn.resize(db + L.dlen, 0.0);
        for (int j = 0; j < m; ++j) {
            const StepCoef& c = P.step[k0 + j];
            const int na = cnt[j + 1], nl = cnt[j] - 2 * na, a0 = st[j + 1], c0 = st[j];
            const int lb = c0 - 2 * a0;
            int32_t* ucp = reinterpret_cast<int32_t*>(up.data() + ub + L.ucp[j]);
            int32_t* dcp = reinterpret_cast<int32_t*>(dn.data() + db + L.dcp[j]);
            for (int i = 0; i <= na; ++i) ucp[i] = dcp[i] = c.cptr[a0 + i] - c0;
            for (int i = 0; i < na; ++i) {
                up[ub + L.us[j] + i] = c.saa[a0 + i];
                up[ub + L.us[j] + na + i] = c.sab[a0 + i];
                up[ub + L.us[j] + 2 * na + i] = c.sbb[a0 + i];
            }
            for (int i = 0; i < nl; ++i) {
                up[ub + L.ul[j] + i] = c.l1[lb + i];
                up[ub + L.ul[j] + nl + i] = c.l2[lb + i];
                dn[db + L.dl[j] + i] = c.l0[lb + i];
                dn[db + L.dl[j] + nl + i] = c.l1[lb + i];
                dn[db + L.dl[j] + 2 * nl + i] = c.l2[lb + i];
            }
        }
        uoff[b + 1] = (int32_t)up.size();
        doff[b + 1] = (int32_t)dn.size();
        xoff[b + 1] = xoff[b] + L.xlen;
    }
}

}  // namespace

struct lap_hierarchy {
    HostPlan plan;
    lap_params params{};
    bool host_only = false;
    bool with_msp = true;
    int64_t n = 0;
    int device = 0;
    double setup_seconds = 0.0;
    int64_t dev_bytes = 0;
    std::vector<void*> allocs;
    // device data
    int32_t* perm0 = nullptr;    // tree position -> input vertex
    Sell A{};
    std::vector<LevelDev> lv;    // host copy of the level table
    double* top_pinv = nullptr;
    int kt = 1;                  // first level of the one-block tail
    TailDesc* d_tail = nullptr;
    double* tail_pack = nullptr;
    size_t tail_lds = 0;
    struct Segment {
        bool group = false;
        int k0 = 0, k1 = 1;
        GroupDev gd{};
        size_t lds_up = 0, lds_down = 0;   // bytes of dynamic LDS
    };
    std::vector<Segment> segs;   // levels [1, kt), in order
    // workspace: input order
    double *x = nullptr, *p[2] = {nullptr, nullptr}, *q = nullptr, *zn = nullptr;
    double *bh = nullptr, *xc = nullptr;
    // workspace: tree order
    double *r = nullptr, *z = nullptr;
    Scal* S = nullptr;
    double* part = nullptr;      // per-block partial sums of the last producer
    double* part2 = nullptr;     // per-block ||r||^2 of the update kernel
    Scal* stage = nullptr;       // pinned host copy of S
    hipStream_t cap = nullptr;   // private capture stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int chunk = 8;

    template <class T>
    T* dalloc(size_t count) {
        void* ptr = nullptr;
        const size_t bytes = (count ? count : 1) * sizeof(T);
        if (hipMalloc(&ptr, bytes) != hipSuccess) throw std::bad_alloc();
        allocs.push_back(ptr);
        dev_bytes += (int64_t)bytes;
        return static_cast<T*>(ptr);
    }
    // Uploads complete before return (host vectors may be temporaries).
    template <class T>
    T* upload(const std::vector<T>& v, hipStream_t s) {
        T* d = dalloc<T>(v.size());
        if (!v.empty()) {
            HIPCHK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        return d;
    }
    ~lap_hierarchy() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
        for (void* ptr : allocs) (void)hipFree(ptr);
        if (stage) (void)hipHostFree(stage);
    }
};

namespace {

// One-block finish of the partials at `part` (G blocks); kFinRho may also
// take the update kernel's ||r||^2 partials (G2 blocks at part2).
template <int OP>
void finish(lap_hierarchy* h, hipStream_t s, int G, int G2 = 0, const double* part = nullptr) {
    hipLaunchKernelGGL(k_finish<OP>, dim3(1), dim3(kFinThreads), 0, s, G, (int)h->n,
                       part ? part : h->part, G2, h->part2, h->S);
}

// The preconditioner: level-0 restriction (with the x, r update when
// do_update), the middle levels, the tail and back, z with its reductions.
// Optional timing of one part of the iteration (lap_profile_kernel): the
// part's first and last kernels carry HIP events that take the kernels' own
// start and end timestamps, so the part is timed in the cache state of a
// real iteration, with no marker packets between the kernels.
struct Marks {
    int kernel = -1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipEvent_t start(int k) const { return kernel == k ? e0 : nullptr; }
    hipEvent_t stop(int k) const { return kernel == k ? e1 : nullptr; }
};

template <class F, class... A>
void launch_timed(F kern, dim3 grid, dim3 block, uint32_t lds, hipStream_t s, hipEvent_t e0,
                  hipEvent_t e1, A... args) {
    if (e0 || e1) hipExtLaunchKernelGGL(kern, grid, block, lds, s, e0, e1, 0, args...);
    else hipLaunchKernelGGL(kern, grid, block, lds, s, args...);
}

void enqueue_precond(lap_hierarchy* h, hipStream_t s, int do_update, const double* pcur,
                     const Marks& mk = Marks{}) {
    const int T = h->plan.nlev() - 1;
    const int n = (int)h->n;
    if (!h->with_msp || T == 0) {
        if (do_update) {
            hipLaunchKernelGGL(k_update_none, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->perm0, h->x,
                               h->r, pcur, h->q, h->S, h->part2);
            if (h->with_msp) finish<kFinRr>(h, s, nblk(n), 0, h->part2);
        }
        if (!h->with_msp) {
            hipLaunchKernelGGL(k_prec_none, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->perm0, h->r,
                               h->z, h->zn, h->S, h->part);
            finish<kFinRho>(h, s, nblk(n), do_update ? nblk(n) : 0);
        } else {
            hipLaunchKernelGGL(k_top_only, dim3(1), dim3(kBlock), 0, s, n, h->perm0, h->top_pinv,
                               h->r, h->z, h->zn, h->S);
        }
        return;
    }
    const LevelDev& s0 = h->lv[0];
    const int g0 = s0.nb;
    launch_timed(k_update_up0, dim3(g0), dim3(kBlock), 0, s,
                 mk.kernel == LAP_KERNEL_PRECOND ? mk.e0 : mk.start(LAP_KERNEL_UPDATE),
                 mk.stop(LAP_KERNEL_UPDATE), s0, (const int32_t*)h->perm0, h->x, h->r, pcur,
                 (const double*)h->q, h->lv[1].r, h->S, h->part2, do_update);
    for (const auto& G : h->segs) {
        if (G.group)
            hipLaunchKernelGGL(k_up_grp, dim3(G.gd.nblocks), dim3(kGrpThreads), G.lds_up, s, G.gd,
                               h->S);
        else
            hipLaunchKernelGGL(k_up, dim3(h->lv[G.k0].nb), dim3(kBlock), 0, s, h->lv[G.k0],
                               h->lv[G.k0].r, h->lv[G.k0 + 1].r, h->S);
    }
    hipLaunchKernelGGL(k_tail, dim3(1), dim3(kTailThreads), h->tail_lds, s, h->d_tail,
                       h->tail_pack, h->lv[h->kt].r, h->lv[h->kt].y, h->S);
    for (auto it = h->segs.rbegin(); it != h->segs.rend(); ++it) {
        const auto& G = *it;
        if (G.group)
            hipLaunchKernelGGL(k_down_grp, dim3(G.gd.nblocks), dim3(kGrpThreads), G.lds_down, s,
                               G.gd, h->S);
        else
            hipLaunchKernelGGL(k_down, dim3(h->lv[G.k0].nb), dim3(kBlock), 0, s,
                               h->lv[G.k0], h->lv[G.k0].r, h->lv[G.k0].y, h->lv[G.k0 + 1].y, h->S);
    }
    launch_timed(k_down0, dim3(g0), dim3(kBlock), 0, s, mk.start(LAP_KERNEL_DOWN0),
                 mk.kernel == LAP_KERNEL_PRECOND ? mk.e1 : mk.stop(LAP_KERNEL_DOWN0), s0,
                 (const int32_t*)h->perm0, (const double*)h->r, h->zn, (const double*)h->lv[1].y,
                 h->S, h->part);
    finish<kFinRho>(h, s, g0, do_update ? g0 : 0);
}

// One PCG iteration reading p[par] and writing p[1-par].
void enqueue_iteration(lap_hierarchy* h, hipStream_t s, int par, const Marks& mk = Marks{}) {
    const int n = (int)h->n;
    launch_timed(k_spmv_p, dim3(nblk(n)), dim3(kBlock), 0, s, mk.start(LAP_KERNEL_SPMV),
                 mk.stop(LAP_KERNEL_SPMV), n, h->A, (const double*)h->zn,
                 (const double*)h->p[par], h->p[1 - par], h->q, h->S, h->part);
    finish<kFinPq>(h, s, nblk(n));
    enqueue_precond(h, s, 1, h->p[1 - par], mk);
}

void build_graph(lap_hierarchy* h) {
    HIPCHK(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < h->chunk; ++i) enqueue_iteration(h, h->cap, i & 1);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamEndCapture(h->cap, &h->graph));
    HIPCHK(hipGraphInstantiate(&h->exec, h->graph, nullptr, nullptr, 0));
}

void upload_plan(lap_hierarchy* h, hipStream_t s) {
    const HostPlan& P = h->plan;
    const int L = P.nlev();
    const int T = L - 1;
    const int64_t n = h->n;
    h->perm0 = h->upload(P.perm[0], s);
    h->A.off = h->upload(P.sell_off, s);
    h->A.width = h->upload(P.sell_width, s);
    h->A.col = h->upload(P.sell_col, s);
    h->A.w = h->upload(P.sell_w, s);
    h->with_msp = (h->params.precond == LAP_PREC_MSP);
    h->r = h->dalloc<double>(n);
    h->z = h->dalloc<double>(n);
    // the tail: the lowest level from which all coarser levels fit in LDS
    const int tail_max = env_int("LAPGPU_TAIL_MAX", 1 << 30);
    h->kt = T;
    for (int k = 1; k <= T; ++k)
        if (P.lv[k].g.n <= tail_max && T - k <= kMaxTailSteps &&
            tail_lds_doubles(P, k) * sizeof(double) <= kTailLdsBytes) {
            h->kt = k;
            break;
        }
    h->lv.assign(L, LevelDev{});
    for (int k = 0; k < L; ++k) {
        LevelDev& d = h->lv[k];
        d.n = (int32_t)P.lv[k].g.n;
        d.nc = k < T ? (int32_t)P.lv[k + 1].g.n : 0;
        if (k >= 1) {
            d.r = h->dalloc<double>(d.n);
            d.y = h->dalloc<double>(d.n);
        } else {
            d.r = h->r;
            d.y = h->z;
        }
        if (k < T) {
            const StepCoef& c = P.step[k];
            d.cptr = h->upload(c.cptr, s);
            d.saa = h->upload(c.saa, s);
            d.sab = h->upload(c.sab, s);
            d.sbb = h->upload(c.sbb, s);
            d.l0 = h->upload(c.l0, s);
            d.l1 = h->upload(c.l1, s);
            d.l2 = h->upload(c.l2, s);
            d.ea = h->dalloc<double>(d.nc);
            d.eb = h->dalloc<double>(d.nc);
            const std::vector<int32_t> bst = block_partition(c.cptr);
            d.nb = (int32_t)bst.size() - 1;
            d.bst = h->upload(bst, s);
        }
    }
    h->top_pinv = h->upload(P.top_pinv, s);
    // middle levels [1, kt): groups of consecutive levels where whole
    // subtrees fit a block, single per-level kernels elsewhere
    h->segs.clear();
    const int cap = env_int("LAPGPU_GRP_CAP", 1024);
    const int maxlev = std::min(kMaxGroupLevels, env_int("LAPGPU_GRP_MAXLEV", kMaxGroupLevels));
    const int first_grouped = std::max(1, env_int("LAPGPU_GRP_FIRST", 2));
    for (int k0 = 1; T >= 1 && k0 < h->kt;) {
        lap_hierarchy::Segment sg;
        bool placed = false;
        for (int m = std::min(maxlev, h->kt - k0); m >= 1 && !placed && k0 >= first_grouped; --m) {
            std::vector<int32_t> D;
            int nb = 0;
            if (!plan_group(P, k0, k0 + m, cap, D, nb, sg.lds_up, sg.lds_down)) continue;
            sg.group = true;
            sg.k0 = k0;
            sg.k1 = k0 + m;
            sg.gd.k0 = k0;
            sg.gd.k1 = k0 + m;
            sg.gd.nblocks = nb;
            sg.gd.D = h->upload(D, s);
            std::vector<int32_t> uoff, doff, xoff;
            std::vector<double> up, dn;
            pack_group(P, k0, k0 + m, nb, D, uoff, doff, xoff, up, dn);
            sg.gd.uoff = h->upload(uoff, s);
            sg.gd.doff = h->upload(doff, s);
            sg.gd.xoff = h->upload(xoff, s);
            sg.gd.upack = h->upload(up, s);
            sg.gd.dpack = h->upload(dn, s);
            sg.gd.scr = h->dalloc<double>(xoff.back());
            sg.gd.r_top = h->lv[k0 + m].r;
            sg.gd.y_top = h->lv[k0 + m].y;
            sg.gd.r_in = h->lv[k0].r;
            sg.gd.y_out = h->lv[k0].y;
            placed = true;
        }
        if (!placed) {
            sg.group = false;
            sg.k0 = k0;
            sg.k1 = k0 + 1;
        }
        k0 = sg.k1;
        h->segs.push_back(sg);
    }
    if (T >= 1) {
        TailDesc desc{};
        std::vector<double> pack;
        build_tail(P, h->kt, desc, pack);
        h->tail_pack = h->upload(pack, s);
        h->d_tail = h->dalloc<TailDesc>(1);
        HIPCHK(hipMemcpyAsync(h->d_tail, &desc, sizeof(desc), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
        h->tail_lds = (size_t)desc.total * sizeof(double);
        HIPCHK(hipFuncSetAttribute((const void*)k_tail,
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)kTailLdsBytes));
        HIPCHK(hipFuncSetAttribute((const void*)k_up_grp,
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   kGrpLdsDoubles * 8));
        HIPCHK(hipFuncSetAttribute((const void*)k_down_grp,
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   kGrpLdsDoubles * 8));
    }
    h->x = h->dalloc<double>(n);
    h->q = h->dalloc<double>(n);
    h->zn = h->dalloc<double>(n);
    h->bh = h->dalloc<double>(n);
    h->xc = h->dalloc<double>(n);
    h->p[0] = h->dalloc<double>(n);
    h->p[1] = h->dalloc<double>(n);
    h->S = h->dalloc<Scal>(1);
    int gmax = nblk(n);
    for (const LevelDev& d : h->lv) gmax = std::max(gmax, (int)d.nb);
    h->part = h->dalloc<double>((size_t)kMaxGridPart * gmax + 64);
    h->part2 = h->dalloc<double>((size_t)gmax + 64);
    HIPCHK(hipHostMalloc((void**)&h->stage, sizeof(Scal), hipHostMallocDefault));
    std::memset(h->stage, 0, sizeof(Scal));
    HIPCHK(hipMemcpyAsync(h->S, h->stage, sizeof(Scal), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipGetLastError());
    h->chunk = std::max(2, env_int("LAPGPU_CHUNK", 8) & ~1);
    build_graph(h);
}

lap_status to_status(int done) {
    switch (done) {
        case 1: return LAP_OK;
        case 2: return LAP_ENOCONV;
        case 3: return LAP_EBREAKDOWN;
        case 4: return LAP_EINVAL;
        default: return LAP_EDEVICE;
    }
}

lap_status solve_one(lap_hierarchy* h, const double* b, double* x, double tol,
                     lap_solve_info* info, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const int n = (int)h->n;
    // reset the scalars and set the run parameters
    std::memset(h->stage, 0, sizeof(Scal));
    h->stage->tol2 = tol * tol;
    h->stage->maxit = h->params.max_iter;
    HIPCHK(hipMemcpyAsync(h->S, h->stage, sizeof(Scal), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_sum, dim3(nblk(n)), dim3(kBlock), 0, s, n, b, h->part);
    finish<kFinBsum>(h, s, nblk(n));
    hipLaunchKernelGGL(k_init, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->perm0, b, h->bh, h->r,
                       h->x, h->p[0], h->p[1], h->S, h->part);
    finish<kFinBn2>(h, s, nblk(n));
    enqueue_precond(h, s, 0, h->p[0]);
    HIPCHK(hipGetLastError());
    // chunks of iterations; one chunk in flight beyond the one being checked
    hipEvent_t ev;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    const int max_chunks = h->params.max_iter / h->chunk + 2;
    try {
        HIPCHK(hipGraphLaunch(h->exec, s));
        for (int c = 0; c < max_chunks; ++c) {
            HIPCHK(hipMemcpyAsync(h->stage, h->S, sizeof(Scal), hipMemcpyDeviceToHost, s));
            HIPCHK(hipEventRecord(ev, s));
            HIPCHK(hipGraphLaunch(h->exec, s));
            HIPCHK(hipEventSynchronize(ev));
            if (h->stage->done) break;
        }
    } catch (const HipErr&) {
        (void)hipEventDestroy(ev);
        throw;
    }
    (void)hipEventDestroy(ev);
    // mean-free x (input order), true residual
    hipLaunchKernelGGL(k_sum, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->x, h->part);
    finish<kFinXsum>(h, s, nblk(n));
    hipLaunchKernelGGL(k_center_out, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->x, h->xc, x, h->S);
    hipLaunchKernelGGL(k_resid, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->A, h->xc, h->bh,
                       h->part);
    finish<kFinRes2>(h, s, nblk(n));
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(h->stage, h->S, sizeof(Scal), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const Scal& S = *h->stage;
    const lap_status st = S.done == 0 ? LAP_ENOCONV : to_status(S.done);
    if (info) {
        const double bn = std::sqrt(S.bn2);
        info->iterations = S.iter;
        info->refinements = 0;
        info->relres_true = bn > 0 ? std::sqrt(S.res2) / bn : 0.0;
        info->relres_recursive = bn > 0 ? std::sqrt(S.rr) / bn : 0.0;
        info->status = st;
        info->seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return st;
}

int rank_status(lap_status s) {
    switch (s) {
        case LAP_OK: return 0;
        case LAP_ENOCONV: return 1;
        case LAP_EBREAKDOWN: return 2;
        default: return 3;
    }
}

}  // namespace

// =================================================================== C ABI

extern "C" {

lap_status lap_default_params(lap_params* p) {
    if (!p) return LAP_EINVAL;
    p->mu = 0.8;
    p->max_levels = 0;
    p->n_top = 2;
    p->mwm_seed = 0;
    p->precond = LAP_PREC_MSP;
    p->precision = LAP_FP64;
    p->max_iter = 1000;
    p->flags = 0;
    return LAP_OK;
}

const char* lap_status_str(lap_status s) {
    switch (s) {
        case LAP_OK: return "LAP_OK";
        case LAP_EINVAL: return "LAP_EINVAL";
        case LAP_EDISCONNECTED: return "LAP_EDISCONNECTED";
        case LAP_ENOMEM: return "LAP_ENOMEM";
        case LAP_EDEVICE: return "LAP_EDEVICE";
        case LAP_ENOCONV: return "LAP_ENOCONV";
        case LAP_EBREAKDOWN: return "LAP_EBREAKDOWN";
        case LAP_EUNSUPPORTED: return "LAP_EUNSUPPORTED";
    }
    return "LAP_UNKNOWN";
}

lap_status lap_setup(const lap_graph* g, const lap_params* p, void* stream, lap_hierarchy** out) {
    if (!out) return LAP_EINVAL;
    *out = nullptr;
    if (!g || !p || !g->u || !g->v || !g->w) return LAP_EINVAL;
    if (p->precond != LAP_PREC_MSP && p->precond != LAP_PREC_NONE)
        return p->precond == LAP_PREC_PEGP ? LAP_EUNSUPPORTED : LAP_EINVAL;
    if (p->precision != LAP_FP64) return LAP_EINVAL;
    if (p->max_iter < 0) return LAP_EINVAL;
    const auto t0 = std::chrono::steady_clock::now();
    lap_hierarchy* h = new (std::nothrow) lap_hierarchy();
    if (!h) return LAP_ENOMEM;
    h->params = *p;
    h->host_only = (p->flags & LAP_FLAG_HOST_ONLY) != 0;
    try {
        const int rc = build_plan(g->n, g->m, g->u, g->v, g->w, p->mu, p->max_levels, p->n_top,
                                  p->mwm_seed, h->host_only, h->plan);
        if (rc != kOk) {
            delete h;
            return (lap_status)rc;
        }
        h->n = g->n;
        if (!h->host_only) {
            int ndev = 0;
            if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
                std::snprintf(g_last_error, sizeof(g_last_error), "no HIP device visible");
                delete h;
                return LAP_EDEVICE;
            }
            HIPCHK(hipGetDevice(&h->device));
            upload_plan(h, (hipStream_t)stream);
        }
    } catch (const std::bad_alloc&) {
        delete h;
        return LAP_ENOMEM;
    } catch (const HipErr&) {
        delete h;
        return LAP_EDEVICE;
    }
    h->setup_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = h;
    return LAP_OK;
}

lap_status lap_solve(lap_hierarchy* h, const double* b, double* x, int32_t nrhs, int64_t ld,
                     double tol, lap_solve_info* info, void* stream) {
    if (!h || !b || !x || nrhs < 1 || ld < h->n || !(tol > 0.0) || !std::isfinite(tol))
        return LAP_EINVAL;
    if (h->host_only) return LAP_EUNSUPPORTED;
    lap_status worst = LAP_OK;
    try {
        for (int c = 0; c < nrhs; ++c) {
            const lap_status st = solve_one(h, b + (int64_t)c * ld, x + (int64_t)c * ld, tol,
                                            info ? info + c : nullptr, (hipStream_t)stream);
            if (rank_status(st) > rank_status(worst)) worst = st;
        }
    } catch (const HipErr&) {
        return LAP_EDEVICE;
    }
    return worst;
}

lap_status lap_apply_laplacian(lap_hierarchy* h, const double* x, double* y, void* stream) {
    if (!h || !x || !y) return LAP_EINVAL;
    if (h->host_only) return LAP_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const int n = (int)h->n;
    hipLaunchKernelGGL(k_spmv_plain, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->A, x, y);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        record_error("k_spmv_plain launch", e, __LINE__);
        return LAP_EDEVICE;
    }
    return LAP_OK;
}

lap_status lap_apply_precond(lap_hierarchy* h, const double* r, double* z, void* stream) {
    if (!h || !r || !z) return LAP_EINVAL;
    if (h->host_only) return LAP_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const int n = (int)h->n;
    try {
        std::memset(h->stage, 0, sizeof(Scal));
        h->stage->first = 1;
        HIPCHK(hipMemcpyAsync(h->S, h->stage, sizeof(Scal), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_gather, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->perm0, r, h->r);
        enqueue_precond(h, s, 0, h->p[0]);
        hipLaunchKernelGGL(k_shift_out, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->zn, z, h->S);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s));
    } catch (const HipErr&) {
        return LAP_EDEVICE;
    }
    return LAP_OK;
}

lap_status lap_profile_kernel(lap_hierarchy* h, int32_t kernel, int32_t reps, void* stream,
                              double* avg_ms, double* alg_bytes) {
    if (!h || reps < 1 || kernel < 0 || kernel > LAP_KERNEL_ITER) return LAP_EINVAL;
    if (h->host_only) return LAP_EUNSUPPORTED;
    const int T = h->plan.nlev() - 1;
    const bool levels = h->with_msp && T >= 1;
    if ((kernel == LAP_KERNEL_UPDATE || kernel == LAP_KERNEL_DOWN0 ||
         kernel == LAP_KERNEL_PRECOND) && !levels)
        return LAP_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    // Algorithmic bytes: FP64 values, int32 indices, each datum a step needs
    // counted once (a permuted access counts as one value).
    const double n = (double)h->n, nnz = (double)h->plan.lv[0].g.nnz();
    auto lvn = [&](int k) { return (double)h->plan.lv[k].g.n; };
    // step k (level k -> k+1), up: r_k; cptr, pair coefficients, leftover
    // coefficients (2); eta a/b and the restricted value written.
    auto step_up = [&](int k) {
        const double nc = lvn(k + 1), nl = lvn(k) - 2.0 * lvn(k + 1);
        return 8.0 * lvn(k) + 4.0 * nc + 24.0 * nc + 16.0 * nl + 24.0 * nc;
    };
    // down: cptr, eta a/b, y_k+1; leftover coefficients (3) and residuals;
    // y_k written.
    auto step_down = [&](int k) {
        const double nc = lvn(k + 1), nl = lvn(k) - 2.0 * lvn(k + 1);
        return 4.0 * nc + 16.0 * nc + 8.0 * nc + 24.0 * nl + 8.0 * nl + 8.0 * lvn(k);
    };
    const double spmv = 32.0 * n + 12.0 * nnz;
    // update_up0: x, p, q, r in; x, r out; plus the step-0 restriction
    // without re-reading r.
    const double upd = levels ? 48.0 * n + step_up(0) - 8.0 * n : 48.0 * n;
    // down0: step-0 prolongation (its residual read serves the dots too);
    // z written once, in input order
    const double down0 = levels ? step_down(0) - 8.0 * (lvn(0) - 2.0 * lvn(1)) + 8.0 * n : 24.0 * n;
    // middle levels and the tail (their data is not re-counted by update/down0)
    double mid = 0.0;
    for (int k = 1; levels && k < T; ++k) mid += step_up(k) + step_down(k);
    double bytes = 0.0;
    switch (kernel) {
        case LAP_KERNEL_SPMV: bytes = spmv; break;
        case LAP_KERNEL_UPDATE: bytes = upd; break;
        case LAP_KERNEL_DOWN0: bytes = down0; break;
        case LAP_KERNEL_PRECOND: bytes = upd + mid + down0; break;
        default: bytes = spmv + (levels ? upd + mid + down0 : 96.0 * n); break;
    }
    // ITER: two events around all timed iterations; a part: its own kernels'
    // timestamps in every timed iteration
    const bool whole = kernel == LAP_KERNEL_ITER;
    std::vector<hipEvent_t> ev(whole ? 2 : 2 * (size_t)reps, nullptr);
    auto destroy = [&]() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    try {
        std::memset(h->stage, 0, sizeof(Scal));
        h->stage->maxit = 0x7fffffff;
        h->stage->rho = 1.0;
        h->stage->bn2 = 1.0;
        HIPCHK(hipMemcpyAsync(h->S, h->stage, sizeof(Scal), hipMemcpyHostToDevice, s));
        for (auto& e : ev) HIPCHK(hipEventCreate(&e));
        enqueue_iteration(h, s, 1);   // untimed
        if (whole) HIPCHK(hipEventRecord(ev[0], s));
        for (int i = 0; i < reps; ++i) {
            Marks mk;
            if (!whole) {
                mk.kernel = kernel;
                mk.e0 = ev[2 * i];
                mk.e1 = ev[2 * i + 1];
            }
            enqueue_iteration(h, s, i & 1, mk);
        }
        if (whole) HIPCHK(hipEventRecord(ev[1], s));
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s));
        double total = 0.0;
        for (size_t i = 0; i < ev.size(); i += 2) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
            total += ms;
        }
        if (avg_ms) *avg_ms = total / reps;
        if (alg_bytes) *alg_bytes = bytes;
        HIPCHK(hipMemcpyAsync(h->stage, h->S, sizeof(Scal), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const bool ran = h->stage->done == 0;
        destroy();
        return ran ? LAP_OK : LAP_EBREAKDOWN;
    } catch (const HipErr&) {
        destroy();
        return LAP_EDEVICE;
    }
}

lap_status lap_hierarchy_info(const lap_hierarchy* h, lap_hierarchy_desc* d) {
    if (!h || !d) return LAP_EINVAL;
    std::memset(d, 0, sizeof(*d));
    d->nlev = h->plan.nlev();
    d->tail_level = h->kt;
    for (int k = 0; k < d->nlev && k < LAP_MAX_LEVELS; ++k) {
        d->sizes[k] = h->plan.lv[k].g.n;
        d->ntilde += d->sizes[k];
    }
    d->nnz = h->plan.lv[0].g.nnz();
    d->device_bytes = h->dev_bytes;
    d->setup_seconds = h->setup_seconds;
    return LAP_OK;
}

lap_status lap_export_level(const lap_hierarchy* h, int32_t level, int64_t* agg, int8_t* matched) {
    if (!h || level < 0 || level >= h->plan.nlev() - 1) return LAP_EINVAL;
    const Level& L = h->plan.lv[level];
    if (agg) std::memcpy(agg, L.agg.data(), L.agg.size() * sizeof(int64_t));
    if (matched) std::memcpy(matched, L.matched.data(), L.matched.size());
    return LAP_OK;
}

lap_status lap_export_graph(const lap_hierarchy* h, int32_t level, int64_t* ptr, int64_t* col,
                            double* w) {
    if (!h || level < 0 || level >= h->plan.nlev() || !ptr) return LAP_EINVAL;
    const Adjacency& g = h->plan.lv[level].g;
    std::memcpy(ptr, g.ptr.data(), g.ptr.size() * sizeof(int64_t));
    if (col)
        for (int64_t k = 0; k < g.nnz(); ++k) col[k] = g.col[k];
    if (w) std::memcpy(w, g.w.data(), g.w.size() * sizeof(double));
    return LAP_OK;
}

void lap_free(lap_hierarchy* h) { delete h; }

const char* lap_last_error(void) { return g_last_error; }

}  // extern "C"
