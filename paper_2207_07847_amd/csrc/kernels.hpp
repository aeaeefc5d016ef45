// Device kernels of the MSP-preconditioned conjugate-gradient solve.
//
// Vectors live in the tree numbering of the host plan: the children of every
// aggregate are a contiguous range whose first two entries are the matched
// pair.  Level k has n_k nodes; step k maps level k onto level k+1.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "setup.hpp"

namespace lapgpu {

constexpr int kBlock = 256;        // threads per block of the streaming kernels
constexpr int kTailThreads = 1024; // threads of the one-block coarse tail
constexpr int kFinThreads = 1024;  // threads of the one-block reduction finish
constexpr int kFinUnroll = 8;      // partials per thread loaded at once by a finish
constexpr int kMaxGridPart = 3;    // values reduced per block
constexpr int kAggPerBlock = 256;  // aggregates per block of a level kernel
constexpr int kCapP = 2048;        // children per block staged in LDS; an
                                   // aggregate with more gets a block alone
constexpr int kWaveAgg = 32;       // aggregates with more children are
                                   // restricted by a whole wavefront

// Scalars of one PCG run, resident in device memory.
struct Scal {
    double rho;     // r^T (z - zbar) of the current z
    double pq;      // p^T L p
    double alpha;
    double beta;
    double zbar;    // mean of the current z
    double rr;      // ||r||^2
    double bn2;     // ||b^||^2
    double tol2;    // tol^2
    double bsum;    // sum of b
    double xsum;    // sum of x
    double res2;    // ||b^ - L x||^2
    double spare;
    int32_t iter;   // products with L performed
    int32_t maxit;
    int32_t done;   // 0 running, 1 converged, 2 max_iter, 3 breakdown, 4 bad input
    int32_t first;  // next preconditioner result starts a new direction (beta = 0)
};

// Level table entry (device copy of per-level pointers).  T is the value
// type of the vectors and coefficients (double, or float for the inner
// solve of mixed precision).
template <class T>
struct LevelDev {
    int32_t n;          // nodes on this level
    int32_t nc;         // aggregates formed from it (nodes on the next level)
    T* r;               // restricted residual (levels >= 1)
    T* y;               // correction (levels >= 1)
    const int32_t* cptr;// children range of each aggregate
    const T* saa;       // theta * inverse 2x2 Schur complement of the pair
    const T* sab;
    const T* sbb;
    const T* l0;        // leftover t: theta / D_tt
    const T* l1;        //             w(t, a) / D_tt
    const T* l2;        //             w(t, b) / D_tt
    T* ea;              // eta of the pair member a (theta-scaled)
    T* eb;
    const int32_t* bst; // block partition: block b owns aggregates [bst[b], bst[b+1])
    int32_t nb;         // blocks of the partition
};

// Layout of the coarse tail in LDS (offsets in values of the solve's type
// from the start of the dynamic shared buffer).  The read-only part
// [0, pack) is a byte copy of a device buffer built by the host; the rest is
// work space.
struct TailStep {
    int32_t nk, nc, nl;                // children, aggregates, leftovers
    int32_t cptr;                      // int32[nc+1], stored in value slots
    int32_t saa, sab, sbb, l0, l1, l2; // coefficients
    int32_t ea, eb;                    // work: pair corrections
    int32_t nbig, big;                 // aggregates with > kTailBig children:
                                       // count, int32 list in value slots
};
constexpr int kTailBig = 64;
constexpr int kMaxTailSteps = 62;
struct TailDesc {
    int32_t nsteps;                    // levels kt .. top-1
    int32_t nt;                        // nodes on the top level
    int32_t pack;                      // doubles copied from the device pack
    int32_t total;                     // doubles of LDS used
    int32_t pinv;                      // theta_top * pinv(L_top), nt*nt
    int32_t r[kMaxTailSteps + 1];      // work: r of level kt+s (s = 0..nsteps)
    int32_t y[kMaxTailSteps + 1];      // work: y of level kt+s
    TailStep st[kMaxTailSteps];
};

// Block b of the fused level-0/1 kernels: its level-2 nodes [A0, A1), their
// level-1 children [J0, J1) and level-0 grandchildren [t0, t1), computed on
// the host so a block reads all three ranges with one load.
struct Blk01 {
    int32_t A0, A1, J0, J1, t0, t1, pad0, pad1;
};

// The descriptor fields the tail needs before anything else, passed by
// value so its first loads do not wait for them.
struct TailArgs {
    int32_t npack;   // TailDesc::pack
    int32_t nsteps;  // TailDesc::nsteps
    int32_t n0;      // nodes on level kt
    int32_t r0;      // TailDesc::r[0]
};

// A group of consecutive levels [k0, k1) processed block-locally: block b
// owns the level-k1 nodes [D[m][b], D[m][b+1]) (m = k1 - k0) and, on every
// level j = k0 + i, their descendants [D[i][b], D[i][b+1]), contiguous in the
// tree numbering.  Each block's coefficients are pre-packed contiguously in
// the order of its LDS carve, so staging is one flat copy; the up-sweep
// leaves its intermediate values in a per-block scratch chunk laid out for
// the down-sweep's carve.
constexpr int kGrpThreads = 512;
constexpr int kMaxGroupLevels = 12;
template <class T>
struct GroupDev {
    int32_t k0, k1, nblocks;
    const int32_t* D;        // (m+1) rows of nblocks+1 entries
    const int32_t* uoff;     // up pack offset of each block (nblocks+1)
    const int32_t* doff;     // down pack offset of each block
    const int32_t* xoff;     // scratch offset of each block
    const T* upack;          // per level: cp (local), pair coefficients, l1, l2
    const T* dpack;          // per level: cp (local), l0, l1, l2
    T* scr;                  // per level: r (levels 1..m-1), then eta a, eta b
    T* r_top;                // level k1 residual (output of the up-sweep)
    const T* y_top;          // level k1 correction (input of the down-sweep)
    const T* r_in;           // level k0 residual (input)
    T* y_out;                // level k0 correction (output)
};

// Offsets (in values) inside one block's up pack, down pack, scratch chunk
// and LDS carves, from the block's per-level counts; `ipv` int32 children
// offsets fit one value slot (2 for double, 1 for float).  Shared by host
// and device so the layouts agree exactly.
struct GrpLayout {
    int32_t ucp[kMaxGroupLevels], us[kMaxGroupLevels], ul[kMaxGroupLevels], ulen;
    int32_t dcp[kMaxGroupLevels], dl[kMaxGroupLevels], dlen;
    int32_t xr[kMaxGroupLevels], xe[kMaxGroupLevels], xlen;
    int32_t ur[kMaxGroupLevels + 1], utotal;                 // up LDS: upack | r_0..r_m
    int32_t dx, dr0, dy[kMaxGroupLevels + 1], dtotal;        // down LDS: dpack | scr | r_0 | y_0..y_m
};

__host__ __device__ inline void grp_layout(int m, const int32_t* cnt, int ipv, GrpLayout& L) {
    int32_t u = 0, d = 0, x = 0;
    for (int j = 0; j < m; ++j) {
        const int32_t na = cnt[j + 1], nl = cnt[j] - 2 * cnt[j + 1];
        const int32_t cps = (na + 1 + ipv - 1) / ipv;
        L.ucp[j] = u; u += cps;
        L.us[j] = u;  u += 3 * na;
        L.ul[j] = u;  u += 2 * nl;
        L.dcp[j] = d; d += cps;
        L.dl[j] = d;  d += 3 * nl;
        L.xr[j] = x;  if (j >= 1) x += cnt[j];
        L.xe[j] = x;  x += 2 * na;
    }
    L.ulen = u;
    L.dlen = d;
    L.xlen = x;
    int32_t o = u;
    for (int j = 0; j <= m; ++j) { L.ur[j] = o; o += cnt[j]; }
    L.utotal = o;
    o = d;
    L.dx = o; o += x;
    L.dr0 = o; o += cnt[0];
    for (int j = 0; j <= m; ++j) { L.dy[j] = o; o += cnt[j]; }
    L.dtotal = o;
}

// Fine Laplacian for the SpMV.  Light rows: sliced ELL, 64 rows per slice
// (one wavefront), slot k of a slice's rows stored contiguously; slice s
// holds the rows row[s*64 .. s*64+63] (row == nullptr: the identity, slot =
// row), width[s] slots each, padding pointing at the row itself with w = 0.
// Heavy rows (degree above kHeavyDeg) are left out of the slices and stored
// as CSR; heavy block b handles the heavy rows [hblk[b], hblk[b+1]): one
// wavefront per row, or the whole block for a single row of degree above
// kHeavyBlockDeg.
template <class T>
struct Sell {
    int32_t nlight;          // rows in the slices
    int32_t nheavyblk;       // heavy blocks
    const int32_t* off;      // slice -> first slot
    const int32_t* width;    // slice -> slots per row
    const int32_t* col;
    const T* w;
    const int32_t* row;      // slot -> row (nullptr: identity)
    const int32_t* hblk;     // heavy block -> first heavy row (nheavyblk+1)
    const int32_t* hrow;     // heavy row -> row
    const int32_t* hptr;     // heavy row -> first entry
    const int32_t* hcol;
    const T* hw;
};

// PEGP on the device (one workgroup, expanded vector in LDS): the factored
// grounded system of PegpPlan (setup.hpp) and the tree links for the
// restriction and prolongation of P(mu).
constexpr int kPegpThreads = 1024;
constexpr int kPegpMaxLevels = 64;
constexpr int kPegpMaxNodes = 19456;     // expanded nodes held in LDS (152 KB)
// dynamic LDS of the PEGP solve kernels: 160 KB less room for their static arrays
constexpr size_t kPegpLdsBytes = 160 * 1024 - 1024;
struct PegpDev {
    int32_t nt, nlev, ground, nflev, nblev;
    int32_t desc_lds;                    // level descriptors copied to LDS (after the vector)
    int32_t off[kPegpMaxLevels + 1];     // level -> first expanded index
    const int32_t* cptr[kPegpMaxLevels]; // children ranges of level k+1 nodes
    const double* diag;
    // level lists packed for the solve: per level a descriptor, row -> node,
    // the padded entries (columns and values)
    const int32_t *fdesc, *frow, *fpcol;
    const double* fpval;
    const int32_t *bdesc, *brow, *bpcol;
    const double* bpval;
    // dense tail (nd rows, 0: none): tail position -> node, the strict lower
    // factor of the tail row-major (forward) and column-major (backward), the
    // forward coupling (CSR by tail position, columns are nodes), the
    // backward coupling (nbc rows bcrow, columns are tail positions)
    int32_t nd, ndp, nbc;                 // tail rows, padded to whole superblocks (the
                                         // dense arrays' dimension), coupling rows
    const int32_t *drow, *dcptr, *dccol, *bcrow, *bcptr, *bccol;
    const double *dlr, *dlc, *dd, *dcval, *bcval;
    // device scratch of one apply: the expanded vector between the
    // single-workgroup kernels, the tail's values, the backward coupling sums
    double *fg, *ty, *cpl;
    // the explicit operator (PegpPlan::op; opn = 0: not formed)
    int32_t opn, opld;
    const double* op;
};
constexpr int kPegpOpRows = 4;           // rows of the operator per workgroup (one per wavefront)

}  // namespace lapgpu
