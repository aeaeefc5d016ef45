// Device kernels of the MSP-preconditioned conjugate-gradient solve.
//
// Vectors live in the tree numbering of the host plan: the children of every
// aggregate are a contiguous range whose first two entries are the matched
// pair.  Level k has n_k nodes; step k maps level k onto level k+1.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lapgpu {

constexpr int kBlock = 256;        // threads per block of the streaming kernels
constexpr int kTailThreads = 1024; // threads of the one-block coarse tail
constexpr int kMaxGridPart = 3;    // values reduced per block

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

// Level table entry (device copy of per-level pointers).
struct LevelDev {
    int32_t n;          // nodes on this level
    int32_t nc;         // aggregates formed from it (nodes on the next level)
    double* r;          // restricted residual (levels >= 1)
    double* y;          // correction (levels >= 1)
    const int32_t* cptr;// children range of each aggregate
    const double* saa;  // theta * inverse 2x2 Schur complement of the pair
    const double* sab;
    const double* sbb;
    const double* l0;   // leftover t: theta / D_tt
    const double* l1;   //             w(t, a) / D_tt
    const double* l2;   //             w(t, b) / D_tt
    double* ea;         // eta of the pair member a (theta-scaled)
    double* eb;
};

// Layout of the coarse tail in LDS (offsets in doubles from the start of the
// dynamic shared buffer).  The read-only part [0, pack) is a byte copy of a
// device buffer built by the host; the rest is work space.
struct TailStep {
    int32_t nk, nc, nl;                // children, aggregates, leftovers
    int32_t cptr;                      // int32[nc+1], stored in double slots
    int32_t saa, sab, sbb, l0, l1, l2; // coefficients
    int32_t ea, eb;                    // work: pair corrections
};
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

struct Sell {
    const int32_t* off;
    const int32_t* width;
    const int32_t* col;
    const double* w;
};

}  // namespace lapgpu
