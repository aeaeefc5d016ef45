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
    uint32_t cnt[8];// arrival counters of the last-block reductions
};

enum { kCntSpmv = 0, kCntUpd = 1, kCntDown = 2, kCntInit = 3, kCntFin = 4, kCntMisc = 5 };

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

struct Sell {
    const int32_t* off;
    const int32_t* width;
    const int32_t* col;
    const double* w;
};

}  // namespace lapgpu
