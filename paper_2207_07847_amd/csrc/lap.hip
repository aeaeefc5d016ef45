// Host side of the MI355X (gfx950) Laplacian solver and its C ABI
// (include/lap.h): device upload of the host plan, the PCG driver (chunks of
// iterations replayed from hipGraphs), FP64 and mixed-precision solves.
// The kernels are in device.hpp.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <new>
#include <stdexcept>
#include <thread>
#include <type_traits>
#include <vector>

#include "block.hpp"
#include "device.hpp"
#include "kernels.hpp"
#include "lap.h"
#include "setup.hpp"

// Scratch of lap_apply_laplacian_noalloc, the variant of lap_apply_laplacian
// for callers that cannot allocate: the two permuted n-vectors that the
// other entry point keeps in the hierarchy.  Each device that runs the
// library holds one copy until the process ends; every call on a device
// shares it (calls that overlap in time on one device race).
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;  // 64 MiB: n <= 4,194,304
constexpr int kNoallocMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

using namespace lapgpu;

namespace {

inline int nblk(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

struct HipErr {};
thread_local char g_last_error[256] = "";

// Device allocator of hierarchies set up from now on (lap_set_allocator):
// null functions mean hipMalloc / hipFree.  A hierarchy keeps the pair it
// was set up with until lap_free.
struct Allocator {
    lap_alloc_fn alloc = nullptr;
    lap_free_fn free = nullptr;
    void* ctx = nullptr;
};
std::mutex g_alloc_mu;
Allocator g_alloc;

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

#include "devsetup.hpp"

int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    return v ? std::atoi(v) : dflt;
}

double env_double(const char* name, double dflt) {
    const char* v = std::getenv(name);
    return v ? std::atof(v) : dflt;
}

constexpr size_t kTailLdsBytes = 152 * 1024;
// dynamic LDS + the tail's static descriptor copy and reduction space fit a CU
static_assert(kTailLdsBytes + sizeof(TailDesc) + 3 * (kTailThreads / 64) * sizeof(double) <=
                  160 * 1024,
              "tail LDS");
constexpr int kProfGroup = 10;          // timed iterations per fresh run (profiling)
constexpr double kReliableDrop = 1e-2;  // ||r||^2 drop between reliable updates
constexpr size_t kGrpLdsBytes = 64 * 1024;

// int32 entries that fit one value slot of type T.
template <class T>
constexpr int ipv() { return (int)(sizeof(T) / sizeof(int32_t)); }

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

// Partition of the level-2 nodes for the fused level-0/1 kernels: runs of
// level-1 aggregates whose level-1 children fit kAggPerBlock and level-0
// grandchildren fit kCapP.  Empty when one aggregate alone does not fit.
std::vector<int32_t> block_partition01(const std::vector<int32_t>& c0,
                                       const std::vector<int32_t>& c1) {
    const int32_t n2 = (int32_t)c1.size() - 1;
    std::vector<int32_t> bst{0};
    int32_t A0 = 0;
    auto fits = [&](int32_t a, int32_t b) {
        return b - a <= kAggPerBlock && c1[b] - c1[a] <= kAggPerBlock &&
               c0[c1[b]] - c0[c1[a]] <= kCapP;
    };
    while (A0 < n2) {
        if (!fits(A0, A0 + 1)) return {};
        int32_t A1 = A0 + 1;
        while (A1 < n2 && fits(A0, A1 + 1)) ++A1;
        bst.push_back(A1);
        A0 = A1;
    }
    return bst;
}

std::vector<int32_t> big_aggregates(const std::vector<int32_t>& cptr) {
    std::vector<int32_t> big;
    for (size_t J = 0; J + 1 < cptr.size(); ++J)
        if (cptr[J + 1] - cptr[J] > kTailBig) big.push_back((int32_t)J);
    return big;
}

// Values of type T the tail needs in LDS when it starts at level kt.
size_t tail_lds_units(const HostPlan& P, int kt, int iv) {
    const int T = P.nlev() - 1;
    size_t d = 0;
    for (int k = kt; k < T; ++k) {
        const size_t nk = P.lv[k].g.n, nc = P.lv[k + 1].g.n, nl = nk - 2 * nc;
        const size_t nbig = big_aggregates(P.step[k].cptr).size();
        d += (nc + 1 + iv - 1) / iv + 3 * nc + 3 * nl + 2 * nc + (nbig + iv - 1) / iv;
    }
    for (int k = kt; k <= T; ++k) d += 2 * P.lv[k].g.n;     // r, y
    d += P.lv[T].g.n * P.lv[T].g.n;                        // top pseudo-inverse
    return d;
}

// Pack the tail coefficients of levels kt..T into one buffer and lay out
// the LDS work space after it.
template <class T>
void build_tail(const HostPlan& P, int kt, TailDesc& D, std::vector<T>& pack) {
    const int top = P.nlev() - 1;
    D.nsteps = top - kt;
    D.nt = (int32_t)P.lv[top].g.n;
    auto put = [&](const std::vector<double>& src) {
        const int32_t off = (int32_t)pack.size();
        for (double x : src) pack.push_back((T)x);
        return off;
    };
    auto put_ints = [&](const std::vector<int32_t>& src) {
        const int32_t off = (int32_t)pack.size();
        pack.resize(pack.size() + (src.size() + ipv<T>() - 1) / ipv<T>(), T(0));
        if (!src.empty()) std::memcpy(pack.data() + off, src.data(), src.size() * sizeof(int32_t));
        return off;
    };
    for (int s = 0; s < D.nsteps; ++s) {
        const int k = kt + s;
        const StepCoef& c = P.step[k];
        TailStep& t = D.st[s];
        t.nk = (int32_t)P.lv[k].g.n;
        t.nc = (int32_t)P.lv[k + 1].g.n;
        t.nl = t.nk - 2 * t.nc;
        t.cptr = put_ints(c.cptr);
        t.saa = put(c.saa);
        t.sab = put(c.sab);
        t.sbb = put(c.sbb);
        t.l0 = put(c.l0);
        t.l1 = put(c.l1);
        t.l2 = put(c.l2);
        const std::vector<int32_t> big = big_aggregates(c.cptr);
        t.nbig = (int32_t)big.size();
        t.big = put_ints(big);
    }
    D.pinv = put(P.top_pinv);
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
// LDS layouts (up and down) fit `units` values.  Fails if one subtree alone
// does not fit.  lds_up / lds_down are in values.
bool plan_group(const HostPlan& P, int k0, int k1, int cap, int iv, int32_t units,
                std::vector<int32_t>& D, int& nblocks, int32_t& lds_up, int32_t& lds_down) {
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
        grp_layout(m, cnt, iv, lay);
        return cnt[0] <= cap && lay.utotal <= units && lay.dtotal <= units;
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
    lds_up = up;
    lds_down = dn;
    return true;
}

// Pack one group's per-block coefficients in the order of grp_layout.
template <class T>
void pack_group(const HostPlan& P, int k0, int k1, int nblocks, const std::vector<int32_t>& D,
                std::vector<int32_t>& uoff, std::vector<int32_t>& doff,
                std::vector<int32_t>& xoff, std::vector<T>& up, std::vector<T>& dn) {
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
        grp_layout(m, cnt, ipv<T>(), L);
        const size_t ub = up.size(), db = dn.size();
        up.resize(ub + L.ulen, T(0));
        dn.resize(db + L.dlen, T(0));
        for (int j = 0; j < m; ++j) {
            const StepCoef& c = P.step[k0 + j];
            const int na = cnt[j + 1], nl = cnt[j] - 2 * na, a0 = st[j + 1], c0 = st[j];
            const int lb = c0 - 2 * a0;
            std::vector<int32_t> cp(na + 1);
            for (int i = 0; i <= na; ++i) cp[i] = c.cptr[a0 + i] - c0;
            std::memcpy(up.data() + ub + L.ucp[j], cp.data(), cp.size() * sizeof(int32_t));
            std::memcpy(dn.data() + db + L.dcp[j], cp.data(), cp.size() * sizeof(int32_t));
            for (int i = 0; i < na; ++i) {
                up[ub + L.us[j] + i] = (T)c.saa[a0 + i];
                up[ub + L.us[j] + na + i] = (T)c.sab[a0 + i];
                up[ub + L.us[j] + 2 * na + i] = (T)c.sbb[a0 + i];
            }
            for (int i = 0; i < nl; ++i) {
                up[ub + L.ul[j] + i] = (T)c.l1[lb + i];
                up[ub + L.ul[j] + nl + i] = (T)c.l2[lb + i];
                dn[db + L.dl[j] + i] = (T)c.l0[lb + i];
                dn[db + L.dl[j] + nl + i] = (T)c.l1[lb + i];
                dn[db + L.dl[j] + 2 * nl + i] = (T)c.l2[lb + i];
            }
        }
        uoff[b + 1] = (int32_t)up.size();
        doff[b + 1] = (int32_t)dn.size();
        xoff[b + 1] = xoff[b] + L.xlen;
    }
}

template <class T>
std::vector<T> convert(const std::vector<double>& v) {
    return std::vector<T>(v.begin(), v.end());
}

// Device data and workspace of one value type: the SpMV matrix, the
// preconditioner levels, the captured iteration graph.
template <class T>
struct Engine {
    bool on = false;
    Sell<T> A{};
    int nlb = 0;                 // light blocks of the SpMV grid; heavy blocks follow
    std::vector<LevelDev<T>> lv;
    T* top_pinv = nullptr;
    int kt = 1;                  // first level of the one-block tail
    TailDesc* d_tail = nullptr;
    T* tail_pack = nullptr;
    size_t tail_lds = 0;         // bytes
    TailArgs tail_args{};
    struct Segment {
        bool group = false;
        int k0 = 0, k1 = 1;
        GroupDev<T> gd{};
        size_t lds_up = 0, lds_down = 0;   // bytes of dynamic LDS
    };
    std::vector<Segment> segs;   // levels [1, kt) ([2, kt) when fuse01), in order
    bool fuse01 = false;         // levels 0 and 1 in the same kernels
    Blk01* blk01 = nullptr;      // fused level-0/1 block ranges
    int nb01 = 0;
    // workspace: input order
    T *x = nullptr, *p[2] = {nullptr, nullptr}, *q = nullptr, *zn = nullptr;
    T* ph = nullptr;             // compact copy of p's hot columns (nhot)
    // workspace: tree order
    T *r = nullptr, *z = nullptr;
    hipStream_t cap = nullptr;   // private capture stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int spmv_grid() const { return nlb + A.nheavyblk; }
    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
        exec = nullptr;
        graph = nullptr;
        cap = nullptr;
    }
};

// Chunked work list over segments [ptr[i], ptr[i+1]) (rows of a matrix or
// children of aggregates): segments longer than `chunk` are split, their
// chunks writing partial rows to scratch slots that a combine pass adds.
template <class P>
struct ChunkHost {
    std::vector<int32_t> id, t0, t1, slot, multi, mfirst{0};
    void build(const std::vector<P>& ptr, int chunk) {
        const size_t nseg = ptr.size() - 1;
        int32_t ns = 0;
        for (size_t i = 0; i < nseg; ++i) {
            const P a = ptr[i], b = ptr[i + 1];
            if (b - a <= chunk) {
                id.push_back((int32_t)i);
                t0.push_back((int32_t)a);
                t1.push_back((int32_t)b);
                slot.push_back(-1);
                continue;
            }
            multi.push_back((int32_t)i);
            for (P c = a; c < b; c += chunk) {
                id.push_back((int32_t)i);
                t0.push_back((int32_t)c);
                t1.push_back((int32_t)std::min<P>(b, c + chunk));
                slot.push_back(ns++);
            }
            mfirst.push_back(ns);
        }
    }
    int32_t nslots() const { return mfirst.back(); }
};

// Device data of the block solve of one value type: the Laplacian in CSR
// (solve order) with its chunk list, per step the up and down chunk lists,
// the block vectors of every level.
template <class T>
struct EngineM {
    bool on = false;
    // sizes picked by the autotuner: matrix entries per SpMM work item (rows
    // above it are split), workgroups of the SpMM, children per work item of
    // the restriction and prolongation
    int chunk = kMmChunk, grid = kMmMaxGrid, seg = kMmChunk;
    Csr<T> A{};
    Chunks CA{};
    T* scrA = nullptr;           // partial rows of split SpMM rows
    std::vector<LevelDev<T>> lv; // block vectors r, y, ea, eb (rows of kCols)
    std::vector<Chunks> up, down;
    std::vector<T*> scrU;        // per step: 3 partial rows per split chunk
    T* top_pinv = nullptr;
    T *x = nullptr, *p[2] = {nullptr, nullptr}, *q = nullptr, *zn = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
        exec = nullptr;
        graph = nullptr;
        cap = nullptr;
    }
};

inline int mm_grid(int64_t items, int cap = kMmMaxGrid) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((items + kMmWaves - 1) / kMmWaves, cap));
}

}  // namespace

struct lap_hierarchy {
    HostPlan plan;
    lap_params params{};
    bool host_only = false;
    bool with_msp = true;
    bool mixed = false;          // solves use mixed precision
    bool has_fp32 = false;       // the FP32 engine exists
    bool pegp = false;           // preconditioner: PEGP (FP64 solves only)
    PegpPlan pegp_plan;
    PegpDev pegp_dev{};
    size_t pegp_lds = 0;
    int64_t n = 0;
    int device = 0;
    double setup_seconds = 0.0;
    int64_t dev_bytes = 0;
    std::vector<void*> allocs;
    std::vector<size_t> alloc_bytes;
    // integer data shared by both engines
    int32_t* perm0 = nullptr;    // tree position -> input vertex
    // The solve order (x, p, q, the SpMV's copy of z, bh) is the input order
    // for meshes and the tree order otherwise (HostPlan::spmv_tree):
    const int32_t* t2s = nullptr;   // tree position -> solve position (null: same)
    const int32_t* sperm = nullptr; // solve position -> input vertex (null: same)
    bool fuse_p = true;             // SpMV forms p on the fly (else a p pass first)
    // hot columns of the separate-p SpMV (k_spmv_q): nhot most referenced
    // columns, their list and the column arrays that name them by rank
    int32_t nhot = 0;
    const int32_t *hot = nullptr, *hot_col = nullptr, *hot_hcol = nullptr;
    std::vector<const int32_t*> cptr, bst;
    std::vector<int32_t> nb;
    Sell<double> Ai{};           // the index arrays of the SpMV matrix (weights unset)
    Engine<double> e64;          // FP64 solve (matrix always: residuals, apply)
    Engine<float> e32;           // inner solve of mixed precision
    // block solve (LAP_FLAG_MULTI_RHS): kCols columns at once
    bool has_block = false;
    EngineM<double> m64;         // FP64 block solve
    EngineM<float> m32;          // FP32 inner block solve (mixed precision)
    Csr<double> A64m{};          // FP64 CSR for block residuals
    Chunks CA64{};
    double* scrA64 = nullptr;
    double *bhm = nullptr, *xm = nullptr, *rm = nullptr, *xcm = nullptr;   // FP64 block vectors
    ScalM* Sm = nullptr;         // scalars of the inner block runs
    ScalM* Smo = nullptr;        // scalars of the outer block loop
    ScalM* stagem = nullptr;     // pinned host copy
    double* partm = nullptr;     // per-block per-column partials
    double* partm2 = nullptr;
    // FP64 vectors in input order
    double *bh = nullptr, *xc = nullptr, *x64 = nullptr, *r64 = nullptr;
    // FGMRES on the expanded system (LAP_FLAG_FGMRES), allocated by the first
    // such solve: a basis of fg_m + 1 expanded vectors of fg_nt values
    int fg_m = 0;
    int64_t fg_nt = 0;
    std::vector<int64_t> fg_off;         // level offsets in an expanded vector
    double* fg_V = nullptr;
    double* fg_w = nullptr;
    double *fg_y = nullptr, *fg_x = nullptr, *fg_r = nullptr;   // n each, solve order
    double* fg_part = nullptr;           // partial dot products
    double* fg_h = nullptr;              // dot results / coefficients on the device
    double* fg_hh = nullptr;             // pinned host copy
    Scal* S = nullptr;           // scalars of the PCG run
    Scal* So = nullptr;          // scalars of the outer refinement loop
    double* part = nullptr;      // per-block partial sums of the last producer
    double* part2 = nullptr;     // per-block ||r||^2 of the update kernel
    Scal* stage = nullptr;       // pinned host copy of S or So
    int chunk = 8;
    double mm_tune_seconds = 0.0;  // block-solve autotuner time in lap_setup
    double inner_tol = 1e-4;
    double reliable_drop = kReliableDrop;
    bool reliable = true;        // mixed precision by reliable updates (else restarts)

    Allocator allocator;         // device memory of this hierarchy
    void dev_free(void* ptr) {
        if (allocator.free) allocator.free(ptr, allocator.ctx);
        else (void)hipFree(ptr);
    }
    template <class T>
    T* dalloc(size_t count) {
        void* ptr = nullptr;
        const size_t bytes = (count ? count : 1) * sizeof(T);
        if (allocator.alloc) {
            ptr = allocator.alloc(bytes, allocator.ctx);
            if (!ptr) throw std::bad_alloc();
        } else if (hipMalloc(&ptr, bytes) != hipSuccess) {
            throw std::bad_alloc();
        }
        allocs.push_back(ptr);
        alloc_bytes.push_back(bytes);
        dev_bytes += (int64_t)bytes;
        return static_cast<T*>(ptr);
    }
    // Frees every allocation made after mark() returned `mk` (the caller has
    // synchronized the work that used them).
    size_t mark() const { return allocs.size(); }
    void release_to(size_t mk) {
        while (allocs.size() > mk) {
            dev_free(allocs.back());
            dev_bytes -= (int64_t)alloc_bytes.back();
            allocs.pop_back();
            alloc_bytes.pop_back();
        }
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
        e64.release();
        e32.release();
        m64.release();
        m32.release();
        for (void* ptr : allocs) dev_free(ptr);
        if (stage) (void)hipHostFree(stage);
        if (stagem) (void)hipHostFree(stagem);
        if (fg_hh) (void)hipHostFree(fg_hh);
    }
    template <class P>
    Chunks upload_chunks(const ChunkHost<P>& c, hipStream_t s) {
        Chunks d{};
        d.nitems = (int32_t)c.id.size();
        d.id = upload(c.id, s);
        d.t0 = upload(c.t0, s);
        d.t1 = upload(c.t1, s);
        d.slot = upload(c.slot, s);
        d.nmulti = (int32_t)c.multi.size();
        d.multi = upload(c.multi, s);
        d.mfirst = upload(c.mfirst, s);
        return d;
    }
};

namespace {

// One-block finish of the partials at `part` (G blocks) into the scalars
// at S; kFinRho may also take the update kernel's ||r||^2 partials (G2
// blocks at part2).
template <int OP>
void finish(lap_hierarchy* h, hipStream_t s, Scal* S, int G, int G2 = 0,
            const double* part = nullptr) {
    hipLaunchKernelGGL(k_finish<OP>, dim3(1), dim3(kFinThreads), 0, s, G, (int)h->n,
                       part ? part : h->part, G2, h->part2, S);
}

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

// The preconditioner: level-0 restriction (with the x, r update when
// do_update), the middle levels, the tail and back, z with its reductions.
template <class T>
void enqueue_precond(lap_hierarchy* h, Engine<T>& e, hipStream_t s, int do_update,
                     const Marks& mk = Marks{}) {
    const int Tl = h->plan.nlev() - 1;
    const int n = (int)h->n;
    Scal* S = h->S;
    if constexpr (std::is_same<T, double>::value) {
        if (h->pegp) {
            if (do_update) {
                hipLaunchKernelGGL(k_update_none<T>, dim3(nblk(n)), dim3(kBlock), 0, s, n,
                                   h->t2s, e.r, (const T*)e.q, S, h->part2);
                finish<kFinRr>(h, s, S, nblk(n), 0, h->part2);
            }
            const PegpDev& P = h->pegp_dev;
            if (P.opn > 0) {
                // the explicit operator: one matrix-vector product
                const int grid = (P.opn + kPegpOpRows - 1) / kPegpOpRows;
                launch_timed(k_pegp_op, dim3(grid), dim3(kBlock),
                             (uint32_t)(P.opld * sizeof(double)), s,
                             mk.start(LAP_KERNEL_PEGP_OP), mk.stop(LAP_KERNEL_PEGP_OP), P,
                             h->t2s, (const double*)e.r, e.zn, (const Scal*)S, h->part);
                finish<kFinRho>(h, s, S, grid);
                return;
            }
            hipLaunchKernelGGL(k_pegp_fwd, dim3(1), dim3(kPegpThreads), h->pegp_lds, s, P,
                               (const double*)e.r, (const Scal*)S);
            if (P.nd > 0) {
                const int per = kBlock / 64;   // a wavefront per row
                hipLaunchKernelGGL(k_pegp_tail_rhs, dim3((P.nd + per - 1) / per), dim3(kBlock), 0,
                                   s, P, (const Scal*)S);
                const int nblk = P.ndp / kTailS;
                for (int b = -1; b + 1 < nblk; ++b) {
                    // workgroup 0, and a wavefront per row past the next superblock
                    const int rest = std::max(0, P.ndp - (b + 2) * kTailS);
                    const int grid = 1 + (b >= 0 ? (rest + per - 1) / per : 0);
                    hipLaunchKernelGGL(k_pegp_tail_fwd, dim3(grid), dim3(kBlock), 0, s, P, b,
                                       (const Scal*)S);
                }
                for (int b = nblk; b > 0; --b) {
                    // workgroup 0, and the rows before the superblock being
                    // solved: a thread each for the diagonal, then a wavefront each
                    const int before = (b - 1) * kTailS;
                    const int grid = 1 + (b == nblk ? (before + kBlock - 1) / kBlock
                                                    : (before + per - 1) / per);
                    hipLaunchKernelGGL(k_pegp_tail_bwd, dim3(grid), dim3(kBlock), 0, s, P, b,
                                       nblk, (const Scal*)S);
                }
                if (P.nbc > 0)
                    hipLaunchKernelGGL(k_pegp_tail_back, dim3((P.nbc + per - 1) / per),
                                       dim3(kBlock), 0, s, P, (const Scal*)S);
            }
            hipLaunchKernelGGL(k_pegp_bwd, dim3(1), dim3(kPegpThreads), h->pegp_lds, s, P,
                               h->t2s, (const double*)e.r, e.z, e.zn, S);
            return;
        }
    }
    if (!h->with_msp || Tl == 0) {
        if (do_update) {
            hipLaunchKernelGGL(k_update_none<T>, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->t2s,
                               e.r, (const T*)e.q, S, h->part2);
            if (h->with_msp) finish<kFinRr>(h, s, S, nblk(n), 0, h->part2);
        }
        if (!h->with_msp) {
            hipLaunchKernelGGL(k_prec_none<T>, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->t2s,
                               (const T*)e.r, e.z, e.zn, S, h->part);
            finish<kFinRho>(h, s, S, nblk(n), do_update ? nblk(n) : 0);
        } else {
            hipLaunchKernelGGL(k_top_only<T>, dim3(1), dim3(kBlock), 0, s, n, h->t2s,
                               (const T*)e.top_pinv, (const T*)e.r, e.z, e.zn, S);
        }
        return;
    }
    const LevelDev<T>& s0 = e.lv[0];
    const int g0 = e.fuse01 ? e.nb01 : s0.nb;
    if (e.fuse01)
        launch_timed(k_update_up01<T>, dim3(g0), dim3(kBlock), 0, s,
                     mk.kernel == LAP_KERNEL_PRECOND ? mk.e0 : mk.start(LAP_KERNEL_UPDATE),
                     mk.stop(LAP_KERNEL_UPDATE), s0, e.lv[1], (const Blk01*)e.blk01, h->t2s,
                     e.r, (const T*)e.q, e.lv[2].r, S, h->part2, do_update);
    else
        launch_timed(k_update_up0<T>, dim3(g0), dim3(kBlock), 0, s,
                     mk.kernel == LAP_KERNEL_PRECOND ? mk.e0 : mk.start(LAP_KERNEL_UPDATE),
                     mk.stop(LAP_KERNEL_UPDATE), s0, h->t2s, e.r, (const T*)e.q, e.lv[1].r, S, h->part2, do_update);
    for (const auto& G : e.segs) {
        if (G.group)
            hipLaunchKernelGGL(k_up_grp<T>, dim3(G.gd.nblocks), dim3(kGrpThreads), G.lds_up, s,
                               G.gd, (const Scal*)S);
        else
            hipLaunchKernelGGL(k_up<T>, dim3(e.lv[G.k0].nb), dim3(kBlock), 0, s, e.lv[G.k0],
                               (const T*)e.lv[G.k0].r, e.lv[G.k0 + 1].r, (const Scal*)S);
    }
    hipLaunchKernelGGL(k_tail<T>, dim3(1), dim3(kTailThreads), e.tail_lds, s,
                       (const TailDesc*)e.d_tail, e.tail_args, (const T*)e.tail_pack,
                       (const T*)e.lv[e.kt].r,
                       e.lv[e.kt].y, (const Scal*)S);
    for (auto it = e.segs.rbegin(); it != e.segs.rend(); ++it) {
        const auto& G = *it;
        if (G.group)
            hipLaunchKernelGGL(k_down_grp<T>, dim3(G.gd.nblocks), dim3(kGrpThreads), G.lds_down,
                               s, G.gd, (const Scal*)S);
        else
            hipLaunchKernelGGL(k_down<T>, dim3(e.lv[G.k0].nb), dim3(kBlock), 0, s, e.lv[G.k0],
                               (const T*)e.lv[G.k0].r, e.lv[G.k0].y, (const T*)e.lv[G.k0 + 1].y,
                               (const Scal*)S);
    }
    if (e.fuse01)
        launch_timed(k_down01<T>, dim3(g0), dim3(kBlock), 0, s, mk.start(LAP_KERNEL_DOWN0),
                     mk.kernel == LAP_KERNEL_PRECOND ? mk.e1 : mk.stop(LAP_KERNEL_DOWN0), s0,
                     e.lv[1], (const Blk01*)e.blk01, h->t2s, (const T*)e.r, e.zn,
                     (const T*)e.lv[2].y, S,
                     h->part);
    else
        launch_timed(k_down0<T>, dim3(g0), dim3(kBlock), 0, s, mk.start(LAP_KERNEL_DOWN0),
                     mk.kernel == LAP_KERNEL_PRECOND ? mk.e1 : mk.stop(LAP_KERNEL_DOWN0), s0,
                     h->t2s, (const T*)e.r, e.zn, (const T*)e.lv[1].y, S, h->part);
    finish<kFinRho>(h, s, S, g0, do_update ? g0 : 0);
}

// One PCG iteration reading p[par] and writing p[1-par].
template <class T>
void enqueue_iteration(lap_hierarchy* h, Engine<T>& e, hipStream_t s, int par,
                       const Marks& mk = Marks{}) {
    if (h->fuse_p) {
        launch_timed(k_spmv_p<T>, dim3(e.spmv_grid()), dim3(kBlock), 0, s,
                     mk.start(LAP_KERNEL_SPMV), mk.stop(LAP_KERNEL_SPMV), e.nlb, e.A,
                     (const T*)e.zn, (const T*)e.p[par], e.p[1 - par], e.q, e.x, h->S,
                     h->part);
    } else {
        const int n = (int)h->n;
        launch_timed(k_pupd<T>, dim3(nblk(n) + nblk(h->nhot)), dim3(kBlock), 0, s,
                     mk.start(LAP_KERNEL_SPMV), (hipEvent_t) nullptr, n, (const T*)e.zn,
                     (const T*)e.p[par], e.p[1 - par], e.x, (const Scal*)h->S, h->nhot, h->hot,
                     e.ph);
        Sell<T> A = e.A;
        if (h->nhot > 0) {
            A.col = h->hot_col;
            A.hcol = h->hot_hcol;
        }
        launch_timed(k_spmv_q<T>, dim3(e.spmv_grid()), dim3(kBlock), 0, s, (hipEvent_t) nullptr,
                     mk.stop(LAP_KERNEL_SPMV), e.nlb, A, (const T*)e.p[1 - par],
                     (const T*)e.ph, e.q, h->S, h->part);
    }
    finish<kFinPq>(h, s, h->S, e.spmv_grid());
    enqueue_precond(h, e, s, 1, mk);
}

template <class T>
void build_graph(lap_hierarchy* h, Engine<T>& e) {
    HIPCHK(hipStreamCreateWithFlags(&e.cap, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(e.cap, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < h->chunk; ++i) enqueue_iteration(h, e, e.cap, i & 1);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamEndCapture(e.cap, &e.graph));
    HIPCHK(hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0));
}

// Integer data of the plan used by both engines.
void upload_shared(lap_hierarchy* h, hipStream_t s) {
    const HostPlan& P = h->plan;
    const int T = P.nlev() - 1;
    h->perm0 = h->upload(P.perm[0], s);
    h->t2s = P.spmv_tree ? nullptr : h->perm0;
    h->sperm = P.spmv_tree ? h->perm0 : nullptr;
    const int fz = env_int("LAPGPU_FUSE_P", -1);
    h->fuse_p = fz < 0 ? !P.spmv_tree : fz != 0;
    h->cptr.assign(T, nullptr);
    h->bst.assign(T, nullptr);
    h->nb.assign(T, 0);
    for (int k = 0; k < T; ++k) {
        h->cptr[k] = h->upload(P.step[k].cptr, s);
        const std::vector<int32_t> b = block_partition(P.step[k].cptr);
        h->nb[k] = (int32_t)b.size() - 1;
        h->bst[k] = h->upload(b, s);
    }
    Sell<double>& A = h->Ai;
    A.nlight = P.sell_nlight;
    A.nheavyblk = (int32_t)P.heavy_blk.size() - 1;
    A.off = h->upload(P.sell_off, s);
    A.width = h->upload(P.sell_width, s);
    A.col = h->upload(P.sell_col, s);
    A.row = P.sell_row.empty() ? nullptr : h->upload(P.sell_row, s);
    A.hblk = h->upload(P.heavy_blk, s);
    A.hrow = h->upload(P.heavy_row, s);
    A.hptr = h->upload(P.heavy_ptr, s);
    A.hcol = h->upload(P.heavy_col, s);
    // hot columns: only for the separate-p SpMV over a vector well beyond
    // what the L2 of one XCD holds (4 MB); a copy of 2^16 values (512 KB)
    // took the SpMV of a 3.9M-vertex Chung-Lu graph from 846 to 707 us
    // (2^18: 714 us, 2^20: 757 us)
    int64_t nh = h->fuse_p || h->n < (int64_t)1 << 19 ? 0 : std::min<int64_t>(h->n / 8, 1 << 16);
    nh = env_int("LAPGPU_HOT_COLS", (int)nh);
    if (!h->fuse_p && nh > 0) {
        std::vector<int32_t> hot, col, hcol;
        hot_columns(P, h->n, nh, hot, col, hcol);
        h->nhot = (int32_t)hot.size();
        h->hot = h->upload(hot, s);
        h->hot_col = h->upload(col, s);
        h->hot_hcol = h->upload(hcol, s);
    }
}

// The SpMV matrix, the preconditioner and the workspace of one value type.
template <class T>
void upload_engine(lap_hierarchy* h, Engine<T>& e, hipStream_t s, bool with_levels) {
    const HostPlan& P = h->plan;
    const int L = P.nlev();
    const int Tl = L - 1;
    const int64_t n = h->n;
    e.on = true;
    {
        const Sell<double>& I = h->Ai;
        e.A.nlight = I.nlight;
        e.A.nheavyblk = I.nheavyblk;
        e.A.off = I.off;
        e.A.width = I.width;
        e.A.col = I.col;
        e.A.row = I.row;
        e.A.hblk = I.hblk;
        e.A.hrow = I.hrow;
        e.A.hptr = I.hptr;
        e.A.hcol = I.hcol;
        e.A.w = h->upload(convert<T>(P.sell_w), s);
        e.A.hw = h->upload(convert<T>(P.heavy_w), s);
        e.nlb = nblk(P.sell_nlight);
    }
    e.x = h->dalloc<T>(n);
    e.q = h->dalloc<T>(n);
    e.zn = h->dalloc<T>(n);
    e.p[0] = h->dalloc<T>(n);
    e.p[1] = h->dalloc<T>(n);
    e.r = h->dalloc<T>(n);
    e.z = h->dalloc<T>(n);
    if (h->nhot > 0) e.ph = h->dalloc<T>(h->nhot);
    if (!with_levels) return;
    // the tail: the lowest level from which all coarser levels fit in LDS
    const int tail_max = env_int("LAPGPU_TAIL_MAX", 1 << 30);
    e.kt = Tl;
    for (int k = 1; k <= Tl; ++k)
        if (P.lv[k].g.n <= tail_max && Tl - k <= kMaxTailSteps &&
            tail_lds_units(P, k, ipv<T>()) * sizeof(T) <= kTailLdsBytes) {
            e.kt = k;
            break;
        }
    e.lv.assign(L, LevelDev<T>{});
    for (int k = 0; k < L; ++k) {
        LevelDev<T>& d = e.lv[k];
        d.n = (int32_t)P.lv[k].g.n;
        d.nc = k < Tl ? (int32_t)P.lv[k + 1].g.n : 0;
        if (k >= 1) {
            d.r = h->dalloc<T>(d.n);
            d.y = h->dalloc<T>(d.n);
        } else {
            d.r = e.r;
            d.y = e.z;
        }
        if (k < Tl) {
            const StepCoef& c = P.step[k];
            d.cptr = h->cptr[k];
            d.bst = h->bst[k];
            d.nb = h->nb[k];
            d.saa = h->upload(convert<T>(c.saa), s);
            d.sab = h->upload(convert<T>(c.sab), s);
            d.sbb = h->upload(convert<T>(c.sbb), s);
            d.l0 = h->upload(convert<T>(c.l0), s);
            d.l1 = h->upload(convert<T>(c.l1), s);
            d.l2 = h->upload(convert<T>(c.l2), s);
            d.ea = h->dalloc<T>(d.nc);
            d.eb = h->dalloc<T>(d.nc);
        }
    }
    e.top_pinv = h->upload(convert<T>(P.top_pinv), s);
    if (Tl == 0) return;
    e.fuse01 = false;
    if (Tl >= 2 && e.kt >= 2 && env_int("LAPGPU_FUSE01", 1) != 0) {
        const std::vector<int32_t> b01 = block_partition01(P.step[0].cptr, P.step[1].cptr);
        if (!b01.empty()) {
            e.fuse01 = true;
            e.nb01 = (int)b01.size() - 1;
            std::vector<Blk01> d01(e.nb01);
            for (int b = 0; b < e.nb01; ++b) {
                Blk01& d = d01[b];
                d.A0 = b01[b];
                d.A1 = b01[b + 1];
                d.J0 = P.step[1].cptr[d.A0];
                d.J1 = P.step[1].cptr[d.A1];
                d.t0 = P.step[0].cptr[d.J0];
                d.t1 = P.step[0].cptr[d.J1];
                d.pad0 = d.pad1 = 0;
            }
            e.blk01 = h->upload(d01, s);
        }
    }
    // middle levels [1, kt) (from 2 when levels 0 and 1 are fused): groups
    // of consecutive levels where whole subtrees fit a block, single
    // per-level kernels elsewhere
    e.segs.clear();
    const int cap = env_int("LAPGPU_GRP_CAP", 1024);
    const int maxlev = std::min(kMaxGroupLevels, env_int("LAPGPU_GRP_MAXLEV", kMaxGroupLevels));
    const int first_grouped = std::max(1, env_int("LAPGPU_GRP_FIRST", 2));
    const int32_t units = (int32_t)(kGrpLdsBytes / sizeof(T));
    for (int k0 = e.fuse01 ? 2 : 1; k0 < e.kt;) {
        typename Engine<T>::Segment sg;
        bool placed = false;
        for (int m = std::min(maxlev, e.kt - k0); m >= 1 && !placed && k0 >= first_grouped; --m) {
            std::vector<int32_t> D;
            int nbk = 0;
            int32_t lu = 0, ld = 0;
            if (!plan_group(P, k0, k0 + m, cap, ipv<T>(), units, D, nbk, lu, ld)) continue;
            sg.group = true;
            sg.k0 = k0;
            sg.k1 = k0 + m;
            sg.lds_up = (size_t)lu * sizeof(T);
            sg.lds_down = (size_t)ld * sizeof(T);
            sg.gd.k0 = k0;
            sg.gd.k1 = k0 + m;
            sg.gd.nblocks = nbk;
            sg.gd.D = h->upload(D, s);
            std::vector<int32_t> uoff, doff, xoff;
            std::vector<T> up, dn;
            pack_group(P, k0, k0 + m, nbk, D, uoff, doff, xoff, up, dn);
            sg.gd.uoff = h->upload(uoff, s);
            sg.gd.doff = h->upload(doff, s);
            sg.gd.xoff = h->upload(xoff, s);
            sg.gd.upack = h->upload(up, s);
            sg.gd.dpack = h->upload(dn, s);
            sg.gd.scr = h->dalloc<T>(xoff.back());
            sg.gd.r_top = e.lv[k0 + m].r;
            sg.gd.y_top = e.lv[k0 + m].y;
            sg.gd.r_in = e.lv[k0].r;
            sg.gd.y_out = e.lv[k0].y;
            placed = true;
        }
        if (!placed) {
            sg.group = false;
            sg.k0 = k0;
            sg.k1 = k0 + 1;
        }
        k0 = sg.k1;
        e.segs.push_back(sg);
    }
    TailDesc desc{};
    std::vector<T> pack;
    build_tail(P, e.kt, desc, pack);
    e.tail_pack = h->upload(pack, s);
    e.d_tail = h->dalloc<TailDesc>(1);
    HIPCHK(hipMemcpyAsync(e.d_tail, &desc, sizeof(desc), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    e.tail_lds = (size_t)desc.total * sizeof(T);
    e.tail_args.npack = desc.pack;
    e.tail_args.nsteps = desc.nsteps;
    e.tail_args.n0 = desc.nsteps > 0 ? desc.st[0].nk : desc.nt;
    e.tail_args.r0 = desc.r[0];
    HIPCHK(hipFuncSetAttribute((const void*)k_tail<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kTailLdsBytes));
    HIPCHK(hipFuncSetAttribute((const void*)k_up_grp<T>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGrpLdsBytes));
    HIPCHK(hipFuncSetAttribute((const void*)k_down_grp<T>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGrpLdsBytes));
}

// The factored PEGP system on the device.
void upload_pegp(lap_hierarchy* h, hipStream_t s) {
    const PegpPlan& G = h->pegp_plan;
    const HostPlan& P = h->plan;
    PegpDev& d = h->pegp_dev;
    d.nt = G.nt;
    d.nlev = P.nlev();
    d.ground = G.ground;
    for (int k = 0; k <= d.nlev; ++k) d.off[k] = G.off[k];
    for (int k = 0; k + 1 < d.nlev; ++k) d.cptr[k] = h->cptr[k];
    d.diag = h->upload(G.diag, s);
    d.nflev = (int32_t)G.flev.size() - 1;
    d.fdesc = h->upload(G.fdesc, s);
    d.frow = h->upload(G.frow, s);
    d.fpcol = h->upload(G.fpcol, s);
    d.fpval = h->upload(G.fpval, s);
    d.nblev = (int32_t)G.blev.size() - 1;
    d.bdesc = h->upload(G.bdesc, s);
    d.brow = h->upload(G.brow, s);
    d.bpcol = h->upload(G.bpcol, s);
    d.bpval = h->upload(G.bpval, s);
    d.nd = G.nd;
    d.ndp = G.ndp;
    d.nbc = (int32_t)G.bcrow.size();
    d.drow = h->upload(G.drow, s);
    d.dlr = h->upload(G.dlr, s);
    d.dlc = h->upload(G.dlc, s);
    d.dd = h->upload(G.dd, s);
    d.dcptr = h->upload(G.dcptr, s);
    d.dccol = h->upload(G.dccol, s);
    d.dcval = h->upload(G.dcval, s);
    d.bcrow = h->upload(G.bcrow, s);
    d.bcptr = h->upload(G.bcptr, s);
    d.bccol = h->upload(G.bccol, s);
    d.bcval = h->upload(G.bcval, s);
    d.fg = h->dalloc<double>(G.nt);
    // (the padding rows of the tail vector stay 0: nothing writes them
    // but the dense solve, which keeps them 0)
    d.ty = h->dalloc<double>(std::max(G.ndp, 1));
    HIPCHK(hipMemsetAsync(d.ty, 0, (size_t)std::max(G.ndp, 1) * sizeof(double), s));
    d.cpl = h->dalloc<double>(G.bcrow.size());
    // the vector, then (16-byte aligned) the larger level descriptor table
    // when it fits beside it
    const size_t vec = ((size_t)G.nt * sizeof(double) + 15) / 16 * 16;
    const size_t tab = (size_t)std::max(d.nflev, d.nblev) * kPegpDescInts * sizeof(int32_t);
    d.desc_lds = vec + tab <= kPegpLdsBytes;
    h->pegp_lds = d.desc_lds ? vec + tab : (size_t)G.nt * sizeof(double);
    HIPCHK(hipFuncSetAttribute((const void*)k_pegp_fwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)h->pegp_lds));
    HIPCHK(hipFuncSetAttribute((const void*)k_pegp_bwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)h->pegp_lds));
    // the explicit operator, when formed (its host copy is not kept)
    d.opn = G.opn;
    d.opld = G.opld;
    d.op = nullptr;
    if (G.opn > 0) {
        d.op = h->upload(G.op, s);
        HIPCHK(hipStreamSynchronize(s));
        std::vector<double>().swap(h->pegp_plan.op);
        HIPCHK(hipFuncSetAttribute((const void*)k_pegp_op,
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)(G.opld * sizeof(double))));
    }
}

void upload_plan(lap_hierarchy* h, hipStream_t s) {
    const int64_t n = h->n;
    h->with_msp = (h->params.precond == LAP_PREC_MSP);
    // the off-tree sparsifier is solved like PEGP, on its own subgraph
    h->pegp = (h->params.precond == LAP_PREC_PEGP || h->params.precond == LAP_PREC_OFFTREE ||
               h->params.precond == LAP_PREC_SPANNING);
    h->mixed = (h->params.precision == LAP_MIXED_FP32_FP64);
    upload_shared(h, s);
    if (h->pegp) upload_pegp(h, s);
    // a mixed-precision hierarchy carries the FP64 solve as well
    // (lap_set_precision switches between them)
    upload_engine(h, h->e64, s, h->with_msp);
    if (h->mixed) upload_engine(h, h->e32, s, h->with_msp);
    h->bh = h->dalloc<double>(n);
    h->xc = h->dalloc<double>(n);
    // the refinement of mixed precision and the residual replacements of
    // FP64 solves
    h->x64 = h->dalloc<double>(n);
    h->r64 = h->dalloc<double>(n);
    h->S = h->dalloc<Scal>(1);
    h->So = h->dalloc<Scal>(1);
    int gmax = std::max(nblk(n), h->e64.spmv_grid());
    for (int b : h->nb) gmax = std::max(gmax, b);
    gmax = std::max(gmax, std::max(h->e64.nb01, h->e32.nb01));
    if (h->pegp) gmax = std::max(gmax, (h->pegp_dev.opn + kPegpOpRows - 1) / kPegpOpRows);
    h->part = h->dalloc<double>((size_t)kMaxGridPart * gmax + 64);
    h->part2 = h->dalloc<double>((size_t)gmax + 64);
    HIPCHK(hipHostMalloc((void**)&h->stage, sizeof(Scal), hipHostMallocDefault));
    std::memset(h->stage, 0, sizeof(Scal));
    HIPCHK(hipMemcpyAsync(h->S, h->stage, sizeof(Scal), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->So, h->stage, sizeof(Scal), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipGetLastError());
    // Iterations per captured chunk.  The PCG loop keeps one chunk in flight
    // beyond the one it checks, so up to two chunks run past convergence as
    // iterations that return at once; each still costs its dispatches.  A
    // PEGP iteration is about 30 dispatches and a few hundred microseconds,
    // so two iterations already cover the host's check.  From 2^20 vertices
    // an iteration takes ~100 us or more and solves run long, so longer
    // chunks (fewer graph launches) pay for the overshoot: 3,369 -> 3,339 ms
    // on a 128^3 grid solve of 23,702 iterations with 32 instead of 8.
    const int dflt = h->pegp ? 2 : h->n >= ((int64_t)1 << 20) ? 32 : 8;
    h->chunk = std::max(2, env_int("LAPGPU_CHUNK", dflt) & ~1);
    h->inner_tol = env_double("LAPGPU_INNER_TOL", 1e-4);
    h->reliable_drop = env_double("LAPGPU_RELIABLE_DROP", kReliableDrop);
    h->reliable = env_int("LAPGPU_MIXED_RESTART", 0) == 0;
    build_graph(h, h->e64);
    if (h->mixed) build_graph(h, h->e32);
    h->has_fp32 = h->mixed;
}

// ------------------------------------------------------------ block solve

template <class T>
void upload_block_engine(lap_hierarchy* h, EngineM<T>& m, const Engine<T>& e, hipStream_t s) {
    const HostPlan& P = h->plan;
    const int L = P.nlev();
    const int Tl = L - 1;
    const int64_t n = h->n;
    const size_t K = kCols;
    m.on = true;
    {
        const Adjacency& g = P.solve_graph();
        m.A.n = (int32_t)n;
        m.A.ptr = h->upload(g.ptr, s);
        m.A.col = h->upload(g.col, s);
        m.A.w = h->upload(convert<T>(g.w), s);
    }
    m.x = h->dalloc<T>(n * K);
    m.q = h->dalloc<T>(n * K);
    m.zn = h->dalloc<T>(n * K);
    m.p[0] = h->dalloc<T>(n * K);
    m.p[1] = h->dalloc<T>(n * K);
    m.lv.assign(L, LevelDev<T>{});
    m.up.assign(std::max(Tl, 0), Chunks{});
    m.down.assign(std::max(Tl, 0), Chunks{});
    m.scrU.assign(std::max(Tl, 0), nullptr);
    for (int k = 0; k < L; ++k) {
        LevelDev<T>& d = m.lv[k];
        d.n = (int32_t)P.lv[k].g.n;
        d.nc = k < Tl ? (int32_t)P.lv[k + 1].g.n : 0;
        d.r = h->dalloc<T>((size_t)d.n * K);
        d.y = h->dalloc<T>((size_t)d.n * K);
        if (k < Tl && h->with_msp) {
            const LevelDev<T>& c = e.lv[k];
            d.cptr = c.cptr;
            d.saa = c.saa;
            d.sab = c.sab;
            d.sbb = c.sbb;
            d.l0 = c.l0;
            d.l1 = c.l1;
            d.l2 = c.l2;
            d.ea = h->dalloc<T>((size_t)d.nc * K);
            d.eb = h->dalloc<T>((size_t)d.nc * K);
        }
    }
    if (h->with_msp) m.top_pinv = e.top_pinv;
}

// Work lists of the block SpMM (entries per item `chunk`) and of the
// restriction / prolongation (children per item `seg`), with their scratch.
// Returns false (nothing built) when the split rows' scratch would exceed
// `max_scratch` bytes.
template <class T>
bool build_spmm_chunks(lap_hierarchy* h, EngineM<T>& m, int chunk, size_t max_scratch,
                       hipStream_t s) {
    ChunkHost<int64_t> ch;
    ch.build(h->plan.solve_graph().ptr, chunk);
    const size_t scr = (size_t)std::max(1, ch.nslots()) * kCols * sizeof(T);
    if (scr > max_scratch) return false;
    m.CA = h->upload_chunks(ch, s);
    m.scrA = h->dalloc<T>(scr / sizeof(T));
    m.chunk = chunk;
    return true;
}

template <class T>
void build_level_chunks(lap_hierarchy* h, EngineM<T>& m, int seg, hipStream_t s) {
    const HostPlan& P = h->plan;
    const int Tl = P.nlev() - 1;
    const size_t K = kCols;
    m.seg = seg;
    if (!h->with_msp) return;
    for (int k = 0; k < Tl; ++k) {
        ChunkHost<int32_t> cu;
        cu.build(P.step[k].cptr, seg);
        m.up[k] = h->upload_chunks(cu, s);
        m.down[k] = m.up[k];
        m.scrU[k] = h->dalloc<T>((size_t)std::max(1, cu.nslots()) * 3 * K);
    }
}

void upload_block(lap_hierarchy* h, hipStream_t s) {
    const int64_t n = h->n;
    const size_t K = kCols;
    if (h->has_fp32) upload_block_engine(h, h->m32, h->e32, s);
    upload_block_engine(h, h->m64, h->e64, s);
    h->A64m = h->m64.A;
    h->bhm = h->dalloc<double>(n * K);
    h->xm = h->dalloc<double>(n * K);
    h->rm = h->dalloc<double>(n * K);
    h->xcm = h->dalloc<double>(n * K);
    h->Sm = h->dalloc<ScalM>(1);
    h->Smo = h->dalloc<ScalM>(1);
    h->partm = h->dalloc<double>((size_t)3 * kMmMaxGrid * K + 64);
    h->partm2 = h->dalloc<double>((size_t)kMmMaxGrid * K + 64);
    HIPCHK(hipHostMalloc((void**)&h->stagem, sizeof(ScalM), hipHostMallocDefault));
    std::memset(h->stagem, 0, sizeof(ScalM));
    h->has_block = true;
}

template <int OP>
void finish_m(lap_hierarchy* h, hipStream_t s, ScalM* S, int G, int G2 = 0,
              const ServeCtl* ctl = nullptr) {
    hipLaunchKernelGGL(k_mm_finish<OP>, dim3(1), dim3(1024), 0, s, G, (int)h->n,
                       (const double*)h->partm, G2, (const double*)h->partm2, S, ctl);
}

// The block preconditioner: level-0 update (when do_update), restriction
// and local solves up the levels, the top, prolongation back, z with its
// per-column sums.
template <class T>
void enqueue_mm_precond(lap_hierarchy* h, EngineM<T>& m, hipStream_t s, int do_update,
                        const T* pcur) {
    const int Tl = h->plan.nlev() - 1;
    const int n = (int)h->n;
    ScalM* S = h->Sm;
    const int gn = mm_grid(n);
    LevelDev<T>& l0 = m.lv[0];
    if (do_update)
        hipLaunchKernelGGL(k_mm_update<T>, dim3(gn), dim3(kMmWaves * 64), 0, s, n, h->t2s, m.x,
                           l0.r, pcur, (const T*)m.q, (const ScalM*)S, h->partm2);
    if (!h->with_msp) {
        hipLaunchKernelGGL(k_mm_copy<T>, dim3(gn), dim3(kMmWaves * 64), 0, s, n, (const T*)l0.r,
                           l0.y, (const ScalM*)S);
    } else {
        for (int k = 0; k < Tl; ++k) {
            const Chunks& C = m.up[k];
            hipLaunchKernelGGL(k_mm_up<T>, dim3(mm_grid(C.nitems)), dim3(kMmWaves * 64), 0, s,
                               m.lv[k], C, (const T*)m.lv[k].r, m.lv[k + 1].r, m.scrU[k],
                               (const ScalM*)S);
            if (C.nmulti > 0)
                hipLaunchKernelGGL(k_mm_up_combine<T>, dim3(mm_grid(C.nmulti)),
                                   dim3(kMmWaves * 64), 0, s, m.lv[k], C, m.lv[k + 1].r,
                                   (const T*)m.scrU[k], (const ScalM*)S);
        }
        hipLaunchKernelGGL(k_mm_top<T>, dim3(1), dim3(kMmWaves * 64), 0, s,
                           (int)h->plan.lv[Tl].g.n, (const T*)m.top_pinv, (const T*)m.lv[Tl].r,
                           m.lv[Tl].y, (const ScalM*)S);
        for (int k = Tl - 1; k >= 0; --k) {
            const Chunks& C = m.down[k];
            hipLaunchKernelGGL(k_mm_down<T>, dim3(mm_grid(C.nitems)), dim3(kMmWaves * 64), 0, s,
                               m.lv[k], C, (const T*)m.lv[k].r, m.lv[k].y,
                               (const T*)m.lv[k + 1].y, (const ScalM*)S);
        }
    }
    hipLaunchKernelGGL(k_mm_zout<T>, dim3(gn), dim3(kMmWaves * 64), 0, s, n, h->t2s,
                       (const T*)l0.r, (const T*)l0.y, m.zn, (const ScalM*)S, h->partm);
    finish_m<kMmRho>(h, s, S, gn, do_update ? gn : 0);
}

template <class T>
void enqueue_mm_iteration(lap_hierarchy* h, EngineM<T>& m, hipStream_t s, int par,
                          hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
    const int n = (int)h->n;
    ScalM* S = h->Sm;
    hipLaunchKernelGGL(k_mm_pupd<T>, dim3(mm_grid(n)), dim3(kMmWaves * 64), 0, s, n,
                       (const T*)m.zn, (const T*)m.p[par], m.p[1 - par], (const ScalM*)S);
    const int ga = mm_grid(m.CA.nitems, m.grid);
    launch_timed(k_mm_spmm<T>, dim3(ga), dim3(kMmWaves * 64), 0, s, e0, e1, m.A, m.CA,
                 (const T*)m.p[1 - par], m.q, m.scrA, (const ScalM*)S, h->partm);
    int gc = 0;
    if (m.CA.nmulti > 0) {
        // split rows: their Q rows and p^T q shares come from the combine
        gc = mm_grid(m.CA.nmulti);
        hipLaunchKernelGGL(k_mm_spmm_combine<T>, dim3(gc), dim3(kMmWaves * 64), 0, s, m.CA,
                           (const T*)m.p[1 - par], m.q, (const T*)m.scrA, (const ScalM*)S,
                           h->partm2);
    }
    finish_m<kMmPq>(h, s, S, ga, gc);
    enqueue_mm_precond(h, m, s, 1, (const T*)m.p[1 - par]);
}

template <class T>
void build_mm_graph(lap_hierarchy* h, EngineM<T>& m) {
    HIPCHK(hipStreamCreateWithFlags(&m.cap, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(m.cap, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < h->chunk; ++i) enqueue_mm_iteration(h, m, m.cap, i & 1);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamEndCapture(m.cap, &m.graph));
    HIPCHK(hipGraphInstantiate(&m.exec, m.graph, nullptr, nullptr, 0));
}

// ------------------------------------------------------------ autotuner
//
// The block solve's work decomposition is picked per hierarchy and value
// type by timing candidates on the device at set-up, on the hierarchy's own
// matrix and levels:
//   - SpMM: matrix entries per work item (rows with more are split into
//     chunks whose partial rows a combine pass adds) x workgroups of the
//     launch (each takes a contiguous range of items): the pair with the
//     shortest SpMM (+ combine) time;
//   - restriction / prolongation: children per work item, by the time of
//     one block preconditioner application.
// Environment: LAPGPU_MM_TUNE=0 keeps the defaults untimed;
// LAPGPU_MM_CHUNK, LAPGPU_MM_GRID, LAPGPU_MM_SEG pin one size each.
constexpr int kTuneChunks[] = {32, 64, 128, 256, 512};
constexpr int kTuneGrids[] = {256, 512, 1024, 2048};
constexpr int kTuneSegs[] = {32, 64, 128, 256};
constexpr int kTuneReps = 3;
constexpr size_t kTuneMaxScratch = size_t(512) << 20;  // split-row scratch of a candidate
static_assert(2048 <= 3 * kMmMaxGrid, "the SpMM's partials fit the partial buffer");
static_assert(kPegpThreads == kPegpSolveThreads, "the PEGP plan is made for the solve's workgroup");
static_assert(kTailS == kPegpTailBlock, "the PEGP tail is padded to the solve's superblocks");

// Average time per call of `launch` over kTuneReps calls after one warm-up.
template <class F>
double tune_time_us(hipStream_t s, F&& launch) {
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    launch();
    HIPCHK(hipEventRecord(a, s));
    for (int i = 0; i < kTuneReps; ++i) launch();
    HIPCHK(hipEventRecord(b, s));
    HIPCHK(hipEventSynchronize(b));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    HIPCHK(hipGetLastError());
    return 1e3 * ms / kTuneReps;
}

template <class T>
void tune_block(lap_hierarchy* h, EngineM<T>& m, hipStream_t s) {
    const int n = (int)h->n;
    const size_t K = kCols;
    const bool tune = env_int("LAPGPU_MM_TUNE", 1) != 0;
    const int pin_c = env_int("LAPGPU_MM_CHUNK", 0), pin_g = env_int("LAPGPU_MM_GRID", 0),
              pin_s = env_int("LAPGPU_MM_SEG", 0);
    std::vector<int> cs, gs, ss;
    auto pick = [&](std::vector<int>& out, int pin, int dflt, const int* cand, int nc) {
        if (pin > 0) out = {pin};
        else if (!tune) out = {dflt};
        else out.assign(cand, cand + nc);
    };
    pick(cs, pin_c, kMmChunk, kTuneChunks, (int)std::size(kTuneChunks));
    pick(gs, pin_g, kMmMaxGrid, kTuneGrids, (int)std::size(kTuneGrids));
    pick(ss, pin_s, kMmChunk, kTuneSegs, (int)std::size(kTuneSegs));
    for (int g : gs)
        if (g < 1 || g > 2048) throw std::invalid_argument("LAPGPU_MM_GRID outside 1..2048");
    int bc = cs[0], bg = gs[0], bs = ss[0];
    if (cs.size() * gs.size() > 1 || ss.size() > 1) {
        // timed on zero vectors with every column running
        HIPCHK(hipMemsetAsync(h->Sm, 0, sizeof(ScalM), s));
        HIPCHK(hipMemsetAsync(m.p[0], 0, (size_t)n * K * sizeof(T), s));
        HIPCHK(hipMemsetAsync(m.lv[0].r, 0, (size_t)n * K * sizeof(T), s));
        double best = 1e300;
        for (int c : cs) {
            const size_t mk = h->mark();
            if (!build_spmm_chunks(h, m, c, kTuneMaxScratch, s)) continue;
            for (int g : gs) {
                const double t = tune_time_us(s, [&]() {
                    hipLaunchKernelGGL(k_mm_spmm<T>, dim3(mm_grid(m.CA.nitems, g)),
                                       dim3(kMmWaves * 64), 0, s, m.A, m.CA, (const T*)m.p[0],
                                       m.q, m.scrA, (const ScalM*)h->Sm, h->partm);
                    if (m.CA.nmulti > 0)
                        hipLaunchKernelGGL(k_mm_spmm_combine<T>, dim3(mm_grid(m.CA.nmulti)),
                                           dim3(kMmWaves * 64), 0, s, m.CA, (const T*)m.p[0],
                                           m.q, (const T*)m.scrA, (const ScalM*)h->Sm,
                                           h->partm2);
                });
                if (t < best) {
                    best = t;
                    bc = c;
                    bg = g;
                }
            }
            HIPCHK(hipStreamSynchronize(s));
            h->release_to(mk);
        }
        best = 1e300;
        for (int sg : ss) {
            if (ss.size() == 1) break;
            const size_t mk = h->mark();
            build_level_chunks(h, m, sg, s);
            const double t = tune_time_us(s, [&]() {
                enqueue_mm_precond(h, m, s, 0, (const T*)m.p[0]);
            });
            if (t < best) {
                best = t;
                bs = sg;
            }
            HIPCHK(hipStreamSynchronize(s));
            h->release_to(mk);
        }
    }
    if (!build_spmm_chunks(h, m, bc, SIZE_MAX, s))
        throw std::runtime_error("block SpMM chunk list");
    build_level_chunks(h, m, bs, s);
    m.grid = bg;
}

void setup_block(lap_hierarchy* h, hipStream_t s) {
    upload_block(h, s);
    const auto t0 = std::chrono::steady_clock::now();
    if (h->m32.on) tune_block(h, h->m32, s);
    tune_block(h, h->m64, s);
    h->mm_tune_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    h->CA64 = h->m64.CA;
    h->scrA64 = h->m64.scrA;
    build_mm_graph(h, h->m64);
    if (h->m32.on) build_mm_graph(h, h->m32);
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

Scal read_scal(lap_hierarchy* h, const Scal* S, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(h->stage, S, sizeof(Scal), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return *h->stage;
}

// PCG on engine e for the right-hand side rhs (FP64, solve order, projected
// here): x = 0 start, stop at ||r|| <= tol ||rhs^|| or after maxit products
// with L.  Returns the final scalars.
template <class T>
Scal run_pcg(lap_hierarchy* h, Engine<T>& e, const double* rhs, double tol, int maxit,
             hipStream_t s) {
    const int n = (int)h->n;
    std::memset(h->stage, 0, sizeof(Scal));
    h->stage->tol2 = tol * tol;
    h->stage->maxit = maxit;
    HIPCHK(hipMemcpyAsync(h->S, h->stage, sizeof(Scal), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_sum, dim3(nblk(n)), dim3(kBlock), 0, s, n, rhs, h->part);
    finish<kFinBsum>(h, s, h->S, nblk(n));
    hipLaunchKernelGGL(k_init<T>, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->t2s, rhs, e.r, e.x,
                       e.p[0], e.p[1], (const Scal*)h->S, h->part);
    finish<kFinBn2>(h, s, h->S, nblk(n));
    enqueue_precond(h, e, s, 0);
    HIPCHK(hipGetLastError());
    // chunks of iterations; one chunk in flight beyond the one being checked
    hipEvent_t ev;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    const int max_chunks = maxit / h->chunk + 2;
    try {
        HIPCHK(hipGraphLaunch(e.exec, s));
        for (int c = 0; c < max_chunks; ++c) {
            HIPCHK(hipMemcpyAsync(h->stage, h->S, sizeof(Scal), hipMemcpyDeviceToHost, s));
            HIPCHK(hipEventRecord(ev, s));
            HIPCHK(hipGraphLaunch(e.exec, s));
            HIPCHK(hipEventSynchronize(ev));
            if (h->stage->done) break;
        }
    } catch (const HipErr&) {
        (void)hipEventDestroy(ev);
        throw;
    }
    (void)hipEventDestroy(ev);
    const Scal R = read_scal(h, h->S, s);
    // the last iteration's step (iteration k wrote its p to p[k & 1])
    if (R.iter > 0)
        hipLaunchKernelGGL(k_last_step<T>, dim3(nblk(n)), dim3(kBlock), 0, s, n, e.x,
                           (const T*)e.p[R.iter & 1], (T*)nullptr, (const Scal*)h->S);
    HIPCHK(hipGetLastError());
    return R;
}

// Mean-free x (solve order) into the caller's buffer (input order) and the
// true FP64 residual ||bh - L x||^2 into So->res2.
void finalize_x(lap_hierarchy* h, const double* xsrc, double* x, hipStream_t s) {
    const int n = (int)h->n;
    hipLaunchKernelGGL(k_sum, dim3(nblk(n)), dim3(kBlock), 0, s, n, xsrc, h->part);
    finish<kFinXsum>(h, s, h->So, nblk(n));
    hipLaunchKernelGGL(k_center_out, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->sperm, xsrc,
                       h->xc, x, (const Scal*)h->So);
    const Engine<double>& e = h->e64;
    hipLaunchKernelGGL(k_resid, dim3(e.spmv_grid()), dim3(kBlock), 0, s, e.nlb, e.A,
                       (const double*)h->xc, (const double*)h->bh, (double*)nullptr, h->part);
    finish<kFinRes2>(h, s, h->So, e.spmv_grid());
    HIPCHK(hipGetLastError());
}

// bh = b - mean(b) in solve order; for mixed precision also x64 = 0 and
// r64 = bh.  ||bh||^2 lands in So->res2.
void begin_solve(lap_hierarchy* h, const double* b, bool outer, hipStream_t s) {
    const int n = (int)h->n;
    std::memset(h->stage, 0, sizeof(Scal));
    HIPCHK(hipMemcpyAsync(h->So, h->stage, sizeof(Scal), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_sum, dim3(nblk(n)), dim3(kBlock), 0, s, n, b, h->part);
    finish<kFinBsum>(h, s, h->So, nblk(n));
    hipLaunchKernelGGL(k_init_outer, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->sperm, b, h->bh,
                       outer ? h->x64 : nullptr, outer ? h->r64 : nullptr, (const Scal*)h->So,
                       h->part);
    finish<kFinRes2>(h, s, h->So, nblk(n));
    HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------ spectrum
//
// The extreme eigenvalues of M L_G on range(L_G), from PCG's own
// coefficients: k PCG steps with step lengths alpha_j and direction updates
// beta_j (p_j = z_j + beta_j p_{j-1}) are k steps of Lanczos on M L_G, with
// the tridiagonal T_k: T_jj = 1/alpha_j + beta_j/alpha_{j-1} (beta_0 = 0),
// T_j,j+1 = sqrt(beta_{j+1})/alpha_j (Saad, Iterative Methods for Sparse
// Linear Systems, Sec. 6.7.3).  The iterations run one at a time on the
// FP64 engine, the scalars read back after each.

constexpr double kSpectrumStop = 1e-10;  // relative residual that ends the run

// Number of eigenvalues of the symmetric tridiagonal (d, e) below x: the
// negative pivots of the LDL^T factorisation of T - x I (Sturm count).
static int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x) {
    int c = 0;
    double q = 1.0;
    for (size_t i = 0; i < d.size(); ++i) {
        q = d[i] - x - (i > 0 ? e[i - 1] * e[i - 1] / q : 0.0);
        if (q == 0.0) q = -1e-300;
        if (q < 0.0) ++c;
    }
    return c;
}

// The idx-th smallest eigenvalue of (d, e) by bisection inside the
// Gershgorin interval, to a relative width of 1e-15.
static double tridiag_eig(const std::vector<double>& d, const std::vector<double>& e, int idx) {
    const size_t k = d.size();
    double lo = HUGE_VAL, hi = -HUGE_VAL;
    for (size_t i = 0; i < k; ++i) {
        const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(e[i]) : 0.0);
        lo = std::min(lo, d[i] - r);
        hi = std::max(hi, d[i] + r);
    }
    for (int it = 0; it < 400; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(hi - lo > 1e-15 * std::max(std::fabs(lo), std::fabs(hi))) || mid == lo || mid == hi)
            break;
        if (sturm_count(d, e, mid) > idx) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// PCG from x = 0 on b (device, original order) to `steps` steps or the
// relative residual kSpectrumStop; alpha_0.. and beta_1.. of the steps
// taken (a breakdown step is not taken).  Returns the final scalars.
static Scal pcg_coefficients(lap_hierarchy* h, const double* b, int steps,
                             std::vector<double>& alpha, std::vector<double>& beta,
                             hipStream_t s) {
    Engine<double>& e = h->e64;
    const int n = (int)h->n;
    begin_solve(h, b, false, s);
    std::memset(h->stage, 0, sizeof(Scal));
    h->stage->tol2 = kSpectrumStop * kSpectrumStop;
    h->stage->maxit = steps;
    HIPCHK(hipMemcpyAsync(h->S, h->stage, sizeof(Scal), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_sum, dim3(nblk(n)), dim3(kBlock), 0, s, n, (const double*)h->bh,
                       h->part);
    finish<kFinBsum>(h, s, h->S, nblk(n));
    hipLaunchKernelGGL(k_init<double>, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->t2s,
                       (const double*)h->bh, e.r, e.x, e.p[0], e.p[1], (const Scal*)h->S,
                       h->part);
    finish<kFinBn2>(h, s, h->S, nblk(n));
    enqueue_precond(h, e, s, 0);
    HIPCHK(hipGetLastError());
    Scal R = read_scal(h, h->S, s);
    for (int i = 0; i < steps && R.done == 0; ++i) {
        enqueue_iteration(h, e, s, i & 1);
        HIPCHK(hipGetLastError());
        R = read_scal(h, h->S, s);
        if (R.alpha > 0.0 && std::isfinite(R.alpha)) alpha.push_back(R.alpha);
        else break;
        // a run that stops (converged, or at `steps`) forms no new direction
        if (R.done != 0) break;
        beta.push_back(R.beta);
    }
    return R;
}

// ------------------------------------------------------------ FGMRES
//
// FGMRES on the expanded system L_G~ x~ = P(mu)^T b^ (Sec. 2.2; the solver
// of Sec. 4), right-preconditioned by the grounded inverse of L_T~ (MSP) or
// L_H~ (PEGP), without restarts up to the basis size.  Every basis vector
// lies in the range of P(mu)^T (b~ does, and so does every L_G~ M~ v~), so
// v~ = P(mu)^T u with u its level-0 block, and
//   L_G~ M~ v~ = P(mu)^T L_G (P(mu) M~ P(mu)^T) u = P(mu)^T L_G (M u),
// M the preconditioner of the PCG path (up to a constant, which L_G
// removes).  A step is: M on the level-0 block, the product with L_G, the
// expansion P(mu)^T (level sums), classical Gram-Schmidt twice against the
// basis; the Givens rotations of the small Hessenberg matrix run on the
// host.  At the end x = P(mu) M~ V y = M (sum_i y_i u_i).  A step is one
// product with L_G~, as in the paper's step counts.

constexpr int kFgDotBlocks = 128;       // row blocks of a dot product
constexpr size_t kFgMaxBasisBytes = size_t(8) << 30;

void fg_alloc(lap_hierarchy* h, int m_req) {
    const HostPlan& P = h->plan;
    const int L = P.nlev();
    std::vector<int64_t> off(L + 1, 0);
    for (int k = 0; k < L; ++k) off[k + 1] = off[k] + P.lv[k].g.n;
    const int64_t nt = off[L];
    const int m_mem = (int)std::max<int64_t>(1, (int64_t)(kFgMaxBasisBytes / (8 * nt)) - 1);
    const int m = std::max(1, std::min(m_req, m_mem));
    if (h->fg_V && h->fg_m == m) return;
    if (h->fg_V) throw std::runtime_error("FGMRES basis size changed");
    h->fg_m = m;
    h->fg_nt = nt;
    h->fg_off = off;
    h->fg_V = h->dalloc<double>((size_t)(m + 1) * nt);
    h->fg_w = h->dalloc<double>(nt);
    h->fg_y = h->dalloc<double>(h->n);
    h->fg_x = h->dalloc<double>(h->n);
    h->fg_r = h->dalloc<double>(h->n);
    h->fg_part = h->dalloc<double>((size_t)(m + 1) * kFgDotBlocks);
    h->fg_h = h->dalloc<double>(2 * (size_t)(m + 1) + 2);
    HIPCHK(hipHostMalloc((void**)&h->fg_hh, sizeof(double) * (2 * (size_t)(m + 1) + 2),
                         hipHostMallocDefault));
}

// w = P(mu)^T y (y in solve order)
void fg_expand(lap_hierarchy* h, const double* y, double* w, hipStream_t s) {
    const int n = (int)h->n, L = h->plan.nlev();
    hipLaunchKernelGGL(k_fg_level0, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->t2s, y, w);
    for (int k = 0; k + 1 < L; ++k) {
        const int nc = (int)h->plan.lv[k + 1].g.n;
        hipLaunchKernelGGL(k_fg_restrict, dim3(nblk(nc)), dim3(kBlock), 0, s, nc,
                           (const int32_t*)h->cptr[k], (const double*)(w + h->fg_off[k]),
                           w + h->fg_off[k + 1], -h->params.mu);
    }
}

// out[0..k) = V_i . w for the first k basis vectors (device)
void fg_dots(lap_hierarchy* h, int k, const double* V, const double* w, double* out,
             hipStream_t s) {
    const int64_t nt = h->fg_nt;
    const int G = (int)std::min<int64_t>(kFgDotBlocks, (nt + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_fg_mdot, dim3(G, k), dim3(kBlock), 0, s, nt, V, nt, w, h->fg_part);
    hipLaunchKernelGGL(k_fg_dot_finish, dim3(k), dim3(kBlock), 0, s, G,
                       (const double*)h->fg_part, out);
}

lap_status solve_fgmres(lap_hierarchy* h, const double* b, double* x, double tol,
                        lap_solve_info* info, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!h->with_msp && !h->pegp) return LAP_EUNSUPPORTED;
    fg_alloc(h, env_int("LAPGPU_FGMRES_RESTART", 1000));
    const int n = (int)h->n, m = h->fg_m;
    const int64_t nt = h->fg_nt;
    Engine<double>& e = h->e64;
    begin_solve(h, b, false, s);
    const double bn2 = read_scal(h, h->So, s).res2;
    if (!std::isfinite(bn2)) return LAP_EINVAL;
    // the preconditioner kernels run while S->done is 0
    std::memset(h->stage, 0, sizeof(Scal));
    HIPCHK(hipMemcpyAsync(h->S, h->stage, sizeof(Scal), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(h->fg_x, 0, sizeof(double) * n, s));
    double* V = h->fg_V;
    double* w = h->fg_w;
    double* hh = h->fg_hh;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    auto Hc = [&](int i, int j) -> double& { return H[(size_t)j * (m + 1) + i]; };
    auto norm2 = [&](const double* v) {
        fg_dots(h, 1, v, v, h->fg_h, s);
        HIPCHK(hipMemcpyAsync(hh, h->fg_h, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return hh[0];
    };
    const int maxit = h->params.max_iter;
    int total = 0;
    double beta0 = 0.0, est = 1.0;
    lap_status st = LAP_ENOCONV;
    const double* rsrc = h->bh;   // residual of the current cycle (solve order)
    for (bool first = true; total < maxit; first = false) {
        fg_expand(h, rsrc, V, s);
        const double beta = std::sqrt(norm2(V));
        if (first) beta0 = beta;
        if (!(beta0 > 0.0) || beta <= tol * beta0) {
            est = beta0 > 0.0 ? beta / beta0 : 0.0;
            st = LAP_OK;
            break;
        }
        hipLaunchKernelGGL(k_fg_axpby, dim3(nblk(nt)), dim3(kBlock), 0, s, nt, 1.0 / beta,
                           (const double*)V, 0.0, V);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        bool conv = false;
        for (int j = 0; j < m && total < maxit; ++j) {
            double* vj = V + (size_t)j * nt;
            // z = M u_j (u_j: level 0 of v_j, tree order), then L z, expanded
            HIPCHK(hipMemcpyAsync(e.r, vj, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
            enqueue_precond(h, e, s, 0);
            hipLaunchKernelGGL(k_spmv_plain, dim3(e.spmv_grid()), dim3(kBlock), 0, s, e.nlb,
                               e.A, (const double*)e.zn, h->fg_y);
            fg_expand(h, h->fg_y, w, s);
            // classical Gram-Schmidt, twice
            double* h1 = h->fg_h;
            double* h2 = h->fg_h + (m + 1);
            fg_dots(h, j + 1, V, w, h1, s);
            hipLaunchKernelGGL(k_fg_maxpy, dim3(nblk(nt)), dim3(kBlock), 0, s, nt, j + 1,
                               (const double*)V, nt, (const double*)h1, -1.0, w);
            fg_dots(h, j + 1, V, w, h2, s);
            hipLaunchKernelGGL(k_fg_maxpy, dim3(nblk(nt)), dim3(kBlock), 0, s, nt, j + 1,
                               (const double*)V, nt, (const double*)h2, -1.0, w);
            fg_dots(h, 1, w, w, h->fg_h + 2 * (m + 1), s);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(hh, h->fg_h, sizeof(double) * (2 * (size_t)(m + 1) + 1),
                                  hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            ++total;
            for (int i = 0; i <= j; ++i) Hc(i, j) = hh[i] + hh[(m + 1) + i];
            const double hn = std::sqrt(std::max(hh[2 * (m + 1)], 0.0));
            Hc(j + 1, j) = hn;
            for (int i = 0; i < j; ++i) {
                const double a = Hc(i, j), c = Hc(i + 1, j);
                Hc(i, j) = cs[i] * a + sn[i] * c;
                Hc(i + 1, j) = -sn[i] * a + cs[i] * c;
            }
            const double den = std::hypot(Hc(j, j), Hc(j + 1, j));
            cs[j] = den == 0.0 ? 1.0 : Hc(j, j) / den;
            sn[j] = den == 0.0 ? 0.0 : Hc(j + 1, j) / den;
            Hc(j, j) = den;
            Hc(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            est = std::fabs(g[j + 1]) / beta0;
            if (std::fabs(g[j + 1]) <= tol * beta0) {
                conv = true;
                break;
            }
            if (!(hn > 0.0) || !std::isfinite(hn)) break;
            hipLaunchKernelGGL(k_fg_axpby, dim3(nblk(nt)), dim3(kBlock), 0, s, nt, 1.0 / hn,
                               (const double*)w, 0.0, V + (size_t)(j + 1) * nt);
        }
        if (k == 0) break;
        for (int i = k - 1; i >= 0; --i) {
            double t = g[i];
            for (int c = i + 1; c < k; ++c) t -= Hc(i, c) * y[c];
            y[i] = t / Hc(i, i);
        }
        if (!std::all_of(y.begin(), y.begin() + k, [](double v) { return std::isfinite(v); })) {
            st = LAP_EBREAKDOWN;
            break;
        }
        // x += M (sum_i y_i u_i): the level-0 blocks combined into e.r
        std::copy(y.begin(), y.begin() + k, hh);
        HIPCHK(hipMemcpyAsync(h->fg_h, hh, sizeof(double) * k, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemsetAsync(e.r, 0, sizeof(double) * n, s));
        hipLaunchKernelGGL(k_fg_maxpy, dim3(nblk(n)), dim3(kBlock), 0, s, (int64_t)n, k,
                           (const double*)V, nt, (const double*)h->fg_h, 1.0, e.r);
        enqueue_precond(h, e, s, 0);
        hipLaunchKernelGGL(k_fg_axpby, dim3(nblk(n)), dim3(kBlock), 0, s, (int64_t)n, 1.0,
                           (const double*)e.zn, 1.0, h->fg_x);
        HIPCHK(hipStreamSynchronize(s));
        if (conv) {
            st = LAP_OK;
            break;
        }
        // restart from the true residual
        hipLaunchKernelGGL(k_resid, dim3(e.spmv_grid()), dim3(kBlock), 0, s, e.nlb, e.A,
                           (const double*)h->fg_x,
                           (const double*)h->bh, h->fg_r, h->part);
        rsrc = h->fg_r;
    }
    finalize_x(h, h->fg_x, x, s);
    // LAP_OK: the expanded residual met tol (the stop test of Sec. 4); the
    // residual of the original system is reported as measured
    const Scal O = read_scal(h, h->So, s);
    if (info) {
        const double bn = std::sqrt(bn2);
        info->iterations = total;
        info->refinements = 0;
        info->relres_true = bn > 0 ? std::sqrt(O.res2) / bn : 0.0;
        info->relres_recursive = est;
        info->status = st;
        info->seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return st;
}

// Residual replacements after a converged recurrence whose true residual
// still misses tol (Sec. 4 stops on the residual of the original system).
constexpr int kMaxReplacements = 3;

// FP64 PCG (Sec. 4, App. A.4).  When the recursive residual meets tol the
// mean-free x and its true residual t = b^ - L x are formed; if ||t|| is
// still above tol ||b^||, the run restarts from x with r = t - mean(t)
// (at most kMaxReplacements times, under the same cap on products with L):
// the correction d solves L d = t from d = 0 to the same absolute residual
// tol ||b^||, and x += d.  A true residual above tol after the last
// replacement, or no products left, gives LAP_ENOCONV.
lap_status solve_fp64(lap_hierarchy* h, const double* b, double* x, double tol,
                      lap_solve_info* info, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const int n = (int)h->n;
    const Engine<double>& e = h->e64;
    begin_solve(h, b, false, s);
    const int maxit = h->params.max_iter;
    Scal R = run_pcg(h, h->e64, h->bh, tol, maxit, s);
    const double bn2 = R.bn2;
    finalize_x(h, h->e64.x, x, s);
    Scal O = read_scal(h, h->So, s);
    int iters = R.iter, reps = 0;
    lap_status st = R.done == 0 ? LAP_ENOCONV : to_status(R.done);
    while (st == LAP_OK && !(O.res2 <= tol * tol * bn2)) {
        if (reps == kMaxReplacements || iters >= maxit || !(O.res2 > 0.0) ||
            !std::isfinite(O.res2)) {
            st = LAP_ENOCONV;
            break;
        }
        ++reps;
        // x64 = x (mean-free), r64 = t = b^ - L x; then L d = t from d = 0
        HIPCHK(hipMemcpyAsync(h->x64, h->xc, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_resid, dim3(e.spmv_grid()), dim3(kBlock), 0, s, e.nlb, e.A,
                           (const double*)h->xc, (const double*)h->bh, h->r64, h->part);
        HIPCHK(hipGetLastError());
        R = run_pcg(h, h->e64, h->r64, tol * std::sqrt(bn2 / O.res2), maxit - iters, s);
        iters += R.iter;
        hipLaunchKernelGGL(k_fg_axpby, dim3(nblk(n)), dim3(kBlock), 0, s, (int64_t)n, 1.0,
                           (const double*)h->e64.x, 1.0, h->x64);
        finalize_x(h, h->x64, x, s);
        O = read_scal(h, h->So, s);
        st = R.done == 0 ? LAP_ENOCONV : to_status(R.done);
    }
    if (info) {
        const double bn = std::sqrt(bn2);
        info->iterations = iters;
        info->refinements = reps;
        info->relres_true = bn > 0 ? std::sqrt(O.res2) / bn : 0.0;
        // the recursive residual of the last run, relative to b^
        info->relres_recursive = bn2 > 0 ? std::sqrt(R.rr / bn2) : 0.0;
        info->status = st;
        info->seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return st;
}

// Mixed precision (iterative refinement): the residual r = b^ - L x, x and
// every inner product stay FP64; each correction d solves L d = r by PCG
// with the FP32 SpMV and preconditioner (FP32 arithmetic, FP64 reductions)
// to a relative residual of inner_tol, then x += d.
lap_status solve_mixed(lap_hierarchy* h, const double* b, double* x, double tol,
                       lap_solve_info* info, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const int n = (int)h->n;
    const Engine<double>& e = h->e64;
    begin_solve(h, b, true, s);
    const double bn2 = read_scal(h, h->So, s).res2;
    if (!std::isfinite(bn2)) return LAP_EINVAL;
    double res2 = bn2;
    int iters = 0, refs = 0, stalls = 0;
    lap_status st = LAP_ENOCONV;
    const int max_refs = 40;
    while (true) {
        if (res2 <= tol * tol * bn2) {
            st = LAP_OK;
            break;
        }
        if (iters >= h->params.max_iter || refs >= max_refs) break;
        const double rel_needed = tol * std::sqrt(bn2 / res2);
        const double itol = std::max(h->inner_tol, 0.5 * rel_needed);
        const Scal R = run_pcg(h, h->e32, h->r64, itol, h->params.max_iter - iters, s);
        iters += R.iter;
        ++refs;
        if (R.iter == 0 && R.done != 1) {
            st = to_status(R.done);
            break;
        }
        hipLaunchKernelGGL(k_add_corr, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->x64,
                           (const float*)h->e32.x);
        hipLaunchKernelGGL(k_resid, dim3(e.spmv_grid()), dim3(kBlock), 0, s, e.nlb, e.A,
                           (const double*)h->x64, (const double*)h->bh, h->r64, h->part);
        finish<kFinRes2>(h, s, h->So, e.spmv_grid());
        HIPCHK(hipGetLastError());
        const double nr2 = read_scal(h, h->So, s).res2;
        if (!std::isfinite(nr2)) {
            st = LAP_EBREAKDOWN;
            break;
        }
        // a refinement that does not halve the residual is a stall
        stalls = nr2 > 0.25 * res2 ? stalls + 1 : 0;
        res2 = nr2;
        if (stalls >= 3) break;
    }
    finalize_x(h, h->x64, x, s);
    const Scal O = read_scal(h, h->So, s);
    if (st == LAP_OK && !(O.res2 <= tol * tol * bn2 * 1.0001)) st = LAP_ENOCONV;
    if (info) {
        const double bn = std::sqrt(bn2);
        info->iterations = iters;
        info->refinements = refs;
        info->relres_true = bn > 0 ? std::sqrt(O.res2) / bn : 0.0;
        info->relres_recursive = bn > 0 ? std::sqrt(res2) / bn : 0.0;
        info->status = st;
        info->seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return st;
}

int rank_status(lap_status s);

ScalM read_scalm(lap_hierarchy* h, const ScalM* S, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(h->stagem, S, sizeof(ScalM), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return *h->stagem;
}

// Inner block PCG on engine m for the right-hand sides rhs (FP64 block,
// solve order): columns with active[c] false take no part; column c stops
// at ||r|| <= sqrt(tol2[c]) ||r_0||.
template <class T>
ScalM run_mm_pcg(lap_hierarchy* h, EngineM<T>& m, const double* rhs, const bool* active,
                 const double* tol2, int maxit, hipStream_t s) {
    const int n = (int)h->n, gn = mm_grid(n);
    ScalM& st = *h->stagem;
    std::memset(&st, 0, sizeof(ScalM));
    for (int c = 0; c < kCols; ++c) {
        st.done[c] = active[c] ? 0 : 5;
        st.tol2[c] = tol2[c];
    }
    st.maxit = maxit;
    HIPCHK(hipMemcpyAsync(h->Sm, &st, sizeof(ScalM), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_mm_colsum, dim3(gn), dim3(kMmWaves * 64), 0, s, n, rhs, h->partm);
    finish_m<kMmSum>(h, s, h->Sm, gn);
    hipLaunchKernelGGL(k_mm_init<T>, dim3(gn), dim3(kMmWaves * 64), 0, s, n, h->t2s, rhs,
                       m.lv[0].r, m.x, m.p[0], m.p[1], (const ScalM*)h->Sm, h->partm);
    finish_m<kMmBn2>(h, s, h->Sm, gn);
    enqueue_mm_precond(h, m, s, 0, (const T*)m.p[0]);
    HIPCHK(hipGetLastError());
    hipEvent_t ev;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    const int max_chunks = maxit / h->chunk + 2;
    try {
        HIPCHK(hipGraphLaunch(m.exec, s));
        for (int c = 0; c < max_chunks; ++c) {
            HIPCHK(hipMemcpyAsync(&h->stagem->all_done, &h->Sm->all_done, sizeof(int32_t),
                                  hipMemcpyDeviceToHost, s));
            HIPCHK(hipEventRecord(ev, s));
            HIPCHK(hipGraphLaunch(m.exec, s));
            HIPCHK(hipEventSynchronize(ev));
            if (h->stagem->all_done) break;
        }
    } catch (const HipErr&) {
        (void)hipEventDestroy(ev);
        throw;
    }
    (void)hipEventDestroy(ev);
    return read_scalm(h, h->Sm, s);
}

// r = bh - L x for the block (FP64), per-column ||r||^2 into So->res2.
void block_residual(lap_hierarchy* h, const double* x, hipStream_t s) {
    const Chunks& C = h->CA64;
    const int ga = mm_grid(C.nitems, h->m64.grid);
    hipLaunchKernelGGL(k_mm_resid, dim3(ga), dim3(kMmWaves * 64), 0, s, h->A64m, C, x,
                       (const double*)h->bhm, h->rm, h->scrA64, h->partm);
    int gc = 0;
    if (C.nmulti > 0) {
        gc = mm_grid(C.nmulti);
        hipLaunchKernelGGL(k_mm_resid_combine, dim3(gc), dim3(kMmWaves * 64), 0, s, C,
                           (const double*)h->bhm, h->rm, (const double*)h->scrA64, h->partm2);
    }
    finish_m<kMmRes2>(h, s, h->Smo, ga, gc);
    HIPCHK(hipGetLastError());
}

// Up to kCols right-hand sides at once (caller's columns c < nrhs at
// b + c*ld).  Mixed precision: each refinement runs the FP32 block PCG on
// the FP64 residuals of the columns not yet converged; FP64: the FP64
// block PCG, refined only if a column's recursive residual drifted.
lap_status solve_block(lap_hierarchy* h, const double* b, double* x, int nrhs, int64_t ld,
                       double tol, lap_solve_info* info, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const int n = (int)h->n, gn = mm_grid(n);
    std::memset(h->stagem, 0, sizeof(ScalM));
    HIPCHK(hipMemcpyAsync(h->Smo, h->stagem, sizeof(ScalM), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_mm_colsum_in, dim3(gn), dim3(kMmWaves * 64), 0, s, n, b, ld, nrhs,
                       h->partm);
    finish_m<kMmSum>(h, s, h->Smo, gn);
    hipLaunchKernelGGL(k_mm_begin, dim3(gn), dim3(kMmWaves * 64), 0, s, n, h->sperm, b, ld, nrhs,
                       h->bhm, h->xm, h->rm, (const ScalM*)h->Smo, h->partm);
    finish_m<kMmRes2>(h, s, h->Smo, gn);
    HIPCHK(hipGetLastError());
    ScalM O = read_scalm(h, h->Smo, s);
    double bn2[kCols], res2[kCols], tol2[kCols];
    bool active[kCols];
    int iters[kCols] = {0}, stalls[kCols] = {0};
    lap_status st[kCols];
    for (int c = 0; c < kCols; ++c) {
        bn2[c] = res2[c] = O.res2[c];
        active[c] = c < nrhs;
        st[c] = LAP_ENOCONV;
        if (c < nrhs && !std::isfinite(bn2[c])) {
            st[c] = LAP_EINVAL;
            active[c] = false;
        }
    }
    int refs = 0;
    const bool mixed = h->mixed && h->m32.on;
    while (refs < 40) {
        bool any = false;
        for (int c = 0; c < nrhs; ++c) {
            if (!active[c]) continue;
            if (res2[c] <= tol * tol * bn2[c]) {
                st[c] = LAP_OK;
                active[c] = false;
            } else if (iters[c] >= h->params.max_iter || stalls[c] >= 3) {
                active[c] = false;
            }
            any |= active[c];
            const double need = tol * std::sqrt(bn2[c] / std::max(res2[c], 1e-300));
            const double it = mixed ? std::max(h->inner_tol, 0.5 * need) : 0.9 * need;
            tol2[c] = it * it;
        }
        if (!any) break;
        int maxit = 0;
        for (int c = 0; c < nrhs; ++c)
            if (active[c]) maxit = std::max(maxit, h->params.max_iter - iters[c]);
        ScalM R;
        if (mixed) R = run_mm_pcg(h, h->m32, h->rm, active, tol2, maxit, s);
        else R = run_mm_pcg(h, h->m64, h->rm, active, tol2, maxit, s);
        ++refs;
        for (int c = 0; c < nrhs; ++c)
            if (active[c]) iters[c] += R.iter[c];
        if (mixed)
            hipLaunchKernelGGL(k_mm_addcorr<float>, dim3(gn), dim3(kMmWaves * 64), 0, s, n,
                               h->xm, (const float*)h->m32.x);
        else
            hipLaunchKernelGGL(k_mm_addcorr<double>, dim3(gn), dim3(kMmWaves * 64), 0, s, n,
                               h->xm, (const double*)h->m64.x);
        block_residual(h, h->xm, s);
        O = read_scalm(h, h->Smo, s);
        for (int c = 0; c < nrhs; ++c) {
            if (!active[c]) continue;
            if (R.done[c] == 3 && R.iter[c] == 0) {
                st[c] = LAP_EBREAKDOWN;
                active[c] = false;
                continue;
            }
            if (!std::isfinite(O.res2[c])) {
                st[c] = LAP_EBREAKDOWN;
                active[c] = false;
                continue;
            }
            stalls[c] = O.res2[c] > 0.25 * res2[c] ? stalls[c] + 1 : 0;
            res2[c] = O.res2[c];
        }
    }
    // mean-free x to the caller, true residuals
    hipLaunchKernelGGL(k_mm_colsum, dim3(gn), dim3(kMmWaves * 64), 0, s, n, (const double*)h->xm,
                       h->partm);
    finish_m<kMmSum>(h, s, h->Smo, gn);
    hipLaunchKernelGGL(k_mm_out, dim3(gn), dim3(kMmWaves * 64), 0, s, n, h->sperm,
                       (const double*)h->xm, h->xcm, x, ld, nrhs, (const ScalM*)h->Smo);
    block_residual(h, h->xcm, s);
    O = read_scalm(h, h->Smo, s);
    lap_status worst = LAP_OK;
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int c = 0; c < nrhs; ++c) {
        if (st[c] == LAP_OK && !(O.res2[c] <= tol * tol * bn2[c] * 1.0001)) st[c] = LAP_ENOCONV;
        if (info) {
            const double bn = std::sqrt(bn2[c]);
            info[c].iterations = iters[c];
            info[c].refinements = refs;
            info[c].relres_true = bn > 0 ? std::sqrt(O.res2[c]) / bn : 0.0;
            info[c].relres_recursive = bn > 0 ? std::sqrt(res2[c]) / bn : 0.0;
            info[c].status = st[c];
            info[c].seconds = secs;
        }
        if (rank_status(st[c]) > rank_status(worst)) worst = st[c];
    }
    return worst;
}

// Mixed precision with reliable updates (van der Vorst and Ye's residual
// replacement, as used for mixed-precision CG): one FP32 PCG run keeps its
// search direction throughout; whenever its residual has fallen by
// kReliableDrop since the last replacement (or it meets the tolerance),
// the FP32 correction moves into the FP64 x, the residual is replaced by
// the FP64 b^ - L x, z = M r and rho are recomputed, and beta is rescaled
// to the new rho so the next direction stays consistent.  The stop test is
// on that FP64 residual.
lap_status solve_mixed_reliable(lap_hierarchy* h, const double* b, double* x, double tol,
                                lap_solve_info* info, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const int n = (int)h->n;
    const Engine<double>& e = h->e64;
    Engine<float>& f = h->e32;
    begin_solve(h, b, true, s);
    const double bn2 = read_scal(h, h->So, s).res2;
    if (!std::isfinite(bn2)) return LAP_EINVAL;
    // FP32 run from r = b^ (x32 = 0, p = 0)
    std::memset(h->stage, 0, sizeof(Scal));
    h->stage->tol2 = tol * tol;
    h->stage->maxit = h->params.max_iter;
    HIPCHK(hipMemcpyAsync(h->S, h->stage, sizeof(Scal), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_sum, dim3(nblk(n)), dim3(kBlock), 0, s, n, (const double*)h->r64,
                       h->part);
    finish<kFinBsum>(h, s, h->S, nblk(n));
    hipLaunchKernelGGL(k_init<float>, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->t2s,
                       (const double*)h->r64, f.r, f.x, f.p[0], f.p[1], (const Scal*)h->S,
                       h->part);
    finish<kFinBn2>(h, s, h->S, nblk(n));
    enqueue_precond(h, f, s, 0);
    HIPCHK(hipGetLastError());
    double res2 = bn2, rr_last = bn2;
    int refs = 0;
    lap_status st = LAP_ENOCONV;
    while (true) {
        HIPCHK(hipGraphLaunch(f.exec, s));
        Scal S = read_scal(h, h->S, s);
        const bool replace = S.done == 1 || (S.done == 0 && S.rr <= h->reliable_drop * rr_last);
        if (S.done != 0 && S.done != 1) {
            st = to_status(S.done);
            break;
        }
        if (!replace) continue;
        // reliable update: the run's last step into its x first (and its p
        // into p[0], where the next chunk reads p_old)
        if (S.iter > 0)
            hipLaunchKernelGGL(k_last_step<float>, dim3(nblk(n)), dim3(kBlock), 0, s, n, f.x,
                               (const float*)f.p[S.iter & 1], (S.iter & 1) ? f.p[0] : nullptr,
                               (const Scal*)h->S);
        hipLaunchKernelGGL(k_move_corr, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->x64, f.x);
        hipLaunchKernelGGL(k_resid, dim3(e.spmv_grid()), dim3(kBlock), 0, s, e.nlb, e.A,
                           (const double*)h->x64, (const double*)h->bh, h->r64, h->part);
        finish<kFinRes2>(h, s, h->So, e.spmv_grid());
        HIPCHK(hipGetLastError());
        const double nr2 = read_scal(h, h->So, s).res2;
        ++refs;
        if (!std::isfinite(nr2)) {
            st = LAP_EBREAKDOWN;
            break;
        }
        res2 = nr2;
        if (res2 <= tol * tol * bn2) {
            st = LAP_OK;
            break;
        }
        if (S.iter >= h->params.max_iter) break;
        hipLaunchKernelGGL(k_residual_in, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->t2s,
                           (const double*)h->r64, f.r);
        // continue the run: beta_new = rho' / rho_prev with rho_prev =
        // rho / beta (the finish divides the new rho by the stored one)
        Scal& st2 = *h->stage;
        st2 = S;
        st2.done = 0;
        st2.first = S.beta > 0.0 ? 0 : 1;
        st2.rho = S.beta > 0.0 ? S.rho / S.beta : S.rho;
        st2.alpha = 0.0;  // the last step is in x already
        HIPCHK(hipMemcpyAsync(h->S, &st2, sizeof(Scal), hipMemcpyHostToDevice, s));
        enqueue_precond(h, f, s, 0);
        HIPCHK(hipGetLastError());
        rr_last = res2;
    }
    const Scal R = read_scal(h, h->S, s);
    finalize_x(h, h->x64, x, s);
    const Scal O = read_scal(h, h->So, s);
    if (st == LAP_OK && !(O.res2 <= tol * tol * bn2 * 1.0001)) st = LAP_ENOCONV;
    if (info) {
        const double bn = std::sqrt(bn2);
        info->iterations = R.iter;
        info->refinements = refs;
        info->relres_true = bn > 0 ? std::sqrt(O.res2) / bn : 0.0;
        info->relres_recursive = bn > 0 ? std::sqrt(res2) / bn : 0.0;
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

// Preconditioner applied once to r (FP64, input order, mean-free) into z
// (FP64, input order, mean removed), with engine e.
template <class T>
void apply_precond(lap_hierarchy* h, Engine<T>& e, const double* r, double* z, hipStream_t s) {
    const int n = (int)h->n;
    std::memset(h->stage, 0, sizeof(Scal));
    h->stage->first = 1;
    HIPCHK(hipMemcpyAsync(h->S, h->stage, sizeof(Scal), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_gather<T>, dim3(nblk(n)), dim3(kBlock), 0, s, n,
                       (const int32_t*)h->perm0, r, e.r);
    enqueue_precond(h, e, s, 0);
    hipLaunchKernelGGL(k_shift_out<T>, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->sperm,
                       (const T*)e.zn, z, (const Scal*)h->S);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
}

// Algorithmic bytes of one part of an iteration (lap_profile_kernel): the
// data each kernel must move once, values of vb bytes, int32 indices.
double part_bytes(const lap_hierarchy* h, int kernel, double vb, bool levels, bool fused01) {
    const int T = h->plan.nlev() - 1;
    const HostPlan& P = h->plan;
    const double n = (double)h->n;
    const double nnz = (double)P.lv[0].g.nnz();
    auto lvn = [&](int k) { return (double)P.lv[k].g.n; };
    // step k (level k -> k+1), up: r_k; cptr, pair coefficients, leftover
    // coefficients (2); eta a/b and the restricted value written.
    auto step_up = [&](int k) {
        const double nc = lvn(k + 1), nl = lvn(k) - 2.0 * lvn(k + 1);
        return vb * lvn(k) + 4.0 * nc + 3.0 * vb * nc + 2.0 * vb * nl + 3.0 * vb * nc;
    };
    // down: cptr, eta a/b, y_k+1; leftover coefficients (3) and residuals;
    // y_k written.
    auto step_down = [&](int k) {
        const double nc = lvn(k + 1), nl = lvn(k) - 2.0 * lvn(k + 1);
        return 4.0 * nc + 2.0 * vb * nc + vb * nc + 3.0 * vb * nl + vb * nl + vb * lvn(k);
    };
    // SpMV: z, p_old, x read, p, q, x written (the previous step x +=
    // alpha p_old rides along); col and w per stored entry (with a separate
    // p pass, p is read back once more by the SpMV)
    const double spmv = (h->fuse_p ? 6.0 : 7.0) * vb * n + (4.0 + vb) * nnz;
    // fused levels 0 and 1: the update kernel also restricts level 1 (its r1
    // stays in LDS but is written once for the down-sweep), down0 also
    // prolongs level 1 (y1 stays in LDS)
    // update: q, r read, r written
    double upd = levels ? 3.0 * vb * n + step_up(0) - vb * n : 3.0 * vb * n;
    double down0 = levels ? step_down(0) - vb * (lvn(0) - 2.0 * lvn(1)) + vb * n : 3.0 * vb * n;
    if (levels && fused01) {
        upd += step_up(1) - vb * lvn(1);
        down0 += step_down(1) - vb * lvn(1) - vb * lvn(1);
    }
    double mid = 0.0;
    for (int k = fused01 ? 2 : 1; levels && k < T; ++k) mid += step_up(k) + step_down(k);
    switch (kernel) {
        case LAP_KERNEL_SPMV: return spmv;
        case LAP_KERNEL_UPDATE: return upd;
        case LAP_KERNEL_DOWN0: return down0;
        case LAP_KERNEL_PRECOND: return upd + mid + down0;
        default: return spmv + upd + mid + down0;
    }
}

template <class T>
lap_status profile(lap_hierarchy* h, Engine<T>& e, int32_t kernel, int32_t reps, hipStream_t s,
                   double* avg_ms, double* alg_bytes) {
    const int T_ = h->plan.nlev() - 1;
    const bool levels = h->with_msp && T_ >= 1;
    if ((kernel == LAP_KERNEL_UPDATE || kernel == LAP_KERNEL_DOWN0 ||
         kernel == LAP_KERNEL_PRECOND) && !levels)
        return LAP_EUNSUPPORTED;
    const PegpDev& G = h->pegp_dev;
    if (kernel == LAP_KERNEL_PEGP_OP && !(h->pegp && G.opn > 0)) return LAP_EUNSUPPORTED;
    // the explicit PEGP operator: its opn x opn entries as stored, r gathered
    // through t2s (value and index), z written
    const double bytes =
        kernel == LAP_KERNEL_PEGP_OP
            ? 8.0 * (double)G.opn * (double)G.opn + 20.0 * (double)h->n
            : part_bytes(h, kernel, (double)sizeof(T), levels, e.fuse01);
    // ITER: two events around all timed iterations; a part: its own kernels'
    // timestamps in every timed iteration
    const bool whole = kernel == LAP_KERNEL_ITER;
    const int groups = (reps + kProfGroup - 1) / kProfGroup;
    std::vector<hipEvent_t> ev(whole ? 2 * (size_t)groups : 2 * (size_t)reps, nullptr);
    auto destroy = [&]() {
        for (hipEvent_t x : ev)
            if (x) (void)hipEventDestroy(x);
    };
    try {
        for (auto& x : ev) HIPCHK(hipEventCreate(&x));
        // a fresh PCG run from a fixed right-hand side every kProfGroup
        // timed iterations, so no run nears convergence while timed
        const int n = (int)h->n;
        hipLaunchKernelGGL(k_pattern, dim3(nblk(n)), dim3(kBlock), 0, s, (int64_t)n, h->xc);
        for (int i0 = 0; i0 < reps; i0 += kProfGroup) {
            std::memset(h->stage, 0, sizeof(Scal));
            h->stage->maxit = 0x7fffffff;
            HIPCHK(hipMemcpyAsync(h->S, h->stage, sizeof(Scal), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_sum, dim3(nblk(n)), dim3(kBlock), 0, s, n, (const double*)h->xc,
                               h->part);
            finish<kFinBsum>(h, s, h->S, nblk(n));
            hipLaunchKernelGGL(k_init<T>, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->t2s,
                               (const double*)h->xc, e.r, e.x, e.p[0], e.p[1], (const Scal*)h->S,
                               h->part);
            finish<kFinBn2>(h, s, h->S, nblk(n));
            enqueue_precond(h, e, s, 0);
            const int i1 = std::min(reps, i0 + kProfGroup);
            if (whole) HIPCHK(hipEventRecord(ev[2 * (i0 / kProfGroup)], s));
            for (int i = i0; i < i1; ++i) {
                Marks mk;
                if (!whole) {
                    mk.kernel = kernel;
                    mk.e0 = ev[2 * i];
                    mk.e1 = ev[2 * i + 1];
                }
                enqueue_iteration(h, e, s, i & 1, mk);
            }
            if (whole) HIPCHK(hipEventRecord(ev[2 * (i0 / kProfGroup) + 1], s));
        }
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
        const bool ran = read_scal(h, h->S, s).done == 0;
        destroy();
        return ran ? LAP_OK : LAP_EBREAKDOWN;
    } catch (const HipErr&) {
        destroy();
        return LAP_EDEVICE;
    }
}

template <class T>
lap_status profile_block(lap_hierarchy* h, EngineM<T>& m, int32_t kernel, int32_t reps,
                         hipStream_t s, double* avg_ms, double* alg_bytes) {
    const double vb = (double)sizeof(T), n = (double)h->n, K = kCols;
    const double nnz = (double)h->plan.lv[0].g.nnz();
    const double spmm = 2.0 * n * K * vb + (4.0 + vb) * nnz;
    const bool whole = kernel == LAP_KERNEL_BLOCK_ITER;
    const int groups = (reps + kProfGroup - 1) / kProfGroup;
    std::vector<hipEvent_t> ev(whole ? 2 * (size_t)groups : 2 * (size_t)reps, nullptr);
    auto destroy = [&]() {
        for (hipEvent_t x : ev)
            if (x) (void)hipEventDestroy(x);
    };
    try {
        for (auto& x : ev) HIPCHK(hipEventCreate(&x));
        const int nn = (int)h->n, gn = mm_grid(nn);
        const int64_t cnt = (int64_t)nn * kCols;
        hipLaunchKernelGGL(k_pattern, dim3((unsigned)((cnt + kBlock - 1) / kBlock)), dim3(kBlock),
                           0, s, cnt, h->xcm);
        for (int i0 = 0; i0 < reps; i0 += kProfGroup) {
            ScalM& st = *h->stagem;
            std::memset(&st, 0, sizeof(ScalM));
            st.maxit = 0x7fffffff;
            HIPCHK(hipMemcpyAsync(h->Sm, &st, sizeof(ScalM), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_mm_colsum, dim3(gn), dim3(kMmWaves * 64), 0, s, nn,
                               (const double*)h->xcm, h->partm);
            finish_m<kMmSum>(h, s, h->Sm, gn);
            hipLaunchKernelGGL(k_mm_init<T>, dim3(gn), dim3(kMmWaves * 64), 0, s, nn, h->t2s,
                               (const double*)h->xcm, m.lv[0].r, m.x, m.p[0], m.p[1],
                               (const ScalM*)h->Sm, h->partm);
            finish_m<kMmBn2>(h, s, h->Sm, gn);
            enqueue_mm_precond(h, m, s, 0, (const T*)m.p[0]);
            const int i1 = std::min(reps, i0 + kProfGroup);
            if (whole) HIPCHK(hipEventRecord(ev[2 * (i0 / kProfGroup)], s));
            for (int i = i0; i < i1; ++i) {
                if (whole) enqueue_mm_iteration(h, m, s, i & 1);
                else enqueue_mm_iteration(h, m, s, i & 1, ev[2 * i], ev[2 * i + 1]);
            }
            if (whole) HIPCHK(hipEventRecord(ev[2 * (i0 / kProfGroup) + 1], s));
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s));
        double total = 0.0;
        for (size_t i = 0; i < ev.size(); i += 2) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
            total += ms;
        }
        if (avg_ms) *avg_ms = total / reps;
        if (alg_bytes) *alg_bytes = whole ? 0.0 : spmm;
        destroy();
        return LAP_OK;
    } catch (const HipErr&) {
        destroy();
        return LAP_EDEVICE;
    }
}

// ---------------------------------------------------------------- serving

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct SrvRequest {
    int64_t tag = 0;
    int graph = 0, nrhs = 0;
    double tol = 0.0;
    const double* b = nullptr;      // caller's host buffers
    double* x = nullptr;
    double* db = nullptr;           // device staging: right-hand sides, solutions
    double* dx = nullptr;
    double* pin = nullptr;          // pinned staging (b in, then x out)
    size_t bytes = 0;               // device staging bytes (budget)
    int cols_left = 0;
    int32_t it_max = 0;
    double rel_max = 0.0;
    lap_status status = LAP_OK;
    hipEvent_t done_ev = nullptr;
    double t_submit = 0.0, t_admit = 0.0;
};

struct SrvLane {
    lap_hierarchy* h = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;        // end of the chunk in flight (and its status copy)
    bool busy = false;
    SrvRequest* slot_req[kCols] = {};
    int slot_col[kCols] = {};
    std::deque<SrvRequest*> pending;
    ServeCtl* dctl = nullptr;       // device
    ServeCtl* pctl = nullptr;       // pinned, written only after the previous copy ran
    ScalM* pst = nullptr;           // pinned status copy after each chunk
};

// Pinned host buffers reused by size (page-locking is slow).
struct PinPool {
    std::multimap<size_t, double*> free_;
    double* get(size_t count) {
        auto it = free_.lower_bound(count);
        if (it != free_.end() && it->first <= 2 * count) {
            double* p = it->second;
            free_.erase(it);
            return p;
        }
        void* p = nullptr;
        if (hipHostMalloc(&p, count * sizeof(double), hipHostMallocDefault) != hipSuccess)
            return nullptr;
        sizes_[p] = count;
        return static_cast<double*>(p);
    }
    void put(double* p) { free_.insert({sizes_[p], p}); }
    ~PinPool() {
        for (auto& kv : sizes_) (void)hipHostFree(kv.first);
    }
    std::map<void*, size_t> sizes_;
};

}  // namespace

struct lap_server {
    int device = 0;
    int64_t budget = 0;             // 0: unlimited
    int64_t used = 0;               // resident hierarchies + request staging
    int64_t resident = 0;           // resident hierarchies
    std::vector<SrvLane> lanes;
    std::mutex mu;
    std::condition_variable cv_out;
    std::deque<SrvRequest*> inbox, outbox;
    std::vector<SrvRequest*> copying;
    int64_t inflight = 0;           // submitted and not yet polled out
    std::thread worker;
    std::atomic<bool> stop{false};
    std::atomic<bool> cancel{false};
    std::atomic<bool> failed{false};
    PinPool pins;
};

namespace {

bool lane_active(const SrvLane& L) {
    for (int c = 0; c < kCols; ++c)
        if (L.slot_req[c]) return true;
    return false;
}

// One chunk boundary of a lane: hand out stopped columns, admit queued
// requests, launch the next chunk if any column is running.
void srv_boundary(lap_server* S, SrvLane& L) {
    lap_hierarchy* h = L.h;
    EngineM<double>& m = h->m64;
    const int n = (int)h->n, gn = mm_grid(n);
    const ScalM& st = *L.pst;
    ServeCtl& ctl = *L.pctl;
    std::memset(&ctl, 0, sizeof(ServeCtl));
    bool extract = false, admit = false;
    std::vector<SrvRequest*> touched;
    for (int c = 0; c < kCols; ++c) {
        SrvRequest* r = L.slot_req[c];
        if (!r || st.done[c] == 0) continue;
        const int j = L.slot_col[c];
        ctl.dst[c] = r->dx + (size_t)j * n;
        r->it_max = std::max(r->it_max, st.iter[c]);
        const double rel = st.bn2[c] > 0 ? std::sqrt(st.rr[c] / st.bn2[c]) : 0.0;
        r->rel_max = std::max(r->rel_max, rel);
        const lap_status cs = to_status(st.done[c]);
        if (rank_status(cs) > rank_status(r->status)) r->status = cs;
        L.slot_req[c] = nullptr;
        if (--r->cols_left == 0) touched.push_back(r);
        extract = true;
    }
    // admission: whole requests, first come first served, while slots and
    // the HBM budget allow
    int nfree = 0;
    for (int c = 0; c < kCols; ++c) nfree += L.slot_req[c] == nullptr;
    std::vector<SrvRequest*> admitted;
    while (!L.pending.empty()) {
        SrvRequest* r = L.pending.front();
        if (r->nrhs > nfree) break;
        const size_t bytes = 2 * (size_t)n * r->nrhs * sizeof(double);
        // over budget: wait for running requests to finish (a request that
        // would not fit even alone is admitted once nothing else runs)
        if (S->budget > 0 && S->used + (int64_t)bytes > S->budget && S->used > S->resident)
            break;
        void* db = nullptr;
        if (hipMallocAsync(&db, bytes, L.s) != hipSuccess) break;
        r->db = static_cast<double*>(db);
        r->dx = r->db + (size_t)n * r->nrhs;
        r->bytes = bytes;
        S->used += (int64_t)bytes;
        r->pin = S->pins.get((size_t)n * r->nrhs);
        std::memcpy(r->pin, r->b, (size_t)n * r->nrhs * sizeof(double));
        HIPCHK(hipMemcpyAsync(r->db, r->pin, (size_t)n * r->nrhs * sizeof(double),
                              hipMemcpyHostToDevice, L.s));
        r->t_admit = now_s();
        int j = 0;
        for (int c = 0; c < kCols && j < r->nrhs; ++c) {
            if (L.slot_req[c]) continue;
            L.slot_req[c] = r;
            L.slot_col[c] = j;
            ctl.src[c] = r->db + (size_t)j * n;
            ctl.tol2[c] = r->tol * r->tol;
            ++j;
        }
        r->cols_left = r->nrhs;
        nfree -= r->nrhs;
        L.pending.pop_front();
        admitted.push_back(r);
        admit = true;
    }
    if (extract || admit)
        HIPCHK(hipMemcpyAsync(L.dctl, L.pctl, sizeof(ServeCtl), hipMemcpyHostToDevice, L.s));
    if (extract) {
        hipLaunchKernelGGL(k_srv_xsum<double>, dim3(gn), dim3(kMmWaves * 64), 0, L.s, n,
                           (const double*)m.x, h->partm);
        finish_m<kMmSum>(h, L.s, h->Sm, gn);
        hipLaunchKernelGGL(k_srv_extract<double>, dim3(gn), dim3(kMmWaves * 64), 0, L.s, n,
                           h->sperm, (const ServeCtl*)L.dctl, (const double*)m.x,
                           (const ScalM*)h->Sm);
        for (SrvRequest* r : touched) {
            // every column of r has been extracted: copy out, then done
            HIPCHK(hipMemcpyAsync(r->pin, r->dx, (size_t)n * r->nrhs * sizeof(double),
                                  hipMemcpyDeviceToHost, L.s));
            HIPCHK(hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming));
            HIPCHK(hipEventRecord(r->done_ev, L.s));
            HIPCHK(hipFreeAsync(r->db, L.s));
            S->copying.push_back(r);
        }
    }
    if (admit) {
        hipLaunchKernelGGL(k_srv_colsum, dim3(gn), dim3(kMmWaves * 64), 0, L.s, n,
                           (const ServeCtl*)L.dctl, h->partm);
        finish_m<kMmSum>(h, L.s, h->Sm, gn);
        hipLaunchKernelGGL(k_srv_admit<double>, dim3(gn), dim3(kMmWaves * 64), 0, L.s, n,
                           (const int32_t*)h->perm0, (const ServeCtl*)L.dctl, m.lv[0].r, m.x,
                           m.p[0], m.p[1], (const ScalM*)h->Sm, h->partm);
        finish_m<kMmAdmit>(h, L.s, h->Sm, gn, 0, (const ServeCtl*)L.dctl);
        enqueue_mm_precond(h, m, L.s, 0, (const double*)m.p[0]);
    }
    HIPCHK(hipGetLastError());
    if (lane_active(L)) {
        HIPCHK(hipGraphLaunch(m.exec, L.s));
        HIPCHK(hipMemcpyAsync(L.pst, h->Sm, sizeof(ScalM), hipMemcpyDeviceToHost, L.s));
        HIPCHK(hipEventRecord(L.ev, L.s));
        L.busy = true;
    }
}

void srv_loop(lap_server* S) {
    (void)hipSetDevice(S->device);
    try {
        while (true) {
            bool work = false;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                while (!S->inbox.empty()) {
                    SrvRequest* r = S->inbox.front();
                    S->inbox.pop_front();
                    S->lanes[r->graph].pending.push_back(r);
                }
            }
            for (SrvLane& L : S->lanes) {
                if (L.busy) {
                    work = true;
                    if (hipEventQuery(L.ev) != hipSuccess) continue;
                    L.busy = false;
                }
                if (lane_active(L) || !L.pending.empty()) {
                    work = true;
                    srv_boundary(S, L);
                }
            }
            for (size_t i = 0; i < S->copying.size();) {
                SrvRequest* r = S->copying[i];
                work = true;
                if (hipEventQuery(r->done_ev) != hipSuccess) {
                    ++i;
                    continue;
                }
                const size_t cnt = (size_t)S->lanes[r->graph].h->n * r->nrhs;
                std::memcpy(r->x, r->pin, cnt * sizeof(double));
                S->pins.put(r->pin);
                (void)hipEventDestroy(r->done_ev);
                S->used -= (int64_t)r->bytes;
                S->copying[i] = S->copying.back();
                S->copying.pop_back();
                {
                    std::lock_guard<std::mutex> lk(S->mu);
                    S->outbox.push_back(r);
                }
                S->cv_out.notify_all();
            }
            if (S->cancel.load()) {
                // drop what has not started; let chunks and copies in flight
                // finish, then retire their requests without results
                bool inflight = !S->copying.empty();
                for (SrvLane& L : S->lanes) {
                    for (SrvRequest* r : L.pending) delete r;
                    L.pending.clear();
                    if (L.busy) {
                        if (hipEventQuery(L.ev) != hipSuccess) {
                            inflight = true;
                            continue;
                        }
                        L.busy = false;
                    }
                    for (int c = 0; c < kCols; ++c) {
                        SrvRequest* r = L.slot_req[c];
                        if (!r) continue;
                        for (int d = c; d < kCols; ++d)
                            if (L.slot_req[d] == r) L.slot_req[d] = nullptr;
                        (void)hipFreeAsync(r->db, L.s);
                        S->pins.put(r->pin);
                        delete r;
                    }
                }
                if (!inflight) break;
                std::this_thread::sleep_for(std::chrono::microseconds(50));
                continue;
            }
            if (!work) {
                if (S->stop.load()) {
                    std::lock_guard<std::mutex> lk(S->mu);
                    if (S->inbox.empty()) break;
                    continue;
                }
                std::this_thread::sleep_for(std::chrono::microseconds(50));
            } else {
                std::this_thread::yield();
            }
        }
    } catch (const HipErr&) {
        S->failed.store(true);
        S->cv_out.notify_all();
    }
}

// y = L x in the caller's order.  When the solve order differs from the
// input order (sperm), x is gathered into w0 in solve order, the product
// goes to w1 and is scattered back: w0 and w1 are n-vector work buffers.
lap_status apply_laplacian(lap_hierarchy* h, const double* x, double* y, double* w0, double* w1,
                           hipStream_t s) {
    const Engine<double>& e = h->e64;
    const int n = (int)h->n;
    if (h->sperm) {
        hipLaunchKernelGGL(k_gather<double>, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->sperm, x,
                           w0);
        hipLaunchKernelGGL(k_spmv_plain, dim3(e.spmv_grid()), dim3(kBlock), 0, s, e.nlb, e.A,
                           (const double*)w0, w1);
        hipLaunchKernelGGL(k_shift_out<double>, dim3(nblk(n)), dim3(kBlock), 0, s, n, h->sperm,
                           (const double*)w1, y, (const Scal*)nullptr);
    } else {
        hipLaunchKernelGGL(k_spmv_plain, dim3(e.spmv_grid()), dim3(kBlock), 0, s, e.nlb, e.A, x,
                           y);
    }
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) {
        record_error("k_spmv_plain launch", err, __LINE__);
        return LAP_EDEVICE;
    }
    return LAP_OK;
}

// Device address of this device's copy of `scratch`, taken once per device
// with that device current (the array's name is only a host-side stand-in)
// and kept for the life of the process.
lap_status noalloc_scratch(int dev, double** out) {
    static std::mutex mu;
    static void* ptr[kNoallocMaxDevices] = {};
    if (dev < 0 || dev >= kNoallocMaxDevices) {
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "lap_apply_laplacian_noalloc: device %d beyond the %d supported", dev,
                      kNoallocMaxDevices);
        return LAP_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            record_error("hipGetSymbolAddress(scratch)", e, __LINE__);
            return LAP_EDEVICE;
        }
        ptr[dev] = p;
    }
    *out = static_cast<double*>(ptr[dev]);
    return LAP_OK;
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
    p->offtree_frac = 0.1;
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

lap_status lap_set_allocator(lap_alloc_fn alloc, lap_free_fn free_fn, void* ctx) {
    if ((alloc == nullptr) != (free_fn == nullptr)) return LAP_EINVAL;
    std::lock_guard<std::mutex> lock(g_alloc_mu);
    g_alloc.alloc = alloc;
    g_alloc.free = free_fn;
    g_alloc.ctx = alloc ? ctx : nullptr;
    return LAP_OK;
}

lap_status lap_setup(const lap_graph* g, const lap_params* p, void* stream, lap_hierarchy** out) {
    if (!out) return LAP_EINVAL;
    *out = nullptr;
    if (!g || !p || !g->u || !g->v || !g->w) return LAP_EINVAL;
    if (p->precond != LAP_PREC_MSP && p->precond != LAP_PREC_NONE &&
        p->precond != LAP_PREC_PEGP && p->precond != LAP_PREC_OFFTREE &&
        p->precond != LAP_PREC_SPANNING)
        return LAP_EINVAL;
    if (p->precision != LAP_FP64 && p->precision != LAP_MIXED_FP32_FP64) return LAP_EINVAL;
    // PEGP: FP64 single solves only
    const bool offtree = p->precond == LAP_PREC_OFFTREE || p->precond == LAP_PREC_SPANNING;
    const bool pegp_like = p->precond == LAP_PREC_PEGP || offtree;
    if (offtree && !(p->offtree_frac >= 0.0 && p->offtree_frac <= 1.0)) return LAP_EINVAL;
    if (pegp_like &&
        (p->precision != LAP_FP64 || (p->flags & LAP_FLAG_MULTI_RHS)))
        return LAP_EUNSUPPORTED;
    if (p->max_iter < 0) return LAP_EINVAL;
    const auto t0 = std::chrono::steady_clock::now();
    lap_hierarchy* h = new (std::nothrow) lap_hierarchy();
    if (!h) return LAP_ENOMEM;
    h->params = *p;
    h->host_only = (p->flags & LAP_FLAG_HOST_ONLY) != 0;
    {
        std::lock_guard<std::mutex> lock(g_alloc_mu);
        h->allocator = g_alloc;
    }
    try {
        // only the MSP solves the top level on chip (a dense pseudo-inverse)
        const bool any_top = h->host_only || p->precond != LAP_PREC_MSP;
        const bool dev_setup = (p->flags & LAP_FLAG_DEVICE_SETUP) && !h->host_only;
        if (dev_setup) {
            int ndev = 0;
            if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
                std::snprintf(g_last_error, sizeof(g_last_error), "no HIP device visible");
                delete h;
                return LAP_EDEVICE;
            }
        }
        DeviceGraphBuilder dgb((hipStream_t)stream);
        const int rc = build_plan(g->n, g->m, g->u, g->v, g->w, p->mu, p->max_levels, p->n_top,
                                  p->mwm_seed, any_top, h->plan, dev_setup ? &dgb : nullptr,
                                  (p->flags & LAP_FLAG_PARALLEL_MATCHING) ? 1 : 0);
        if (rc != kOk) {
            delete h;
            return (lap_status)rc;
        }
        h->n = g->n;
        if (pegp_like) {
            int64_t nt = 0;
            for (int k = 0; k < h->plan.nlev(); ++k) nt += h->plan.lv[k].g.n;
            if (nt > kPegpMaxNodes || h->plan.nlev() > kPegpMaxLevels) {
                delete h;
                return LAP_EUNSUPPORTED;
            }
            const int prc =
                build_pegp(h->plan, p->mu, h->pegp_plan, offtree ? p->offtree_frac : -1.0,
                           p->precond == LAP_PREC_SPANNING ? 1 : 0);
            if (prc != kOk) {
                delete h;
                return (lap_status)prc;
            }
        }
        if (!h->host_only) {
            int ndev = 0;
            if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
                std::snprintf(g_last_error, sizeof(g_last_error), "no HIP device visible");
                delete h;
                return LAP_EDEVICE;
            }
            HIPCHK(hipGetDevice(&h->device));
            upload_plan(h, (hipStream_t)stream);
            if (p->flags & LAP_FLAG_MULTI_RHS) setup_block(h, (hipStream_t)stream);
        }
    } catch (const std::bad_alloc&) {
        delete h;
        return LAP_ENOMEM;
    } catch (const HipErr&) {
        delete h;
        return LAP_EDEVICE;
    } catch (const std::invalid_argument& ex) {
        std::snprintf(g_last_error, sizeof(g_last_error), "%s", ex.what());
        delete h;
        return LAP_EINVAL;
    } catch (const std::exception& ex) {
        std::snprintf(g_last_error, sizeof(g_last_error), "%s", ex.what());
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
        if (nrhs > 1 && h->has_block) {
            for (int c0 = 0; c0 < nrhs; c0 += kCols) {
                const int nb = std::min(kCols, nrhs - c0);
                const lap_status st = solve_block(h, b + (int64_t)c0 * ld, x + (int64_t)c0 * ld,
                                                  nb, ld, tol, info ? info + c0 : nullptr,
                                                  (hipStream_t)stream);
                if (rank_status(st) > rank_status(worst)) worst = st;
            }
            return worst;
        }
        const bool fgmres = (h->params.flags & LAP_FLAG_FGMRES) != 0;
        if (fgmres && h->mixed) return LAP_EUNSUPPORTED;
        for (int c = 0; c < nrhs; ++c) {
            const double* bc = b + (int64_t)c * ld;
            double* xc = x + (int64_t)c * ld;
            lap_solve_info* ic = info ? info + c : nullptr;
            const lap_status st =
                fgmres ? solve_fgmres(h, bc, xc, tol, ic, (hipStream_t)stream)
                : !h->mixed ? solve_fp64(h, bc, xc, tol, ic, (hipStream_t)stream)
                : h->reliable ? solve_mixed_reliable(h, bc, xc, tol, ic, (hipStream_t)stream)
                              : solve_mixed(h, bc, xc, tol, ic, (hipStream_t)stream);
            if (rank_status(st) > rank_status(worst)) worst = st;
        }
    } catch (const HipErr&) {
        return LAP_EDEVICE;
    }
    return worst;
}

lap_status lap_set_precision(lap_hierarchy* h, int32_t precision) {
    if (!h) return LAP_EINVAL;
    if (precision != LAP_FP64 && precision != LAP_MIXED_FP32_FP64) return LAP_EINVAL;
    if (h->host_only) return LAP_EUNSUPPORTED;
    if (precision == LAP_MIXED_FP32_FP64 && !h->has_fp32) return LAP_EUNSUPPORTED;
    h->mixed = precision == LAP_MIXED_FP32_FP64;
    return LAP_OK;
}

lap_status lap_apply_laplacian(lap_hierarchy* h, const double* x, double* y, void* stream) {
    if (!h || !x || !y) return LAP_EINVAL;
    if (h->host_only) return LAP_EUNSUPPORTED;
    // the permuted copies go through two FP64 work vectors of the hierarchy
    return apply_laplacian(h, x, y, h->xc, h->bh, (hipStream_t)stream);
}

lap_status lap_apply_laplacian_noalloc(lap_hierarchy* h, const double* x, double* y,
                                       void* stream) {
    if (!h || !x || !y) return LAP_EINVAL;
    if (h->host_only) return LAP_EUNSUPPORTED;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return LAP_EDEVICE;
    if (dev != h->device) {
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "lap_apply_laplacian_noalloc: current device %d, hierarchy on device %d",
                      dev, h->device);
        return LAP_EINVAL;
    }
    if (!h->sperm) return apply_laplacian(h, x, y, nullptr, nullptr, (hipStream_t)stream);
    const size_t need = 2 * sizeof(double) * (size_t)h->n;
    if (need > kNoallocScratchBytes) {
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "lap_apply_laplacian_noalloc: n = %lld needs %zu bytes of scratch, the "
                      "maximum is %zu (n <= %zu for this graph)",
                      (long long)h->n, need, kNoallocScratchBytes,
                      kNoallocScratchBytes / (2 * sizeof(double)));
        return LAP_EUNSUPPORTED;
    }
    double* scr = nullptr;
    const lap_status st = noalloc_scratch(dev, &scr);
    if (st != LAP_OK) return st;
    return apply_laplacian(h, x, y, scr, scr + h->n, (hipStream_t)stream);
}

lap_status lap_apply_precond(lap_hierarchy* h, const double* r, double* z, void* stream) {
    if (!h || !r || !z) return LAP_EINVAL;
    if (h->host_only) return LAP_EUNSUPPORTED;
    try {
        if (h->mixed) apply_precond(h, h->e32, r, z, (hipStream_t)stream);
        else apply_precond(h, h->e64, r, z, (hipStream_t)stream);
    } catch (const HipErr&) {
        return LAP_EDEVICE;
    }
    return LAP_OK;
}

lap_status lap_profile_kernel(lap_hierarchy* h, int32_t kernel, int32_t reps, void* stream,
                              double* avg_ms, double* alg_bytes) {
    if (!h || reps < 1 || kernel < 0 || kernel > LAP_KERNEL_PEGP_OP) return LAP_EINVAL;
    if (h->host_only) return LAP_EUNSUPPORTED;
    if (kernel == LAP_KERNEL_BLOCK_SPMM || kernel == LAP_KERNEL_BLOCK_ITER) {
        if (!h->has_block) return LAP_EUNSUPPORTED;
        return h->mixed ? profile_block(h, h->m32, kernel, reps, (hipStream_t)stream, avg_ms,
                                        alg_bytes)
                        : profile_block(h, h->m64, kernel, reps, (hipStream_t)stream, avg_ms,
                                        alg_bytes);
    }
    return h->mixed ? profile(h, h->e32, kernel, reps, (hipStream_t)stream, avg_ms, alg_bytes)
                    : profile(h, h->e64, kernel, reps, (hipStream_t)stream, avg_ms, alg_bytes);
}

lap_status lap_hierarchy_info(const lap_hierarchy* h, lap_hierarchy_desc* d) {
    if (!h || !d) return LAP_EINVAL;
    std::memset(d, 0, sizeof(*d));
    d->nlev = h->plan.nlev();
    d->tail_level = h->mixed ? h->e32.kt : h->e64.kt;
    for (int k = 0; k < d->nlev && k < LAP_MAX_LEVELS; ++k) {
        d->sizes[k] = h->plan.lv[k].g.n;
        d->ntilde += d->sizes[k];
    }
    d->nnz = h->plan.lv[0].g.nnz();
    d->device_bytes = h->dev_bytes;
    d->setup_seconds = h->setup_seconds;
    d->spmv_fused = h->fuse_p ? 1 : 0;
    d->pegp_operator_n = h->pegp ? h->pegp_dev.opn : 0;
    if (h->has_block) {
        d->mm_chunk[0] = h->m64.chunk;
        d->mm_grid[0] = h->m64.grid;
        d->mm_seg[0] = h->m64.seg;
        if (h->m32.on) {
            d->mm_chunk[1] = h->m32.chunk;
            d->mm_grid[1] = h->m32.grid;
            d->mm_seg[1] = h->m32.seg;
        }
        d->mm_tune_seconds = h->mm_tune_seconds;
    }
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

lap_status lap_export_offtree(const lap_hierarchy* h, int64_t* count, int64_t* a, int64_t* b,
                              double* w, double* stretch, int8_t* kept) {
    if (!h || !count ||
        (h->params.precond != LAP_PREC_OFFTREE && h->params.precond != LAP_PREC_SPANNING))
        return LAP_EINVAL;
    const PegpPlan& G = h->pegp_plan;
    const size_t c = G.ot_a.size();
    *count = (int64_t)c;
    if (a) std::memcpy(a, G.ot_a.data(), c * sizeof(int64_t));
    if (b) std::memcpy(b, G.ot_b.data(), c * sizeof(int64_t));
    if (w) std::memcpy(w, G.ot_w.data(), c * sizeof(double));
    if (stretch) std::memcpy(stretch, G.ot_stretch.data(), c * sizeof(double));
    if (kept) std::memcpy(kept, G.ot_kept.data(), c);
    return LAP_OK;
}

lap_status lap_server_create(int64_t hbm_budget_bytes, lap_server** out) {
    if (!out || hbm_budget_bytes < 0) return LAP_EINVAL;
    *out = nullptr;
    lap_server* S = new (std::nothrow) lap_server();
    if (!S) return LAP_ENOMEM;
    S->budget = hbm_budget_bytes;
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return LAP_EDEVICE;
    }
    *out = S;
    return LAP_OK;
}

lap_status lap_server_add(lap_server* S, lap_hierarchy* h, int32_t* graph_id) {
    if (!S || !h || !graph_id) return LAP_EINVAL;
    if (h->host_only || !h->has_block) return LAP_EUNSUPPORTED;
    if (S->worker.joinable()) return LAP_EINVAL;        // before the first submit only
    if (S->budget > 0 && S->used + h->dev_bytes > S->budget) return LAP_ENOMEM;
    SrvLane L;
    L.h = h;
    try {
        HIPCHK(hipStreamCreateWithFlags(&L.s, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&L.ev, hipEventDisableTiming));
        L.dctl = h->dalloc<ServeCtl>(1);
        HIPCHK(hipHostMalloc((void**)&L.pctl, sizeof(ServeCtl), hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void**)&L.pst, sizeof(ScalM), hipHostMallocDefault));
        std::memset(L.pctl, 0, sizeof(ServeCtl));
        std::memset(L.pst, 0, sizeof(ScalM));
        // all slots idle: a ScalM with every column stopped
        ScalM& st = *h->stagem;
        std::memset(&st, 0, sizeof(ScalM));
        for (int c = 0; c < kCols; ++c) st.done[c] = 5;
        st.maxit = h->params.max_iter;
        st.all_done = 1;
        HIPCHK(hipMemcpyAsync(h->Sm, &st, sizeof(ScalM), hipMemcpyHostToDevice, L.s));
        HIPCHK(hipStreamSynchronize(L.s));
    } catch (const std::bad_alloc&) {
        return LAP_ENOMEM;
    } catch (const HipErr&) {
        return LAP_EDEVICE;
    }
    S->used += h->dev_bytes;
    S->resident += h->dev_bytes;
    *graph_id = (int32_t)S->lanes.size();
    S->lanes.push_back(L);
    return LAP_OK;
}

lap_status lap_server_submit(lap_server* S, int32_t graph, const double* b, double* x,
                             int32_t nrhs, double tol, int64_t tag) {
    if (!S || !b || !x || graph < 0 || graph >= (int32_t)S->lanes.size() || nrhs < 1 ||
        nrhs > kCols || !(tol > 0.0) || !std::isfinite(tol))
        return LAP_EINVAL;
    if (S->failed.load()) return LAP_EDEVICE;
    SrvRequest* r = new (std::nothrow) SrvRequest();
    if (!r) return LAP_ENOMEM;
    r->tag = tag;
    r->graph = graph;
    r->nrhs = nrhs;
    r->tol = tol;
    r->b = b;
    r->x = x;
    r->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->inbox.push_back(r);
        ++S->inflight;
        if (!S->worker.joinable()) S->worker = std::thread(srv_loop, S);
    }
    return LAP_OK;
}

lap_status lap_server_poll(lap_server* S, lap_request_result* out, int32_t max, int32_t wait_ms,
                           int32_t* count) {
    if (!S || !count || max < 0 || (max > 0 && !out)) return LAP_EINVAL;
    *count = 0;
    std::unique_lock<std::mutex> lk(S->mu);
    if (wait_ms > 0 && S->outbox.empty())
        S->cv_out.wait_for(lk, std::chrono::milliseconds(wait_ms),
                           [&] { return !S->outbox.empty() || S->failed.load(); });
    if (S->failed.load() && S->outbox.empty()) return LAP_EDEVICE;
    int32_t k = 0;
    while (k < max && !S->outbox.empty()) {
        SrvRequest* r = S->outbox.front();
        S->outbox.pop_front();
        lap_request_result& o = out[k++];
        o.tag = r->tag;
        o.graph = r->graph;
        o.nrhs = r->nrhs;
        o.status = r->status;
        o.iterations_max = r->it_max;
        o.relres_max = r->rel_max;
        o.queue_seconds = r->t_admit - r->t_submit;
        o.total_seconds = now_s() - r->t_submit;
        --S->inflight;
        delete r;
    }
    *count = k;
    return LAP_OK;
}

void lap_server_destroy(lap_server* S) {
    if (!S) return;
    S->stop.store(true);
    S->cancel.store(true);
    if (S->worker.joinable()) S->worker.join();
    for (SrvLane& L : S->lanes) {
        if (L.s) {
            (void)hipStreamSynchronize(L.s);
            (void)hipStreamDestroy(L.s);
        }
        if (L.ev) (void)hipEventDestroy(L.ev);
        if (L.pctl) (void)hipHostFree(L.pctl);
        if (L.pst) (void)hipHostFree(L.pst);
        for (SrvRequest* r : L.pending) delete r;
    }
    for (SrvRequest* r : S->outbox) delete r;
    delete S;
}

lap_status lap_estimate_spectrum(lap_hierarchy* h, const double* b, int32_t steps, double* lmin,
                                 double* lmax, int32_t* taken, void* stream) {
    if (!h || !b || !lmin || !lmax || steps < 1) return LAP_EINVAL;
    if (h->host_only || (!h->with_msp && !h->pegp)) return LAP_EUNSUPPORTED;
    try {
        std::vector<double> alpha, beta;
        const Scal R = pcg_coefficients(h, b, steps, alpha, beta, (hipStream_t)stream);
        if (R.done == 4) return LAP_EINVAL;
        if (taken) *taken = (int32_t)alpha.size();
        if (alpha.empty()) return LAP_EBREAKDOWN;
        const size_t k = alpha.size();
        std::vector<double> d(k), e(k > 0 ? k - 1 : 0);
        for (size_t j = 0; j < k; ++j) {
            d[j] = 1.0 / alpha[j] + (j > 0 ? beta[j - 1] / alpha[j - 1] : 0.0);
            if (j + 1 < k) e[j] = std::sqrt(beta[j]) / alpha[j];
        }
        *lmin = tridiag_eig(d, e, 0);
        *lmax = tridiag_eig(d, e, (int)k - 1);
    } catch (const HipErr&) {
        return LAP_EDEVICE;
    }
    return LAP_OK;
}

lap_status lap_select_mu(const lap_graph* g, const lap_params* p, const double* mus, int32_t nmu,
                         const double* b, int32_t steps, double* kappa, int32_t* best,
                         void* stream) {
    if (!g || !p || !mus || !b || !best || nmu < 1 || steps < 1) return LAP_EINVAL;
    lap_status first_err = LAP_OK;
    double best_k = HUGE_VAL;
    *best = -1;
    for (int32_t i = 0; i < nmu; ++i) {
        lap_params q = *p;
        q.mu = mus[i];
        lap_hierarchy* h = nullptr;
        double k = HUGE_VAL;
        lap_status st = lap_setup(g, &q, stream, &h);
        if (st == LAP_OK) {
            double lo = 0.0, hi = 0.0;
            st = lap_estimate_spectrum(h, b, steps, &lo, &hi, nullptr, stream);
            if (st == LAP_OK && lo > 0.0) k = hi / lo;
            lap_free(h);
        }
        if (st != LAP_OK && first_err == LAP_OK) first_err = st;
        if (kappa) kappa[i] = k;
        if (k < best_k) {
            best_k = k;
            *best = i;
        }
    }
    return *best >= 0 ? LAP_OK : first_err;
}

void lap_free(lap_hierarchy* h) { delete h; }

const char* lap_last_error(void) { return g_last_error; }

}  // extern "C"
