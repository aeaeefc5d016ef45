// Host-side setup of the MSP hierarchy (Hu & Lin, arXiv 2207.07847).
//
// Builds, on the CPU, everything the device solve reads:
//   * the aggregation hierarchy by maximal weighted matching (Sec. 2.2) and
//     the coarse graphs P^T L P;
//   * a renumbering of every level in which the children of each aggregate
//     are contiguous (matched pair first), so restriction and prolongation
//     are segmented sums and broadcasts over ranges;
//   * the closed-form coefficients of the MSP solve (Sec. 3.3): per
//     aggregate the inverse of the 2x2 Schur complement of its sparsifier
//     block, per leftover member its elimination coefficients, per level the
//     weight theta_j, and the pseudo-inverse of the top-level Laplacian;
//   * the fine Laplacian in sliced-ELL form in the graph's own order.
#pragma once

#include <cstdint>
#include <vector>

namespace lapgpu {

enum Status { kOk = 0, kInval = 1, kDisconnected = 2, kNoMem = 3, kDevice = 4,
              kNoConv = 5, kBreakdown = 6, kUnsupported = 7 };

constexpr int kSlice = 64;        // rows per sliced-ELL slice (one wave)
constexpr int kTopMax = 64;       // largest top level solved on chip
constexpr int kHeavyDeg = 64;     // rows of higher degree leave the slices
constexpr int kHeavyBlockDeg = 4096;  // ... and above this get a block alone
constexpr int kSigma = 65536;     // rows sorted by degree within windows of this
constexpr int kHeavyWaves = 4;    // heavy rows per heavy block (one per wave)

// Symmetric weighted adjacency, neighbours ascending, no diagonal.
struct Adjacency {
    int64_t n = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> col;
    std::vector<double> w;
    int64_t nnz() const { return ptr.empty() ? 0 : ptr.back(); }
};

struct Level {
    Adjacency g;                   // graph of this level, own numbering
    std::vector<int64_t> agg;      // node -> aggregate (next level); empty on top
    std::vector<int8_t> matched;   // 1: paired by the matching, 0: leftover
};

// Per aggregation step k (level k -> level k+1), in tree numbering.
struct StepCoef {
    std::vector<int32_t> cptr;               // children of aggregate J: [cptr[J], cptr[J+1])
    std::vector<double> saa, sab, sbb;       // theta_k * inverse Schur complement (pair)
    std::vector<double> l0, l1, l2;          // leftover t: theta_k/D_tt, w_ta/D_tt, w_tb/D_tt
};

struct HostPlan {
    double mu = 0.8;
    std::vector<Level> lv;                   // original numbering per level
    std::vector<std::vector<int32_t>> perm;  // perm[k][tree id] = level-k id
    std::vector<std::vector<int32_t>> inv;   // inv[k][level-k id] = tree id
    std::vector<StepCoef> step;              // nlev-1 entries
    std::vector<double> theta;               // theta_k, k = 0..nlev-1
    std::vector<double> top_pinv;            // theta_top * pinv(L_top), row-major
    // fine Laplacian for the SpMV, in the solve order: the graph's own order
    // (spmv_tree false) or the tree order of level 0 (spmv_tree true; then
    // solve position t is input vertex perm[0][t]).  Light rows in sliced
    // ELL (64 rows per slice, column-major), heavy rows in CSR.
    bool spmv_tree = false;
    Adjacency solve_g;                       // the graph in tree order (spmv_tree)
    const Adjacency& solve_graph() const { return spmv_tree ? solve_g : lv[0].g; }
    int32_t sell_nlight = 0;
    std::vector<int32_t> sell_off;           // slice -> first slot
    std::vector<int32_t> sell_width;         // slice -> slots per row
    std::vector<int32_t> sell_col;
    std::vector<double> sell_w;
    std::vector<int32_t> sell_row;           // slot -> row; empty: identity
    std::vector<int32_t> heavy_blk;          // heavy block -> first heavy row
    std::vector<int32_t> heavy_row;          // heavy row -> row
    std::vector<int32_t> heavy_ptr;
    std::vector<int32_t> heavy_col;
    std::vector<double> heavy_w;
    int nlev() const { return (int)lv.size(); }
};

// PEGP (Sec. 3.1-3.2) as the factored grounded system S = D L_H~ D, D =
// diag(mu^-k) on level k, over the expanded nodes in tree numbering (node t
// of level k has expanded index off[k] + t).  L_H~ keeps the negative
// off-diagonal entries of L_G~ = P(mu)^T L_G P(mu), whose magnitudes are
// mu^(k+l) w_AB: w_AB = total fine weight between disjoint aggregates A, B
// (kept when k + l is even) or, for B inside A, the weight from B to
// outside A (kept when k + l is odd); so S(A,B) = -w_AB and S(A,A) =
// sum_B mu^(l-k) w_AB.  The last expanded node is grounded; the rest is
// factored S = L diag(d) L^T in a minimum-degree order, and both
// triangular solves are level-scheduled.
struct PegpPlan {
    int32_t nt = 0;                          // expanded nodes
    int32_t ground = 0;                      // grounded expanded node
    std::vector<int32_t> off;                // level -> first expanded index (nlev+1)
    std::vector<double> diag;                // d of each expanded node (ground: 1)
    // forward: levels of rows, row v = sum over earlier-eliminated u of l_vu
    std::vector<int32_t> flev, frow, fptr, fcol;
    std::vector<double> fval;
    // backward: levels of nodes, node v = sum over later-eliminated u of l_uv
    std::vector<int32_t> blev, brow, bptr, bcol;
    std::vector<double> bval;
    int64_t nnz_s = 0, nnz_l = 0;            // off-diagonals of S (both halves), of L
    // Dense tail: the trailing forward levels of at most kPegpTailWidth rows
    // (the nearly dense last-eliminated block of the minimum-degree order),
    // solved by dense blocked substitution over the whole device.  No other
    // row depends on the tail in the forward pass, and the tail depends on no
    // other row in the backward pass; the level lists above leave it out.
    int32_t nd = 0;                          // tail rows (0: none)
    int32_t ndp = 0;                         // nd rounded up to a multiple of kPegpTailBlock
    std::vector<int32_t> drow;               // tail position -> expanded node
    // ndp x ndp strict lower L_tt, row- and column-major, and the diagonal
    // of the tail by position; the padding rows and columns are 0 (diagonal
    // 1), so every block of the dense solve is whole and solves to 0 there
    std::vector<double> dlr, dlc, dd;
    // Coupling of the tail with the other nodes: forward, the tail rows'
    // entries on the other nodes (CSR by tail position, columns are nodes);
    // backward, the other rows' entries on the tail (rows bcrow, columns are
    // tail positions).  The backward level lists hold only the other rows'
    // entries on each other.
    std::vector<int32_t> dcptr, dccol;
    std::vector<double> dcval;
    std::vector<int32_t> bcrow, bcptr, bccol;
    std::vector<double> bcval;
    // log2 of the lanes that share a row, per forward / backward level
    std::vector<int32_t> flg, blg;
    // The levels packed for the solve: per level a descriptor of
    // kPegpDescInts ints {base, NT | g << 12 | U << 16, P | nr << 16, r0}:
    // 2^g lanes per row, the rows [r0, r0 + nr) of the level list dealt to P
    // passes of NT threads, U entries per thread and pass; the entry of pass
    // p, round u, thread t at base + (p U + u) NT + t, its column as the
    // node's byte offset in a vector of doubles, node * 8 (padding: value 0
    // on node 0).  A thread's entries are found from the descriptor alone, so a
    // level's loads can be issued before the previous level is done.
    std::vector<int32_t> fdesc, bdesc, fpcol, bpcol;
    std::vector<double> fpval, bpval;
    // The explicit operator M = P(mu) L_H~^+ P(mu)^T on mean-free vectors
    // of the fine level (tree order), formed column by column through the
    // factor: op[i * opld + j] = (M (e_j - 1/n))_i - mean, opld = n rounded
    // up to a multiple of kPegpOpAlign (padding 0).  Empty when n exceeds
    // kPegpOpMax or the operator is switched off.
    int32_t opn = 0, opld = 0;
    std::vector<double> op;
    // Off-tree sparsifier (build_pegp with offtree_frac >= 0): the positive
    // edges of H~ outside the tree (T~ or the spanning tree), each with its expanded ends in
    // the levels' own numbering (level offset + node id), weight (of H~),
    // stretch in T~ and whether it was added back.
    std::vector<int64_t> ot_a, ot_b;
    std::vector<double> ot_w, ot_stretch;
    std::vector<int8_t> ot_kept;
};
constexpr int kPegpSolveThreads = 1024;      // threads of the PEGP solve workgroup
constexpr int kPegpDescInts = 4;
constexpr int kPegpTailWidth = 24;
constexpr int kPegpOpMax = 8192;             // largest fine level applied as an explicit operator
constexpr int kPegpOpAlign = 128;            // row length of the operator: whole wavefront loads
constexpr int kPegpTailBlock = 192;           // rows per kernel (superblock) of the dense tail solve
constexpr int kPegpMinDense = 64;
constexpr int kPegpMaxDense = 4096;
// The factored grounded system of PEGP (offtree_frac < 0: all of H~), or,
// with 0 <= offtree_frac <= 1, of a tree plus the ceil(frac * count)
// off-tree edges of H~ of largest stretch in it (Sec. 3.3): the MSP tree T~
// (tree 0) or a maximum-weight spanning tree of H~ (tree 1).
int build_pegp(const HostPlan& plan, double mu, PegpPlan& out, double offtree_frac = -1.0,
               int tree = 0);

int build_adjacency(int64_t n, int64_t m, const int64_t* u, const int64_t* v,
                    const double* w, Adjacency& out);
bool is_connected(const Adjacency& g);
int64_t match_aggregate(const Adjacency& g, const std::vector<int64_t>* order,
                        std::vector<int64_t>& agg, std::vector<int8_t>& matched);
void coarse_graph(const Adjacency& f, const std::vector<int64_t>& agg, int64_t nc,
                  Adjacency& c);
// Full host setup; returns a Status.  any_top allows top levels larger
// than kTopMax (no on-chip dense top solve: host-only setups, PEGP, plain
// CG); their top pseudo-inverse is then not formed.
// Graph construction done elsewhere (on the device): the same outputs as
// build_adjacency (after validate_edges) and coarse_graph, bit for bit.
struct GraphBuilder {
    virtual int adjacency(int64_t n, int64_t m, const int64_t* u, const int64_t* v,
                          const double* w, Adjacency& out) = 0;
    virtual void coarse(const Adjacency& f, const std::vector<int64_t>& agg, int64_t nc,
                        Adjacency& c) = 0;
    // The locally dominant matching of match_locally_dominant, bit for bit;
    // false: not available here (the host computes it).
    virtual bool match(const Adjacency& g, std::vector<int64_t>& agg,
                       std::vector<int8_t>& matched, int64_t& nc) {
        (void)g; (void)agg; (void)matched; (void)nc;
        return false;
    }
    virtual ~GraphBuilder() = default;
};
// matching: 0 the visit-order matching of Sec. 2.2 (seed: the order), 1 the
// locally dominant (greedy) matching of a parallel setup.
int build_plan(int64_t n, int64_t m, const int64_t* u, const int64_t* v,
               const double* w, double mu, int max_levels, int64_t n_top,
               uint64_t seed, bool any_top, HostPlan& plan, GraphBuilder* gb = nullptr,
               int matching = 0);
int64_t match_locally_dominant(const Adjacency& g, std::vector<int64_t>& agg,
                               std::vector<int8_t>& matched);
// kOk when the edge list is a valid input: n >= 2, 0 <= u, v < n, u != v,
// w > 0 finite; kInval otherwise.
int validate_edges(int64_t n, int64_t m, const int64_t* u, const int64_t* v, const double* w);
// The SpMV layout of the fine Laplacian g (part of build_plan).
void build_sell(const Adjacency& g, HostPlan& plan);
// Whether g is mesh-like for the SpMV: no row above kHeavyDeg and slices of
// consecutive rows padded by at most 15 %.
bool mesh_like(const Adjacency& g);
// The hot columns of the SpMV matrix: the `count` columns referenced most
// often (ties to the smaller column), hot[k] = column of rank k, and copies
// of the matrix's column arrays in which every reference to a hot column c
// reads ~rank(c) (negative), so a kernel can gather those values from a
// compact copy of the vector.  Padding slots keep their own row.
void hot_columns(const HostPlan& plan, int64_t n, int64_t count, std::vector<int32_t>& hot,
                 std::vector<int32_t>& sell_col, std::vector<int32_t>& heavy_col);
// g renumbered: new id of old vertex i is inv[i], rows ascending.
void permute_graph(const Adjacency& g, const std::vector<int32_t>& perm,
                   const std::vector<int32_t>& inv, Adjacency& out);

}  // namespace lapgpu
