// Host-side setup of the MSP hierarchy; see setup.hpp.
#include "setup.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <atomic>
#include <thread>
#include <unordered_map>

namespace lapgpu {

// ---------------------------------------------------------------- graph

// Sec. 2.1: undirected, positively weighted.  Rows are filled by a
// counting pass, then each row is ordered by (neighbour, edge position) and
// parallel edges merged in edge-position order (same order in both rows, so
// the merged weights are exactly symmetric).
int validate_edges(int64_t n, int64_t m, const int64_t* u, const int64_t* v, const double* w) {
    if (n < 2 || m < 1 || n > INT32_MAX - 1) return kInval;
    for (int64_t e = 0; e < m; ++e) {
        if (u[e] < 0 || u[e] >= n || v[e] < 0 || v[e] >= n || u[e] == v[e]) return kInval;
        if (!(w[e] > 0.0) || !std::isfinite(w[e])) return kInval;
    }
    return kOk;
}

int build_adjacency(int64_t n, int64_t m, const int64_t* u, const int64_t* v,
                    const double* w, Adjacency& out) {
    if (validate_edges(n, m, u, v, w) != kOk) return kInval;
    std::vector<int64_t> start(n + 1, 0);
    for (int64_t e = 0; e < m; ++e) { ++start[u[e] + 1]; ++start[v[e] + 1]; }
    for (int64_t i = 0; i < n; ++i) start[i + 1] += start[i];
    std::vector<std::pair<int32_t, int64_t>> slot(2 * m);   // (neighbour, edge)
    std::vector<int64_t> fillp(start.begin(), start.end() - 1);
    for (int64_t e = 0; e < m; ++e) {
        slot[fillp[u[e]]++] = {(int32_t)v[e], e};
        slot[fillp[v[e]]++] = {(int32_t)u[e], e};
    }
    out.n = n;
    out.ptr.assign(n + 1, 0);
    out.col.clear();
    out.w.clear();
    out.col.reserve(2 * m);
    out.w.reserve(2 * m);
    for (int64_t i = 0; i < n; ++i) {
        auto b = slot.begin() + start[i], e = slot.begin() + start[i + 1];
        std::sort(b, e);
        for (auto it = b; it != e; ++it) {
            if (it != b && it->first == (it - 1)->first) {
                out.w.back() += w[it->second];
            } else {
                out.col.push_back(it->first);
                out.w.push_back(w[it->second]);
            }
        }
        out.ptr[i + 1] = (int64_t)out.col.size();
    }
    return kOk;
}

bool is_connected(const Adjacency& g) {
    std::vector<char> seen(g.n, 0);
    std::vector<int32_t> stack{0};
    seen[0] = 1;
    int64_t count = 1;
    while (!stack.empty()) {
        int32_t i = stack.back();
        stack.pop_back();
        for (int64_t k = g.ptr[i]; k < g.ptr[i + 1]; ++k) {
            int32_t j = g.col[k];
            if (!seen[j]) { seen[j] = 1; ++count; stack.push_back(j); }
        }
    }
    return count == g.n;
}

// ---------------------------------------------------------- aggregation

// Maximal weighted matching of Sec. 2.2.  First pass: in visit order, an
// unaggregated vertex opens a new aggregate with its heaviest unaggregated
// neighbour (ties: smaller id).  Second pass: each vertex still alone joins
// the aggregate of its heaviest neighbour (ties: smaller id); all of its
// neighbours were paired in the first pass.
int64_t match_aggregate(const Adjacency& g, const std::vector<int64_t>* order,
                        std::vector<int64_t>& agg, std::vector<int8_t>& matched) {
    const int64_t n = g.n;
    agg.assign(n, -1);
    matched.assign(n, 0);
    int64_t next = 0;
    for (int64_t t = 0; t < n; ++t) {
        const int64_t v = order ? (*order)[t] : t;
        if (agg[v] >= 0) continue;
        int64_t pick = -1;
        double pw = -1.0;
        for (int64_t k = g.ptr[v]; k < g.ptr[v + 1]; ++k) {
            const int32_t nb = g.col[k];
            if (agg[nb] >= 0) continue;
            if (g.w[k] > pw) { pw = g.w[k]; pick = nb; }   // ascending nb: first max wins
        }
        if (pick >= 0) {
            agg[v] = agg[pick] = next++;
            matched[v] = matched[pick] = 1;
        }
    }
    for (int64_t v = 0; v < n; ++v) {
        if (matched[v]) continue;
        int64_t pick = -1;
        double pw = -1.0;
        for (int64_t k = g.ptr[v]; k < g.ptr[v + 1]; ++k)
            if (g.w[k] > pw) { pw = g.w[k]; pick = g.col[k]; }
        agg[v] = agg[pick];
    }
    return next;
}

// Aggregation of the parallel setup: the matching by rounds of locally
// dominant pairs.  In every round each free vertex points at its heaviest
// free neighbour (ties: smaller id), and two vertices pointing at each other
// pair up; rounds go on until no free vertex has a free neighbour.  With
// that tie rule an edge's rank (weight descending, then the smaller (i, j))
// is a strict total order, and the result is the greedy matching in that
// order: the heaviest edge left is always mutual.  Pair ids follow the
// smaller end; each vertex left free joins its heaviest neighbour's
// aggregate (ties: smaller id), as in the second pass above.  The device
// runs the same rounds with a thread per vertex (devsetup.hpp).
int64_t match_locally_dominant(const Adjacency& g, std::vector<int64_t>& agg,
                               std::vector<int8_t>& matched) {
    const int64_t n = g.n;
    std::vector<int64_t> mate(n, -1), ptr(n, -1);
    auto heaviest = [&](int64_t v, bool free_only) {
        int64_t pick = -1;
        double pw = -1.0;
        for (int64_t k = g.ptr[v]; k < g.ptr[v + 1]; ++k) {
            const int32_t nb = g.col[k];
            if (free_only && mate[nb] >= 0) continue;
            if (g.w[k] > pw) { pw = g.w[k]; pick = nb; }   // ascending nb: first max wins
        }
        return pick;
    };
    for (bool changed = true; changed;) {
        for (int64_t v = 0; v < n; ++v) ptr[v] = mate[v] < 0 ? heaviest(v, true) : -1;
        changed = false;
        for (int64_t v = 0; v < n; ++v) {
            const int64_t u = ptr[v];
            if (u >= 0 && ptr[u] == v) {
                mate[v] = u;
                changed = true;
            }
        }
    }
    agg.assign(n, -1);
    matched.assign(n, 0);
    int64_t next = 0;
    for (int64_t v = 0; v < n; ++v)
        if (mate[v] > v) {
            agg[v] = agg[mate[v]] = next++;
            matched[v] = matched[mate[v]] = 1;
        }
    for (int64_t v = 0; v < n; ++v)
        if (mate[v] < 0) agg[v] = agg[heaviest(v, false)];
    return next;
}

// Coarse graph of P^T L P: edges between different aggregates, weights
// accumulated per unordered aggregate pair in ascending fine (i, j), i < j.
// Contributions are bucketed by the smaller aggregate id in scan order (a
// stable counting sort), then merged per bucket with a position table.
void coarse_graph(const Adjacency& f, const std::vector<int64_t>& agg, int64_t nc,
                  Adjacency& c) {
    std::vector<int64_t> bstart(nc + 1, 0);
    for (int64_t i = 0; i < f.n; ++i)
        for (int64_t k = f.ptr[i]; k < f.ptr[i + 1]; ++k) {
            const int32_t j = f.col[k];
            if (j > i && agg[j] != agg[i]) ++bstart[std::min(agg[i], agg[j]) + 1];
        }
    for (int64_t a = 0; a < nc; ++a) bstart[a + 1] += bstart[a];
    std::vector<int32_t> bkey(bstart[nc]);
    std::vector<double> bval(bstart[nc]);
    std::vector<int64_t> fp(bstart.begin(), bstart.end() - 1);
    for (int64_t i = 0; i < f.n; ++i)
        for (int64_t k = f.ptr[i]; k < f.ptr[i + 1]; ++k) {
            const int32_t j = f.col[k];
            if (j <= i || agg[j] == agg[i]) continue;
            const int64_t lo = std::min(agg[i], agg[j]), hi = std::max(agg[i], agg[j]);
            bkey[fp[lo]] = (int32_t)hi;
            bval[fp[lo]] = f.w[k];
            ++fp[lo];
        }
    // unique upper-triangle edges per row, ascending
    std::vector<int64_t> where(nc, -1);
    std::vector<int64_t> ustart(nc + 1, 0);
    std::vector<int32_t> ukey;
    std::vector<double> uval;
    ukey.reserve(bstart[nc]);
    uval.reserve(bstart[nc]);
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t a = 0; a < nc; ++a) {
        row.clear();
        for (int64_t e = bstart[a]; e < bstart[a + 1]; ++e) {
            const int32_t b = bkey[e];
            if (where[b] >= 0) {
                row[where[b]].second += bval[e];
            } else {
                where[b] = (int64_t)row.size();
                row.push_back({b, bval[e]});
            }
        }
        for (auto& p : row) where[p.first] = -1;
        std::sort(row.begin(), row.end(),
                  [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) {
                      return x.first < y.first;
                  });
        for (auto& p : row) { ukey.push_back(p.first); uval.push_back(p.second); }
        ustart[a + 1] = (int64_t)ukey.size();
    }
    // symmetric CSR: row x = (entries from rows a < x, ascending a) + own list
    c.n = nc;
    c.ptr.assign(nc + 1, 0);
    for (int64_t a = 0; a < nc; ++a)
        for (int64_t e = ustart[a]; e < ustart[a + 1]; ++e) {
            ++c.ptr[a + 1];
            ++c.ptr[ukey[e] + 1];
        }
    for (int64_t a = 0; a < nc; ++a) c.ptr[a + 1] += c.ptr[a];
    c.col.assign(c.ptr[nc], 0);
    c.w.assign(c.ptr[nc], 0.0);
    std::vector<int64_t> lowfill(c.ptr.begin(), c.ptr.end() - 1);
    std::vector<int64_t> nlow(nc, 0);
    for (int64_t a = 0; a < nc; ++a)
        for (int64_t e = ustart[a]; e < ustart[a + 1]; ++e) ++nlow[ukey[e]];
    std::vector<int64_t> highfill(nc);
    for (int64_t a = 0; a < nc; ++a) highfill[a] = c.ptr[a] + nlow[a];
    for (int64_t a = 0; a < nc; ++a)
        for (int64_t e = ustart[a]; e < ustart[a + 1]; ++e) {
            const int32_t b = ukey[e];
            c.col[highfill[a]] = b;
            c.w[highfill[a]] = uval[e];
            ++highfill[a];
            c.col[lowfill[b]] = (int32_t)a;
            c.w[lowfill[b]] = uval[e];
            ++lowfill[b];
        }
}

// ------------------------------------------------------------- helpers

static uint64_t mix64(uint64_t& s) {      // SplitMix64 (Steele, Lea, Flood 2014)
    uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Fisher-Yates shuffle driven by SplitMix64 seeded with seed + level index.
static std::vector<int64_t> visit_order(int64_t n, uint64_t seed) {
    std::vector<int64_t> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    uint64_t s = seed;
    for (int64_t i = n - 1; i > 0; --i) {
        const int64_t j = (int64_t)(mix64(s) % (uint64_t)(i + 1));
        std::swap(ord[i], ord[j]);
    }
    return ord;
}

// Pseudo-inverse of a connected Laplacian: (L + J/t)^-1 - J/t, J = 1 1^T.
static bool laplacian_pinv(const Adjacency& g, std::vector<double>& out) {
    const int t = (int)g.n;
    std::vector<double> A(t * t, 1.0 / t), I(t * t, 0.0);
    for (int i = 0; i < t; ++i) {
        for (int64_t k = g.ptr[i]; k < g.ptr[i + 1]; ++k) {
            A[i * t + g.col[k]] -= g.w[k];
            A[i * t + i] += g.w[k];
        }
        I[i * t + i] = 1.0;
    }
    // Gauss-Jordan with partial pivoting (A is SPD).
    for (int c = 0; c < t; ++c) {
        int p = c;
        for (int r = c + 1; r < t; ++r)
            if (std::fabs(A[r * t + c]) > std::fabs(A[p * t + c])) p = r;
        if (A[p * t + c] == 0.0) return false;
        if (p != c)
            for (int k = 0; k < t; ++k) {
                std::swap(A[p * t + k], A[c * t + k]);
                std::swap(I[p * t + k], I[c * t + k]);
            }
        const double d = 1.0 / A[c * t + c];
        for (int k = 0; k < t; ++k) { A[c * t + k] *= d; I[c * t + k] *= d; }
        for (int r = 0; r < t; ++r) {
            if (r == c || A[r * t + c] == 0.0) continue;
            const double f = A[r * t + c];
            for (int k = 0; k < t; ++k) {
                A[r * t + k] -= f * A[c * t + k];
                I[r * t + k] -= f * I[c * t + k];
            }
        }
    }
    out.resize(t * t);
    for (int i = 0; i < t * t; ++i) out[i] = I[i] - 1.0 / t;
    return true;
}

// Level weight of the additive form of P(mu) L_T~^+ P(mu)^T:
//   theta_k = s_k^2 mu^(-2k),  s_k = sum_{i<=k} (-mu)^i = (1 - (-mu)^(k+1)) / (1 + mu).
static double level_theta(double mu, int k) {
    const double s = (1.0 - std::pow(-mu, k + 1)) / (1.0 + mu);
    return s * s * std::pow(mu, -2.0 * k);
}

// ---------------------------------------------------------------- plan

int build_plan(int64_t n, int64_t m, const int64_t* u, const int64_t* v,
               const double* w, double mu, int max_levels, int64_t n_top,
               uint64_t seed, bool any_top, HostPlan& plan, GraphBuilder* gb, int matching) {
    if (!(mu > 0.0 && mu < 1.0) || n_top < 2 || max_levels < 0) return kInval;
    plan = HostPlan();
    plan.mu = mu;
    plan.lv.emplace_back();
    int rc = gb ? gb->adjacency(n, m, u, v, w, plan.lv[0].g)
                : build_adjacency(n, m, u, v, w, plan.lv[0].g);
    if (rc != kOk) return rc;
    if (!is_connected(plan.lv[0].g)) return kDisconnected;

    // 1. hierarchy
    while ((max_levels == 0 || (int)plan.lv.size() < max_levels) &&
           plan.lv.back().g.n > n_top && plan.lv.size() < 60) {
        Level& f = plan.lv.back();
        std::vector<int64_t> agg;
        std::vector<int8_t> mt;
        int64_t nc;
        if (matching == 1) {
            nc = (gb && gb->match(f.g, agg, mt, nc)) ? nc : match_locally_dominant(f.g, agg, mt);
        } else if (seed != 0) {
            std::vector<int64_t> ord = visit_order(f.g.n, seed + (uint64_t)plan.lv.size());
            nc = match_aggregate(f.g, &ord, agg, mt);
        } else {
            nc = match_aggregate(f.g, nullptr, agg, mt);
        }
        if (nc < 2 || nc >= f.g.n) break;
        Level c;
        if (gb) gb->coarse(f.g, agg, nc, c.g);
        else coarse_graph(f.g, agg, nc, c.g);
        f.agg.swap(agg);
        f.matched.swap(mt);
        plan.lv.push_back(std::move(c));
    }
    const int L = plan.nlev();
    const int T = L - 1;
    if (plan.lv[T].g.n > kTopMax && !any_top) return kUnsupported;

    // 2. tree numbering, top level first
    plan.perm.assign(L, {});
    plan.inv.assign(L, {});
    plan.step.assign(T, {});
    {
        const int64_t nt = plan.lv[T].g.n;
        plan.perm[T].resize(nt);
        plan.inv[T].resize(nt);
        std::iota(plan.perm[T].begin(), plan.perm[T].end(), 0);
        std::iota(plan.inv[T].begin(), plan.inv[T].end(), 0);
    }
    for (int k = T - 1; k >= 0; --k) {
        const Level& f = plan.lv[k];
        const int64_t nk = f.g.n, nc = plan.lv[k + 1].g.n;
        StepCoef& sc = plan.step[k];
        sc.cptr.assign(nc + 1, 0);
        for (int64_t i = 0; i < nk; ++i) ++sc.cptr[plan.inv[k + 1][f.agg[i]] + 1];
        for (int64_t J = 0; J < nc; ++J) sc.cptr[J + 1] += sc.cptr[J];
        std::vector<int32_t> pos(sc.cptr.begin(), sc.cptr.end() - 1);
        plan.perm[k].resize(nk);
        plan.inv[k].resize(nk);
        for (int pass = 1; pass >= 0; --pass)      // matched members, then leftovers
            for (int64_t i = 0; i < nk; ++i) {
                if (f.matched[i] != pass) continue;
                const int32_t J = plan.inv[k + 1][f.agg[i]];
                plan.perm[k][pos[J]] = (int32_t)i;
                plan.inv[k][i] = pos[J]++;
            }
    }

    // 3. MSP coefficients
    plan.theta.resize(L);
    for (int k = 0; k < L; ++k) plan.theta[k] = level_theta(mu, k);
    for (int k = 0; k < T; ++k) {
        const Level& f = plan.lv[k];
        StepCoef& sc = plan.step[k];
        const int64_t nc = plan.lv[k + 1].g.n;
        const double th = plan.theta[k];
        const int64_t nleft = f.g.n - 2 * nc;
        sc.saa.resize(nc); sc.sab.resize(nc); sc.sbb.resize(nc);
        sc.l0.resize(nleft); sc.l1.resize(nleft); sc.l2.resize(nleft);
        for (int64_t J = 0; J < nc; ++J) {
            const int32_t b0 = sc.cptr[J], b1 = sc.cptr[J + 1];
            if (b1 - b0 < 2) return kInval;   // cannot happen: every aggregate has a pair
            const int32_t a = plan.perm[k][b0], b = plan.perm[k][b0 + 1];
            const int64_t aggid = f.agg[a];
            // pair block of L_B + mu diag(ext)
            double wab = 0.0, ia = 0.0, ib = 0.0, ea = 0.0, eb = 0.0;
            for (int64_t q = f.g.ptr[a]; q < f.g.ptr[a + 1]; ++q) {
                if (f.agg[f.g.col[q]] == aggid) { ia += f.g.w[q]; if (f.g.col[q] == b) wab = f.g.w[q]; }
                else ea += f.g.w[q];
            }
            for (int64_t q = f.g.ptr[b]; q < f.g.ptr[b + 1]; ++q) {
                if (f.agg[f.g.col[q]] == aggid) ib += f.g.w[q];
                else eb += f.g.w[q];
            }
            double Saa = ia + mu * ea, Sbb = ib + mu * eb, Sab = -wab;
            for (int32_t t = b0 + 2; t < b1; ++t) {
                const int32_t x = plan.perm[k][t];
                double wa = 0.0, wb = 0.0, ex = 0.0;
                for (int64_t q = f.g.ptr[x]; q < f.g.ptr[x + 1]; ++q) {
                    const int32_t y = f.g.col[q];
                    if (f.agg[y] != aggid) ex += f.g.w[q];
                    else if (y == a) wa += f.g.w[q];
                    else if (y == b) wb += f.g.w[q];
                    else return kInval;     // leftovers are never adjacent
                }
                const double dxx = wa + wb + mu * ex;
                Saa -= wa * wa / dxx;
                Sbb -= wb * wb / dxx;
                Sab -= wa * wb / dxx;
                const int64_t li = t - 2 * (int64_t)(J + 1);
                sc.l0[li] = th / dxx;
                sc.l1[li] = wa / dxx;
                sc.l2[li] = wb / dxx;
            }
            const double det = Saa * Sbb - Sab * Sab;
            if (!(det > 0.0)) return kInval;
            sc.saa[J] = th * Sbb / det;
            sc.sbb[J] = th * Saa / det;
            sc.sab[J] = -th * Sab / det;
        }
    }
    if (plan.lv[T].g.n <= kTopMax) {
        if (!laplacian_pinv(plan.lv[T].g, plan.top_pinv)) return kInval;
        for (double& x : plan.top_pinv) x *= plan.theta[T];
    }

    // 4. fine Laplacian for the SpMV.  A mesh keeps its own order (its
    //    neighbour gathers are contiguous across a wavefront); any other
    //    graph is renumbered in the tree order of the hierarchy, where every
    //    aggregate (a vertex with its heaviest neighbours) is contiguous and
    //    the level-0 restriction and prolongation need no permutation.
    const char* ord = std::getenv("LAPGPU_SPMV_ORDER");
    if (ord && std::strcmp(ord, "tree") == 0) plan.spmv_tree = true;
    else if (ord && std::strcmp(ord, "natural") == 0) plan.spmv_tree = false;
    else plan.spmv_tree = !mesh_like(plan.lv[0].g);
    if (plan.spmv_tree && T >= 1) {
        permute_graph(plan.lv[0].g, plan.perm[0], plan.inv[0], plan.solve_g);
        build_sell(plan.solve_g, plan);
    } else {
        plan.spmv_tree = false;
        build_sell(plan.lv[0].g, plan);
    }
    return kOk;
}

bool mesh_like(const Adjacency& g) {
    int64_t nnz = 0, pad = 0;
    for (int64_t s = 0; s * kSlice < g.n; ++s) {
        int64_t wmax = 0;
        for (int64_t t = s * kSlice; t < std::min<int64_t>(g.n, (s + 1) * kSlice); ++t) {
            const int64_t d = g.ptr[t + 1] - g.ptr[t];
            if (d > kHeavyDeg) return false;
            wmax = std::max(wmax, d);
            nnz += d;
        }
        pad += wmax * kSlice;
    }
    return pad * 100 <= nnz * 115;
}

void permute_graph(const Adjacency& g, const std::vector<int32_t>& perm,
                   const std::vector<int32_t>& inv, Adjacency& out) {
    out.n = g.n;
    out.ptr.assign(g.n + 1, 0);
    out.col.resize(g.nnz());
    out.w.resize(g.nnz());
    for (int64_t t = 0; t < g.n; ++t) out.ptr[t + 1] = out.ptr[t] + (g.ptr[perm[t] + 1] - g.ptr[perm[t]]);
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t t = 0; t < g.n; ++t) {
        const int64_t i = perm[t];
        row.clear();
        for (int64_t k = g.ptr[i]; k < g.ptr[i + 1]; ++k) row.push_back({inv[g.col[k]], g.w[k]});
        std::sort(row.begin(), row.end(),
                  [](const std::pair<int32_t, double>& a, const std::pair<int32_t, double>& b) {
                      return a.first < b.first;
                  });
        for (size_t q = 0; q < row.size(); ++q) {
            out.col[out.ptr[t] + q] = row[q].first;
            out.w[out.ptr[t] + q] = row[q].second;
        }
    }
}

// Sliced ELL in the given vertex order: for meshes and grids that
// order keeps the neighbour gathers of a wavefront within a few cache
// lines.  Rows of degree above kHeavyDeg go to a CSR part processed a row
// per wavefront (or per block).  When slices of consecutive rows would be
// padded by more than 15 %, rows are sorted by degree within windows of
// kSigma rows first (sliced ELL with sorting windows), so a slice's rows
// have similar degrees.
static int env_or(const char* name, int dflt) {
    const char* v = std::getenv(name);
    return v ? std::atoi(v) : dflt;
}

void build_sell(const Adjacency& g, HostPlan& plan) {
    const int64_t n = g.n;
    const int64_t heavy_deg = std::max(16, env_or("LAPGPU_HEAVY_DEG", kHeavyDeg));
    const int64_t sigma = std::max(kSlice, env_or("LAPGPU_SIGMA", kSigma));
    auto deg = [&](int64_t i) { return g.ptr[i + 1] - g.ptr[i]; };
    std::vector<int32_t> light, heavy;
    for (int64_t i = 0; i < n; ++i) (deg(i) > heavy_deg ? heavy : light).push_back((int32_t)i);
    const int64_t nl = (int64_t)light.size();
    int64_t nnz_l = 0, pad_id = 0;
    for (int64_t s = 0; s * kSlice < nl; ++s) {
        int64_t wmax = 0;
        for (int64_t t = s * kSlice; t < std::min<int64_t>(nl, (s + 1) * kSlice); ++t) {
            wmax = std::max<int64_t>(wmax, deg(light[t]));
            nnz_l += deg(light[t]);
        }
        pad_id += wmax * kSlice;
    }
    const bool sorted = pad_id * 100 > nnz_l * 115;
    if (sorted)
        for (int64_t w0 = 0; w0 < nl; w0 += sigma) {
            const auto b = light.begin() + w0, e = light.begin() + std::min<int64_t>(nl, w0 + sigma);
            std::stable_sort(b, e, [&](int32_t x, int32_t y) { return deg(x) > deg(y); });
        }
    const int64_t nslice = (nl + kSlice - 1) / kSlice;
    plan.sell_nlight = (int32_t)nl;
    plan.sell_off.assign(nslice + 1, 0);
    plan.sell_width.assign(nslice, 0);
    for (int64_t s = 0; s < nslice; ++s) {
        int64_t wmax = 0;
        for (int64_t t = s * kSlice; t < std::min<int64_t>(nl, (s + 1) * kSlice); ++t)
            wmax = std::max<int64_t>(wmax, deg(light[t]));
        plan.sell_width[s] = (int32_t)wmax;
        plan.sell_off[s + 1] = plan.sell_off[s] + (int32_t)(wmax * kSlice);
    }
    plan.sell_col.assign(plan.sell_off[nslice], 0);
    plan.sell_w.assign(plan.sell_off[nslice], 0.0);
    for (int64_t t = 0; t < nl; ++t) {
        const int64_t s = t / kSlice, lane = t % kSlice, r = light[t];
        for (int64_t k = 0; k < plan.sell_width[s]; ++k) {
            const int64_t slot = plan.sell_off[s] + k * kSlice + lane;
            if (k < deg(r)) {
                plan.sell_col[slot] = g.col[g.ptr[r] + k];
                plan.sell_w[slot] = g.w[g.ptr[r] + k];
            } else {
                plan.sell_col[slot] = (int32_t)r;   // padding: w = 0 on the row itself
                plan.sell_w[slot] = 0.0;
            }
        }
    }
    plan.sell_row.clear();
    if (sorted || !heavy.empty()) plan.sell_row = light;
    // heavy rows: CSR, grouped into blocks
    plan.heavy_row = heavy;
    plan.heavy_ptr.assign(heavy.size() + 1, 0);
    plan.heavy_col.clear();
    plan.heavy_w.clear();
    plan.heavy_blk.assign(1, 0);
    int32_t in_blk = 0;
    for (size_t h = 0; h < heavy.size(); ++h) {
        const int64_t r = heavy[h];
        for (int64_t q = g.ptr[r]; q < g.ptr[r + 1]; ++q) {
            plan.heavy_col.push_back(g.col[q]);
            plan.heavy_w.push_back(g.w[q]);
        }
        plan.heavy_ptr[h + 1] = (int32_t)plan.heavy_col.size();
        if (deg(r) > kHeavyBlockDeg) {
            if (in_blk > 0) plan.heavy_blk.push_back((int32_t)h);
            plan.heavy_blk.push_back((int32_t)h + 1);
            in_blk = 0;
        } else if (++in_blk == kHeavyWaves) {
            plan.heavy_blk.push_back((int32_t)h + 1);
            in_blk = 0;
        }
    }
    if (in_blk > 0) plan.heavy_blk.push_back((int32_t)heavy.size());
}

void hot_columns(const HostPlan& plan, int64_t n, int64_t count, std::vector<int32_t>& hot,
                 std::vector<int32_t>& sell_col, std::vector<int32_t>& heavy_col) {
    std::vector<int64_t> refs(n, 0);
    // light slots: only the real entries (a padding slot holds its own row
    // with weight 0)
    for (size_t t = 0; t < plan.sell_col.size(); ++t)
        if (plan.sell_w[t] != 0.0) ++refs[plan.sell_col[t]];
    for (int32_t c : plan.heavy_col) ++refs[c];
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    count = std::min<int64_t>(count, n);
    std::partial_sort(order.begin(), order.begin() + count, order.end(), [&](int32_t a, int32_t b) {
        return refs[a] != refs[b] ? refs[a] > refs[b] : a < b;
    });
    hot.assign(order.begin(), order.begin() + count);
    std::vector<int32_t> rank(n, -1);
    for (int64_t k = 0; k < count; ++k) rank[hot[k]] = (int32_t)k;
    sell_col = plan.sell_col;
    for (size_t t = 0; t < sell_col.size(); ++t)
        if (plan.sell_w[t] != 0.0 && rank[sell_col[t]] >= 0) sell_col[t] = ~rank[sell_col[t]];
    heavy_col = plan.heavy_col;
    for (int32_t& c : heavy_col)
        if (rank[c] >= 0) c = ~rank[c];
}

// ------------------------------------------------------------------ PEGP

// How many lanes share a row in the rows [r0, r1) of a PEGP solve level
// (log2).  Rows are dealt round-robin to groups of G lanes; a lane loads
// eight entries a round, so a group spends max(1, ceil(len / 8G)) rounds on
// a row plus a little per reduction step.  The pick minimises the busiest
// group's time.
static int32_t pegp_lanes(const std::vector<int32_t>& ptr, int32_t r0, int32_t r1) {
    int32_t best = 0;
    double best_cost = 1e300;
    for (int g = 0; g <= 6; ++g) {
        const int64_t G = 1 << g, NG = kPegpSolveThreads / G;
        double worst = 0.0;
        for (int64_t s = 0; s < NG && r0 + s < r1; ++s) {
            double c = 0.0;
            for (int64_t r = r0 + s; r < r1; r += NG) {
                const int64_t len = ptr[r + 1] - ptr[r];
                c += (double)std::max<int64_t>(1, (len + 8 * G - 1) / (8 * G)) + 0.1 * g;
            }
            worst = std::max(worst, c);
        }
        if (worst < best_cost) {
            best_cost = worst;
            best = g;
        }
    }
    return best;
}

// The level lists (lev, ptr, col, val) with lanes per level lg packed as
// the descriptors and padded entry arrays the solve reads.
static bool pegp_pack(const std::vector<int32_t>& lev, const std::vector<int32_t>& lg,
                      const std::vector<int32_t>& ptr, const std::vector<int32_t>& col,
                      const std::vector<double>& val, std::vector<int32_t>& desc,
                      std::vector<double>& pval, std::vector<int32_t>& pcol) {
    desc.clear();
    pval.clear();
    pcol.clear();
    for (size_t l = 0; l + 1 < lev.size(); ++l) {
        const int32_t r0 = lev[l], r1 = lev[l + 1], nr = r1 - r0, g = lg[l];
        const int32_t G = 1 << g, NG = kPegpSolveThreads / G;
        const int32_t np = (nr + NG - 1) / NG, nt = np > 1 ? kPegpSolveThreads : nr * G;
        int32_t maxlen = 0;
        for (int32_t r = r0; r < r1; ++r) maxlen = std::max(maxlen, ptr[r + 1] - ptr[r]);
        const int32_t U = std::max(1, (maxlen + G - 1) / G);
        if (U >= 1 << 15 || np >= 1 << 16 || nr >= 1 << 15 ||
            pval.size() + (size_t)np * U * nt > (size_t)INT32_MAX)
            return false;
        const int32_t base = (int32_t)pval.size();
        pval.resize(base + (size_t)np * U * nt, 0.0);
        pcol.resize(pval.size(), 0);
        for (int32_t rr = 0; rr < nr; ++rr) {
            const int32_t p = rr / NG, grp = rr % NG, r = r0 + rr;
            for (int32_t e = 0; e < ptr[r + 1] - ptr[r]; ++e) {
                const int32_t t = grp * G + e % G, u = e / G;
                const size_t i = (size_t)base + ((size_t)p * U + u) * nt + t;
                pval[i] = val[ptr[r] + e];
                pcol[i] = col[ptr[r] + e] * (int32_t)sizeof(double);
            }
        }
        const int32_t d[kPegpDescInts] = {base, nt | g << 12 | U << 16, np | nr << 16, r0};
        desc.insert(desc.end(), d, d + kPegpDescInts);
    }
    return true;
}

// Columns of the explicit PEGP operator (see PegpPlan::op): for r = e_j -
// 1/n, the scaled right-hand side D P(mu)^T r has, on a level-k node A,
// (-1)^k times the sum of r over A's fine descendants; the grounded solve
// S y' = D P(mu)^T r runs through the factor S = L diag(d) L^T in
// elimination order, and z = P(mu) D y' = sum_k (-1)^k y'(ancestor on level
// k), made mean-free.  Columns are spread over host threads.
static void pegp_operator(const HostPlan& P, const std::vector<int32_t>& off,
                          const std::vector<std::vector<int32_t>>& par,
                          const std::vector<int32_t>& order,
                          const std::vector<std::vector<std::pair<int32_t, double>>>& rowL,
                          const std::vector<std::vector<std::pair<int32_t, double>>>& colL,
                          const std::vector<double>& diag, PegpPlan& out) {
    const int L = P.nlev(), T = L - 1;
    const int32_t n = (int32_t)P.lv[0].g.n, nt = off[L], m = nt - 1;
    const int32_t ld = (n + kPegpOpAlign - 1) / kPegpOpAlign * kPegpOpAlign;
    // the factor as CSR in elimination order
    std::vector<int32_t> fp(m + 1, 0), bp(m + 1, 0), fi, bi;
    std::vector<double> fv, bv;
    for (int32_t q = 0; q < m; ++q) {
        const int32_t v = order[q];
        for (auto& e : rowL[v]) {
            fi.push_back(e.first);
            fv.push_back(e.second);
        }
        fp[q + 1] = (int32_t)fi.size();
        for (auto& e : colL[v]) {
            bi.push_back(e.first);
            bv.push_back(e.second);
        }
        bp[q + 1] = (int32_t)bi.size();
    }
    // fine descendants of every expanded node, and the level of each
    std::vector<double> cnt(nt, 0.0);
    std::vector<int> lev(nt, 0);
    for (int k = 0; k < L; ++k)
        for (int32_t e = off[k]; e < off[k + 1]; ++e) lev[e] = k;
    for (int32_t t = 0; t < n; ++t) cnt[t] = 1.0;
    for (int k = 0; k < T; ++k)
        for (int32_t t = 0; t < off[k + 1] - off[k]; ++t) cnt[off[k + 1] + par[k][t]] += cnt[off[k] + t];
    out.opn = n;
    out.opld = ld;
    out.op.assign((size_t)n * ld, 0.0);
    auto column = [&](int32_t j, std::vector<double>& w, std::vector<double>& acc) {
        for (int32_t e = 0; e < nt; ++e) w[e] = -cnt[e] / (double)n * ((lev[e] & 1) ? -1.0 : 1.0);
        for (int32_t a = j, k = 0;; ++k) {
            w[off[k] + a] += (k & 1) ? -1.0 : 1.0;
            if (k == T) break;
            a = par[k][a];
        }
        for (int32_t q = 0; q < m; ++q) {
            const int32_t v = order[q];
            double x = w[v];
            for (int32_t i = fp[q]; i < fp[q + 1]; ++i) x -= fv[i] * w[fi[i]];
            w[v] = x;
        }
        for (int32_t q = 0; q < m; ++q) w[order[q]] /= diag[order[q]];
        for (int32_t q = m - 1; q >= 0; --q) {
            const int32_t v = order[q];
            double x = w[v];
            for (int32_t i = bp[q]; i < bp[q + 1]; ++i) x -= bv[i] * w[bi[i]];
            w[v] = x;
        }
        w[nt - 1] = 0.0;  // the grounded node
        // z = sum over levels of (-1)^k y'(ancestor), top down
        for (int32_t e = off[T]; e < nt; ++e) acc[e] = (T & 1) ? -w[e] : w[e];
        for (int k = T - 1; k >= 0; --k)
            for (int32_t t = 0; t < off[k + 1] - off[k]; ++t)
                acc[off[k] + t] = ((k & 1) ? -w[off[k] + t] : w[off[k] + t]) +
                                  acc[off[k + 1] + par[k][t]];
        double mean = 0.0;
        for (int32_t t = 0; t < n; ++t) mean += acc[t];
        mean /= (double)n;
        for (int32_t t = 0; t < n; ++t) out.op[(size_t)t * ld + j] = acc[t] - mean;
    };
    const int nth = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
    std::atomic<int32_t> next{0};
    auto work = [&]() {
        std::vector<double> w(nt), acc(nt);
        for (int32_t j; (j = next.fetch_add(1)) < n;) column(j, w, acc);
    };
    std::vector<std::thread> pool;
    for (int i = 1; i < nth; ++i) pool.emplace_back(work);
    work();
    for (auto& t : pool) t.join();
}

// The off-tree sparsifier of Sec. 3.3 on top of the MSP tree T~ (the
// sparsifier of the MSP preconditioner: edges inside an aggregate on every
// level below the top, links from a node to its own aggregate on the next
// level, all top-level edges).  The positive edges of H~ outside T~ are
// ranked by their stretch in T~, w_e times the effective resistance between
// the ends through T~ (the distance of def. stretch-edge, taken as the
// resistance, as for the total stretch of the bound after it), and the
// ceil(frac * count) largest are kept (ties to the smaller pair in the
// levels' own numbering).  Effective resistances come from a grounded
// LDL^T of the tree Laplacian L_T~ (edge weights mu^(k+l) w_AB): for the
// right-hand side e_a - e_b, w = L^-1 (e_a - e_b) touches only the
// elimination-tree paths of a and b, and R = sum_v w_v^2 / d_v.  The
// weights span mu^(2(l-1)), and a running diagonal would lose the small
// pivots of coarse nodes to cancellation; every pivot is instead the sum of
// the magnitudes of its remaining off-diagonal entries (the Schur
// complements of a Laplacian are Laplacians; Grassmann, Taksar and
// Heyman's elimination without subtraction), the grounded node included.
// use[q] is cleared for every H~ edge keys[q] left out.  False: T~ is not
// positive definite once grounded (not connected).
static bool select_offtree(const HostPlan& P, const std::vector<int32_t>& off,
                           const std::vector<std::vector<int32_t>>& par, double mu,
                           const std::vector<uint64_t>& keys,
                           const std::unordered_map<uint64_t, double>& acc, double frac,
                           std::vector<char>& use, PegpPlan& out) {
    const int L = P.nlev(), T = L - 1;
    const int32_t nt = off[L], m = nt - 1;
    std::vector<int> lev(nt);
    std::vector<int32_t> own(nt);
    for (int k = 0; k < L; ++k)
        for (int32_t t = 0; t < off[k + 1] - off[k]; ++t) {
            lev[off[k] + t] = k;
            own[off[k] + t] = P.perm[k][t];
        }
    auto in_tree = [&](int32_t a, int32_t b) {  // a < b: lev(a) <= lev(b)
        const int ka = lev[a], kb = lev[b];
        const int32_t ta = a - off[ka], tb = b - off[kb];
        if (ka == kb) return ka == T || par[ka][ta] == par[kb][tb];
        return kb == ka + 1 && par[ka][ta] == tb;
    };
    // the tree Laplacian's off-diagonal entries (negative), rows as hash
    // maps (fill is added as it comes)
    std::vector<std::unordered_map<int32_t, double>> A(nt);
    std::vector<int32_t> offq;  // off-tree edges (indices into keys)
    for (size_t q = 0; q < keys.size(); ++q) {
        const double w = acc.at(keys[q]);
        if (!(w > 0.0)) continue;
        const int32_t a = (int32_t)(keys[q] >> 32), b = (int32_t)(keys[q] & 0xffffffffu);
        if (!in_tree(a, b)) {
            offq.push_back((int32_t)q);
            continue;
        }
        const double we = std::pow(mu, lev[a] + lev[b]) * w;
        A[a][b] -= we;
        A[b][a] -= we;
    }
    // elimination order: level by level from the finest, on each level
    // below the top the leftovers before the matched nodes; the last top
    // node is grounded
    std::vector<int32_t> order, pos(nt, -1);
    for (int k = 0; k < L; ++k)
        for (int pass = 0; pass < 2; ++pass)
            for (int32_t t = 0; t < off[k + 1] - off[k]; ++t) {
                const bool matched = k < T && P.lv[k].matched[P.perm[k][t]];
                if (k == T ? pass == 0 : (pass == 0) != matched) order.push_back(off[k] + t);
            }
    order.pop_back();  // nt - 1, the ground
    for (int32_t q = 0; q < m; ++q) pos[order[q]] = q;
    std::vector<double> piv(nt, 0.0);
    std::vector<std::vector<std::pair<int32_t, double>>> col(nt);  // l_uv, u later
    std::vector<int32_t> etp(nt, -1);                                // elimination-tree parent
    for (int32_t q = 0; q < m; ++q) {
        const int32_t v = order[q];
        // remaining neighbours: later in the order, or the ground (pos -1)
        auto live = [&](int32_t u) { return u != v && (pos[u] > q || u == nt - 1); };
        double dv = 0.0;
        for (auto& e : A[v])
            if (live(e.first)) dv -= e.second;
        if (!(dv > 0.0) || !std::isfinite(dv)) return false;
        piv[v] = dv;
        // the multipliers l_uv of the remaining neighbours (the ground's
        // only enter the Schur updates: its column is not solved for)
        std::vector<std::pair<int32_t, double>> c;
        for (auto& e : A[v])
            if (live(e.first)) c.push_back({e.first, e.second / dv});
        std::sort(c.begin(), c.end());
        // off-diagonal Schur updates only (they add entries of one sign)
        for (auto& e1 : c)
            for (auto& e2 : c)
                if (e2.first != e1.first) A[e1.first][e2.first] -= e1.second * dv * e2.second;
        int32_t best = -1;
        for (auto& e : c)
            if (e.first != nt - 1) {
                col[v].push_back(e);
                if (best < 0 || pos[e.first] < pos[best]) best = e.first;
            }
        etp[v] = best;
        A[v].clear();
    }
    // stretch of every off-tree edge
    const size_t cnt = offq.size();
    std::vector<double> stretch(cnt);
    std::vector<double> wv(nt, 0.0);
    std::vector<int32_t> path;
    for (size_t i = 0; i < cnt; ++i) {
        const uint64_t key = keys[offq[i]];
        const int32_t a = (int32_t)(key >> 32), b = (int32_t)(key & 0xffffffffu);
        path.clear();
        for (int32_t v = a; v >= 0 && v != nt - 1; v = etp[v]) path.push_back(v);
        for (int32_t v = b; v >= 0 && v != nt - 1; v = etp[v]) path.push_back(v);
        // (the ground's column is not part of the factor: etp stops there)
        std::sort(path.begin(), path.end(), [&](int32_t x, int32_t y) { return pos[x] < pos[y]; });
        path.erase(std::unique(path.begin(), path.end()), path.end());
        if (a != nt - 1) wv[a] += 1.0;
        if (b != nt - 1) wv[b] -= 1.0;
        double R = 0.0;
        for (int32_t v : path) {
            const double x = wv[v];
            for (auto& e : col[v]) wv[e.first] -= e.second * x;
            R += x * x / piv[v];
        }
        for (int32_t v : path) wv[v] = 0.0;
        stretch[i] = std::pow(mu, lev[a] + lev[b]) * acc.at(key) * R;
    }
    // ranking: stretch descending, ties to the smaller pair (own numbering)
    auto pair_of = [&](size_t i) {
        const uint64_t key = keys[offq[i]];
        const int32_t a = (int32_t)(key >> 32), b = (int32_t)(key & 0xffffffffu);
        const int64_t oa = off[lev[a]] + own[a], ob = off[lev[b]] + own[b];
        return std::make_pair(std::min(oa, ob), std::max(oa, ob));
    };
    std::vector<size_t> rank(cnt);
    std::iota(rank.begin(), rank.end(), 0);
    std::sort(rank.begin(), rank.end(), [&](size_t x, size_t y) {
        if (stretch[x] != stretch[y]) return stretch[x] > stretch[y];
        return pair_of(x) < pair_of(y);
    });
    const size_t keep = (size_t)std::ceil(frac * (double)cnt - 1e-12);
    std::vector<int8_t> kept(cnt, 0);
    for (size_t r = 0; r < std::min(keep, cnt); ++r) kept[rank[r]] = 1;
    out.ot_a.resize(cnt);
    out.ot_b.resize(cnt);
    out.ot_w.resize(cnt);
    out.ot_stretch = stretch;
    out.ot_kept = kept;
    for (size_t i = 0; i < cnt; ++i) {
        const auto pr = pair_of(i);
        out.ot_a[i] = pr.first;
        out.ot_b[i] = pr.second;
        const uint64_t key = keys[offq[i]];
        const int32_t a = (int32_t)(key >> 32), b = (int32_t)(key & 0xffffffffu);
        out.ot_w[i] = std::pow(mu, lev[a] + lev[b]) * acc.at(key);
        if (!kept[i]) use[offq[i]] = 0;
    }
    return true;
}

// The other tree: a maximum-weight spanning tree of H~ (Kruskal: heaviest
// edge first, weights within kTieRel of each other, runs of sorted
// weights with every consecutive gap inside it, taken as equal and
// ordered by the smaller pair in the levels' own numbering; an edge
// joining two components is taken), and its off-tree edges ranked by
// stretch, w_e times the resistance of the tree path between the ends
// (the sum of 1 / w along it), as select_offtree ranks them for T~.  H~
// has structurally equal weights (the pairs (i, parent(j)) and (j,
// parent(i)) of one fine edge, for one), which FP64 evaluations of H~ may
// round apart by far less than kTieRel.
constexpr double kTieRel = 1e-9;
static bool select_spanning(const HostPlan& P, const std::vector<int32_t>& off, double mu,
                            const std::vector<uint64_t>& keys,
                            const std::unordered_map<uint64_t, double>& acc, double frac,
                            std::vector<char>& use, PegpPlan& out) {
    const int L = P.nlev();
    const int32_t nt = off[L];
    std::vector<int> lev(nt);
    std::vector<int32_t> own(nt);
    for (int k = 0; k < L; ++k)
        for (int32_t t = 0; t < off[k + 1] - off[k]; ++t) {
            lev[off[k] + t] = k;
            own[off[k] + t] = P.perm[k][t];
        }
    const size_t ne = keys.size();
    std::vector<double> we(ne, 0.0);
    std::vector<std::pair<int64_t, int64_t>> pr(ne);
    std::vector<size_t> cand;
    for (size_t q = 0; q < ne; ++q) {
        const double w = acc.at(keys[q]);
        const int32_t a = (int32_t)(keys[q] >> 32), b = (int32_t)(keys[q] & 0xffffffffu);
        const int64_t oa = off[lev[a]] + own[a], ob = off[lev[b]] + own[b];
        pr[q] = {std::min(oa, ob), std::max(oa, ob)};
        if (!(w > 0.0)) continue;
        we[q] = std::pow(mu, lev[a] + lev[b]) * w;
        cand.push_back(q);
    }
    std::sort(cand.begin(), cand.end(), [&](size_t x, size_t y) { return we[x] > we[y]; });
    std::vector<int32_t> group(ne, 0);
    for (size_t r = 1; r < cand.size(); ++r) {
        const double a = we[cand[r - 1]], b = we[cand[r]];
        group[cand[r]] = group[cand[r - 1]] + (a - b > kTieRel * a ? 1 : 0);
    }
    std::sort(cand.begin(), cand.end(), [&](size_t x, size_t y) {
        if (group[x] != group[y]) return group[x] < group[y];
        return pr[x] < pr[y];
    });
    std::vector<int32_t> dsu(nt);
    std::iota(dsu.begin(), dsu.end(), 0);
    auto find = [&](int32_t a) {
        while (dsu[a] != a) a = dsu[a] = dsu[dsu[a]];
        return a;
    };
    std::vector<char> in_tree(ne, 0);
    std::vector<std::vector<std::pair<int32_t, double>>> tadj(nt);
    int32_t taken = 0;
    for (size_t q : cand) {
        const int32_t a = (int32_t)(keys[q] >> 32), b = (int32_t)(keys[q] & 0xffffffffu);
        const int32_t ra = find(a), rb = find(b);
        if (ra == rb) continue;
        dsu[ra] = rb;
        in_tree[q] = 1;
        tadj[a].push_back({b, we[q]});
        tadj[b].push_back({a, we[q]});
        ++taken;
    }
    if (taken != nt - 1) return false;  // H~ not connected
    // the tree rooted at the ground: parents, depths, edge weights upward,
    // and ancestor tables for the meeting points of paths
    std::vector<int32_t> parent(nt, -1), depth(nt, 0), bfs;
    std::vector<double> up_w(nt, 0.0);
    bfs.reserve(nt);
    bfs.push_back(nt - 1);
    parent[nt - 1] = nt - 1;
    for (size_t i = 0; i < bfs.size(); ++i) {
        const int32_t a = bfs[i];
        for (auto& e : tadj[a])
            if (parent[e.first] < 0) {
                parent[e.first] = a;
                depth[e.first] = depth[a] + 1;
                up_w[e.first] = e.second;
                bfs.push_back(e.first);
            }
    }
    int LOG = 1;
    while ((1 << LOG) < nt) ++LOG;
    std::vector<std::vector<int32_t>> anc(LOG, std::vector<int32_t>(nt));
    anc[0] = parent;
    for (int k = 1; k < LOG; ++k)
        for (int32_t v = 0; v < nt; ++v) anc[k][v] = anc[k - 1][anc[k - 1][v]];
    auto meet = [&](int32_t a, int32_t b) {
        if (depth[a] < depth[b]) std::swap(a, b);
        for (int k = LOG - 1; k >= 0; --k)
            if (depth[a] - (1 << k) >= depth[b]) a = anc[k][a];
        if (a == b) return a;
        for (int k = LOG - 1; k >= 0; --k)
            if (anc[k][a] != anc[k][b]) {
                a = anc[k][a];
                b = anc[k][b];
            }
        return parent[a];
    };
    std::vector<size_t> offq;
    for (size_t q : cand)
        if (!in_tree[q]) offq.push_back(q);
    std::sort(offq.begin(), offq.end());
    const size_t cnt = offq.size();
    std::vector<double> stretch(cnt);
    for (size_t i = 0; i < cnt; ++i) {
        const uint64_t key = keys[offq[i]];
        const int32_t a = (int32_t)(key >> 32), b = (int32_t)(key & 0xffffffffu);
        const int32_t c = meet(a, b);
        double R = 0.0;
        for (int32_t v = a; v != c; v = parent[v]) R += 1.0 / up_w[v];
        for (int32_t v = b; v != c; v = parent[v]) R += 1.0 / up_w[v];
        stretch[i] = we[offq[i]] * R;
    }
    std::vector<size_t> rank(cnt);
    std::iota(rank.begin(), rank.end(), 0);
    std::sort(rank.begin(), rank.end(), [&](size_t x, size_t y) {
        if (stretch[x] != stretch[y]) return stretch[x] > stretch[y];
        return pr[offq[x]] < pr[offq[y]];
    });
    const size_t keep = (size_t)std::ceil(frac * (double)cnt - 1e-12);
    std::vector<int8_t> kept(cnt, 0);
    for (size_t r = 0; r < std::min(keep, cnt); ++r) kept[rank[r]] = 1;
    out.ot_a.resize(cnt);
    out.ot_b.resize(cnt);
    out.ot_w.resize(cnt);
    out.ot_stretch = stretch;
    out.ot_kept = kept;
    for (size_t i = 0; i < cnt; ++i) {
        out.ot_a[i] = pr[offq[i]].first;
        out.ot_b[i] = pr[offq[i]].second;
        out.ot_w[i] = we[offq[i]];
    }
    for (size_t q = 0; q < ne; ++q) use[q] = in_tree[q];
    for (size_t i = 0; i < cnt; ++i)
        if (kept[i]) use[offq[i]] = 1;
    return true;
}

int build_pegp(const HostPlan& P, double mu, PegpPlan& out, double offtree_frac, int tree) {
    const int L = P.nlev();
    const int T = L - 1;
    out = PegpPlan();
    out.off.assign(L + 1, 0);
    for (int k = 0; k < L; ++k) out.off[k + 1] = out.off[k] + (int32_t)P.lv[k].g.n;
    const int32_t nt = out.off[L];
    out.nt = nt;
    // parent (tree numbering) of every node of levels 0..T-1
    std::vector<std::vector<int32_t>> par(T);
    for (int k = 0; k < T; ++k) {
        par[k].resize(P.lv[k].g.n);
        const std::vector<int32_t>& cp = P.step[k].cptr;
        for (size_t J = 0; J + 1 < cp.size(); ++J)
            for (int32_t t = cp[J]; t < cp[J + 1]; ++t) par[k][t] = (int32_t)J;
    }
    auto lev = [&](int32_t e) {
        return (int)(std::upper_bound(out.off.begin(), out.off.end(), e) - out.off.begin()) - 1;
    };
    // edge weights w_AB from the fine edges, keyed by (min, max) expanded index
    std::unordered_map<uint64_t, double> acc;
    acc.reserve((size_t)P.lv[0].g.nnz() * L);
    auto add = [&](int32_t a, int32_t b, double w) {
        const uint64_t key = a < b ? ((uint64_t)a << 32) | (uint32_t)b : ((uint64_t)b << 32) | (uint32_t)a;
        acc[key] += w;
    };
    const Adjacency& g = P.lv[0].g;
    std::vector<int32_t> ai(L), bj(L);
    for (int64_t i = 0; i < g.n; ++i)
        for (int64_t q = g.ptr[i]; q < g.ptr[i + 1]; ++q) {
            const int64_t j = g.col[q];
            if (j < i) continue;
            const double w = g.w[q];
            ai[0] = P.inv[0][i];
            bj[0] = P.inv[0][j];
            for (int k = 0; k < T; ++k) {
                ai[k + 1] = par[k][ai[k]];
                bj[k + 1] = par[k][bj[k]];
            }
            int c = 0;                         // first common level
            while (c < L && ai[c] != bj[c]) ++c;
            // disjoint pairs (both below c), k + l even
            for (int k = 0; k < c; ++k)
                for (int l = k & 1; l < c; l += 2) add(out.off[k] + ai[k], out.off[l] + bj[l], w);
            // nested pairs: B = level-l node, A = its level-k ancestor (l < k
            // < c), k + l odd: the edge leaves A
            for (int k = 1; k < c; ++k)
                for (int l = 0; l < k; ++l)
                    if ((k + l) & 1) {
                        add(out.off[k] + ai[k], out.off[l] + ai[l], w);
                        add(out.off[k] + bj[k], out.off[l] + bj[l], w);
                    }
        }
    // S: off-diagonals -w_AB, diagonal sum_B mu^(l-k) w_AB
    std::vector<std::vector<std::pair<int32_t, double>>> adj(nt);
    std::vector<double> sdiag(nt, 0.0);
    std::vector<uint64_t> keys;
    keys.reserve(acc.size());
    for (auto& kv : acc) keys.push_back(kv.first);
    std::sort(keys.begin(), keys.end());
    std::vector<char> use(keys.size(), 1);
    if (offtree_frac >= 0.0 &&
        !(tree == 1 ? select_spanning(P, out.off, mu, keys, acc, offtree_frac, use, out)
                    : select_offtree(P, out.off, par, mu, keys, acc, offtree_frac, use, out)))
        return kInval;
    for (size_t q = 0; q < keys.size(); ++q) {
        if (!use[q]) continue;
        const uint64_t key = keys[q];
        const double w = acc[key];
        if (!(w > 0.0)) continue;
        const int32_t a = (int32_t)(key >> 32), b = (int32_t)(key & 0xffffffffu);
        const int ka = lev(a), kb = lev(b);
        adj[a].push_back({b, -w});
        adj[b].push_back({a, -w});
        sdiag[a] += std::pow(mu, kb - ka) * w;
        sdiag[b] += std::pow(mu, ka - kb) * w;
    }
    for (auto& r : adj) out.nnz_s += (int64_t)r.size();
    out.ground = nt - 1;
    // minimum-degree elimination on bitsets, numeric LDL^T on a dense copy
    const int32_t m = nt - 1;                 // the grounded node is left out
    if ((int64_t)m * m > (int64_t)400 * 1000 * 1000) return kUnsupported;
    const int32_t words = (m + 63) / 64;
    std::vector<uint64_t> bits((size_t)m * words, 0);
    std::vector<double> A((size_t)m * m, 0.0);
    for (int32_t a = 0; a < m; ++a) {
        A[(size_t)a * m + a] = sdiag[a];
        for (auto& e : adj[a])
            if (e.first < m) {
                A[(size_t)a * m + e.first] = e.second;
                bits[(size_t)a * words + (e.first >> 6)] |= 1ull << (e.first & 63);
            }
    }
    std::vector<char> gone(m, 0);
    std::vector<int32_t> deg(m), order, pos(m);
    for (int32_t a = 0; a < m; ++a) {
        int d = 0;
        for (int32_t wi = 0; wi < words; ++wi) d += __builtin_popcountll(bits[(size_t)a * words + wi]);
        deg[a] = d;
    }
    std::vector<std::vector<std::pair<int32_t, double>>> colL(m);   // l_uv for later u
    out.diag.assign(nt, 1.0);
    std::vector<int32_t> nb;
    for (int32_t step = 0; step < m; ++step) {
        int32_t v = -1;
        for (int32_t a = 0; a < m; ++a)
            if (!gone[a] && (v < 0 || deg[a] < deg[v])) v = a;
        gone[v] = 1;
        pos[v] = step;
        order.push_back(v);
        nb.clear();
        const uint64_t* bv = &bits[(size_t)v * words];
        for (int32_t wi = 0; wi < words; ++wi)
            for (uint64_t x = bv[wi]; x; x &= x - 1) {
                const int32_t u = wi * 64 + __builtin_ctzll(x);
                if (!gone[u]) nb.push_back(u);
            }
        const double dv = A[(size_t)v * m + v];
        if (!(dv > 0.0)) return kInval;
        out.diag[v] = dv;
        for (int32_t u : nb) colL[v].push_back({u, A[(size_t)u * m + v] / dv});
        for (size_t x = 0; x < nb.size(); ++x) {
            const int32_t u = nb[x];
            const double luv = A[(size_t)u * m + v] / dv;
            double* Au = &A[(size_t)u * m];
            for (size_t y = 0; y < nb.size(); ++y) {
                const int32_t w2 = nb[y];
                Au[w2] -= luv * A[(size_t)v * m + w2];
            }
            uint64_t* bu = &bits[(size_t)u * words];
            for (int32_t wi = 0; wi < words; ++wi) bu[wi] |= bv[wi];
            bu[u >> 6] &= ~(1ull << (u & 63));
            bu[v >> 6] &= ~(1ull << (v & 63));
        }
        for (int32_t u : nb) {
            int d = 0;
            const uint64_t* bu = &bits[(size_t)u * words];
            for (int32_t wi = 0; wi < words; ++wi) {
                uint64_t x = bu[wi];
                // count only nodes still present
                while (x) {
                    const int32_t z = wi * 64 + __builtin_ctzll(x);
                    x &= x - 1;
                    d += !gone[z];
                }
            }
            deg[u] = d;
        }
    }
    // rows of L (forward, gather) and columns (backward, gather), levels
    std::vector<std::vector<std::pair<int32_t, double>>> rowL(m);
    for (int32_t v = 0; v < m; ++v)
        for (auto& e : colL[v]) rowL[e.first].push_back({v, e.second});
    for (int32_t v = 0; v < m; ++v) out.nnz_l += (int64_t)colL[v].size();
    std::vector<int32_t> lf(m, 0), lb(m, 0);
    for (int32_t v : order) {
        int d = 0;
        for (auto& e : rowL[v]) d = std::max(d, lf[e.first] + 1);
        lf[v] = d;
    }
    for (auto it = order.rbegin(); it != order.rend(); ++it) {
        int d = 0;
        for (auto& e : colL[*it]) d = std::max(d, lb[e.first] + 1);
        lb[*it] = d;
    }
    // level schedule of the nodes with keep[v] (all when keep is empty)
    auto schedule = [&](const std::vector<int32_t>& lv, const std::vector<std::vector<std::pair<int32_t, double>>>& ent,
                        std::vector<int32_t>& levp, std::vector<int32_t>& rows, std::vector<int32_t>& ptr,
                        std::vector<int32_t>& col, std::vector<double>& val,
                        const std::vector<char>& keep) {
        auto kept = [&](int32_t v) { return keep.empty() || keep[v]; };
        int nl = 0, nr = 0;
        for (int32_t v = 0; v < m; ++v)
            if (kept(v)) {
                nl = std::max(nl, lv[v] + 1);
                ++nr;
            }
        levp.assign(nl + 1, 0);
        for (int32_t v = 0; v < m; ++v)
            if (kept(v)) ++levp[lv[v] + 1];
        for (int l = 0; l < nl; ++l) levp[l + 1] += levp[l];
        rows.assign(nr, 0);
        std::vector<int32_t> fill(levp.begin(), levp.end() - 1);
        for (int32_t v : order)
            if (kept(v)) rows[fill[lv[v]]++] = v;
        const int32_t m = nr;
        ptr.assign(m + 1, 0);
        col.clear();
        val.clear();
        for (int32_t r = 0; r < m; ++r) {
            for (auto& e : ent[rows[r]]) {
                col.push_back(e.first);
                val.push_back(e.second);
            }
            ptr[r + 1] = (int32_t)col.size();
        }
    };
    schedule(lf, rowL, out.flev, out.frow, out.fptr, out.fcol, out.fval, {});
    // the dense tail: trailing forward levels of at most kPegpTailWidth rows
    const int nfl = (int)out.flev.size() - 1;
    int lt = nfl;
    int32_t nd = 0;
    while (lt > 0) {
        const int32_t wdt = out.flev[lt] - out.flev[lt - 1];
        if (wdt > kPegpTailWidth || nd + wdt > kPegpMaxDense) break;
        nd += wdt;
        --lt;
    }
    if (nd < kPegpMinDense || env_or("LAPGPU_PEGP_DENSE", 1) == 0) {
        nd = 0;
        lt = nfl;
    }
    std::vector<int32_t> tpos(m, -1);
    out.nd = nd;
    const int32_t ndp = (nd + kPegpTailBlock - 1) / kPegpTailBlock * kPegpTailBlock;
    out.ndp = ndp;
    out.drow.assign(out.frow.begin() + out.flev[lt], out.frow.begin() + out.flev[nfl]);
    for (int32_t p = 0; p < nd; ++p) tpos[out.drow[p]] = p;
    out.dlr.assign((size_t)ndp * ndp, 0.0);
    out.dlc.assign((size_t)ndp * ndp, 0.0);
    out.dd.assign(ndp, 1.0);
    for (int32_t p = 0; p < nd; ++p) out.dd[p] = out.diag[out.drow[p]];
    out.dcptr.assign(nd + 1, 0);
    for (int32_t p = 0; p < nd; ++p) {
        for (auto& e : rowL[out.drow[p]]) {
            const int32_t q = tpos[e.first];
            if (q >= 0) {
                // dependencies lie on earlier levels: earlier tail positions
                if (q >= p) return kInval;
                out.dlr[(size_t)p * ndp + q] = e.second;
                out.dlc[(size_t)q * ndp + p] = e.second;
            } else {
                out.dccol.push_back(e.first);
                out.dcval.push_back(e.second);
            }
        }
        out.dcptr[p + 1] = (int32_t)out.dccol.size();
    }
    out.flev.resize(lt + 1);
    // backward levels of the other rows, counted over their dependencies on
    // each other only: the tail is solved first, and its contributions to
    // the other rows are applied in one pass before the levels
    std::vector<char> keep;
    const std::vector<std::vector<std::pair<int32_t, double>>>* bent = &colL;
    std::vector<std::vector<std::pair<int32_t, double>>> colN;
    if (nd > 0) {
        keep.assign(m, 1);
        for (int32_t p = 0; p < nd; ++p) keep[out.drow[p]] = 0;
        colN.resize(m);
        out.bcptr.assign(1, 0);
        for (int32_t v = 0; v < m; ++v) {
            if (!keep[v]) continue;
            const size_t k0 = out.bccol.size();
            for (auto& e : colL[v]) {
                if (keep[e.first]) {
                    colN[v].push_back(e);
                } else {
                    out.bccol.push_back(tpos[e.first]);
                    out.bcval.push_back(e.second);
                }
            }
            if (out.bccol.size() > k0) {
                out.bcrow.push_back(v);
                out.bcptr.push_back((int32_t)out.bccol.size());
            }
        }
        bent = &colN;
        std::fill(lb.begin(), lb.end(), 0);
        for (auto it = order.rbegin(); it != order.rend(); ++it) {
            if (!keep[*it]) continue;
            int d = 0;
            for (auto& e : colN[*it]) d = std::max(d, lb[e.first] + 1);
            lb[*it] = d;
        }
    }
    schedule(lb, *bent, out.blev, out.brow, out.bptr, out.bcol, out.bval, keep);
    // lanes per row of every level and coupling pass
    out.flg.resize(out.flev.size() - 1);
    for (size_t l = 0; l + 1 < out.flev.size(); ++l)
        out.flg[l] = pegp_lanes(out.fptr, out.flev[l], out.flev[l + 1]);
    out.blg.resize(out.blev.size() - 1);
    for (size_t l = 0; l + 1 < out.blev.size(); ++l)
        out.blg[l] = pegp_lanes(out.bptr, out.blev[l], out.blev[l + 1]);
    if (!pegp_pack(out.flev, out.flg, out.fptr, out.fcol, out.fval, out.fdesc, out.fpval,
                   out.fpcol) ||
        !pegp_pack(out.blev, out.blg, out.bptr, out.bcol, out.bval, out.bdesc, out.bpval,
                   out.bpcol))
        return kUnsupported;
    if (P.lv[0].g.n <= kPegpOpMax && env_or("LAPGPU_PEGP_OPERATOR", 1) != 0)
        pegp_operator(P, out.off, par, order, rowL, colL, out.diag, out);
    return kOk;
}

}  // namespace lapgpu
