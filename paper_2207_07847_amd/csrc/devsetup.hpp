// Graph construction of the setup on the device: the symmetric adjacency of
// the input edge list and the Galerkin coarse graph P^T L P of each
// aggregation step (Sec. 2.2), with the same outputs as the host's
// build_adjacency and coarse_graph, bit for bit.  Both are a stable radix
// sort of (row, column) keys followed by a sum over each run of equal keys
// in the order the host sums them (edges in input order; fine entries in
// CSR order), so every weight is the same double.  The visit-order matching
// of Sec. 2.2 between the two stays on the host (it is sequential by
// definition); the locally dominant matching of the parallel setup runs
// here, in rounds of a thread per vertex.
//
// Included by lap.hip inside its own namespace, after HIPCHK (and
// hipcub at global scope).
#pragma once

constexpr uint64_t kKeyNone = ~0ull;   // sorts after every (row, column) key

__global__ void k_adj_keys(int64_t m, const int64_t* __restrict__ u,
                           const int64_t* __restrict__ v, uint64_t* __restrict__ key,
                           uint32_t* __restrict__ val) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const uint64_t a = (uint64_t)u[e], b = (uint64_t)v[e];
    key[2 * e] = a << 32 | b;
    key[2 * e + 1] = b << 32 | a;
    val[2 * e] = (uint32_t)e;
    val[2 * e + 1] = (uint32_t)e;
}

// head[i] = 1 where a run of equal keys starts (kKeyNone never starts one)
__global__ void k_run_heads(int64_t N, const uint64_t* __restrict__ key,
                            int32_t* __restrict__ head) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    head[i] = key[i] != kKeyNone && (i == 0 || key[i] != key[i - 1]);
}

// For each run start i: output pos[i] gets the column (low half of the key)
// and the weights of the run summed left to right, w[val[i]] first; the row
// (high half) is counted.
__global__ void k_run_sums(int64_t N, const uint64_t* __restrict__ key,
                           const uint32_t* __restrict__ val, const int32_t* __restrict__ head,
                           const int32_t* __restrict__ pos, const double* __restrict__ w,
                           int32_t* __restrict__ col, double* __restrict__ wout,
                           unsigned long long* __restrict__ rowcnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N || !head[i]) return;
    const uint64_t k = key[i];
    double s = w[val[i]];
    for (int64_t t = i + 1; t < N && key[t] == k; ++t) s += w[val[t]];
    const int32_t j = pos[i];
    col[j] = (int32_t)(k & 0xffffffffu);
    wout[j] = s;
    atomicAdd(&rowcnt[k >> 32], 1ull);
}

// Upper-triangle coarse keys of the fine entries: entry k of row i with
// column j > i between different aggregates gives (lo, hi) = the two
// aggregates ordered; every other entry gives kKeyNone.  val = k (CSR order).
__global__ void k_coarse_keys(int64_t n, int64_t nnz, const int64_t* __restrict__ ptr,
                              const int32_t* __restrict__ col, const int32_t* __restrict__ agg,
                              uint64_t* __restrict__ key, uint32_t* __restrict__ val) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    // row of entry k: the last i with ptr[i] <= k
    int64_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (ptr[mid] <= k) lo = mid;
        else hi = mid;
    }
    const int64_t i = lo;
    const int32_t j = col[k];
    uint64_t out = kKeyNone;
    if (j > i && agg[i] != agg[j]) {
        const uint64_t a = (uint64_t)min(agg[i], agg[j]), b = (uint64_t)max(agg[i], agg[j]);
        out = a << 32 | b;
    }
    key[k] = out;
    val[k] = (uint32_t)k;
}

// The symmetric coarse entries of the U unique upper pairs (sorted keys
// ukey, weights uw): both directions, val = the pair's index.
__global__ void k_coarse_mirror(int64_t U, const uint64_t* __restrict__ ukey,
                                uint64_t* __restrict__ key, uint32_t* __restrict__ val) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= U) return;
    const uint64_t k = ukey[p];
    key[2 * p] = k;
    key[2 * p + 1] = (k & 0xffffffffu) << 32 | k >> 32;
    val[2 * p] = (uint32_t)p;
    val[2 * p + 1] = (uint32_t)p;
}

// Entry q of the symmetric CSR: column and weight of its pair; rows counted.
__global__ void k_coarse_fill(int64_t N, const uint64_t* __restrict__ key,
                              const uint32_t* __restrict__ val, const double* __restrict__ uw,
                              int32_t* __restrict__ col, double* __restrict__ w,
                              unsigned long long* __restrict__ rowcnt) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    const uint64_t k = key[q];
    col[q] = (int32_t)(k & 0xffffffffu);
    w[q] = uw[val[q]];
    atomicAdd(&rowcnt[k >> 32], 1ull);
}

// Upper pairs from sorted (key, val = fine entry) runs: key and summed weight.
__global__ void k_coarse_runs(int64_t N, const uint64_t* __restrict__ key,
                              const uint32_t* __restrict__ val, const int32_t* __restrict__ head,
                              const int32_t* __restrict__ pos, const double* __restrict__ fw,
                              uint64_t* __restrict__ ukey, double* __restrict__ uw) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N || !head[i]) return;
    const uint64_t k = key[i];
    double s = fw[val[i]];
    for (int64_t t = i + 1; t < N && key[t] == k; ++t) s += fw[val[t]];
    ukey[pos[i]] = k;
    uw[pos[i]] = s;
}

// Locally dominant matching (the host's match_locally_dominant, bit for
// bit).  One round: every free vertex points at its heaviest free
// neighbour (neighbours ascending: the first maximum is the smaller id)...
// Rows longer than this are scanned by a wavefront (k_ld_point_heavy).
constexpr int kLdHeavy = 64;

__global__ void k_ld_point(int64_t n, const int64_t* __restrict__ ptr,
                           const int32_t* __restrict__ col, const double* __restrict__ w,
                           const int32_t* __restrict__ mate, int32_t* __restrict__ best) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n || ptr[v + 1] - ptr[v] > kLdHeavy) return;
    int32_t pick = -1;
    if (mate[v] < 0) {
        double pw = -1.0;
        for (int64_t k = ptr[v]; k < ptr[v + 1]; ++k) {
            const int32_t nb = col[k];
            if (mate[nb] >= 0) continue;
            if (w[k] > pw) {
                pw = w[k];
                pick = nb;
            }
        }
    }
    best[v] = pick;
}

// The heaviest (free) neighbour of heavy vertex hv[i] by a wavefront: lanes
// stride over the row, then the (weight, id) maxima are combined, larger
// weight first, then the smaller id.
__device__ inline void ld_wave_best(const int64_t* __restrict__ ptr,
                                    const int32_t* __restrict__ col,
                                    const double* __restrict__ w,
                                    const int32_t* __restrict__ mate, int64_t v, bool free_only,
                                    int lane, double& pw, int32_t& pick) {
    pw = -1.0;
    pick = -1;
    for (int64_t k = ptr[v] + lane; k < ptr[v + 1]; k += 64) {
        const int32_t nb = col[k];
        if (free_only && mate[nb] >= 0) continue;
        if (w[k] > pw) {  // a lane's columns ascend: its first maximum is its smallest id
            pw = w[k];
            pick = nb;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double ow = __shfl_xor(pw, off, 64);
        const int32_t op = __shfl_xor(pick, off, 64);
        if (ow > pw || (ow == pw && op >= 0 && (pick < 0 || op < pick))) {
            pw = ow;
            pick = op;
        }
    }
}

__global__ void k_ld_point_heavy(int64_t nh, const int32_t* __restrict__ hv,
                                 const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                 const double* __restrict__ w, const int32_t* __restrict__ mate,
                                 int32_t* __restrict__ best) {
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (i >= nh) return;
    const int64_t v = hv[i];
    if (mate[v] >= 0) {
        if (lane == 0) best[v] = -1;
        return;
    }
    double pw;
    int32_t pick;
    ld_wave_best(ptr, col, w, mate, v, true, lane, pw, pick);
    if (lane == 0) best[v] = pick;
}

// ... and two vertices pointing at each other pair up (each writes its own
// mate); `changed` counts the vertices paired in the round.
__global__ void k_ld_pair(int64_t n, const int32_t* __restrict__ best, int32_t* __restrict__ mate,
                          unsigned int* __restrict__ changed) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t u = best[v];
    if (u >= 0 && best[u] == (int32_t)v) {
        mate[v] = u;
        atomicAdd(changed, 1u);
    }
}

// flag[v] = 1 where v is the smaller end of its pair
__global__ void k_ld_first(int64_t n, const int32_t* __restrict__ mate,
                           int32_t* __restrict__ flag) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) flag[v] = mate[v] > (int32_t)v;
}

// Aggregates: a pair's id is the rank of its smaller end (id = exclusive
// scan of flag); a vertex left free joins its heaviest neighbour's.
__global__ void k_ld_agg(int64_t n, const int64_t* __restrict__ ptr,
                         const int32_t* __restrict__ col, const double* __restrict__ w,
                         const int32_t* __restrict__ mate, const int32_t* __restrict__ id,
                         int32_t* __restrict__ agg, int8_t* __restrict__ matched) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t m = mate[v];
    if (m >= 0) {
        agg[v] = id[min((int32_t)v, m)];
        matched[v] = 1;
        return;
    }
    if (ptr[v + 1] - ptr[v] > kLdHeavy) return;  // k_ld_agg_heavy
    int32_t pick = -1;
    double pw = -1.0;
    for (int64_t k = ptr[v]; k < ptr[v + 1]; ++k)
        if (w[k] > pw) {
            pw = w[k];
            pick = col[k];
        }
    // the matching is maximal: every neighbour of a free vertex is paired
    agg[v] = id[min(pick, mate[pick])];
    matched[v] = 0;
}

__global__ void k_ld_agg_heavy(int64_t nh, const int32_t* __restrict__ hv,
                               const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                               const double* __restrict__ w, const int32_t* __restrict__ mate,
                               const int32_t* __restrict__ id, int32_t* __restrict__ agg,
                               int8_t* __restrict__ matched) {
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (i >= nh) return;
    const int64_t v = hv[i];
    if (mate[v] >= 0) return;  // paired: k_ld_agg
    double pw;
    int32_t pick;
    ld_wave_best(ptr, col, w, mate, v, false, lane, pw, pick);
    if (lane == 0) {
        agg[v] = id[min(pick, mate[pick])];
        matched[v] = 0;
    }
}

class DeviceGraphBuilder : public GraphBuilder {
  public:
    explicit DeviceGraphBuilder(hipStream_t s) : s_(s) {}
    ~DeviceGraphBuilder() override {
        for (void* p : owned_) (void)hipFree(p);
    }

    int adjacency(int64_t n, int64_t m, const int64_t* u, const int64_t* v, const double* w,
                  Adjacency& out) override {
        if (validate_edges(n, m, u, v, w) != kOk) return kInval;
        const int64_t N = 2 * m;
        if (N > (int64_t)INT32_MAX || m > (int64_t)UINT32_MAX) return build_adjacency(n, m, u, v, w, out);
        const size_t mark = owned_.size();
        int64_t* du = up(u, m);
        int64_t* dv = up(v, m);
        double* dw = up(w, m);
        uint64_t *k0 = alloc<uint64_t>(N), *k1 = alloc<uint64_t>(N);
        uint32_t *v0 = alloc<uint32_t>(N), *v1 = alloc<uint32_t>(N);
        hipLaunchKernelGGL(k_adj_keys, dim3(blocks(m)), dim3(kB), 0, s_, m, (const int64_t*)du,
                           (const int64_t*)dv, k0, v0);
        sort_pairs(k0, k1, v0, v1, N, 32 + bits(n));
        runs_to_csr(n, N, k1, v1, dw, out);
        release(mark);
        return kOk;
    }

    void coarse(const Adjacency& f, const std::vector<int64_t>& agg, int64_t nc,
                Adjacency& c) override {
        const int64_t nnz = f.nnz();
        if (nnz > (int64_t)INT32_MAX) {
            coarse_graph(f, agg, nc, c);
            return;
        }
        const size_t mark = owned_.size();
        std::vector<int32_t> a32(agg.begin(), agg.end());
        int64_t* dptr = up(f.ptr.data(), f.n + 1);
        int32_t* dcol = up(f.col.data(), nnz);
        double* dfw = up(f.w.data(), nnz);
        int32_t* dagg = up(a32.data(), f.n);
        uint64_t *k0 = alloc<uint64_t>(nnz), *k1 = alloc<uint64_t>(nnz);
        uint32_t *v0 = alloc<uint32_t>(nnz), *v1 = alloc<uint32_t>(nnz);
        hipLaunchKernelGGL(k_coarse_keys, dim3(blocks(nnz)), dim3(kB), 0, s_, f.n, nnz,
                           (const int64_t*)dptr, (const int32_t*)dcol, (const int32_t*)dagg, k0,
                           v0);
        sort_pairs(k0, k1, v0, v1, nnz, 64);
        int32_t *head = alloc<int32_t>(nnz), *pos = alloc<int32_t>(nnz);
        const int64_t U = heads(nnz, k1, head, pos);
        uint64_t* ukey = alloc<uint64_t>(std::max<int64_t>(U, 1));
        double* uw = alloc<double>(std::max<int64_t>(U, 1));
        hipLaunchKernelGGL(k_coarse_runs, dim3(blocks(nnz)), dim3(kB), 0, s_, nnz,
                           (const uint64_t*)k1, (const uint32_t*)v1, (const int32_t*)head,
                           (const int32_t*)pos, (const double*)dfw, ukey, uw);
        // both directions, sorted by (row, column)
        const int64_t N = 2 * U;
        uint64_t *m0 = alloc<uint64_t>(std::max<int64_t>(N, 1)), *m1 = alloc<uint64_t>(std::max<int64_t>(N, 1));
        uint32_t *mv0 = alloc<uint32_t>(std::max<int64_t>(N, 1)), *mv1 = alloc<uint32_t>(std::max<int64_t>(N, 1));
        if (U > 0) {
            hipLaunchKernelGGL(k_coarse_mirror, dim3(blocks(U)), dim3(kB), 0, s_, U,
                               (const uint64_t*)ukey, m0, mv0);
            sort_pairs(m0, m1, mv0, mv1, N, 32 + bits(nc));
        }
        int32_t* ccol = alloc<int32_t>(std::max<int64_t>(N, 1));
        double* cw = alloc<double>(std::max<int64_t>(N, 1));
        unsigned long long* cnt = alloc<unsigned long long>(nc + 1);
        HIPCHK(hipMemsetAsync(cnt, 0, (nc + 1) * sizeof(unsigned long long), s_));
        if (N > 0)
            hipLaunchKernelGGL(k_coarse_fill, dim3(blocks(N)), dim3(kB), 0, s_, N,
                               (const uint64_t*)m1, (const uint32_t*)mv1, (const double*)uw, ccol,
                               cw, cnt);
        finish_csr(nc, N, cnt, ccol, cw, c);
        release(mark);
    }

    bool match(const Adjacency& g, std::vector<int64_t>& agg, std::vector<int8_t>& matched,
               int64_t& nc) override {
        const int64_t n = g.n, nnz = g.nnz();
        if (n < 2 || n > (int64_t)INT32_MAX || nnz > (int64_t)INT32_MAX) return false;
        const size_t mark = owned_.size();
        int64_t* dptr = up(g.ptr.data(), n + 1);
        int32_t* dcol = up(g.col.data(), nnz);
        double* dw = up(g.w.data(), nnz);
        int32_t* mate = alloc<int32_t>(n);
        int32_t* best = alloc<int32_t>(n);
        unsigned int* changed = alloc<unsigned int>(1);
        HIPCHK(hipMemsetAsync(mate, 0xff, (size_t)n * sizeof(int32_t), s_));  // -1: free
        // rows above kLdHeavy neighbours: a wavefront each
        std::vector<int32_t> heavy;
        for (int64_t v = 0; v < n; ++v)
            if (g.ptr[v + 1] - g.ptr[v] > kLdHeavy) heavy.push_back((int32_t)v);
        const int64_t nh = (int64_t)heavy.size();
        int32_t* dh = nh ? up(heavy.data(), nh) : nullptr;
        const int64_t hblocks = std::max<int64_t>(1, (nh * 64 + kB - 1) / kB);
        // rounds in batches of kLdBatch between checks: a round after the
        // last pairing changes nothing
        constexpr int kLdBatch = 4;
        unsigned int hc = 0;
        int rounds = 0;
        do {
            HIPCHK(hipMemsetAsync(changed, 0, sizeof(unsigned int), s_));
            for (int r = 0; r < kLdBatch; ++r) {
                hipLaunchKernelGGL(k_ld_point, dim3(blocks(n)), dim3(kB), 0, s_, n,
                                   (const int64_t*)dptr, (const int32_t*)dcol, (const double*)dw,
                                   (const int32_t*)mate, best);
                if (nh)
                    hipLaunchKernelGGL(k_ld_point_heavy, dim3(hblocks), dim3(kB), 0, s_, nh,
                                       (const int32_t*)dh, (const int64_t*)dptr,
                                       (const int32_t*)dcol, (const double*)dw,
                                       (const int32_t*)mate, best);
                hipLaunchKernelGGL(k_ld_pair, dim3(blocks(n)), dim3(kB), 0, s_, n,
                                   (const int32_t*)best, mate, changed);
            }
            rounds += kLdBatch;
            HIPCHK(hipMemcpyAsync(&hc, changed, sizeof(hc), hipMemcpyDeviceToHost, s_));
            HIPCHK(hipStreamSynchronize(s_));
        } while (hc != 0);
        if (std::getenv("LAPGPU_DEBUG"))
            std::fprintf(stderr, "[lapgpu] locally dominant matching: n %lld, %d rounds\n",
                         (long long)n, rounds);
        int32_t *flag = alloc<int32_t>(n), *id = alloc<int32_t>(n);
        hipLaunchKernelGGL(k_ld_first, dim3(blocks(n)), dim3(kB), 0, s_, n, (const int32_t*)mate,
                           flag);
        size_t tmp = 0;
        HIPCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp, flag, id, (int)n, s_));
        void* t = alloc<unsigned char>((int64_t)tmp);
        HIPCHK(hipcub::DeviceScan::ExclusiveSum(t, tmp, flag, id, (int)n, s_));
        int32_t* dagg = alloc<int32_t>(n);
        int8_t* dmt = alloc<int8_t>(n);
        hipLaunchKernelGGL(k_ld_agg, dim3(blocks(n)), dim3(kB), 0, s_, n, (const int64_t*)dptr,
                           (const int32_t*)dcol, (const double*)dw, (const int32_t*)mate,
                           (const int32_t*)id, dagg, dmt);
        if (nh)
            hipLaunchKernelGGL(k_ld_agg_heavy, dim3(hblocks), dim3(kB), 0, s_, nh,
                               (const int32_t*)dh, (const int64_t*)dptr, (const int32_t*)dcol,
                               (const double*)dw, (const int32_t*)mate, (const int32_t*)id,
                               dagg, dmt);
        std::vector<int32_t> a32(n);
        int32_t last[2];
        matched.resize(n);
        HIPCHK(hipMemcpyAsync(a32.data(), dagg, (size_t)n * sizeof(int32_t),
                              hipMemcpyDeviceToHost, s_));
        HIPCHK(hipMemcpyAsync(matched.data(), dmt, (size_t)n, hipMemcpyDeviceToHost, s_));
        HIPCHK(hipMemcpyAsync(&last[0], id + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s_));
        HIPCHK(hipMemcpyAsync(&last[1], flag + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s_));
        release(mark);
        agg.assign(a32.begin(), a32.end());
        nc = (int64_t)last[0] + last[1];
        return true;
    }

  private:
    static constexpr int kB = 256;
    hipStream_t s_;
    std::vector<void*> owned_;

    static int64_t blocks(int64_t items) { return std::max<int64_t>(1, (items + kB - 1) / kB); }
    static int bits(int64_t n) {
        int b = 1;
        while (b < 32 && ((int64_t)1 << b) < n) ++b;
        return b;
    }
    template <class T>
    T* alloc(int64_t count) {
        void* p = nullptr;
        HIPCHK(hipMalloc(&p, (size_t)std::max<int64_t>(count, 1) * sizeof(T)));
        owned_.push_back(p);
        return static_cast<T*>(p);
    }
    template <class T>
    T* up(const T* h, int64_t count) {
        T* d = alloc<T>(count);
        HIPCHK(hipMemcpyAsync(d, h, (size_t)count * sizeof(T), hipMemcpyHostToDevice, s_));
        return d;
    }
    void release(size_t mark) {
        HIPCHK(hipStreamSynchronize(s_));
        while (owned_.size() > mark) {
            (void)hipFree(owned_.back());
            owned_.pop_back();
        }
    }
    // stable LSD radix sort of (key, val) on key bits [0, end_bit)
    void sort_pairs(uint64_t* kin, uint64_t* kout, uint32_t* vin, uint32_t* vout, int64_t N,
                    int end_bit) {
        size_t tmp = 0;
        HIPCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, kin, kout, vin, vout, (int)N, 0,
                                                  end_bit, s_));
        void* t = alloc<unsigned char>((int64_t)tmp);
        HIPCHK(hipcub::DeviceRadixSort::SortPairs(t, tmp, kin, kout, vin, vout, (int)N, 0,
                                                  end_bit, s_));
    }
    // run starts of sorted keys and their output positions; the run count
    int64_t heads(int64_t N, const uint64_t* key, int32_t* head, int32_t* pos) {
        hipLaunchKernelGGL(k_run_heads, dim3(blocks(N)), dim3(kB), 0, s_, N, key, head);
        size_t tmp = 0;
        HIPCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp, head, pos, (int)N, s_));
        void* t = alloc<unsigned char>((int64_t)tmp);
        HIPCHK(hipcub::DeviceScan::ExclusiveSum(t, tmp, head, pos, (int)N, s_));
        int32_t last[2];
        HIPCHK(hipMemcpyAsync(&last[0], pos + N - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s_));
        HIPCHK(hipMemcpyAsync(&last[1], head + N - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s_));
        HIPCHK(hipStreamSynchronize(s_));
        return (int64_t)last[0] + last[1];
    }
    // CSR from sorted (row, column) runs: weights summed per run
    void runs_to_csr(int64_t n, int64_t N, const uint64_t* key, const uint32_t* val,
                     const double* w, Adjacency& out) {
        int32_t *head = alloc<int32_t>(N), *pos = alloc<int32_t>(N);
        const int64_t nnz = heads(N, key, head, pos);
        int32_t* col = alloc<int32_t>(nnz);
        double* wo = alloc<double>(nnz);
        unsigned long long* cnt = alloc<unsigned long long>(n + 1);
        HIPCHK(hipMemsetAsync(cnt, 0, (n + 1) * sizeof(unsigned long long), s_));
        hipLaunchKernelGGL(k_run_sums, dim3(blocks(N)), dim3(kB), 0, s_, N, key, val,
                           (const int32_t*)head, (const int32_t*)pos, w, col, wo, cnt);
        finish_csr(n, nnz, cnt, col, wo, out);
    }
    // row counts -> ptr; copy the CSR to the host
    void finish_csr(int64_t n, int64_t nnz, unsigned long long* cnt, const int32_t* col,
                    const double* w, Adjacency& out) {
        HIPCHK(hipGetLastError());
        std::vector<unsigned long long> c(n);
        HIPCHK(hipMemcpyAsync(c.data(), cnt, n * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, s_));
        out.n = n;
        out.ptr.assign(n + 1, 0);
        out.col.resize(nnz);
        out.w.resize(nnz);
        if (nnz > 0) {
            HIPCHK(hipMemcpyAsync(out.col.data(), col, nnz * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, s_));
            HIPCHK(hipMemcpyAsync(out.w.data(), w, nnz * sizeof(double), hipMemcpyDeviceToHost,
                                  s_));
        }
        HIPCHK(hipStreamSynchronize(s_));
        for (int64_t i = 0; i < n; ++i) out.ptr[i + 1] = out.ptr[i] + (int64_t)c[i];
    }
};
