// graph.hip -- the resident data graph G and its label index.
//
// G is undirected, vertex-labelled and simple (Section II-A).  It stays in HBM
// as CSR for the lifetime of the handle.  The label index groups the vertices
// by label and orders each group by degree descending, then id ascending, so
// that the label-and-degree candidate filter of a query vertex u
// (l(v) = l(u), d(v) >= d_q(u)) is a prefix of u's label group, and a vertex's
// rank inside its group decides membership in one comparison.
#include <hipcub/hipcub.hpp>

#include "internal.h"

enum : int {
    BAD_ROWPTR = 1,
    BAD_COL_RANGE = 2,
    BAD_SELF_LOOP = 4,
    BAD_UNSORTED = 8,
    BAD_ASYMMETRIC = 16,
    BAD_LABEL = 32,
};

__global__ void k_check_rows(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ label, int64_t n,
                             int64_t nnz, int* __restrict__ err, unsigned long long* __restrict__ max_deg,
                             int* __restrict__ max_label) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long md = 0;
    int ml = -1;
    int bad = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += stride) {
        int64_t r = row_ptr[v];
        if (v == 0 && r != 0) bad |= BAD_ROWPTR;
        if (v == n) {
            if (r != nnz) bad |= BAD_ROWPTR;
            continue;
        }
        int64_t r1 = row_ptr[v + 1];
        if (r1 < r || r1 > nnz) {
            bad |= BAD_ROWPTR;
            continue;
        }
        unsigned long long d = (unsigned long long)(r1 - r);
        md = d > md ? d : md;
        int l = label[v];
        if (l < 0) bad |= BAD_LABEL;
        ml = l > ml ? l : ml;
    }
    if (bad) atomicOr(err, bad);
    atomicMax(max_deg, md);
    atomicMax(max_label, ml);
}

__device__ inline bool row_contains(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col, int64_t v,
                                    int32_t x) {
    int64_t lo = row_ptr[v], hi = row_ptr[v + 1];
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        int32_t y = col[mid];
        if (y == x) return true;
        if (y < x) lo = mid + 1;
        else hi = mid;
    }
    return false;
}

// One thread per stored edge: range, no self-loop, strictly increasing row, symmetric.
__global__ void k_check_edges(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col, int64_t n,
                              int64_t nnz, int* __restrict__ err) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
        // source vertex: last v with row_ptr[v] <= e
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            int64_t mid = (lo + hi + 1) >> 1;
            if (row_ptr[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        int64_t s = lo;
        int32_t w = col[e];
        if (w < 0 || (int64_t)w >= n) {
            bad |= BAD_COL_RANGE;
            continue;
        }
        if ((int64_t)w == s) bad |= BAD_SELF_LOOP;
        if (e > row_ptr[s] && col[e - 1] >= w) bad |= BAD_UNSORTED;
        if (!row_contains(row_ptr, col, w, (int32_t)s)) bad |= BAD_ASYMMETRIC;
    }
    if (bad) atomicOr(err, bad);
}

__global__ void k_make_keys(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ label, int64_t n,
                            uint64_t* __restrict__ keys, int32_t* __restrict__ ids,
                            unsigned long long* __restrict__ hist) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        uint64_t d = (uint64_t)(row_ptr[v + 1] - row_ptr[v]);
        uint64_t l = (uint64_t)label[v];
        // ascending key = label, then degree descending; the stable sort keeps ids ascending
        keys[v] = (l << 32) | (0xFFFFFFFFull - (d > 0xFFFFFFFFull ? 0xFFFFFFFFull : d));
        ids[v] = (int32_t)v;
        atomicAdd(&hist[l], 1ull);
    }
}

__global__ void k_perm_degrees(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ perm, int64_t n,
                               int64_t* __restrict__ out) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        int32_t v = perm[i];
        out[i] = row_ptr[v + 1] - row_ptr[v];
    }
}

__global__ void k_ranks(const int32_t* __restrict__ perm, const int32_t* __restrict__ label,
                        const int64_t* __restrict__ label_ptr, int64_t n, uint64_t* __restrict__ lab_rank) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        int32_t v = perm[i];
        uint64_t l = (uint64_t)label[v];
        lab_rank[v] = (l << 32) | (uint64_t)(i - label_ptr[l]);
    }
}

// deg_at_least[l][d]: the label groups are degree-descending, so a binary search finds the cut.
__global__ void k_deg_at_least(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ perm,
                               const int64_t* __restrict__ label_ptr, int32_t num_labels,
                               int64_t* __restrict__ out) {
    int64_t total = (int64_t)num_labels * (CSTM_MAX_K + 1);
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        int64_t l = t / (CSTM_MAX_K + 1);
        int64_t d = t % (CSTM_MAX_K + 1);
        int64_t lo = label_ptr[l], hi = label_ptr[l + 1];
        int64_t base = lo;
        while (lo < hi) {  // first position with degree < d
            int64_t mid = lo + ((hi - lo) >> 1);
            int32_t v = perm[mid];
            if (row_ptr[v + 1] - row_ptr[v] >= d) lo = mid + 1;
            else hi = mid;
        }
        out[t] = lo - base;
    }
}

extern "C" cstm_status cstm_graph_load(cstm_ctx* ctx, int64_t n, int64_t nnz, const int64_t* row_ptr,
                                       const int32_t* col, const int32_t* label, int on_device, void* stream,
                                       cstm_graph** out) {
    cstm_graph* g = nullptr;
    cstm_status st = cstm_guard([&] {
        CSTM_REQUIRE(ctx && out, CSTM_EINVAL, "NULL argument");
        *out = nullptr;
        CSTM_REQUIRE(n >= 0 && n < ((int64_t)1 << 31), CSTM_EINVAL, "n must be in [0, 2^31)");
        CSTM_REQUIRE(nnz >= 0, CSTM_EINVAL, "nnz must be >= 0");
        CSTM_REQUIRE(row_ptr && (nnz == 0 || col) && (n == 0 || label), CSTM_EINVAL, "NULL graph array");
        HIP_TRY(hipSetDevice(ctx->device));
        hipStream_t s = (hipStream_t)stream;
        g = new cstm_graph();
        g->ctx = ctx;
        g->mem.ctx = ctx;
        g->n = n;
        g->nnz = nnz;
        if (on_device) {
            g->row_ptr = row_ptr;
            g->col = col;
            g->label = label;
        } else {
            int64_t* rp = g->mem.get_n<int64_t>(n + 1);
            int32_t* cl = g->mem.get_n<int32_t>(nnz ? nnz : 1);
            int32_t* lb = g->mem.get_n<int32_t>(n ? n : 1);
            HIP_TRY(hipMemcpyAsync(rp, row_ptr, (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
            if (nnz) HIP_TRY(hipMemcpyAsync(cl, col, nnz * sizeof(int32_t), hipMemcpyHostToDevice, s));
            if (n) HIP_TRY(hipMemcpyAsync(lb, label, n * sizeof(int32_t), hipMemcpyHostToDevice, s));
            g->row_ptr = rp;
            g->col = cl;
            g->label = lb;
        }
        // validation
        struct Flags {
            int err;
            int max_label;
            unsigned long long max_deg;
        };
        Flags* f = g->mem.get_n<Flags>(1);
        Flags init{0, -1, 0};
        HIP_TRY(hipMemcpyAsync(f, &init, sizeof(Flags), hipMemcpyHostToDevice, s));
        k_check_rows<<<cstm_blocks(n + 1, 256, 4096), 256, 0, s>>>(g->row_ptr, g->label, n, nnz, &f->err, &f->max_deg,
                                                                   &f->max_label);
        HIP_TRY(hipGetLastError());
        Flags got;
        HIP_TRY(hipMemcpyAsync(&got, f, sizeof(Flags), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        CSTM_REQUIRE(!(got.err & BAD_ROWPTR), CSTM_EINVAL, "row_ptr is not a valid CSR offset array");
        CSTM_REQUIRE(!(got.err & BAD_LABEL), CSTM_EINVAL, "negative vertex label");
        if (nnz) {
            k_check_edges<<<cstm_blocks(nnz, 256, 16384), 256, 0, s>>>(g->row_ptr, g->col, n, nnz, &f->err);
            HIP_TRY(hipGetLastError());
            HIP_TRY(hipMemcpyAsync(&got, f, sizeof(Flags), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
        CSTM_REQUIRE(!(got.err & BAD_COL_RANGE), CSTM_EINVAL, "column index out of range");
        CSTM_REQUIRE(!(got.err & BAD_SELF_LOOP), CSTM_EINVAL, "self-loop in G");
        CSTM_REQUIRE(!(got.err & BAD_UNSORTED), CSTM_EINVAL, "CSR row not strictly increasing (unsorted or duplicate)");
        CSTM_REQUIRE(!(got.err & BAD_ASYMMETRIC), CSTM_EINVAL, "CSR is not symmetric (G must be undirected)");
        CSTM_REQUIRE(got.max_label < (1 << 26), CSTM_EINVAL, "labels must be below 2^26");
        g->max_degree = (int64_t)got.max_deg;
        g->num_labels = got.max_label + 1;
        const int32_t L = g->num_labels;
        // label index
        g->perm = g->mem.get_n<int32_t>(n ? n : 1);
        g->lab_rank = g->mem.get_n<uint64_t>(n ? n : 1);
        g->label_ptr.assign((size_t)L + 1, 0);
        g->deg_at_least.assign((size_t)(L > 0 ? L : 0) * (CSTM_MAX_K + 1), 0);
        if (n > 0) {
            uint64_t* keys = g->mem.get_n<uint64_t>(n);
            uint64_t* keys2 = g->mem.get_n<uint64_t>(n);
            int32_t* ids = g->mem.get_n<int32_t>(n);
            unsigned long long* hist = g->mem.get_n<unsigned long long>(L);
            HIP_TRY(hipMemsetAsync(hist, 0, (size_t)L * 8, s));
            k_make_keys<<<cstm_blocks(n, 256, 16384), 256, 0, s>>>(g->row_ptr, g->label, n, keys, ids, hist);
            HIP_TRY(hipGetLastError());
            int end_bit = 32;
            while (end_bit < 64 && ((uint64_t)L >> (end_bit - 32)) > 0) ++end_bit;
            size_t tb = 0;
            std::lock_guard<std::mutex> lk(ctx->scratch_mu);
            HIP_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, keys, keys2, ids, g->perm, (int)n, 0, end_bit, s));
            void* tmp = ctx->scratch(tb);
            HIP_TRY(hipcub::DeviceRadixSort::SortPairs(tmp, tb, keys, keys2, ids, g->perm, (int)n, 0, end_bit, s));
            std::vector<unsigned long long> h((size_t)L);
            HIP_TRY(hipMemcpyAsync(h.data(), hist, (size_t)L * 8, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            for (int32_t l = 0; l < L; ++l) g->label_ptr[l + 1] = g->label_ptr[l] + (int64_t)h[l];
            int64_t* lp = g->mem.get_n<int64_t>((size_t)L + 1);
            HIP_TRY(hipMemcpyAsync(lp, g->label_ptr.data(), ((size_t)L + 1) * 8, hipMemcpyHostToDevice, s));
            k_ranks<<<cstm_blocks(n, 256, 16384), 256, 0, s>>>(g->perm, g->label, lp, n, g->lab_rank);
            HIP_TRY(hipGetLastError());
            int64_t* dal = g->mem.get_n<int64_t>(g->deg_at_least.size());
            k_deg_at_least<<<cstm_blocks((int64_t)g->deg_at_least.size(), 256, 4096), 256, 0, s>>>(
                g->row_ptr, g->perm, lp, L, dal);
            HIP_TRY(hipGetLastError());
            HIP_TRY(hipMemcpyAsync(g->deg_at_least.data(), dal, g->deg_at_least.size() * 8, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            // degree prefix sums in label-index order, for footprint estimates
            int64_t* pd = (int64_t*)keys;  // n int64 entries, free again
            int64_t* ps = (int64_t*)keys2;
            k_perm_degrees<<<cstm_blocks(n, 256, 16384), 256, 0, s>>>(g->row_ptr, g->perm, n, pd);
            HIP_TRY(hipGetLastError());
            HIP_TRY(hipStreamSynchronize(s));
            g->deg_prefix.assign((size_t)n + 1, 0);
            {
                size_t tb2 = 0;
                HIP_TRY(hipcub::DeviceScan::InclusiveSum(nullptr, tb2, pd, ps, (int)n, s));
                void* tmp2 = ctx->scratch(tb2);
                HIP_TRY(hipcub::DeviceScan::InclusiveSum(tmp2, tb2, pd, ps, (int)n, s));
                HIP_TRY(hipMemcpyAsync(g->deg_prefix.data() + 1, ps, (size_t)n * 8, hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
            }
            g->mem.release(keys);
            g->mem.release(keys2);
            g->mem.release(ids);
            g->mem.release(hist);
            g->mem.release(dal);
        }
        *out = g;
    });
    if (st != CSTM_OK && g) delete g;
    return st;
}

extern "C" cstm_status cstm_cst_estimate(const cstm_graph* g, int32_t k, const int32_t* qlabel, int32_t m_q,
                                         const int32_t* qedges, uint64_t* bytes_out) {
    return cstm_guard([&] {
        CSTM_REQUIRE(g && bytes_out, CSTM_EINVAL, "NULL argument");
        CSTM_REQUIRE(k >= 1 && k <= CSTM_MAX_K && qlabel, CSTM_EINVAL, "bad query");
        CSTM_REQUIRE(m_q >= 0 && (m_q == 0 || qedges), CSTM_EINVAL, "bad query edges");
        int deg[CSTM_MAX_K] = {};
        for (int e = 0; e < m_q; ++e) {
            int a = qedges[2 * e], b = qedges[2 * e + 1];
            CSTM_REQUIRE(a >= 0 && a < k && b >= 0 && b < k && a != b, CSTM_EINVAL, "bad query edge");
            deg[a]++;
            deg[b]++;
        }
        int64_t c0[CSTM_MAX_K];
        uint64_t sdeg[CSTM_MAX_K];
        uint64_t bytes = 0, max_c0 = 0;
        for (int u = 0; u < k; ++u) {
            CSTM_REQUIRE(qlabel[u] >= 0, CSTM_EINVAL, "negative query label");
            c0[u] = g->count_ge(qlabel[u], deg[u]);
            sdeg[u] = 0;
            if (c0[u] > 0) {
                int64_t lo = g->label_ptr[qlabel[u]];
                sdeg[u] = (uint64_t)(g->deg_prefix[lo + c0[u]] - g->deg_prefix[lo]);
            }
            if ((uint64_t)c0[u] > max_c0) max_c0 = (uint64_t)c0[u];
            // candidate array and rank table (C(u) is a subset of the filtered label prefix)
            bytes += 8ull * (uint64_t)c0[u];
        }
        // scan, flag, per-owner counts and the path-count vectors of one leaf path
        bytes += (24ull + 8ull * (uint64_t)k) * (max_c0 + 1);
        // every candidate edge list: offsets over its owner, entries (ids and, for
        // non-tree lists, global ids); an edge (v, w) with v in C(a), w in C(b)
        // appears once, so either side's degree sum bounds the entries
        for (int e = 0; e < m_q; ++e) {
            int a = qedges[2 * e], b = qedges[2 * e + 1];
            uint64_t ent = sdeg[a] < sdeg[b] ? sdeg[a] : sdeg[b];
            bytes += 8ull * (max_c0 + 1) + 8ull * ent;
        }
        *bytes_out = bytes + 4096;  // descriptor and small flags
    });
}

extern "C" void cstm_graph_free(cstm_graph* g) {
    if (!g) return;
    (void)hipSetDevice(g->ctx->device);
    (void)hipDeviceSynchronize();
    delete g;
}

extern "C" cstm_status cstm_graph_info(const cstm_graph* g, int64_t* n, int64_t* nnz, int32_t* num_labels,
                                       int64_t* max_degree) {
    return cstm_guard([&] {
        CSTM_REQUIRE(g, CSTM_EINVAL, "NULL graph");
        if (n) *n = g->n;
        if (nnz) *nnz = g->nnz;
        if (num_labels) *num_labels = g->num_labels;
        if (max_degree) *max_degree = g->max_degree;
    });
}
