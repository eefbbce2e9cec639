// graph.hip -- the resident data graph G and its label index.
//
// G is undirected, vertex-labelled and simple (Section II-A).  It stays in HBM
// as CSR for the lifetime of the handle.  The label index groups the vertices
// by label and orders each group by degree descending, then id ascending, so
// that the label-and-degree candidate filter of a query vertex u
// (l(v) = l(u), d(v) >= d_q(u)) is a prefix of u's label group, and a vertex's
// rank inside its group decides membership in one comparison.  A second copy
// of the rows holds each neighbour's packed key, with every row ordered by
// (label, id): the neighbours of one label are then one run, found by binary
// search, so CST construction reads only the run of the label it looks for.
// The index and the copy are built with the library's own radix sort and scan
// (prims.hip).
#include <algorithm>

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

// Sort key of vertex v: label, then degree descending (deg_bits bits hold
// the degree); the stable sort keeps ids ascending among equal keys.
__global__ void k_make_keys(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ label, int64_t n,
                            int deg_bits, uint64_t* __restrict__ keys, int32_t* __restrict__ ids,
                            unsigned long long* __restrict__ hist) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const uint64_t dmax = (1ull << deg_bits) - 1;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const uint64_t d = (uint64_t)(row_ptr[v + 1] - row_ptr[v]);
        const uint64_t l = (uint64_t)label[v];
        keys[v] = (l << deg_bits) | (dmax - d);
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

// Packed key of every vertex: (label << shift) | rank inside its label group.
template <class K>
__global__ void k_ranks(const int32_t* __restrict__ perm, const int32_t* __restrict__ label,
                        const int64_t* __restrict__ label_ptr, int64_t n, int shift, K* __restrict__ key) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int32_t v = perm[i];
        const int32_t l = label[v];
        key[v] = (K)(((K)l << shift) | (K)(i - label_ptr[l]));
    }
}

// Label-grouped rows, built one chunk of rows at a time.  Sort key of row
// entry j of row r: (r - r0, label of col[j]); the stable sort keeps the ids
// ascending inside each (row, label) run.  One wavefront per row.
template <class K>
__global__ void k_regroup_keys(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                               const K* __restrict__ key, int key_shift, int64_t r0, int64_t r1, int64_t base,
                               int label_bits, uint64_t* __restrict__ skey, int32_t* __restrict__ sval) {
    const int lane = threadIdx.x & (CSTM_WAVE - 1);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / CSTM_WAVE;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) / CSTM_WAVE;
    for (int64_t r = r0 + wave; r < r1; r += waves) {
        const uint64_t hi = (uint64_t)(r - r0) << label_bits;
        const int64_t e = row_ptr[r + 1];
        for (int64_t j = row_ptr[r] + lane; j < e; j += CSTM_WAVE) {
            skey[j - base] = hi | (uint64_t)(key[col[j]] >> key_shift);
            sval[j - base] = (int32_t)(j - base);
        }
    }
}

// Entry i of the chunk's sorted order: the key of the neighbour it came from.
template <class K>
__global__ void k_regroup_gather(const int32_t* __restrict__ col, const K* __restrict__ key, int64_t base,
                                 int64_t cnt, const int32_t* __restrict__ sval, K* __restrict__ lkey) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride)
        lkey[base + i] = key[col[base + sval[i]]];
}

// First row of every chunk: chunk c starts at the first row whose first entry
// is at or after c * chunk (out[nchunks] = n); rowbase[c] = row_ptr[out[c]].
__global__ void k_chunk_rows(const int64_t* __restrict__ row_ptr, int64_t n, int64_t chunk, int64_t nchunks,
                             int64_t* __restrict__ out, int64_t* __restrict__ rowbase) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= nchunks; c += stride) {
        int64_t r = n;
        if (c < nchunks) {
            const int64_t t = c * chunk;
            int64_t lo = 0, hi = n;
            while (lo < hi) {
                const int64_t mid = lo + ((hi - lo) >> 1);
                if (row_ptr[mid] < t) lo = mid + 1;
                else hi = mid;
            }
            r = lo;
        }
        out[c] = r;
        rowbase[c] = row_ptr[r];
    }
}

// Edges of G between each pair of labels: pair[a * L + b] counts the row
// entries (v, w) with l(v) = a and l(w) = b.  Each workgroup counts its rows
// (one wavefront per row) in an L x L table in LDS, then adds it to the
// global table.
constexpr int kPairMaxLabels = 128;  // L x L 32-bit counters fit in 64 KiB of LDS
template <class K>
__global__ __launch_bounds__(256) void k_pair_counts(const int64_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ label, const K* __restrict__ lkey,
                                                     int key_shift, int64_t n, int L,
                                                     unsigned long long* __restrict__ pair) {
    __shared__ uint32_t h[kPairMaxLabels * kPairMaxLabels];
    const int LL = L * L;
    for (int i = threadIdx.x; i < LL; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (CSTM_WAVE - 1);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / CSTM_WAVE;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) / CSTM_WAVE;
    for (int64_t v = wave; v < n; v += waves) {
        const int base = label[v] * L;
        const int64_t e = row_ptr[v + 1];
        for (int64_t j = row_ptr[v] + lane; j < e; j += CSTM_WAVE) atomicAdd(&h[base + (int)(lkey[j] >> key_shift)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < LL; i += blockDim.x)
        if (h[i]) atomicAdd(&pair[i], (unsigned long long)h[i]);
}

// Entries per radix sort of the regrouping (a longer row is sorted alone).
constexpr int64_t kRegroupChunk = (int64_t)1 << 28;

static int bits_for(uint64_t x) {  // bits needed to hold every value in [0, x]
    int b = 0;
    while (b < 64 && (x >> b) != 0) ++b;
    return b;
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

// The label-grouped copy of the rows (lkey32 or lkey64, allocated by the
// caller): every row's neighbour keys ordered by (label, id).
static void regroup_rows(cstm_graph* g, int label_bits, hipStream_t s) {
    const int64_t n = g->n, nnz = g->nnz;
    const int64_t nchunks = (nnz + kRegroupChunk - 1) / kRegroupChunk;
    std::vector<int64_t> rows((size_t)nchunks + 1), base((size_t)nchunks + 1);
    {
        int64_t* d = g->mem.get_n<int64_t>(2 * ((size_t)nchunks + 1));
        k_chunk_rows<<<cstm_blocks(nchunks + 1, 256, 64), 256, 0, s>>>(g->row_ptr, n, kRegroupChunk, nchunks, d,
                                                                       d + nchunks + 1);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(rows.data(), d, ((size_t)nchunks + 1) * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(base.data(), d + nchunks + 1, ((size_t)nchunks + 1) * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        g->mem.release(d);
    }
    for (int64_t c = 0; c < nchunks; ++c) {
        const int64_t r0 = rows[(size_t)c], r1 = rows[(size_t)c + 1];
        const int64_t b = base[(size_t)c], cnt = base[(size_t)c + 1] - b;
        if (r1 <= r0 || cnt <= 0) continue;
        CSTM_REQUIRE(cnt < ((int64_t)1 << 31), CSTM_EINVAL, "a row of G is too long to regroup by label");
        uint64_t* skey = g->mem.get_n<uint64_t>(cnt);
        int32_t* sval = g->mem.get_n<int32_t>(cnt);
        const unsigned grid = cstm_blocks((r1 - r0) * CSTM_WAVE, 256, 16384);
        if (g->key32)
            k_regroup_keys<uint32_t><<<grid, 256, 0, s>>>(g->row_ptr, g->col, g->key32, g->key_shift, r0, r1, b,
                                                          label_bits, skey, sval);
        else
            k_regroup_keys<uint64_t><<<grid, 256, 0, s>>>(g->row_ptr, g->col, g->key64, g->key_shift, r0, r1, b,
                                                          label_bits, skey, sval);
        HIP_TRY(hipGetLastError());
        if (label_bits > 0)  // one label: the rows are in order already
            cstm_radix_sort_pairs(g->ctx, skey, sval, cnt, bits_for((uint64_t)(r1 - r0 - 1)) + label_bits, s);
        if (g->key32)
            k_regroup_gather<uint32_t><<<cstm_blocks(cnt, 256, 16384), 256, 0, s>>>(g->col, g->key32, b, cnt, sval,
                                                                                   g->lkey32);
        else
            k_regroup_gather<uint64_t><<<cstm_blocks(cnt, 256, 16384), 256, 0, s>>>(g->col, g->key64, b, cnt, sval,
                                                                                   g->lkey64);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(s));
        g->mem.release(skey);
        g->mem.release(sval);
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
        g->label_ptr.assign((size_t)L + 1, 0);
        g->deg_at_least.assign((size_t)(L > 0 ? L : 0) * (CSTM_MAX_K + 1), 0);
        g->deg_prefix.assign((size_t)n + 1, 0);
        if (n > 0) {
            uint64_t* keys = g->mem.get_n<uint64_t>(n);
            int32_t* ids = g->perm;  // sorted in place into the permutation
            unsigned long long* hist = g->mem.get_n<unsigned long long>(L);
            cstm_fill_words(hist, (size_t)L * 8, 0u, s);
            const int deg_bits = std::max(1, bits_for((uint64_t)g->max_degree));
            const int label_bits = bits_for((uint64_t)(L - 1));
            k_make_keys<<<cstm_blocks(n, 256, 16384), 256, 0, s>>>(g->row_ptr, g->label, n, deg_bits, keys, ids, hist);
            HIP_TRY(hipGetLastError());
            cstm_radix_sort_pairs(ctx, keys, ids, n, deg_bits + label_bits, s);
            std::vector<unsigned long long> h((size_t)L);
            HIP_TRY(hipMemcpyAsync(h.data(), hist, (size_t)L * 8, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            int64_t max_group = 0;
            for (int32_t l = 0; l < L; ++l) {
                g->label_ptr[l + 1] = g->label_ptr[l] + (int64_t)h[l];
                max_group = std::max<int64_t>(max_group, (int64_t)h[l]);
            }
            int64_t* lp = g->mem.get_n<int64_t>((size_t)L + 1);
            HIP_TRY(hipMemcpyAsync(lp, g->label_ptr.data(), ((size_t)L + 1) * 8, hipMemcpyHostToDevice, s));
            // packed (label, rank) keys: 32 bits when both fit
            const int rank_bits = std::max(1, bits_for((uint64_t)(max_group - 1)));
            if (label_bits + rank_bits <= 32) {
                g->key_shift = rank_bits;
                g->key32 = g->mem.get_n<uint32_t>(n);
                k_ranks<uint32_t><<<cstm_blocks(n, 256, 16384), 256, 0, s>>>(g->perm, g->label, lp, n, rank_bits,
                                                                             g->key32);
            } else {
                g->key_shift = 32;
                g->key64 = g->mem.get_n<uint64_t>(n);
                k_ranks<uint64_t><<<cstm_blocks(n, 256, 16384), 256, 0, s>>>(g->perm, g->label, lp, n, 32, g->key64);
            }
            HIP_TRY(hipGetLastError());
            if (nnz > 0) {
                if (g->key32) g->lkey32 = g->mem.get_n<uint32_t>(nnz);
                else g->lkey64 = g->mem.get_n<uint64_t>(nnz);
                regroup_rows(g, label_bits, s);
            }
            int64_t* dal = g->mem.get_n<int64_t>(g->deg_at_least.size());
            k_deg_at_least<<<cstm_blocks((int64_t)g->deg_at_least.size(), 256, 4096), 256, 0, s>>>(
                g->row_ptr, g->perm, lp, L, dal);
            HIP_TRY(hipGetLastError());
            HIP_TRY(hipMemcpyAsync(g->deg_at_least.data(), dal, g->deg_at_least.size() * 8, hipMemcpyDeviceToHost, s));
            // degree prefix sums in label-index order, for footprint estimates and build bounds
            int64_t* pd = (int64_t*)keys;  // n int64 entries, free again
            int64_t* ps = g->mem.get_n<int64_t>(n + 1);
            int64_t* part = g->mem.get_n<int64_t>(kScanPartSlots);
            k_perm_degrees<<<cstm_blocks(n, 256, 16384), 256, 0, s>>>(g->row_ptr, g->perm, n, pd);
            HIP_TRY(hipGetLastError());
            cstm_dscan_i64(pd, ps, nullptr, n, nullptr, part, s);
            HIP_TRY(hipMemcpyAsync(g->deg_prefix.data(), ps, (size_t)(n + 1) * 8, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            g->mem.release(keys);
            g->mem.release(hist);
            g->mem.release(dal);
            g->mem.release(ps);
            g->mem.release(part);
            if (nnz > 0 && L <= kPairMaxLabels) {
                unsigned long long* pc = g->mem.get_n<unsigned long long>((size_t)L * L);
                cstm_fill_words(pc, (size_t)L * L * 8, 0u, s);
                const unsigned grid = cstm_blocks(n * CSTM_WAVE, 256, 2048);
                if (g->key32)
                    k_pair_counts<uint32_t><<<grid, 256, 0, s>>>(g->row_ptr, g->label, g->lkey32, g->key_shift, n, L, pc);
                else
                    k_pair_counts<uint64_t><<<grid, 256, 0, s>>>(g->row_ptr, g->label, g->lkey64, g->key_shift, n, L, pc);
                HIP_TRY(hipGetLastError());
                g->pair_count.assign((size_t)L * L, 0);
                HIP_TRY(hipMemcpyAsync(g->pair_count.data(), pc, (size_t)L * L * 8, hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
                g->mem.release(pc);
            }
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
            // kept: the candidate array; during the build: rank table, top-down
            // set and ranks, refined set, index map, flags and their scan (int32
            // each)
            bytes += 4ull * (uint64_t)c0[u] + 7ull * 4 * ((uint64_t)c0[u] + 1);
        }
        // path-count vectors of one leaf path
        bytes += 8ull * (uint64_t)k * (max_c0 + 1);
        // every candidate edge list: kept offsets over its owner and entries (ids
        // and, for non-tree lists, global ids); an edge (v, w) with v in C(a), w
        // in C(b) appears once, so either side's degree sum bounds the entries.
        // During the build: per-owner counts and offsets, and the owner's label
        // runs (length, start, offset: int64 each), one int32 per run entry
        // (kept ranks or indices; the owner's degree sum and the edges of G
        // between the two labels bound the entries), plus two int64 per part
        // of those runs.
        for (int e = 0; e < m_q; ++e) {
            int a = qedges[2 * e], b = qedges[2 * e + 1];
            // the edges of G between the two labels bound both
            const uint64_t pairs = g->pair_bound(qlabel[a], qlabel[b]);
            uint64_t ent = sdeg[a] < sdeg[b] ? sdeg[a] : sdeg[b];
            ent = ent < pairs ? ent : pairs;
            uint64_t rows = sdeg[a] > sdeg[b] ? sdeg[a] : sdeg[b];
            rows = rows < pairs ? rows : pairs;
            const uint64_t cmax = (uint64_t)(c0[a] > c0[b] ? c0[a] : c0[b]);
            bytes += 8ull * (max_c0 + 1) + 8ull * ent;
            bytes += 40ull * (cmax + 1) + 4ull * rows + 16ull * (rows / 512 + 2);
        }
        *bytes_out = bytes + 65536;  // descriptor, size table, scan scratch and small flags
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

extern "C" cstm_status cstm_graph_label_edges(const cstm_graph* g, uint64_t* out, int64_t cap, int64_t* n_out) {
    return cstm_guard([&] {
        CSTM_REQUIRE(g && n_out, CSTM_EINVAL, "NULL argument");
        CSTM_REQUIRE(cap >= 0 && (cap == 0 || out), CSTM_EINVAL, "bad output array");
        const int64_t n = (int64_t)g->pair_count.size();
        *n_out = n;
        for (int64_t i = 0; i < n && i < cap; ++i) out[i] = g->pair_count[(size_t)i];
    });
}
