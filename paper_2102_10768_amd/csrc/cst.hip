// cst.hip -- CST construction on the device (Section V-A, Definition 2, Algorithm 1).
//
// For a query q the CST holds, per query vertex u, the candidate set C(u) and,
// per query edge, the candidate adjacency lists N^u_{u'}(v) = N_G(v) ∩ C(u').
// Construction follows Algorithm 1:
//   1. C(root): the label/degree filter, i.e. a prefix of the root's label group;
//   2. top-down along the BFS tree t_q: C(u) = candidates of u adjacent to some
//      candidate of its tree parent;
//   3. bottom-up: a candidate stays iff it has a neighbour in C(u_c) for every
//      tree child u_c (children refined first);
//   4. the tree lists, the path-based matching order (Section V-B), and the
//      non-tree candidate edges (stored once, from the earlier to the later
//      endpoint in the order, which is the direction enumeration reads).
// Membership of a data vertex w in C(u) is one range test on w's label-group
// rank plus one lookup in a rank-indexed table, so every scan below is a
// coalesced walk over CSR rows with one gather per neighbour.
#include <algorithm>
#include <cstring>
#include <numeric>

#include "internal.h"

namespace {

__device__ inline int lane_id() { return threadIdx.x & (CSTM_WAVE - 1); }

__device__ inline int64_t global_wave() { return ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / CSTM_WAVE; }

__device__ inline int64_t num_waves() { return ((int64_t)gridDim.x * blockDim.x) / CSTM_WAVE; }

__device__ inline uint64_t ballot(bool p) { return __ballot(p); }

__device__ inline int mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

// Rows of a candidate array laid end to end: entry t of the flattened space is
// entry t - rowoff[i] of the CSR row of candidate i, where rowoff is the
// exclusive prefix sum of the candidates' degrees.  Kernels walk this space in
// tiles of kTile entries, one wavefront per tile, so a hub's long row is shared
// by many wavefronts and short rows are packed together.
constexpr int kTile = 512;

struct Rows {
    const int32_t* cand;    // candidate data-vertex ids
    const int64_t* rowoff;  // n + 1 prefix sums of their degrees
    int64_t n;
    int64_t total;          // rowoff[n]
};

// The candidate whose row holds flattened entry t: the last i in [lo, hi]
// with rowoff[i] <= t (empty rows are skipped by construction).
__device__ inline int64_t owner_of(const int64_t* __restrict__ rowoff, int64_t lo, int64_t hi, int64_t t) {
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (rowoff[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void k_cand_degrees(const int32_t* __restrict__ cand, int64_t n, const int64_t* __restrict__ row_ptr,
                               int64_t* __restrict__ deg) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int32_t v = cand[i];
        deg[i] = row_ptr[v + 1] - row_ptr[v];
    }
}

// Top-down marking: every neighbour of a parent candidate that passes u's
// label/degree filter is marked in u's rank table.
__global__ void k_mark(Rows R, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                       const uint64_t* __restrict__ lab_rank, uint64_t key, int64_t cnt0, int32_t* __restrict__ mark) {
    const int lane = lane_id();
    const int64_t ntiles = (R.total + kTile - 1) / kTile;
    for (int64_t tile = global_wave(); tile < ntiles; tile += num_waves()) {
        const int64_t t0 = tile * kTile, t1 = t0 + kTile < R.total ? t0 + kTile : R.total;
        const int64_t lo = owner_of(R.rowoff, 0, R.n - 1, t0);
        const int64_t hi = owner_of(R.rowoff, lo, R.n - 1, t1 - 1);
        for (int64_t t = t0 + lane; t < t1; t += CSTM_WAVE) {
            const int64_t i = owner_of(R.rowoff, lo, hi, t);
            const int64_t j = row_ptr[R.cand[i]] + (t - R.rowoff[i]);
            const uint64_t d = lab_rank[col[j]] - key;
            if (d < (uint64_t)cnt0) mark[d] = 1;
        }
    }
}

// marks -> candidate indices: C(u) in rank order (degree desc, id asc).
__global__ void k_assign(int32_t* __restrict__ loc, const int32_t* __restrict__ scan, int64_t cnt0,
                         const int32_t* __restrict__ perm_base, int32_t* __restrict__ cand) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < cnt0; r += stride) {
        if (loc[r]) {
            int32_t j = scan[r];
            cand[j] = perm_base[r];
            loc[r] = j;
        } else {
            loc[r] = -1;
        }
    }
}

__global__ void k_iota_root(int32_t* __restrict__ loc, int64_t cnt0, const int32_t* __restrict__ perm_base,
                            int32_t* __restrict__ cand) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < cnt0; r += stride) {
        loc[r] = (int32_t)r;
        cand[r] = perm_base[r];
    }
}

struct ChildRef {
    uint64_t key;
    int64_t cnt0;
    const int32_t* loc;
};
struct ChildSet {
    int32_t n;
    ChildRef c[CSTM_MAX_K];
};

// Bottom-up validity: a candidate needs a neighbour in every refined child set.
__global__ void k_valid(const int32_t* __restrict__ cand, int64_t n, const int64_t* __restrict__ row_ptr,
                        const int32_t* __restrict__ col, const uint64_t* __restrict__ lab_rank, ChildSet ch,
                        int32_t* __restrict__ flag) {
    const int lane = lane_id();
    for (int64_t i = global_wave(); i < n; i += num_waves()) {
        int32_t v = cand[i];
        int64_t b = row_ptr[v], e = row_ptr[v + 1];
        bool ok = true;
        for (int c = 0; c < ch.n && ok; ++c) {
            const ChildRef cr = ch.c[c];
            bool found = false;
            for (int64_t j0 = b; j0 < e && !found; j0 += CSTM_WAVE) {
                int64_t j = j0 + lane;
                bool hit = false;
                if (j < e) {
                    uint64_t d = lab_rank[col[j]] - cr.key;
                    hit = d < (uint64_t)cr.cnt0 && cr.loc[d] >= 0;
                }
                found = ballot(hit) != 0;
            }
            ok = found;
        }
        if (lane == 0) flag[i] = ok ? 1 : 0;
    }
}

__global__ void k_refine(const int32_t* __restrict__ cand_old, const int32_t* __restrict__ flag,
                         const int32_t* __restrict__ scan, int64_t n, const uint64_t* __restrict__ lab_rank,
                         uint64_t key, int32_t* __restrict__ loc, int32_t* __restrict__ cand_new) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        int32_t v = cand_old[i];
        uint64_t r = lab_rank[v] - key;
        if (flag[i]) {
            int32_t j = scan[i];
            cand_new[j] = v;
            loc[r] = j;
        } else {
            loc[r] = -1;
        }
    }
}

// List sizes: |N_G(v) ∩ C(u')| per candidate v of the list's owner, added to
// cnt (zeroed by the caller) once per run of lanes with the same owner; the
// number of list entries in each tile goes to tile_cnt.
__global__ void k_list_count(Rows R, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                             const uint64_t* __restrict__ lab_rank, uint64_t key, int64_t cnt0,
                             const int32_t* __restrict__ loc, unsigned long long* __restrict__ cnt,
                             int64_t* __restrict__ tile_cnt) {
    const int lane = lane_id();
    const int64_t ntiles = (R.total + kTile - 1) / kTile;
    for (int64_t tile = global_wave(); tile < ntiles; tile += num_waves()) {
        const int64_t t0 = tile * kTile, t1 = t0 + kTile < R.total ? t0 + kTile : R.total;
        const int64_t lo = owner_of(R.rowoff, 0, R.n - 1, t0);
        const int64_t hi = owner_of(R.rowoff, lo, R.n - 1, t1 - 1);
        int64_t in_tile = 0;
        for (int64_t s0 = t0; s0 < t1; s0 += CSTM_WAVE) {
            const int64_t t = s0 + lane;
            const bool in = t < t1;
            const int64_t i = in ? owner_of(R.rowoff, lo, hi, t) : hi;
            bool hit = false;
            if (in) {
                const int64_t j = row_ptr[R.cand[i]] + (t - R.rowoff[i]);
                const uint64_t d = lab_rank[col[j]] - key;
                hit = d < (uint64_t)cnt0 && loc[d] >= 0;
            }
            const uint64_t hits = ballot(hit);
            in_tile += __popcll(hits);
            // owners never decrease across lanes: one atomic per run of equal owners
            const int64_t prev = __shfl_up(i, 1, CSTM_WAVE);
            const bool head = lane == 0 || prev != i;
            const uint64_t heads = ballot(head);
            if (head) {
                const uint64_t later = lane == CSTM_WAVE - 1 ? 0ull : (heads >> (lane + 1)) << (lane + 1);
                const uint64_t upto = later ? (later & (~later + 1)) - 1 : ~0ull;  // bits below the next head
                const uint64_t run = upto & ~((1ull << lane) - 1);
                const int c = __popcll(hits & run);
                if (c) atomicAdd(&cnt[i], (unsigned long long)c);
            }
        }
        if (lane == 0) tile_cnt[tile] = in_tile;
    }
}

// Largest list length, from the list offsets.
__global__ void k_max_len(const int64_t* __restrict__ off, int64_t n, int* __restrict__ max_len) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int64_t len = off[i + 1] - off[i];
        m = len > m ? (int)len : m;
    }
    for (int o = CSTM_WAVE / 2; o > 0; o >>= 1) {
        const int y = __shfl_xor(m, o, CSTM_WAVE);
        m = y > m ? y : m;
    }
    if (lane_id() == 0 && m) atomicMax(max_len, m);
}

// List entries, in G's row order (ascending data-vertex id), as indices into
// C(u'): the hits of the flattened space are numbered in order, tile by tile
// from tile_base, which lays the lists of consecutive owners end to end exactly
// as the offsets from the per-owner counts do.
__global__ void k_list_fill(Rows R, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                            const uint64_t* __restrict__ lab_rank, uint64_t key, int64_t cnt0,
                            const int32_t* __restrict__ loc, const int64_t* __restrict__ tile_base,
                            int32_t* __restrict__ adj, int32_t* __restrict__ adj_gid) {
    const int lane = lane_id();
    const int64_t ntiles = (R.total + kTile - 1) / kTile;
    for (int64_t tile = global_wave(); tile < ntiles; tile += num_waves()) {
        const int64_t t0 = tile * kTile, t1 = t0 + kTile < R.total ? t0 + kTile : R.total;
        const int64_t lo = owner_of(R.rowoff, 0, R.n - 1, t0);
        const int64_t hi = owner_of(R.rowoff, lo, R.n - 1, t1 - 1);
        int64_t out = tile_base[tile];
        for (int64_t s0 = t0; s0 < t1; s0 += CSTM_WAVE) {
            const int64_t t = s0 + lane;
            int32_t idx = -1, w = 0;
            if (t < t1) {
                const int64_t i = owner_of(R.rowoff, lo, hi, t);
                const int64_t j = row_ptr[R.cand[i]] + (t - R.rowoff[i]);
                w = col[j];
                const uint64_t d = lab_rank[w] - key;
                if (d < (uint64_t)cnt0) idx = loc[d];
            }
            const uint64_t m = ballot(idx >= 0);
            if (idx >= 0) {
                adj[out + mbcnt(m)] = idx;
                if (adj_gid) adj_gid[out + mbcnt(m)] = w;
            }
            out += __popcll(m);
        }
    }
}

__device__ inline uint64_t sat_add(uint64_t a, uint64_t b) {
    uint64_t s = a + b;
    return s < a ? ~0ull : s;
}

// One step of a path count: val[v] = sum over the list of v of child_val (1 at the leaf).
__global__ void k_path_step(const int64_t* __restrict__ off, const int32_t* __restrict__ adj, int64_t np,
                            const uint64_t* __restrict__ child_val, uint64_t* __restrict__ out) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += stride) {
        int64_t b = off[i], e = off[i + 1];
        uint64_t s = 0;
        if (!child_val) s = (uint64_t)(e - b);
        else
            for (int64_t j = b; j < e; ++j) s = sat_add(s, child_val[adj[j]]);
        out[i] = s;
    }
}

__global__ void k_sum_sat(const uint64_t* __restrict__ v, int64_t n, unsigned long long* __restrict__ total) {
    __shared__ uint64_t part[256];
    uint64_t s = 0;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) s = sat_add(s, v[i]);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] = sat_add(part[threadIdx.x], part[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        unsigned long long add = part[0];
        unsigned long long old = *total, assumed;
        do {
            assumed = old;
            old = atomicCAS(total, assumed, (unsigned long long)sat_add(assumed, add));
        } while (old != assumed);
    }
}

// a * b, or 2^64 - 1 when the product does not fit: with sat_add this gives
// min(exact value, 2^64 - 1) for any sum of products of non-negative integers
__device__ inline uint64_t sat_mul(uint64_t a, uint64_t b) {
    return __umul64hi(a, b) ? ~0ull : a * b;
}

// Workload DP (Section V-C) for one tree edge (u_p -> u): the value of each
// candidate of u_p is multiplied by the sum of the values of its list in C(u).
// Exact unsigned 64-bit integers, saturating at 2^64 - 1.
__global__ void k_workload_step(const int64_t* __restrict__ off, const int32_t* __restrict__ adj, int64_t np,
                                const uint64_t* __restrict__ cu, uint64_t* __restrict__ cp) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += stride) {
        uint64_t sum = 0;
        for (int64_t j = off[i]; j < off[i + 1]; ++j) sum = sat_add(sum, cu[adj[j]]);
        cp[i] = sat_mul(cp[i], sum);
    }
}

__global__ void k_fill_ones(uint64_t* __restrict__ x, int64_t n) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = 1;
}

constexpr int kWaveBlock = 256;

unsigned wave_grid(int64_t items) {
    // one wave per item, at most a few passes per wave
    return cstm_blocks(items * CSTM_WAVE, kWaveBlock, 1u << 16);
}

struct QueryPrep {
    int k;
    int32_t qlabel[CSTM_MAX_K];
    uint32_t adj[CSTM_MAX_K];
    const int32_t* order = nullptr;  // caller's matching order, or nullptr for the path-based one
};

void validate_query(int32_t k, const int32_t* qlabel, int32_t m_q, const int32_t* qedges, QueryPrep& q) {
    CSTM_REQUIRE(k >= 1 && k <= CSTM_MAX_K, CSTM_EINVAL, "query size k must be in 1..32");
    CSTM_REQUIRE(qlabel, CSTM_EINVAL, "qlabel is NULL");
    CSTM_REQUIRE(m_q >= 0 && (m_q == 0 || qedges), CSTM_EINVAL, "bad query edge array");
    q.k = k;
    for (int u = 0; u < k; ++u) {
        CSTM_REQUIRE(qlabel[u] >= 0, CSTM_EINVAL, "negative query label");
        q.qlabel[u] = qlabel[u];
        q.adj[u] = 0;
    }
    for (int e = 0; e < m_q; ++e) {
        int a = qedges[2 * e], b = qedges[2 * e + 1];
        CSTM_REQUIRE(a >= 0 && a < k && b >= 0 && b < k, CSTM_EINVAL, "query edge endpoint out of range");
        CSTM_REQUIRE(a != b, CSTM_EINVAL, "query self-loop");
        CSTM_REQUIRE(!(q.adj[a] >> b & 1u), CSTM_EINVAL, "duplicate query edge");
        q.adj[a] |= 1u << b;
        q.adj[b] |= 1u << a;
    }
    uint32_t seen = 1u, frontier = 1u;
    while (frontier) {
        uint32_t next = 0;
        for (int u = 0; u < k; ++u)
            if (frontier >> u & 1u) next |= q.adj[u];
        next &= ~seen;
        seen |= next;
        frontier = next;
    }
    uint32_t all = k == 32 ? 0xFFFFFFFFu : ((1u << k) - 1u);
    CSTM_REQUIRE(seen == all, CSTM_EINVAL, "query graph is disconnected");
}

struct EventTimer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    explicit EventTimer(hipStream_t st) : s(st) {
        HIP_TRY(hipEventCreate(&a));
        HIP_TRY(hipEventCreate(&b));
        HIP_TRY(hipEventRecord(a, s));
    }
    double stop() {
        float ms = 0;
        HIP_TRY(hipEventRecord(b, s));
        HIP_TRY(hipEventSynchronize(b));
        HIP_TRY(hipEventElapsedTime(&ms, a, b));
        return ms;
    }
    ~EventTimer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace

// Flattened rows of n candidates: degrees, then their prefix sums into rowoff
// (n + 1 entries).  Returns the total number of row entries.
static Rows flat_rows(cstm_cst* c, const int32_t* cand, int64_t n, int64_t* deg, int64_t* rowoff) {
    hipStream_t s = c->stream;
    if (n) {
        k_cand_degrees<<<cstm_blocks(n, 256, 4096), 256, 0, s>>>(cand, n, c->g->row_ptr, deg);
        HIP_TRY(hipGetLastError());
    }
    Rows R;
    R.cand = cand;
    R.rowoff = rowoff;
    R.n = n;
    R.total = cstm_exclusive_scan_i64(c->ctx, deg, rowoff, n, s);
    return R;
}

static unsigned tile_grid(int64_t total) {
    const int64_t tiles = (total + kTile - 1) / kTile;
    return wave_grid(tiles > 0 ? tiles : 1);
}

// The lists of `from` (a query vertex) into `to`, using to's rank table.
// Scratch: deg, rowoff and cnt hold at least #C(from) + 1 int64 entries.
// The longest list goes to the device int *d_max (zeroed by the caller), read
// back once after all lists; blocks the fill kernel still uses go to `later`,
// released after the build's last wait.
static void build_lists(cstm_cst* c, int from, int to, int32_t* const* loc, EdgeLists& el, int* d_max,
                        int64_t* deg, int64_t* rowoff, int64_t* cnt, bool with_gid, std::vector<void*>& later) {
    const cstm_graph* g = c->g;
    hipStream_t s = c->stream;
    const int64_t np = c->ncand[from];
    uint64_t key = (uint64_t)c->qlabel[to] << 32;
    el.off = c->mem.get_n<int64_t>(np + 1);
    const Rows R = flat_rows(c, c->cand[from], np, deg, rowoff);
    const int64_t ntiles = (R.total + kTile - 1) / kTile;
    int64_t* tile_cnt = c->mem.get_n<int64_t>(ntiles + 1);
    if (np) HIP_TRY(hipMemsetAsync(cnt, 0, (size_t)np * sizeof(int64_t), s));
    if (ntiles) {
        k_list_count<<<tile_grid(R.total), kWaveBlock, 0, s>>>(R, g->row_ptr, g->col, g->lab_rank, key, c->cnt0[to],
                                                               loc[to], (unsigned long long*)cnt, tile_cnt);
        HIP_TRY(hipGetLastError());
    }
    el.entries = cstm_exclusive_scan_i64(c->ctx, cnt, el.off, np, s);
    if (np) {
        k_max_len<<<cstm_blocks(np, 256, 1024), 256, 0, s>>>(el.off, np, d_max);
        HIP_TRY(hipGetLastError());
    }
    el.adj = c->mem.get_n<int32_t>(el.entries ? el.entries : 1);
    if (with_gid) el.adj_gid = c->mem.get_n<int32_t>(el.entries ? el.entries : 1);
    if (ntiles && el.entries) {
        int64_t* tile_base = c->mem.get_n<int64_t>(ntiles + 1);
        const int64_t again = cstm_exclusive_scan_i64(c->ctx, tile_cnt, tile_base, ntiles, s);
        CSTM_REQUIRE(again == el.entries, CSTM_EDEVICE, "candidate list counts disagree");
        k_list_fill<<<tile_grid(R.total), kWaveBlock, 0, s>>>(R, g->row_ptr, g->col, g->lab_rank, key, c->cnt0[to],
                                                              loc[to], tile_base, el.adj, el.adj_gid);
        HIP_TRY(hipGetLastError());
        later.push_back(tile_base);
    }
    // the last reader of tile_cnt was the scan above, which waited for the stream
    c->mem.release(tile_cnt);
}

static void build_cst(cstm_cst* c, const QueryPrep& q) {
    const cstm_graph* g = c->g;
    hipStream_t s = c->stream;
    const int k = q.k;
    c->k = k;
    for (int u = 0; u < k; ++u) {
        c->qlabel[u] = q.qlabel[u];
        c->qadj[u] = q.adj[u];
        c->qdeg[u] = __builtin_popcount(q.adj[u]);
        c->cnt0[u] = g->count_ge(q.qlabel[u], c->qdeg[u]);
        c->lb_lo[u] = q.qlabel[u] < g->num_labels ? g->label_ptr[q.qlabel[u]] : 0;
    }
    // root: fewest filtered candidates per unit of query degree, smaller id on ties
    int root = 0;
    if (k > 1) {
        for (int u = 1; u < k; ++u) {
            if (c->cnt0[u] * c->qdeg[root] < c->cnt0[root] * c->qdeg[u]) root = u;
        }
    }
    c->root = root;
    // BFS tree: neighbours in ascending id, parent = first discoverer
    for (int u = 0; u < k; ++u) c->parent[u] = -1;
    uint32_t seen = 1u << root;
    int head = 0, tail = 0;
    c->bfs[tail++] = root;
    while (head < tail) {
        int u = c->bfs[head++];
        for (int w = 0; w < k; ++w) {
            if ((q.adj[u] >> w & 1u) && !(seen >> w & 1u)) {
                seen |= 1u << w;
                c->parent[w] = u;
                c->bfs[tail++] = w;
            }
        }
    }
    for (int a = 0; a < k; ++a)
        for (int b = a + 1; b < k; ++b)
            if ((q.adj[a] >> b & 1u) && c->parent[a] != b && c->parent[b] != a) c->nontree.push_back({a, b});

    for (int u = 0; u < k; ++u)
        if (c->cnt0[u] == 0) c->empty = true;

    int32_t* loc[CSTM_MAX_K] = {};
    if (!c->empty) {
        int64_t max_cnt0 = 0;
        for (int u = 0; u < k; ++u) max_cnt0 = std::max(max_cnt0, c->cnt0[u]);
        int32_t* scan = c->mem.get_n<int32_t>(max_cnt0 + 1);
        int32_t* flag = c->mem.get_n<int32_t>(max_cnt0 + 1);
        int64_t* fdeg = c->mem.get_n<int64_t>(max_cnt0 + 1);
        int64_t* frow = c->mem.get_n<int64_t>(max_cnt0 + 1);
        // 1. root candidates: the filtered prefix of the root's label group
        loc[root] = c->mem.get_n<int32_t>(c->cnt0[root]);
        c->cand[root] = c->mem.get_n<int32_t>(c->cnt0[root]);
        c->ncand[root] = c->cnt0[root];
        k_iota_root<<<cstm_blocks(c->cnt0[root], 256, 4096), 256, 0, s>>>(loc[root], c->cnt0[root],
                                                                          g->perm + c->lb_lo[root], c->cand[root]);
        HIP_TRY(hipGetLastError());
        // 2. top-down construction
        for (int t = 1; t < k && !c->empty; ++t) {
            int u = c->bfs[t], up = c->parent[u];
            loc[u] = c->mem.get_n<int32_t>(c->cnt0[u]);
            HIP_TRY(hipMemsetAsync(loc[u], 0, c->cnt0[u] * sizeof(int32_t), s));
            const Rows R = flat_rows(c, c->cand[up], c->ncand[up], fdeg, frow);
            if (R.total) {
                k_mark<<<tile_grid(R.total), kWaveBlock, 0, s>>>(R, g->row_ptr, g->col, g->lab_rank,
                                                                 (uint64_t)q.qlabel[u] << 32, c->cnt0[u], loc[u]);
                HIP_TRY(hipGetLastError());
            }
            int64_t nu = cstm_exclusive_scan_i32(c->ctx, loc[u], scan, c->cnt0[u], s);
            c->ncand[u] = nu;
            c->cand[u] = c->mem.get_n<int32_t>(nu ? nu : 1);
            k_assign<<<cstm_blocks(c->cnt0[u], 256, 4096), 256, 0, s>>>(loc[u], scan, c->cnt0[u],
                                                                        g->perm + c->lb_lo[u], c->cand[u]);
            HIP_TRY(hipGetLastError());
            if (nu == 0) c->empty = true;
        }
        // 3. bottom-up refinement
        for (int t = k - 1; t >= 0 && !c->empty; --t) {
            int u = c->bfs[t];
            ChildSet ch{};
            for (int w = 0; w < k; ++w) {
                if (c->parent[w] == u) {
                    ch.c[ch.n].key = (uint64_t)q.qlabel[w] << 32;
                    ch.c[ch.n].cnt0 = c->cnt0[w];
                    ch.c[ch.n].loc = loc[w];
                    ch.n++;
                }
            }
            if (ch.n == 0) continue;
            int64_t n = c->ncand[u];
            k_valid<<<wave_grid(n), kWaveBlock, 0, s>>>(c->cand[u], n, g->row_ptr, g->col, g->lab_rank, ch, flag);
            HIP_TRY(hipGetLastError());
            int64_t nn = cstm_exclusive_scan_i32(c->ctx, flag, scan, n, s);
            if (nn != n) {
                int32_t* cn = c->mem.get_n<int32_t>(nn ? nn : 1);
                k_refine<<<cstm_blocks(n, 256, 4096), 256, 0, s>>>(c->cand[u], flag, scan, n, g->lab_rank,
                                                                   (uint64_t)q.qlabel[u] << 32, loc[u], cn);
                HIP_TRY(hipGetLastError());
                HIP_TRY(hipStreamSynchronize(s));
                c->mem.release(c->cand[u]);
                c->cand[u] = cn;
                c->ncand[u] = nn;
            }
            if (nn == 0) c->empty = true;
        }
        c->mem.release(flag);
        c->mem.release(scan);
        c->mem.release(fdeg);
        c->mem.release(frow);
    }

    // 4a. tree lists (longest-list slots: tree edges by child, then non-tree edges)
    const int n_slots = k + (int)c->nontree.size();
    int* d_max = c->mem.get_n<int>(n_slots);
    HIP_TRY(hipMemsetAsync(d_max, 0, (size_t)n_slots * sizeof(int), s));
    std::vector<void*> later;
    int64_t maxn = 1;
    for (int u = 0; u < k; ++u) maxn = std::max(maxn, c->ncand[u]);
    int64_t* d_cnt = c->mem.get_n<int64_t>(maxn + 1);
    int64_t* l_deg = c->mem.get_n<int64_t>(maxn + 1);
    int64_t* l_row = c->mem.get_n<int64_t>(maxn + 1);
    if (!c->empty) {
        for (int t = 1; t < k; ++t) {
            int u = c->bfs[t];
            build_lists(c, c->parent[u], u, loc, c->tree[u], d_max + u, l_deg, l_row, d_cnt, false, later);
        }
    }
    // 4b. matching order: the caller's (checked against the tree) or the path-based one
    if (q.order) {
        uint32_t placed = 0;
        for (int i = 0; i < k; ++i) {
            const int u = q.order[i];
            CSTM_REQUIRE(u >= 0 && u < k && !(placed >> u & 1u), CSTM_EINVAL, "order is not a permutation of 0..k-1");
            CSTM_REQUIRE(i > 0 || u == root, CSTM_EINVAL, "order must start at the CST root");
            CSTM_REQUIRE(i == 0 || (placed >> c->parent[u] & 1u), CSTM_EINVAL,
                         "order must place every vertex after its tree parent");
            placed |= 1u << u;
            c->order[i] = u;
        }
        for (int i = 0; i < k; ++i) c->pos_of[c->order[i]] = i;
    } else {
        std::vector<std::pair<std::pair<uint64_t, int>, std::vector<int>>> paths;
        for (int leaf = 0; leaf < k; ++leaf) {
            bool has_child = false;
            for (int w = 0; w < k; ++w) has_child |= c->parent[w] == leaf;
            if (has_child || (leaf == root && k > 1)) continue;
            std::vector<int> p{leaf};
            while (c->parent[p.back()] >= 0) p.push_back(c->parent[p.back()]);
            std::reverse(p.begin(), p.end());
            uint64_t cnt = 0;
            if (!c->empty) {
                const uint64_t* child_val = nullptr;
                uint64_t* vals[CSTM_MAX_K] = {};
                for (int i = (int)p.size() - 2; i >= 0; --i) {
                    int u = p[i], uc = p[i + 1];
                    vals[i] = c->mem.get_n<uint64_t>(c->ncand[u] ? c->ncand[u] : 1);
                    k_path_step<<<cstm_blocks(c->ncand[u], 256, 4096), 256, 0, s>>>(
                        c->tree[uc].off, c->tree[uc].adj, c->ncand[u], child_val, vals[i]);
                    HIP_TRY(hipGetLastError());
                    child_val = vals[i];
                }
                unsigned long long* tot = (unsigned long long*)d_cnt;
                HIP_TRY(hipMemsetAsync(tot, 0, 8, s));
                if (p.size() == 1) {
                    cnt = (uint64_t)c->ncand[p[0]];
                } else {
                    k_sum_sat<<<cstm_blocks(c->ncand[root], 256, 1024), 256, 0, s>>>(vals[0], c->ncand[root], tot);
                    HIP_TRY(hipGetLastError());
                    HIP_TRY(hipMemcpyAsync(&cnt, tot, 8, hipMemcpyDeviceToHost, s));
                    HIP_TRY(hipStreamSynchronize(s));
                }
                for (int i = 0; i < (int)p.size(); ++i)
                    if (vals[i]) c->mem.release(vals[i]);
            }
            paths.push_back({{cnt, leaf}, p});
        }
        std::sort(paths.begin(), paths.end(),
                  [](const auto& x, const auto& y) { return x.first < y.first; });
        int n = 0;
        uint32_t placed = 0;
        for (auto& pr : paths)
            for (int u : pr.second)
                if (!(placed >> u & 1u)) {
                    placed |= 1u << u;
                    c->order[n++] = u;
                }
        if (n == 0) c->order[n++] = root;
        for (int i = 0; i < k; ++i) c->pos_of[c->order[i]] = i;
    }
    // 4c. non-tree candidate edges, earlier -> later in the order
    for (size_t j = 0; j < c->nontree.size(); ++j) {
        int a = c->nontree[j].first, b = c->nontree[j].second;
        if (c->pos_of[a] > c->pos_of[b]) std::swap(a, b);
        EdgeLists el;
        el.from = c->pos_of[a];
        el.to = c->pos_of[b];
        if (!c->empty) {
            build_lists(c, a, b, loc, el, d_max + k + (int)j, l_deg, l_row, d_cnt, true, later);
        } else {
            el.off = nullptr;
        }
        c->nt.push_back(el);
    }
    // longest lists: one read-back for every edge (also the wait for the fills)
    {
        std::vector<int> h((size_t)n_slots, 0);
        HIP_TRY(hipMemcpyAsync(h.data(), d_max, (size_t)n_slots * sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (!c->empty) {
            for (int t = 1; t < k; ++t) {
                const int u = c->bfs[t];
                c->tree[u].max_len = h[(size_t)u];
                c->d_cst = std::max(c->d_cst, c->tree[u].max_len);
            }
            for (size_t j = 0; j < c->nt.size(); ++j) {
                c->nt[j].max_len = h[(size_t)k + j];
                c->d_cst = std::max(c->d_cst, c->nt[j].max_len);
            }
        }
        for (void* p : later) c->mem.release(p);
    }
    std::sort(c->nt.begin(), c->nt.end(), [](const EdgeLists& x, const EdgeLists& y) {
        return x.to != y.to ? x.to < y.to : x.from < y.from;
    });
    HIP_TRY(hipStreamSynchronize(s));
    for (int u = 0; u < k; ++u)
        if (loc[u]) c->mem.release(loc[u]);
    c->mem.release(d_cnt);
    c->mem.release(l_deg);
    c->mem.release(l_row);
    c->mem.release(d_max);

    // descriptor in order positions
    CstDev& D = c->host_desc;
    std::memset(&D, 0, sizeof(D));
    D.k = k;
    D.n_nt = (int32_t)c->nt.size();
    for (int i = 0; i < k; ++i) {
        int u = c->order[i];
        PosDesc& P = D.pos[i];
        P.u = u;
        P.par = c->parent[u] >= 0 ? c->pos_of[c->parent[u]] : -1;
        P.n = c->ncand[u];
        P.gid = c->cand[u];
        P.toff = c->tree[u].off;
        P.tadj = c->tree[u].adj;
        P.label = c->qlabel[u];
        for (int j = 0; j < i; ++j)
            if (c->qlabel[c->order[j]] == c->qlabel[u]) P.same_mask |= 1u << j;
        P.nt_first = -1;
    }
    for (int e = 0; e < D.n_nt; ++e) {
        const EdgeLists& el = c->nt[e];
        D.nt[e] = NtDesc{el.from, el.to, el.off, el.adj, el.adj_gid};
        PosDesc& P = D.pos[el.to];
        P.nt_mask |= 1u << el.from;
        if (P.nt_first < 0) P.nt_first = e;
    }
    for (int i = 0; i < k; ++i) {
        PosDesc& P = D.pos[i];
        bool repeated = false;
        for (int j = 0; j < k; ++j) repeated |= j != i && D.pos[j].label == P.label;
        P.need_gid = (repeated || P.nt_mask) ? 1 : 0;
    }
    c->dev = c->mem.get_n<CstDev>(1);
    HIP_TRY(hipMemcpyAsync(c->dev, &D, sizeof(CstDev), hipMemcpyHostToDevice, s));
    uint64_t bytes = 0;
    for (int u = 0; u < k; ++u) {
        bytes += 4ull * c->ncand[u];
        if (c->parent[u] >= 0) bytes += 8ull * (c->ncand[c->parent[u]] + 1) + 4ull * c->tree[u].entries;
    }
    for (auto& el : c->nt) bytes += 8ull * (c->ncand[c->order[el.from]] + 1) + 8ull * el.entries;
    c->bytes = bytes;
    HIP_TRY(hipStreamSynchronize(s));
}

extern "C" cstm_status cstm_cst_build_ordered(cstm_ctx* ctx, const cstm_graph* g, int32_t k, const int32_t* qlabel,
                                              int32_t m_q, const int32_t* qedges, const int32_t* order, void* stream,
                                              cstm_cst** out) {
    cstm_cst* c = nullptr;
    cstm_status st = cstm_guard([&] {
        CSTM_REQUIRE(ctx && g && out, CSTM_EINVAL, "NULL argument");
        *out = nullptr;
        QueryPrep q;
        validate_query(k, qlabel, m_q, qedges, q);
        q.order = order;
        HIP_TRY(hipSetDevice(ctx->device));
        c = new cstm_cst();
        c->ctx = ctx;
        c->g = g;
        c->stream = (hipStream_t)stream;
        c->mem.ctx = ctx;
        EventTimer tm(c->stream);
        build_cst(c, q);
        c->t_build = tm.stop();
        *out = c;
    });
    if (st != CSTM_OK && c) {
        // kernels of a half-built tree may still run on the stream: let them
        // finish before their blocks go back to the pool
        (void)hipStreamSynchronize(c->stream);
        delete c;
    }
    return st;
}

extern "C" cstm_status cstm_cst_build(cstm_ctx* ctx, const cstm_graph* g, int32_t k, const int32_t* qlabel,
                                      int32_t m_q, const int32_t* qedges, void* stream, cstm_cst** out) {
    return cstm_cst_build_ordered(ctx, g, k, qlabel, m_q, qedges, nullptr, stream, out);
}

extern "C" void cstm_cst_free(cstm_cst* cst) {
    if (!cst) return;
    (void)hipStreamSynchronize(cst->stream);
    delete cst;
}

extern "C" cstm_status cstm_cst_info_get(const cstm_cst* c, cstm_cst_info* out) {
    return cstm_guard([&] {
        CSTM_REQUIRE(c && out, CSTM_EINVAL, "NULL argument");
        std::memset(out, 0, sizeof(*out));
        out->k = c->k;
        out->root = c->root;
        for (int u = 0; u < CSTM_MAX_K; ++u) {
            out->parent[u] = u < c->k ? c->parent[u] : -1;
            out->order[u] = u < c->k ? c->order[u] : -1;
            out->cand[u] = u < c->k ? c->ncand[u] : 0;
        }
        for (int u = 0; u < c->k; ++u) out->tree_entries += c->tree[u].entries;
        for (auto& el : c->nt) out->nontree_entries += el.entries;
        out->bytes = c->bytes;
        out->d_cst = c->d_cst;
        out->n_nontree = (int32_t)c->nontree.size();
        out->n_parts = c->n_parts;
        out->part_bytes = c->blob_bytes;
        out->max_part_bytes = c->max_blob;
    });
}

extern "C" cstm_status cstm_cst_candidates(const cstm_cst* c, int32_t u, int32_t* out, int64_t cap, int64_t* n_out) {
    return cstm_guard([&] {
        CSTM_REQUIRE(c, CSTM_EINVAL, "NULL cst");
        CSTM_REQUIRE(u >= 0 && u < c->k, CSTM_EINVAL, "query vertex out of range");
        int64_t n = c->ncand[u];
        if (n_out) *n_out = n;
        int64_t w = std::min(n, cap);
        if (out && w > 0) {
            HIP_TRY(hipMemcpyAsync(out, c->cand[u], w * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
        }
    });
}

// W_CST = sum over root candidates of c_root, where c_u(v) is the product over
// u's tree children u' of the sum of c_u'(v') over v's list in C(u') (1 at the
// leaves): the number of tree-shaped paths the CST holds, an upper bound on
// the embeddings below each candidate (Section V-C).  Unsigned 64-bit integer
// arithmetic that saturates at 2^64 - 1, so every value is
// min(exact value, 2^64 - 1).
uint64_t cstm_cst_workload_run(cstm_cst* c) {
    if (c->has_workload) return c->workload;
    if (c->empty) {
        c->root_w.clear();
        c->has_workload = true;
        return c->workload = 0;
    }
    hipStream_t s = c->stream;
    DevArena mem;
    mem.ctx = c->ctx;
    uint64_t* val[CSTM_MAX_K] = {};
    for (int u = 0; u < c->k; ++u) {
        const int64_t n = c->ncand[u];
        val[u] = mem.get_n<uint64_t>(n ? n : 1);
        if (n) {
            k_fill_ones<<<cstm_blocks(n, 256, 4096), 256, 0, s>>>(val[u], n);
            HIP_TRY(hipGetLastError());
        }
    }
    for (int t = c->k - 1; t >= 1; --t) {
        const int u = c->bfs[t], p = c->parent[u];
        const int64_t np = c->ncand[p];
        if (!np) continue;
        k_workload_step<<<cstm_blocks(np, 256, 4096), 256, 0, s>>>(c->tree[u].off, c->tree[u].adj, np, val[u], val[p]);
        HIP_TRY(hipGetLastError());
    }
    const int64_t nr = c->ncand[c->root];
    std::vector<uint64_t> h((size_t)nr);
    if (nr) HIP_TRY(hipMemcpyAsync(h.data(), val[c->root], (size_t)nr * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    uint64_t w = 0;
    for (uint64_t x : h) w = (w + x < w) ? ~0ull : w + x;
    c->root_w = std::move(h);
    c->has_workload = true;
    return c->workload = w;
}

extern "C" cstm_status cstm_cst_workload(cstm_cst* c, uint64_t* w_out) {
    return cstm_guard([&] {
        CSTM_REQUIRE(c && w_out, CSTM_EINVAL, "NULL argument");
        HIP_TRY(hipSetDevice(c->ctx->device));
        *w_out = cstm_cst_workload_run(c);
    });
}

extern "C" cstm_status cstm_cst_times(const cstm_cst* c, double* build_ms, double* partition_ms, double* enumerate_ms) {
    return cstm_guard([&] {
        CSTM_REQUIRE(c, CSTM_EINVAL, "NULL cst");
        if (build_ms) *build_ms = c->t_build;
        if (partition_ms) *partition_ms = c->t_part;
        if (enumerate_ms) *enumerate_ms = c->t_enum;
    });
}
