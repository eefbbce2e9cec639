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
// Membership of a data vertex w in C(u) is one range test on w's packed
// (label, rank) key plus one lookup in a rank-indexed table.  G keeps a copy
// of its rows with the neighbours' keys grouped by label, so for an edge
// (u_p, u) only the run of each candidate's row that carries l(u) is read: a
// binary search finds it, and the run is read in order.  The runs of a
// parent's candidates are walked once per tree edge, in the top-down pass:
// each entry's rank test is kept (`erank`), and the bottom-up test and both
// passes over the tree list read it back in order.  Sizes stay on the device (kernels read them from a small table and
// run grids sized by host-side bounds from the label index), so a build waits
// for the device four times: for the tree-list sizes, the path counts of the
// order, the non-tree list sizes, and at the end.
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

// The label runs of a candidate array's rows, for one label, laid end to
// end: entry t of the flattened space is lkey[beg[i] + t - rowoff[i]], the
// (t - rowoff[i])-th neighbour of candidate i with that label, where rowoff is
// the exclusive prefix sum of the run lengths.  The number of candidates lives
// on the device (*n), and rowoff[*n] is the number of entries.  Kernels walk
// this space in parts: a part is at most kPartRounds rounds of 64 entries of
// one block of 64 candidates (whose runs are contiguous).  A block of at most
// 64 * kPartRounds entries is one part; a longer one (a hub's run) has
// 1 + extra[b] parts, spread over the wavefronts, with exoff the exclusive
// prefix of extra[] over the blocks (exoff[nblocks] = number of extra parts).
// Part p of block b has the index b + exoff[b] + p, so parts are numbered in
// the order of their entries.
constexpr int kPartRounds = 8;

struct Rows {
    const int32_t* cand;    // candidate data-vertex ids
    const int64_t* rowoff;  // n + 1 prefix sums of their run lengths
    const int64_t* beg;     // n: where each candidate's run starts in lkey
    const int64_t* n;       // device: number of candidates
    const int64_t* exoff;   // nblocks + 1: prefix of the extra parts per block
};

constexpr int kWaveBlock = 256;  // threads per workgroup of the run walks

__device__ inline int32_t wave_incl_max(int32_t x) {
    const int lane = lane_id();
    for (int o = 1; o < CSTM_WAVE; o <<= 1) {
        const int32_t y = __shfl_up(x, o, CSTM_WAVE);
        if (lane >= o && y > x) x = y;
    }
    return x;
}

// Extra parts of each block of 64 candidates (beyond its first) and, in
// *nblocks, the number of blocks, for the scan that makes exoff.
__global__ void k_extra_parts(const int64_t* __restrict__ rowoff, const int64_t* __restrict__ n_dev,
                              int64_t* __restrict__ extra, int64_t* __restrict__ nblocks) {
    const int64_t n = *n_dev;
    const int64_t nb = (n + CSTM_WAVE - 1) / CSTM_WAVE;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (first == 0) *nblocks = nb;
    for (int64_t b = first; b < nb; b += stride) {
        const int64_t lo = b * CSTM_WAVE, hi = lo + CSTM_WAVE < n ? lo + CSTM_WAVE : n;
        const int64_t rounds = (rowoff[hi] - rowoff[lo] + CSTM_WAVE - 1) / CSTM_WAVE;
        const int64_t parts = (rounds + kPartRounds - 1) / kPartRounds;
        extra[b] = parts > 1 ? parts - 1 : 0;
    }
}

// Walk the runs part by part.  begin(item) and end(item) run once per part,
// with the part's index; entry(valid, t, i, pos) runs on every lane of every
// round, with the entry's flattened index t, its owner i and its position pos
// in lkey (valid is false for the lanes past the block's last entry, whose t,
// i and pos are not to be used but whose owner i is still a candidate of the
// block).  The owner of an entry is the last lane whose non-empty run starts
// at or before it: the run starts inside a round are marked (starts of
// non-empty runs are distinct) and a prefix maximum carries them forward from
// the owner of the entry before the round, which one ballot finds.  First
// every block's first part (one wavefront per block), then the extra parts of
// long blocks, each found by a binary search over exoff.
template <class Begin, class Entry, class End>
__device__ inline void for_blocks(const Rows& R, Begin&& begin, Entry&& entry, End&& end) {
    __shared__ int32_t s_mark[kWaveBlock / CSTM_WAVE][CSTM_WAVE];
    int32_t* mark = s_mark[threadIdx.x / CSTM_WAVE];
    const int lane = lane_id();
    const int64_t n = *R.n;
    const int64_t nblocks = (n + CSTM_WAVE - 1) / CSTM_WAVE;
    auto part = [&](int64_t blk, int64_t p) {
        const int64_t first = blk * CSTM_WAVE;
        const int64_t last = first + CSTM_WAVE < n ? first + CSTM_WAVE : n;
        const int64_t i = first + lane;
        const bool has = i < last;
        const int64_t r0 = R.rowoff[first];
        const int64_t total = R.rowoff[last] - r0;
        const int64_t start = has ? R.rowoff[i] - r0 : 0;
        const int64_t len = has ? R.rowoff[i + 1] - r0 - start : 0;
        const int64_t beg = has ? R.beg[i] : 0;
        const int64_t item = blk + R.exoff[blk] + p;
        const int64_t tb = p * (int64_t)kPartRounds * CSTM_WAVE;
        const int64_t te = tb + (int64_t)kPartRounds * CSTM_WAVE < total ? tb + (int64_t)kPartRounds * CSTM_WAVE : total;
        begin(item);
        const uint64_t before = ballot(len > 0 && start < tb);
        int32_t carry = before ? 63 - __clzll(before) : 0;  // owner lane of the entry before the part
        for (int64_t t0 = tb; t0 < te; t0 += CSTM_WAVE) {
            mark[lane] = -1;
            __builtin_amdgcn_wave_barrier();
            if (len > 0 && start >= t0 && start < t0 + CSTM_WAVE) mark[start - t0] = lane;
            __builtin_amdgcn_wave_barrier();
            const int32_t m = wave_incl_max(mark[lane]);
            __builtin_amdgcn_wave_barrier();
            const int32_t own = m > carry ? m : carry;
            carry = __builtin_amdgcn_readlane(own, CSTM_WAVE - 1);
            const int64_t tl = t0 + lane;
            const int64_t ostart = __shfl(start, own);
            const int64_t obeg = __shfl(beg, own);
            entry(tl < te, r0 + tl, first + own, obeg + (tl - ostart));
        }
        end(item);
    };
    for (int64_t blk = global_wave(); blk < nblocks; blk += num_waves()) part(blk, 0);
    const int64_t nextra = R.exoff[nblocks];
    for (int64_t e = global_wave(); e < nextra; e += num_waves()) {
        int64_t lo = 0, hi = nblocks - 1;  // the block b with exoff[b] <= e < exoff[b + 1]
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (R.exoff[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        part(lo, 1 + e - R.exoff[lo]);
    }
}

// The run of label l in each candidate's label-grouped row: its start by a
// binary search over the row, its end by a galloping search from the start
// (runs are mostly short, so the end is usually one or two probes away).
template <class K>
__global__ void k_seg(const int32_t* __restrict__ cand, const int64_t* __restrict__ n_dev,
                      const int64_t* __restrict__ row_ptr, const K* __restrict__ lkey, int shift, uint64_t l,
                      int64_t* __restrict__ len, int64_t* __restrict__ beg) {
    const int64_t n = *n_dev;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int32_t v = cand[i];
        int64_t lo = row_ptr[v], hi = row_ptr[v + 1];
        const int64_t e = hi;
        while (lo < hi) {  // first entry with label >= l
            const int64_t mid = lo + ((hi - lo) >> 1);
            if ((uint64_t)(lkey[mid] >> shift) < l) lo = mid + 1;
            else hi = mid;
        }
        const int64_t b = lo;
        // first entry with label > l: nothing to find for an empty run; else
        // probe b + 1, b + 3, b + 7, ... until one passes the run (or the row
        // ends), then search the last gap
        hi = b;
        if (b < e && (uint64_t)(lkey[b] >> shift) == l) {
            int64_t prev = b, step = 1;
            for (;;) {
                const int64_t nxt = prev + step;
                if (nxt >= e || (uint64_t)(lkey[nxt] >> shift) > l) {
                    lo = prev + 1;
                    hi = nxt < e ? nxt : e;
                    break;
                }
                prev = nxt;
                step <<= 1;
            }
        }
        while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            if ((uint64_t)(lkey[mid] >> shift) <= l) lo = mid + 1;
            else hi = mid;
        }
        beg[i] = b;
        len[i] = lo - b;
    }
}

// Top-down marking for a tree edge (u_p -> u): every neighbour of a parent
// candidate that passes u's label/degree filter is marked in u's rank table,
// and each entry's rank (or -1) is kept in erank for the later passes.  R
// holds the runs of label l(u), so only the degree filter (a rank below cnt0)
// is left to test.
template <class K>
__global__ void k_mark(Rows R, const K* __restrict__ lkey, K base, int64_t cnt0, int32_t* __restrict__ mark,
                       int32_t* __restrict__ erank) {
    for_blocks(
        R, [](int64_t) {},
        [&](bool valid, int64_t t, int64_t, int64_t pos) {
            if (!valid) return;
            const uint64_t d = (uint64_t)(K)(lkey[pos] - base);
            const bool hit = d < (uint64_t)cnt0;
            erank[t] = hit ? (int32_t)d : -1;
            if (hit) mark[d] = 1;
        },
        [](int64_t) {});
}

// marks -> candidate indices: C(u) in rank order (degree desc, id asc); each
// candidate's rank is kept in tdrank.
__global__ void k_assign(int32_t* __restrict__ loc, const int32_t* __restrict__ scan, int64_t cnt0,
                         const int32_t* __restrict__ perm_base, int32_t* __restrict__ cand,
                         int32_t* __restrict__ tdrank) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < cnt0; r += stride) {
        if (loc[r]) {
            const int32_t j = scan[r];
            cand[j] = perm_base[r];
            tdrank[j] = (int32_t)r;
            loc[r] = j;
        } else {
            loc[r] = -1;
        }
    }
}

__global__ void k_iota_root(int32_t* __restrict__ loc, int64_t cnt0, const int32_t* __restrict__ perm_base,
                            int32_t* __restrict__ cand, int32_t* __restrict__ tdrank) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < cnt0; r += stride) {
        loc[r] = (int32_t)r;
        cand[r] = perm_base[r];
        tdrank[r] = (int32_t)r;
    }
}

// One tree child of the vertex being refined: the ranks its top-down pass
// kept over the vertex's runs of the child's label (offsets rowoff), and its
// (already refined) rank table.
struct ChildRef {
    const int32_t* erank;
    const int32_t* loc;
    const int64_t* rowoff;
};
struct ChildSet {
    int32_t n;
    ChildRef c[CSTM_MAX_K];
};

// Bottom-up validity: a candidate needs a neighbour in every refined child set.
// One wavefront per candidate, reading the kept ranks of its runs.
__global__ void k_valid(const int64_t* __restrict__ n_dev, ChildSet ch, int32_t* __restrict__ flag) {
    const int lane = lane_id();
    const int64_t n = *n_dev;
    for (int64_t i = global_wave(); i < n; i += num_waves()) {
        bool ok = true;
        for (int c = 0; c < ch.n && ok; ++c) {
            const ChildRef cr = ch.c[c];
            const int64_t b = cr.rowoff[i], e = cr.rowoff[i + 1];
            bool found = false;
            for (int64_t j0 = b; j0 < e && !found; j0 += CSTM_WAVE) {
                const int64_t j = j0 + lane;
                bool hit = false;
                if (j < e) {
                    const int32_t r = cr.erank[j];
                    hit = r >= 0 && cr.loc[r] >= 0;
                }
                found = ballot(hit) != 0;
            }
            ok = found;
        }
        if (lane == 0) flag[i] = ok ? 1 : 0;
    }
}

// Compaction of the top-down set to the refined one; newidx maps a top-down
// index to the refined index (or -1), the rank table follows.
__global__ void k_refine(const int32_t* __restrict__ cand_td, const int32_t* __restrict__ tdrank,
                         const int32_t* __restrict__ flag, const int32_t* __restrict__ scan,
                         const int64_t* __restrict__ n_dev, int32_t* __restrict__ loc, int32_t* __restrict__ cand,
                         int32_t* __restrict__ newidx) {
    const int64_t n = *n_dev;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (flag[i]) {
            const int32_t j = scan[i];
            cand[j] = cand_td[i];
            loc[tdrank[i]] = j;
            newidx[i] = j;
        } else {
            loc[tdrank[i]] = -1;
            newidx[i] = -1;
        }
    }
}

__global__ void k_copy_i64(const int64_t* __restrict__ src, int64_t* __restrict__ dst) { *dst = *src; }

// Adds the hits of one 64-entry step to the per-owner counts: owners never
// decrease across lanes, so one atomic per run of lanes with the same owner.
__device__ inline void add_runs(int64_t owner, int32_t ni, uint64_t hits, unsigned long long* __restrict__ cnt) {
    const int lane = lane_id();
    const int64_t prev = __shfl_up(owner, 1, CSTM_WAVE);
    const bool head = lane == 0 || prev != owner;
    const uint64_t heads = ballot(head);
    if (head && ni >= 0) {
        const uint64_t later = lane == CSTM_WAVE - 1 ? 0ull : (heads >> (lane + 1)) << (lane + 1);
        const uint64_t upto = later ? (later & (~later + 1)) - 1 : ~0ull;  // bits below the next head
        const uint64_t run = upto & ~((1ull << lane) - 1);
        const int c = __popcll(hits & run);
        if (c) atomicAdd(&cnt[ni], (unsigned long long)c);
    }
}

// Tree list (u_p -> u) sizes from the kept ranks: an entry is in the list of
// its (refined) owner when its rank survives in u's rank table.  Per refined
// owner counts go to cnt (zeroed by the caller), per block counts to tile_cnt.
__global__ void k_tree_count(Rows R, const int32_t* __restrict__ newidx, const int32_t* __restrict__ erank,
                             const int32_t* __restrict__ loc, unsigned long long* __restrict__ cnt,
                             int64_t* __restrict__ tile_cnt) {
    const int lane = lane_id();
    int64_t in_tile = 0;
    for_blocks(
        R, [&](int64_t) { in_tile = 0; },
        [&](bool valid, int64_t t, int64_t i, int64_t) {
            const int32_t ni = newidx ? newidx[i] : (int32_t)i;
            bool hit = false;
            if (valid && ni >= 0) {
                const int32_t r = erank[t];
                hit = r >= 0 && loc[r] >= 0;
            }
            const uint64_t hits = ballot(hit);
            in_tile += __popcll(hits);
            add_runs(i, ni, hits, cnt);
        },
        [&](int64_t blk) {
            if (lane == 0) tile_cnt[blk] = in_tile;
        });
}

// Tree list entries, in run order (ascending data-vertex id), as indices
// into C(u): the hits of the flattened space are numbered in order, block by
// block from tile_base, which lays the lists of consecutive owners end to end
// exactly as the offsets from the per-owner counts do.
__global__ void k_tree_fill(Rows R, const int32_t* __restrict__ newidx, const int32_t* __restrict__ erank,
                            const int32_t* __restrict__ loc, const int64_t* __restrict__ tile_base,
                            int32_t* __restrict__ adj) {
    int64_t out = 0;
    for_blocks(
        R, [&](int64_t blk) { out = tile_base[blk]; },
        [&](bool valid, int64_t t, int64_t i, int64_t) {
            int32_t idx = -1;
            if (valid) {
                const int32_t ni = newidx ? newidx[i] : (int32_t)i;
                const int32_t r = erank[t];
                if (ni >= 0 && r >= 0) idx = loc[r];
            }
            const uint64_t m = ballot(idx >= 0);
            if (idx >= 0) adj[out + mbcnt(m)] = idx;
            out += __popcll(m);
        },
        [](int64_t) {});
}

// Non-tree list (a -> b) sizes over a's runs of label l(b): each entry's
// index in C(b) (or -1) is kept in E for the fill, per refined owner counts go
// to cnt, per tile counts to tile_cnt.
template <class K>
__global__ void k_nt_count(Rows R, const int32_t* __restrict__ newidx, const K* __restrict__ lkey, K base,
                           int64_t cnt0, const int32_t* __restrict__ loc, int32_t* __restrict__ E,
                           unsigned long long* __restrict__ cnt, int64_t* __restrict__ tile_cnt) {
    const int lane = lane_id();
    int64_t in_tile = 0;
    for_blocks(
        R, [&](int64_t) { in_tile = 0; },
        [&](bool valid, int64_t t, int64_t i, int64_t pos) {
            const int32_t ni = newidx ? newidx[i] : (int32_t)i;
            int32_t idx = -1;
            if (valid && ni >= 0) {
                const uint64_t d = (uint64_t)(K)(lkey[pos] - base);
                if (d < (uint64_t)cnt0) idx = loc[d];
            }
            if (valid) E[t] = idx;
            const uint64_t hits = ballot(idx >= 0);
            in_tile += __popcll(hits);
            add_runs(i, ni, hits, cnt);
        },
        [&](int64_t blk) {
            if (lane == 0) tile_cnt[blk] = in_tile;
        });
}

// Non-tree list entries from E, with their data-vertex ids from C(b)
// (ascending within each list, since runs keep the ids ascending).
__global__ void k_nt_fill(Rows R, const int32_t* __restrict__ E, const int64_t* __restrict__ tile_base,
                          const int32_t* __restrict__ cand_b, int32_t* __restrict__ adj,
                          int32_t* __restrict__ adj_gid) {
    int64_t out = 0;
    for_blocks(
        R, [&](int64_t blk) { out = tile_base[blk]; },
        [&](bool valid, int64_t t, int64_t, int64_t) {
            const int32_t idx = valid ? E[t] : -1;
            const uint64_t m = ballot(idx >= 0);
            if (idx >= 0) {
                adj[out + mbcnt(m)] = idx;
                adj_gid[out + mbcnt(m)] = cand_b[idx];
            }
            out += __popcll(m);
        },
        [](int64_t) {});
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

// Grid of a run walk over at most `cands` candidates: one wavefront per block
// of 64, at most kMaxWalkWaves (the walk is grid-strided, and the candidate
// bound from the label index is loose, so a larger grid would mostly launch
// idle waves).
constexpr int64_t kMaxWalkWaves = 8192;
unsigned walk_grid(int64_t cands) {
    const int64_t blocks = (cands + CSTM_WAVE - 1) / CSTM_WAVE;
    return wave_grid(blocks < 1 ? 1 : blocks < kMaxWalkWaves ? blocks : kMaxWalkWaves);
}

// Blocks of 64 candidates among at most `cands` (plus one).
int64_t blocks_of(int64_t cands) { return (cands + CSTM_WAVE - 1) / CSTM_WAVE + 1; }

// Slots of a per-part count array over at most `cands` candidates whose runs
// hold at most `entries` entries: a block's extra part covers a full part of
// entries of that block.
int64_t parts_of(int64_t cands, int64_t entries) {
    return blocks_of(cands) + entries / ((int64_t)kPartRounds * CSTM_WAVE) + 1;
}

// The device size table of one build: per query vertex its top-down set size
// and refined set size; per candidate list its entries.
constexpr int kNsz = 0, kNfin = CSTM_MAX_K, kLent = 2 * CSTM_MAX_K;
constexpr int kMetaSlots = 3 * CSTM_MAX_K + CSTM_MAX_NT;

__global__ void k_set_i64(int64_t* __restrict__ p, int64_t v) { *p = v; }

}  // namespace

// One CST build: the query's tree and order on the host, every set and list on
// the device.  Temporaries live in `tmp` until the last wait.
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

    // host bounds from the label index: C(u) lies in the filtered prefix of
    // its label group, so that prefix bounds its size and its degree sum
    // bounds the entries of its rows
    int64_t rbound[CSTM_MAX_K];
    for (int u = 0; u < k; ++u)
        rbound[u] = c->cnt0[u] ? g->deg_prefix[c->lb_lo[u] + c->cnt0[u]] - g->deg_prefix[c->lb_lo[u]] : 0;
    // entries of the runs of label l(b) over a's candidates: a's degree sum,
    // and the edges of G between the two labels
    auto run_bound = [&](int a, int b) -> int64_t {
        const uint64_t pb = g->pair_bound(q.qlabel[a], q.qlabel[b]);
        return (uint64_t)rbound[a] < pb ? rbound[a] : (int64_t)pb;
    };
    const bool k32 = g->key32 != nullptr;
    auto key_base = [&](int u) { return (uint64_t)q.qlabel[u] << g->key_shift; };
    CSTM_REQUIRE(g->nnz == 0 || (k32 ? g->lkey32 != nullptr : g->lkey64 != nullptr), CSTM_EINVAL,
                 "graph has no label-grouped rows");

    DevArena tmp;
    tmp.ctx = c->ctx;
    // destroyed before tmp: a failed build lets its kernels finish before their blocks go back
    struct WaitOnExit {
        hipStream_t s;
        ~WaitOnExit() { (void)hipStreamSynchronize(s); }
    } wait_on_exit{s};
    int64_t* meta = tmp.get_n<int64_t>(kMetaSlots);
    cstm_fill_words(meta, kMetaSlots * sizeof(int64_t), 0u, s);
    int64_t* part = tmp.get_n<int64_t>(kScanPartSlots);  // scan scratch; every scan runs on this one stream
    const int n_slots = k + (int)c->nontree.size();
    int* d_max = tmp.get_n<int>(n_slots);
    cstm_fill_words(d_max, (size_t)n_slots * sizeof(int), 0u, s);
    auto nsz = [&](int u) { return meta + kNsz + u; };
    auto nfin = [&](int u) { return meta + kNfin + u; };

    int32_t* loc[CSTM_MAX_K] = {};     // rank table: rank -> index in C(u), or -1
    int32_t* cand_td[CSTM_MAX_K] = {}; // top-down set (bound-sized)
    int32_t* tdrank[CSTM_MAX_K] = {};  // rank of each top-down candidate
    int32_t* cand_fin[CSTM_MAX_K] = {};  // refined set (top-down set for leaves)
    int32_t* newidx[CSTM_MAX_K] = {};  // top-down index -> refined index (nullptr: identity)
    int32_t* erank[CSTM_MAX_K] = {};   // by tree child: kept ranks over the parent's runs of its label
    Rows trows[CSTM_MAX_K] = {};       // by tree child: the parent's top-down set, runs of the child's label
    // runs of label l over u's top-down set, made once per (u, l)
    struct RunsOf {
        int u;
        int32_t l;
        Rows r;
    };
    std::vector<RunsOf> runs;
    auto runs_of = [&](int u, int32_t l) -> Rows {
        for (const RunsOf& x : runs)
            if (x.u == u && x.l == l) return x.r;
        const int64_t c0 = c->cnt0[u];
        int64_t* len = tmp.get_n<int64_t>(c0 + 1);
        int64_t* beg = tmp.get_n<int64_t>(c0 + 1);
        int64_t* off = tmp.get_n<int64_t>(c0 + 1);
        if (k32)
            k_seg<uint32_t><<<cstm_blocks(c0, 256, 4096), 256, 0, s>>>(cand_td[u], nsz(u), g->row_ptr, g->lkey32,
                                                                        g->key_shift, (uint64_t)l, len, beg);
        else
            k_seg<uint64_t><<<cstm_blocks(c0, 256, 4096), 256, 0, s>>>(cand_td[u], nsz(u), g->row_ptr, g->lkey64,
                                                                        g->key_shift, (uint64_t)l, len, beg);
        HIP_TRY(hipGetLastError());
        cstm_dscan_i64(len, off, nsz(u), c0, nullptr, part, s);
        // extra parts of long blocks: len is free again, and the block count
        // goes to the last size-table slot of this (u, l)
        const int64_t nbb = blocks_of(c0);
        int64_t* exoff = tmp.get_n<int64_t>(nbb + 1);
        int64_t* nb_dev = tmp.get_n<int64_t>(1);
        k_extra_parts<<<cstm_blocks(nbb, 256, 1024), 256, 0, s>>>(off, nsz(u), len, nb_dev);
        HIP_TRY(hipGetLastError());
        cstm_dscan_i64(len, exoff, nb_dev, nbb, nullptr, part, s);
        runs.push_back({u, l, Rows{cand_td[u], off, beg, nsz(u), exoff}});
        return runs.back().r;
    };

    // tree lists: per child, the offsets over the refined parent set (bound-sized) and the tile bases
    int64_t* toff_b[CSTM_MAX_K] = {};
    int64_t* tbase[CSTM_MAX_K] = {};
    if (!c->empty) {
        // 1. root candidates: the filtered prefix of the root's label group
        // a leaf's top-down set is its final set and a refined set is final:
        // both are made in the CST's own memory (bound-sized), so nothing is
        // copied once the sizes are known
        bool leaf[CSTM_MAX_K];
        for (int u = 0; u < k; ++u) {
            leaf[u] = true;
            for (int w = 0; w < k; ++w) leaf[u] = leaf[u] && c->parent[w] != u;
        }
        auto td_mem = [&](int u) { return leaf[u] ? c->mem.get_n<int32_t>(c->cnt0[u]) : tmp.get_n<int32_t>(c->cnt0[u]); };
        const int64_t c0r = c->cnt0[root];
        loc[root] = tmp.get_n<int32_t>(c0r);
        cand_td[root] = td_mem(root);
        tdrank[root] = tmp.get_n<int32_t>(c0r);
        k_iota_root<<<cstm_blocks(c0r, 256, 4096), 256, 0, s>>>(loc[root], c0r, g->perm + c->lb_lo[root],
                                                                cand_td[root], tdrank[root]);
        HIP_TRY(hipGetLastError());
        k_set_i64<<<1, 1, 0, s>>>(nsz(root), c0r);
        HIP_TRY(hipGetLastError());
        // 2. top-down construction, keeping each entry's rank test
        for (int t = 1; t < k; ++t) {
            const int u = c->bfs[t], up = c->parent[u];
            const int64_t c0 = c->cnt0[u];
            trows[u] = runs_of(up, q.qlabel[u]);
            loc[u] = tmp.get_n<int32_t>(c0);
            cstm_fill_words(loc[u], (size_t)c0 * 4, 0u, s);
            erank[u] = tmp.get_n<int32_t>(std::max<int64_t>(run_bound(up, u), 1));
            if (k32)
                k_mark<uint32_t><<<walk_grid(c->cnt0[up]), kWaveBlock, 0, s>>>(
                    trows[u], g->lkey32, (uint32_t)key_base(u), c0, loc[u], erank[u]);
            else
                k_mark<uint64_t><<<walk_grid(c->cnt0[up]), kWaveBlock, 0, s>>>(trows[u], g->lkey64, key_base(u), c0,
                                                                               loc[u], erank[u]);
            HIP_TRY(hipGetLastError());
            int32_t* scan = tmp.get_n<int32_t>(c0 + 1);
            cstm_dscan_i32(loc[u], scan, nullptr, c0, nsz(u), part, s);
            cand_td[u] = td_mem(u);
            tdrank[u] = tmp.get_n<int32_t>(c0);
            k_assign<<<cstm_blocks(c0, 256, 4096), 256, 0, s>>>(loc[u], scan, c0, g->perm + c->lb_lo[u], cand_td[u],
                                                                tdrank[u]);
            HIP_TRY(hipGetLastError());
        }
        // 3. bottom-up refinement, children first, from the kept ranks
        for (int t = k - 1; t >= 0; --t) {
            const int u = c->bfs[t];
            ChildSet ch{};
            for (int w = 0; w < k; ++w)
                if (c->parent[w] == u) ch.c[ch.n++] = ChildRef{erank[w], loc[w], trows[w].rowoff};
            if (ch.n == 0) {
                cand_fin[u] = cand_td[u];
                k_copy_i64<<<1, 1, 0, s>>>(nsz(u), nfin(u));
                HIP_TRY(hipGetLastError());
                continue;
            }
            const int64_t c0 = c->cnt0[u];
            int32_t* flag = tmp.get_n<int32_t>(c0 + 1);
            k_valid<<<wave_grid(std::min<int64_t>(c0, kMaxWalkWaves)), kWaveBlock, 0, s>>>(nsz(u), ch, flag);
            HIP_TRY(hipGetLastError());
            int32_t* scan = tmp.get_n<int32_t>(c0 + 1);
            cstm_dscan_i32(flag, scan, nsz(u), c0, nfin(u), part, s);
            cand_fin[u] = c->mem.get_n<int32_t>(c0);
            newidx[u] = tmp.get_n<int32_t>(c0);
            k_refine<<<cstm_blocks(c0, 256, 4096), 256, 0, s>>>(cand_td[u], tdrank[u], flag, scan, nsz(u), loc[u],
                                                                cand_fin[u], newidx[u]);
            HIP_TRY(hipGetLastError());
        }
        // 4a. tree list sizes (parent -> child), from the kept ranks
        for (int t = 1; t < k; ++t) {
            const int u = c->bfs[t], p = c->parent[u];
            const int64_t c0p = c->cnt0[p], nt = parts_of(c0p, run_bound(p, u));
            // per-owner and per-part counts, zeroed by one fill
            unsigned long long* cnt = tmp.get_n<unsigned long long>(c0p + nt + 2);
            int64_t* tcnt = (int64_t*)(cnt + c0p + 1);
            cstm_fill_words(cnt, (size_t)(c0p + nt + 2) * 8, 0u, s);
            k_tree_count<<<walk_grid(c->cnt0[p]), kWaveBlock, 0, s>>>(trows[u], newidx[p], erank[u], loc[u], cnt, tcnt);
            HIP_TRY(hipGetLastError());
            // the list offsets stay with the CST; the scan also finds the longest list
            toff_b[u] = c->mem.get_n<int64_t>(c0p + 1);
            cstm_dscan_i64((const int64_t*)cnt, toff_b[u], nfin(p), c0p, meta + kLent + u, part, s, d_max + u);
            tbase[u] = tmp.get_n<int64_t>(nt + 1);
            cstm_dscan_i64(tcnt, tbase[u], nullptr, nt, nullptr, part, s);
        }
    }
    // wait 1: the refined set sizes and the tree list sizes
    std::vector<int64_t> hm(kMetaSlots, 0);
    HIP_TRY(hipMemcpyAsync(hm.data(), meta, kMetaSlots * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (!c->empty) {
        for (int u = 0; u < k; ++u) {
            c->ncand[u] = hm[kNfin + u];
            if (c->ncand[u] == 0) c->empty = true;
        }
        // a set emptied by the refinement leaves no embedding: keep no candidates at all
        if (c->empty)
            for (int u = 0; u < k; ++u) c->ncand[u] = 0;
    }
    if (!c->empty) {
        for (int u = 0; u < k; ++u) c->cand[u] = cand_fin[u];
        for (int t = 1; t < k; ++t) {
            const int u = c->bfs[t], p = c->parent[u];
            EdgeLists& el = c->tree[u];
            el.from = -1;
            el.to = -1;
            el.entries = hm[kLent + u];
            el.off = toff_b[u];
            el.adj = c->mem.get_n<int32_t>(el.entries ? el.entries : 1);
            k_tree_fill<<<walk_grid(c->cnt0[p]), kWaveBlock, 0, s>>>(trows[u], newidx[p], erank[u], loc[u], tbase[u],
                                                                    el.adj);
            HIP_TRY(hipGetLastError());
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
    } else if (c->ctx->tune.order_rule == 1) {
        // constraint first: among the vertices whose tree parent is placed,
        // the one with the most placed query neighbours (so non-tree edges
        // are checked as early as the tree allows), then the larger query
        // degree, then the smaller id
        uint32_t placed = 1u << root;
        c->order[0] = root;
        for (int i = 1; i < k; ++i) {
            int best = -1, best_nb = -1;
            for (int u = 0; u < k; ++u) {
                if ((placed >> u & 1u) || !(placed >> c->parent[u] & 1u)) continue;
                const int nb = __builtin_popcount(q.adj[u] & placed);
                if (nb > best_nb || (nb == best_nb && c->qdeg[u] > c->qdeg[best])) {
                    best = u;
                    best_nb = nb;
                }
            }
            placed |= 1u << best;
            c->order[i] = best;
        }
        for (int i = 0; i < k; ++i) c->pos_of[c->order[i]] = i;
    } else {
        // root-to-leaf paths and their numbers of CST path embeddings, all
        // computed before one wait
        std::vector<std::vector<int>> plist;
        for (int leaf = 0; leaf < k; ++leaf) {
            bool has_child = false;
            for (int w = 0; w < k; ++w) has_child |= c->parent[w] == leaf;
            if (has_child || (leaf == root && k > 1)) continue;
            std::vector<int> p{leaf};
            while (c->parent[p.back()] >= 0) p.push_back(c->parent[p.back()]);
            std::reverse(p.begin(), p.end());
            plist.push_back(p);
        }
        const int np = (int)plist.size();
        unsigned long long* d_paths = tmp.get_n<unsigned long long>(std::max(np, 1));
        cstm_fill_words(d_paths, (size_t)std::max(np, 1) * 8, 0u, s);
        std::vector<uint64_t> pcnt((size_t)np, 0);
        if (!c->empty) {
            for (int pi = 0; pi < np; ++pi) {
                const std::vector<int>& p = plist[pi];
                if (p.size() == 1) {
                    pcnt[pi] = (uint64_t)c->ncand[p[0]];
                    continue;
                }
                const uint64_t* child_val = nullptr;
                for (int i = (int)p.size() - 2; i >= 0; --i) {
                    const int u = p[i], uc = p[i + 1];
                    uint64_t* vals = tmp.get_n<uint64_t>(c->ncand[u] ? c->ncand[u] : 1);
                    k_path_step<<<cstm_blocks(c->ncand[u], 256, 4096), 256, 0, s>>>(
                        c->tree[uc].off, c->tree[uc].adj, c->ncand[u], child_val, vals);
                    HIP_TRY(hipGetLastError());
                    child_val = vals;
                }
                k_sum_sat<<<cstm_blocks(c->ncand[root], 256, 1024), 256, 0, s>>>(child_val, c->ncand[root],
                                                                                   d_paths + pi);
                HIP_TRY(hipGetLastError());
            }
            // wait 2: the path counts
            std::vector<unsigned long long> hp((size_t)std::max(np, 1));
            HIP_TRY(hipMemcpyAsync(hp.data(), d_paths, hp.size() * 8, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            for (int pi = 0; pi < np; ++pi)
                if (plist[pi].size() > 1) pcnt[pi] = hp[pi];
        }
        std::vector<int> idx((size_t)np);
        std::iota(idx.begin(), idx.end(), 0);
        std::sort(idx.begin(), idx.end(), [&](int x, int y) {
            return pcnt[x] != pcnt[y] ? pcnt[x] < pcnt[y] : plist[x].back() < plist[y].back();
        });
        int n = 0;
        uint32_t placed = 0;
        for (int pi : idx)
            for (int u : plist[pi])
                if (!(placed >> u & 1u)) {
                    placed |= 1u << u;
                    c->order[n++] = u;
                }
        if (n == 0) c->order[n++] = root;
        for (int i = 0; i < k; ++i) c->pos_of[c->order[i]] = i;
    }
    // 4c. non-tree candidate edges, earlier -> later in the order: sizes, one wait, fills
    std::vector<int32_t*> ntE(c->nontree.size(), nullptr);
    std::vector<int64_t*> ntbase(c->nontree.size(), nullptr);
    std::vector<Rows> ntrows(c->nontree.size());
    for (size_t j = 0; j < c->nontree.size(); ++j) {
        int a = c->nontree[j].first, b = c->nontree[j].second;
        if (c->pos_of[a] > c->pos_of[b]) std::swap(a, b);
        EdgeLists el;
        el.from = c->pos_of[a];
        el.to = c->pos_of[b];
        if (!c->empty) {
            ntrows[j] = runs_of(a, q.qlabel[b]);
            const int64_t nt = parts_of(c->cnt0[a], run_bound(a, b));
            unsigned long long* cnt = tmp.get_n<unsigned long long>(c->ncand[a] + nt + 2);
            int64_t* tcnt = (int64_t*)(cnt + c->ncand[a] + 1);
            cstm_fill_words(cnt, (size_t)(c->ncand[a] + nt + 2) * 8, 0u, s);
            ntE[j] = tmp.get_n<int32_t>(std::max<int64_t>(run_bound(a, b), 1));
            if (k32)
                k_nt_count<uint32_t><<<walk_grid(c->cnt0[a]), kWaveBlock, 0, s>>>(
                    ntrows[j], newidx[a], g->lkey32, (uint32_t)key_base(b), c->cnt0[b], loc[b], ntE[j], cnt, tcnt);
            else
                k_nt_count<uint64_t><<<walk_grid(c->cnt0[a]), kWaveBlock, 0, s>>>(
                    ntrows[j], newidx[a], g->lkey64, key_base(b), c->cnt0[b], loc[b], ntE[j], cnt, tcnt);
            HIP_TRY(hipGetLastError());
            el.off = c->mem.get_n<int64_t>(c->ncand[a] + 1);
            cstm_dscan_i64((const int64_t*)cnt, el.off, nullptr, c->ncand[a], meta + kLent + k + (int)j, part, s,
                           d_max + k + (int)j);
            ntbase[j] = tmp.get_n<int64_t>(nt + 1);
            cstm_dscan_i64(tcnt, ntbase[j], nullptr, nt, nullptr, part, s);
        } else {
            el.off = nullptr;
        }
        c->nt.push_back(el);
    }
    if (!c->empty && !c->nontree.empty()) {
        // wait 3: the non-tree list sizes
        HIP_TRY(hipMemcpyAsync(hm.data(), meta, kMetaSlots * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (size_t j = 0; j < c->nontree.size(); ++j) {
            EdgeLists& el = c->nt[j];
            const int a = c->order[el.from], b = c->order[el.to];
            el.entries = hm[kLent + k + (int)j];
            el.adj = c->mem.get_n<int32_t>(el.entries ? el.entries : 1);
            el.adj_gid = c->mem.get_n<int32_t>(el.entries ? el.entries : 1);
            k_nt_fill<<<walk_grid(c->cnt0[a]), kWaveBlock, 0, s>>>(ntrows[j], ntE[j], ntbase[j], c->cand[b], el.adj,
                                                                  el.adj_gid);
            HIP_TRY(hipGetLastError());
        }
    }
    // wait 4: the longest lists (and every fill before the temporaries go back)
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
    }
    std::sort(c->nt.begin(), c->nt.end(), [](const EdgeLists& x, const EdgeLists& y) {
        return x.to != y.to ? x.to < y.to : x.from < y.from;
    });

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
    c->mem_bytes = c->mem.used();
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
