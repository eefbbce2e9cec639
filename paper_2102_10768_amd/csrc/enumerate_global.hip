// enumerate_global.hip -- enumeration with the CST resident in HBM (L2/MALL) and
// GPU-wide dynamic load balancing.
//
// This is the "CST read from device memory" variant of the paper's matcher
// (FAST-DRAM in Section VII-A), rebuilt for a GPU: the CST of one query is a
// few hundred KB to a few MB, so it stays in each XCD's L2 / the Infinity
// Cache, and every wavefront can work on any part of it.  That removes the
// replication that partitioning into 160 KB LDS images causes on power-law
// graphs, and lets the whole GPU share one query's search.
//
// Work unit: a task = (query slot, level j, a range of the candidate list at
// level j, the mapped candidates of levels 0..j-1).  Wavefronts pop tasks from
// a ring buffer and run the same bounded depth-first expansion as the on-chip
// enumerator (64 candidates per level and round, ballot compaction, deepest
// level first).  When some wavefronts are idle, a busy wavefront donates the
// unexpanded remainder of its shallowest open level as a new task, so a skewed
// search (one hub candidate owning most embeddings) spreads over the machine.
// Edge validation reads the non-tree candidate list of the mapped neighbour,
// stored as ascending data-vertex ids, by binary search.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace {

struct GTask {
    int32_t q;
    int32_t depth;
    int64_t lo, hi;  // depth 0: root candidate indices; else offsets into the level's tree list array
    int32_t prefix[CSTM_MAX_K];
};

// Each counter sits on its own 256-byte line: thousands of wavefronts poll
// them, and sharing a line would serialise every poll behind every update.
struct alignas(256) GLine {
    unsigned long long v;
    unsigned long long pad[31];
};
struct GQueue {
    GLine head;         // next ticket a consumer takes (may run ahead of tail: waiting consumers)
    GLine tail;         // next ticket a producer fills
    GLine outstanding;  // tasks pushed and not finished
    GLine abort;        // first reason to stop wins: 1 no progress for idle_limit, 2 deadline passed
    GLine beat;         // s_memrealtime tick at which some busy wavefront last reported progress
};

// How often (s_memrealtime ticks, 100 MHz) a busy wavefront refreshes the
// progress beat: 1 ms keeps the stores to that line rare.
constexpr uint64_t kBeatTicks = 100000;
// chunks between looks at the stop flag of a query with a count limit
constexpr uint32_t kLimitCheck = 8;

struct GArgs {
    const CstDev* descs;  // nq descriptors, contiguous
    const int32_t* slot;  // count slot of each descriptor
    int nq;
    GQueue* qu;
    GTask* tasks;
    unsigned int* ready;
    unsigned long long qmask;
    int qlog;
    unsigned long long margin;
    unsigned long long* counts;
    int list;
    int32_t* rows;
    uint64_t cap;
    unsigned long long* row_cursor;
    unsigned long long* stats;  // [tasks, donated, N, M, F, wait ticks, busy ticks, summed, chunks] or nullptr
    uint64_t idle_limit;        // s_memrealtime ticks (100 MHz) an idle wave waits while no wave makes progress
    uint64_t deadline;          // absolute s_memrealtime tick to stop at (0 = none)
    int donate_period;          // longest interval in chunks between donation checks (<= 0: never donate)
    int donate_min;             // shortest such interval
    int64_t flat_max;           // expand the last level flattened when the survivors' lists sum to at most this
    int64_t donate_last_min;    // smallest last-level remainder worth donating
    int last_sum;               // > 0: count an unconstrained last level by list lengths
    const unsigned long long* limits;  // per query: stop once its count reaches this (0: none); nullptr: none
    unsigned int* qstop;               // per query: set once its limit was reached
    bool small_lists;                  // every list shorter than 2^23: 128 lengths sum in 32 bits
};

__device__ inline int lane_id() { return threadIdx.x & (CSTM_WAVE - 1); }


__device__ inline int mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

__device__ inline int32_t rl(int32_t x, int l) { return __builtin_amdgcn_readlane(x, l); }
__device__ inline uint32_t rl(uint32_t x, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)x, l); }
__device__ inline int64_t rl(int64_t x, int l) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)x >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ inline uint64_t rl(uint64_t x, int l) { return (uint64_t)rl((int64_t)x, l); }
__device__ inline const void* rlp(const void* p, int l) { return (const void*)rl((uint64_t)(uintptr_t)p, l); }

template <class T>
__device__ inline T setl(T cur, T val, int lane, int l) {
    return lane == l ? val : cur;
}

template <class T>
__device__ inline T ld_acq(T* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ inline T ld_rlx(T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

// Inclusive prefix sum over the 64 lanes with DPP row shifts and row
// broadcasts (VALU only, no LDS permutes); every lane must be active.
__device__ inline int32_t wave_incl_add(int32_t x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
    return x;
}

// Inclusive prefix maximum over the 64 lanes (values >= -1), the same DPP pattern.
__device__ inline int32_t wave_incl_max(int32_t x) {
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x111, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x112, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x114, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x118, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x142, 0xa, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x143, 0xc, 0xf, false));
    return x;
}

// Sum over the 64 lanes; 32-bit when the caller knows it cannot overflow.
__device__ inline int64_t wave_sum(int64_t x, bool small) {
    if (small) return (int64_t)__builtin_amdgcn_readlane(wave_incl_add((int32_t)x), CSTM_WAVE - 1);
    for (int o = CSTM_WAVE / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, CSTM_WAVE);
    return x;
}

// Binary search of x in the ascending array a[lo, hi).
__device__ inline bool contains(const int32_t* a, int64_t lo, int64_t hi, int32_t x) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        int32_t y = a[mid];
        if (y == x) return true;
        if (y < x) lo = mid + 1;
        else hi = mid;
    }
    return false;
}

// Push a task built from the wave's registers: levels 0..depth-1 from pl.
// Returns false (nothing pushed) when the ring is close to full.
__device__ bool push_task(const GArgs& A, int q, int depth, int64_t lo, int64_t hi, int32_t pl, int lane) {
    unsigned long long t = 0;
    bool ok = true;
    if (lane == 0) {
        const long long pending = (long long)(ld_rlx(&A.qu->tail.v) - ld_rlx(&A.qu->head.v));
        if (pending + (long long)A.margin > (long long)A.qmask) {
            ok = false;
        } else {
            atomicAdd(&A.qu->outstanding.v, 1ull);
            t = atomicAdd(&A.qu->tail.v, 1ull);
        }
    }
    ok = __shfl(ok ? 1 : 0, 0) != 0;
    if (!ok) return false;
    t = __shfl(t, 0);
    GTask* T = &A.tasks[t & A.qmask];
    if (lane < CSTM_MAX_K) T->prefix[lane] = lane < depth ? pl : 0;
    if (lane == 0) {
        T->q = q;
        T->depth = depth;
        T->lo = lo;
        T->hi = hi;
    }
    __threadfence();
    if (lane == 0)
        __hip_atomic_store(&A.ready[t & A.qmask], (unsigned int)((t >> A.qlog) + 1), __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// Take the next ticket and wait for its task.  Each waiting wavefront polls
// only its own slot, so an idle machine does not hammer one cache line.
// Returns the slot, -1 when all work is done, -2 on abort (limit or deadline).
__device__ long long pop_task(const GArgs& A, int lane) {
    long long slot = -1;
    if (lane == 0) {
        const unsigned long long h = atomicAdd(&A.qu->head.v, 1ull);
        const unsigned int lap = (unsigned int)((h >> A.qlog) + 1);
        unsigned int* rp = &A.ready[h & A.qmask];
        const uint64_t t0 = now_ticks();
        int polls = 0, nap = 1;
        for (;;) {
            // relaxed polls leave the CU's L1 alone; one acquire fence once the task is there
            if (ld_rlx(rp) == lap) {
                __atomic_thread_fence(__ATOMIC_ACQUIRE);
                slot = (long long)(h & A.qmask);
                break;
            }
            if (++polls >= 16) {
                polls = 0;
                if (ld_rlx(&A.qu->outstanding.v) == 0) {
                    slot = -1;
                    break;
                }
                if (ld_rlx(&A.qu->abort.v)) {
                    slot = -2;
                    break;
                }
                const uint64_t now = now_ticks();
                if (A.deadline && now > A.deadline) {
                    atomicCAS(&A.qu->abort.v, 0ull, 2ull);
                    slot = -2;
                    break;
                }
                // give up only when nothing has progressed for the idle limit:
                // neither this wait nor any busy wavefront's beat is that recent
                const uint64_t beat = ld_rlx(&A.qu->beat.v);
                const uint64_t last = beat > t0 ? beat : t0;
                if (now > last && now - last > A.idle_limit) {
                    atomicCAS(&A.qu->abort.v, 0ull, 1ull);
                    slot = -2;
                    break;
                }
            }
            for (int i = 0; i < nap; ++i) __builtin_amdgcn_s_sleep(16);
            nap = nap < 16 ? nap + 1 : 16;
        }
    }
    return __shfl(slot, 0);
}

// Membership of data vertex x in a tree list: its entries are indices into
// the candidate array gid, in ascending data-vertex order.
__device__ inline bool in_tree_list(const int32_t* tadj, const int32_t* gid, int64_t lo, int64_t hi, int32_t x) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        const int32_t y = gid[tadj[mid]];
        if (y == x) return true;
        if (y < x) lo = mid + 1;
        else hi = mid;
    }
    return false;
}

// Entries of the tree-list range [lo, hi) of the last level that are not
// among the earlier matches of its label (positions in `same`): the count of
// its valid candidates when it closes no non-tree edge.  Those matches are
// distinct, so each one found in the range removes exactly one entry.  The
// match at position L is g_L, at d is g_d, at any other earlier position
// lane jj of pg holds it.
__device__ inline int64_t unused_in_list(const int32_t* tadj, const int32_t* gid, int64_t lo, int64_t hi,
                                         uint32_t same, int d, int32_t g_d, int L, int32_t g_L, int32_t pg) {
    int64_t n = hi - lo;
    while (same) {
        const int jj = __ffs(same) - 1;
        same &= same - 1;
        const int32_t x = jj == L ? g_L : (jj == d ? g_d : rl(pg, jj));
        if (n > 0 && in_tree_list(tadj, gid, lo, hi, x)) --n;
    }
    return n;
}

// The candidates of level L for a partial result whose level-d entry is v
// (d = L - 1) and whose earlier levels are in pl must lie in every list that
// ends at L: the tree list of its parent's candidate and the non-tree list of
// each earlier neighbour's candidate.  The shortest of them is the one read
// (ties keep the tree list); every other list becomes a check.  Returns the
// non-tree edge index of that list, or -1 for the tree list, and its range.
// Only the partial result decides, so a task handed to another wavefront
// picks the same list again.
__device__ inline int pick_list(const CstDev* D, int L, int d, int32_t v, int32_t pl, int32_t my_par,
                                const int64_t* my_toff, uint32_t my_nt, uint32_t my_ntf, int64_t& lo, int64_t& hi) {
    const int p = rl(my_par, L);
    const int64_t* toff = (const int64_t*)rlp(my_toff, L);
    const int32_t x = p == d ? v : rl(pl, p);
    lo = toff[x];
    hi = toff[x + 1];
    int src = -1;
    uint32_t ntm = rl(my_nt, L);
    uint32_t e = rl(my_ntf, L);
    while (ntm) {
        const int jj = __ffs(ntm) - 1;
        ntm &= ntm - 1;
        const NtDesc& N = D->nt[e];
        const int32_t xa = jj == d ? v : rl(pl, jj);
        const int64_t a = N.off[xa], b = N.off[xa + 1];
        if (b - a < hi - lo) {
            lo = a;
            hi = b;
            src = (int)e;
        }
        ++e;
    }
    return src;
}

// Combined length of the level d+1 lists the survivors (lanes with ok) of a
// level-d chunk would read.
__device__ inline int64_t flat_total(const GArgs& A, const CstDev* D, int d, bool ok, int32_t v, int32_t pl,
                                     int32_t my_par, const int64_t* my_toff, uint32_t my_nt, uint32_t my_ntf) {
    int64_t len = 0;
    if (ok) {
        int64_t lo, hi;
        pick_list(D, d + 1, d, v, pl, my_par, my_toff, my_nt, my_ntf, lo, hi);
        len = hi - lo;
    }
    return wave_sum(len, A.small_lists);
}

// The embeddings the survivors of a chunk at the second-to-last level d
// complete, when the last level closes no non-tree edge: per survivor its
// tree-list length, less the earlier matches of the last level's label found
// in that list (same), summed over the wavefront.
__device__ inline int64_t last_total(const GArgs& A, const CstDev* D, int d, bool ok, int32_t v, int32_t g,
                                     int32_t pl, int32_t pg, uint32_t same, int32_t my_par, const int64_t* my_toff,
                                     const int32_t* my_tadj, const int32_t* my_gid, uint32_t my_nt, uint32_t my_ntf) {
    int64_t len = 0;
    if (ok) {
        int64_t lo, hi;
        pick_list(D, d + 1, d, v, pl, my_par, my_toff, my_nt, my_ntf, lo, hi);
        len = same ? unused_in_list((const int32_t*)rlp(my_tadj, d + 1), (const int32_t*)rlp(my_gid, d + 1), lo, hi,
                                    same, d, g, -1, 0, pg)
                   : hi - lo;
    }
    return wave_sum(len, A.small_lists);
}

// Expand level L = d + 1 for every survivor (lanes with ok) of the current
// level-d chunk at once, 64 (survivor, candidate) pairs per round, so short
// lists do not leave lanes idle and no survivor needs a descent of its own.
// L is either the last level (each passing pair is one embedding, written out
// when listing) or, with sum_next, the second-to-last level of a query whose
// last level closes no non-tree edge (each passing pair adds the length of
// its last-level list, less the earlier matches of that level's label, the
// positions in same_last, found in it).  Returns the number of passing pairs.
__device__ __forceinline__ uint64_t flat_expand(const GArgs& A, const CstDev* D, int k, int d, bool ok, int32_t v,
                                                int32_t g, int32_t pl, int32_t pg, int lane, int32_t my_par,
                                                const int64_t* my_toff, const int32_t* my_tadj,
                                                const int32_t* my_gid, uint32_t my_need, uint32_t my_same,
                                                uint32_t my_nt, uint32_t my_ntf, uint32_t my_u, bool sum_next,
                                                uint32_t same_last, uint64_t& cnt, uint64_t& nN, uint64_t& nM,
                                                uint64_t& nS, uint64_t& nC) {
    const int L = d + 1;
    const int pk = rl(my_par, L);
    const int64_t* toffL = (const int64_t*)rlp(my_toff, L);
    const int32_t* tadjL = (const int32_t*)rlp(my_tadj, L);
    const int32_t* gidL = (const int32_t*)rlp(my_gid, L);
    const bool needL = rl(my_need, L) != 0;
    const uint32_t sameL = rl(my_same, L), ntL = rl(my_nt, L), ntfL = rl(my_ntf, L);
    // with sum_next: where the last level's list owner sits
    const int pK = sum_next ? rl(my_par, L + 1) : 0;
    const int64_t* toffK = sum_next ? (const int64_t*)rlp(my_toff, L + 1) : nullptr;
    const int32_t* tadjK = sum_next && same_last ? (const int32_t*)rlp(my_tadj, L + 1) : nullptr;
    const int32_t* gidK = sum_next && same_last ? (const int32_t*)rlp(my_gid, L + 1) : nullptr;
    int64_t b0 = 0;
    int32_t len = 0;  // the caller checked that the lengths sum to at most flat_max < 2^31
    int src = -1;     // the list each survivor reads (pick_list)
    if (ok) {
        int64_t hi = 0;
        src = pick_list(D, L, d, v, pl, my_par, my_toff, my_nt, my_ntf, b0, hi);
        len = (int32_t)(hi - b0);
    }
    const int32_t incl = wave_incl_add(len);  // inclusive prefix over lanes
    const int32_t total = __builtin_amdgcn_readlane(incl, CSTM_WAVE - 1);
    uint64_t passed = 0;
    // Two rounds of 64 pairs per iteration: their owner searches and loads are
    // independent, so each hides the other's latency.
    constexpr int R = 2;
    // Owner lane of each pair: every survivor with a non-empty list marks the
    // round position where its list starts (starts are distinct), and a prefix
    // maximum carries each mark forward to the positions its list covers.
    __shared__ int32_t s_mark[256 / CSTM_WAVE][CSTM_WAVE];
    int32_t* mark = s_mark[threadIdx.x / CSTM_WAVE];
    const int32_t start_me = incl - len;
    int32_t carry = 0;  // owner of the pair just before the current round
    for (int32_t t0 = 0; t0 < total; t0 += R * CSTM_WAVE) {
        int32_t t[R], own[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int32_t base = t0 + r * CSTM_WAVE;
            t[r] = base + lane;
            mark[lane] = -1;
            __builtin_amdgcn_wave_barrier();
            if (len > 0 && start_me >= base && start_me < base + CSTM_WAVE) mark[start_me - base] = lane;
            __builtin_amdgcn_wave_barrier();
            const int32_t m = wave_incl_max(mark[lane]);
            __builtin_amdgcn_wave_barrier();
            own[r] = m > carry ? m : carry;
            carry = __builtin_amdgcn_readlane(own[r], CSTM_WAVE - 1);
        }
        bool val2[R], ok2[R];
        int32_t v2[R], g2[R], vs[R], gs[R], sr[R];
        int64_t at[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int sl = own[r];
            val2[r] = t[r] < total;
            const int32_t start = __shfl(incl, sl) - __shfl(len, sl);
            const int64_t bs = __shfl(b0, sl);
            vs[r] = __shfl(v, sl);
            gs[r] = __shfl(g, sl);
            sr[r] = __shfl(src, sl);
            at[r] = bs + (t[r] - start);
            v2[r] = val2[r] ? (sr[r] < 0 ? tadjL[at[r]] : D->nt[sr[r]].adj[at[r]]) : 0;
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
            g2[r] = (val2[r] && needL) ? (sr[r] < 0 ? gidL[v2[r]] : D->nt[sr[r]].adj_gid[at[r]]) : -1;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            bool okr = val2[r];
            uint32_t same2 = sameL;
            while (same2) {
                const int jj = __ffs(same2) - 1;
                same2 &= same2 - 1;
                okr = okr && g2[r] != (jj == d ? gs[r] : rl(pg, jj));
            }
            uint32_t nt2 = ntL, e2 = ntfL;
            while (nt2) {
                const int jj = __ffs(nt2) - 1;
                nt2 &= nt2 - 1;
                const int ei = (int)e2++;
                if (ei == sr[r]) continue;  // the list this candidate came from
                const NtDesc& N = D->nt[ei];
                const int32_t x = jj == d ? vs[r] : rl(pl, jj);
                if (okr) okr = contains(N.adj_gid, N.off[x], N.off[x + 1], g2[r]);
            }
            if (okr && sr[r] >= 0) {
                // read from a non-tree list: the tree edge is the check
                const int32_t xp = pk == d ? vs[r] : rl(pl, pk);
                okr = in_tree_list(tadjL, gidL, toffL[xp], toffL[xp + 1], g2[r]);
            }
            ok2[r] = okr;
        }
        if (sum_next) {
            int64_t lk = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (ok2[r]) {
                    const int32_t xk = pK == L ? v2[r] : (pK == d ? vs[r] : rl(pl, pK));
                    lk += same_last ? unused_in_list(tadjK, gidK, toffK[xk], toffK[xk + 1], same_last, d, gs[r], L,
                                                     g2[r], pg)
                                    : toffK[xk + 1] - toffK[xk];
                }
            }
            lk = wave_sum(lk, A.small_lists);
            cnt += (uint64_t)lk;
            nN += (uint64_t)lk;
            nS += (uint64_t)lk;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t m2 = __ballot(ok2[r]);
            const uint64_t nv2 = (uint64_t)__popcll(__ballot(val2[r]));
            nN += nv2;
            nC += nv2 ? 1 : 0;
            nM += nv2 * (uint64_t)__popc(ntL);
            passed += (uint64_t)__popcll(m2);
            if (sum_next) continue;
            cnt += (uint64_t)__popcll(m2);
            if (A.list && m2) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(A.row_cursor, (unsigned long long)__popcll(m2));
                base = __shfl(base, 0);
                if (ok2[r]) {
                    const uint64_t row_i = base + (uint64_t)mbcnt(m2);
                    if (row_i < A.cap) {
                        int32_t* row = A.rows + row_i * (uint64_t)k;
                        for (int i = 0; i < k; ++i)
                            row[rl(my_u, i)] = i == L ? g2[r] : (i == d ? gs[r] : rl(pg, i));
                    }
                }
            }
        }
    }
    return passed;
}

__global__ __launch_bounds__(256, 4) void k_enumerate_global(GArgs A) {
    const int lane = lane_id();
    if (A.deadline) A.deadline += now_ticks();  // relative on entry, absolute from here on
    // per-query position records, held one per lane (lane d = position d)
    int cur_q = -1, k = 0;
    const int32_t* my_gid = nullptr;
    const int64_t* my_toff = nullptr;
    const int32_t* my_tadj = nullptr;
    int32_t my_par = -1;
    uint32_t my_same = 0, my_nt = 0, my_ntf = 0, my_u = 0, my_need = 0;
    bool sum_last = false;  // this query's last level is counted by list lengths
    uint32_t same_last = 0;  // then: the earlier positions sharing its label
    const CstDev* D = nullptr;
    uint64_t cnt = 0, nN = 0, nM = 0, nF = 0, nS = 0, nC = 0, ntasks = 0, ndon = 0;
    uint64_t t_wait = 0, t_busy = 0;
    uint64_t my_beat = 0;  // lane 0: when this wavefront last refreshed the progress beat
    // chunks between checks for waiting consumers, adapted per wavefront
    const uint32_t max_period = (uint32_t)(A.donate_period > 0 ? A.donate_period : 64);
    const uint32_t min_period = (uint32_t)A.donate_min < max_period ? (uint32_t)A.donate_min : max_period;
    uint32_t period = A.donate_period > 0 ? min_period : max_period;
    for (;;) {
        const uint64_t w0 = now_ticks();
        const long long slot = pop_task(A, lane);
        const uint64_t w1 = now_ticks();
        t_wait += w1 - w0;
        if (slot < 0) break;
        const GTask* T = &A.tasks[slot];
        const int q = T->q;
        const int j = T->depth;
        if (A.qstop && ld_rlx(&A.qstop[q])) {
            // this query already found its limit: drop the task
            if (lane == 0) atomicAdd(&A.qu->outstanding.v, ~0ull);
            t_busy += now_ticks() - w1;
            continue;
        }
        int64_t lo = T->lo, hi = T->hi;
        // with a count limit, an unpublished count of limit / 16384 or more is
        // published at once (one chunk can add millions of summed embeddings),
        // and the query's stop flag is read at least every kLimitCheck chunks:
        // a late publication or a late look at the flag lets the query run far
        // past its limit
        const unsigned long long lim = A.limits ? A.limits[q] : 0ull;
        const uint64_t publish_at = lim ? ((lim >> 14) ? (lim >> 14) : 1ull) : ~0ull;
        const uint32_t check_cap = lim ? kLimitCheck : ~0u;
        int32_t pre = lane < CSTM_MAX_K ? T->prefix[lane] : 0;
        ++ntasks;
        if (q != cur_q) {
            if (cur_q >= 0 && cnt) {
                if (lane == 0) atomicAdd(&A.counts[A.slot[cur_q]], (unsigned long long)cnt);
                cnt = 0;
            }
            cur_q = q;
            D = &A.descs[q];
            k = D->k;
            if (lane < k) {
                const PosDesc& P = D->pos[lane];
                my_gid = P.gid;
                my_toff = P.toff;
                my_tadj = P.tadj;
                my_par = P.par;
                my_same = P.same_mask;
                my_nt = P.nt_mask;
                my_ntf = (uint32_t)(P.nt_first < 0 ? 0 : P.nt_first);
                my_u = (uint32_t)P.u;
                my_need = (A.list || P.need_gid) ? 1u : 0u;
            }
            // when the last position closes no non-tree edge its tree list holds all
            // results but the earlier matches of its label, which a search finds
            sum_last = A.last_sum > 0 && !A.list && k >= 2 && rl(my_nt, k - 1) == 0;
            same_last = sum_last ? rl(my_same, k - 1) : 0u;
        }
        // level registers: lane d holds level d
        int32_t pl = lane < j ? pre : 0;
        int32_t pg = 0;
        if (lane < j && my_need) pg = my_gid[pl];
        int64_t lc = 0, le = 0;
        uint64_t lm = 0;
        int32_t ls = -1;  // lane d: the list level d reads (-1: tree list, else a non-tree edge)
        lc = setl(lc, lo, lane, j);
        le = setl(le, hi, lane, j);
        if (j > 0) {
            // the task's range lies in the list its prefix picks
            int64_t a, b;
            const int src = pick_list(D, j, j - 1, rl(pl, j - 1), pl, my_par, my_toff, my_nt, my_ntf, a, b);
            ls = setl(ls, (int32_t)src, lane, j);
        }
        int d = j;
        uint32_t since_check = 0;
        for (;;) {
            uint64_t M = rl(lm, d);
            const int64_t cur = rl(lc, d);
            if (M == 0) {
                const int64_t end = rl(le, d);
                if (cur >= end) {
                    if (d == j) break;
                    --d;
                    continue;
                }
                if (d == k - 1 && sum_last && d > 0) {
                    // a donated remainder of a last level counted by list lengths
                    const uint64_t n =
                        same_last ? (uint64_t)unused_in_list((const int32_t*)rlp(my_tadj, d), (const int32_t*)rlp(my_gid, d),
                                                             cur, end, same_last, -1, 0, -1, 0, pg)
                                  : (uint64_t)(end - cur);
                    cnt += n;
                    nN += n;
                    nS += n;
                    lc = setl(lc, end, lane, d);
                    continue;
                }
                const int64_t idx = cur + lane;
                const bool val = idx < end;
                const int32_t* gid = (const int32_t*)rlp(my_gid, d);
                const int32_t* tadj = (const int32_t*)rlp(my_tadj, d);
                const int src = d == 0 ? -1 : rl(ls, d);
                int32_t v = 0;
                if (val) v = d == 0 ? (int32_t)idx : (src < 0 ? tadj[idx] : D->nt[src].adj[idx]);
                const int32_t g = (val && rl(my_need, d)) ? (src < 0 ? gid[v] : D->nt[src].adj_gid[idx]) : -1;
                bool ok = val;
                uint32_t same = rl(my_same, d);
                while (same) {
                    const int jj = __ffs(same) - 1;
                    same &= same - 1;
                    ok = ok && g != rl(pg, jj);
                }
                uint32_t ntm = rl(my_nt, d);
                uint32_t e = rl(my_ntf, d);
                const uint32_t n_nt_here = (uint32_t)__popc(ntm);
                while (ntm) {
                    const int jj = __ffs(ntm) - 1;
                    ntm &= ntm - 1;
                    const int ei = (int)e++;
                    if (ei == src) continue;  // the list these candidates came from
                    const NtDesc& N = D->nt[ei];
                    const int32_t x = rl(pl, jj);
                    if (ok) ok = contains(N.adj_gid, N.off[x], N.off[x + 1], g);
                }
                if (src >= 0 && ok) {
                    // read from a non-tree list: the tree edge is the check
                    const int64_t* toff = (const int64_t*)rlp(my_toff, d);
                    const int32_t xp = rl(pl, rl(my_par, d));
                    ok = in_tree_list(tadj, gid, toff[xp], toff[xp + 1], g);
                }
                const uint64_t m = __ballot(ok);
                {
                    const uint64_t nv = (uint64_t)__popcll(__ballot(val));
                    nN += nv;
                    nM += nv * n_nt_here;
                    ++nC;
                }
                lc = setl(lc, cur + (int64_t)CSTM_WAVE, lane, d);
                if (d == k - 1) {
                    cnt += (uint64_t)__popcll(m);
                    if (A.list && m) {
                        unsigned long long base = 0;
                        if (lane == 0) base = atomicAdd(A.row_cursor, (unsigned long long)__popcll(m));
                        base = __shfl(base, 0);
                        if (ok) {
                            const uint64_t r = base + (uint64_t)mbcnt(m);
                            if (r < A.cap) {
                                int32_t* row = A.rows + r * (uint64_t)k;
                                for (int i = 0; i < k; ++i) row[rl(my_u, i)] = i == d ? g : rl(pg, i);
                            }
                        }
                    }
                } else if (d == k - 2 && sum_last) {
                    // last level counted by list lengths: every survivor adds its list
                    // length, less the earlier matches of that level's label found in it
                    if (m) {
                        const uint64_t n = (uint64_t)last_total(A, D, d, ok, v, g, pl, pg, same_last, my_par, my_toff,
                                                                my_tadj, my_gid, my_nt, my_ntf);
                        cnt += n;
                        nN += n;
                        nS += n;
                        nF += (uint64_t)__popcll(m);
                    }
                } else if (m && ((d == k - 2) || (d == k - 3 && sum_last)) &&
                           flat_total(A, D, d, ok, v, pl, my_par, my_toff, my_nt, my_ntf) <= A.flat_max) {
                    // the next level flattened over all survivors of this chunk: the last
                    // level, or the second-to-last with the unconstrained last level summed
                    const bool sum_next = d == k - 3;
                    const uint64_t passed = flat_expand(A, D, k, d, ok, v, g, pl, pg, lane, my_par, my_toff, my_tadj,
                                                        my_gid, my_need, my_same, my_nt, my_ntf, my_u, sum_next,
                                                        same_last, cnt, nN, nM, nS, nC);
                    nF += (uint64_t)__popcll(m) + (sum_next ? passed : 0);
                } else if (m) {
                    M = m;
                    nF += (uint64_t)__popcll(m);
                }
                // every few chunks: stop on abort or deadline; donate the untouched
                // remainder of the shallowest open level when a consumer is waiting.
                // The interval adapts: short while consumers wait (a narrow search
                // spreads fast), doubling up to donate_period while none do.
                if (++since_check >= (period < check_cap ? period : check_cap) || cnt >= publish_at) {
                    since_check = 0;
                    int want = 0, added = 0;
                    // with a count limit, publish the count found so far; once the
                    // query's count reaches its limit, every task of it stops
                    const bool publish = lim && cnt;
                    if (lane == 0) {
                        const uint64_t now = now_ticks();
                        if (now - my_beat > kBeatTicks) {
                            __hip_atomic_store(&A.qu->beat.v, (unsigned long long)now, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                            my_beat = now;
                        }
                        if (ld_rlx(&A.qu->abort.v)) want = -1;
                        else if (A.deadline && now > A.deadline) {
                            atomicCAS(&A.qu->abort.v, 0ull, 2ull);
                            want = -1;
                        } else if (lim && ld_rlx(&A.qstop[q])) {
                            want = -2;
                        } else if (publish) {
                            added = 1;
                            if (atomicAdd(&A.counts[A.slot[q]], (unsigned long long)cnt) + cnt >= lim) {
                                __hip_atomic_store(&A.qstop[q], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                want = -2;
                            }
                        }
                        if (want == 0 && A.donate_period > 0) {
                            const unsigned long long t2 = ld_rlx(&A.qu->tail.v), h2 = ld_rlx(&A.qu->head.v);
                            want = (long long)(h2 - t2) > 0 ? 1 : 0;
                        }
                    }
                    if (__shfl(added, 0)) cnt = 0;  // lane 0 added it to the query's count
                    want = __shfl(want, 0);
                    if (want < 0) break;
                    if (!want) period = period * 2 < max_period ? period * 2 : max_period;
                    if (want) {
                        // shallowest open level first: its untouched list remainder, or
                        // (above the current level) the survivors not yet descended into,
                        // given away as a range the receiver re-checks
                        // the last level visited holds cheap entries: only large remainders go
                        const int last_visited = sum_last ? k - 2 : k - 1;
                        for (int dd = j; dd <= d; ++dd) {
                            const int64_t c2 = rl(lc, dd), e2 = rl(le, dd);
                            if (dd == last_visited && e2 - c2 < A.donate_last_min) break;
                            if (c2 < e2) {
                                if (push_task(A, q, dd, c2, e2, pl, lane)) {
                                    le = setl(le, c2, lane, dd);
                                    ++ndon;
                                    period = min_period;
                                }
                                break;
                            }
                            const uint64_t Mr = dd < d ? rl(lm, dd) : 0;
                            if (Mr) {
                                const int64_t cs = c2 - (int64_t)CSTM_WAVE;
                                const int64_t from = cs + (int64_t)(__ffsll((unsigned long long)Mr) - 1);
                                const int64_t to = c2 < e2 ? c2 : e2;
                                if (from < to && push_task(A, q, dd, from, to, pl, lane)) {
                                    lm = setl(lm, (uint64_t)0, lane, dd);
                                    ++ndon;
                                    period = min_period;
                                }
                                break;
                            }
                        }
                    }
                }
                if (M == 0) continue;
            }
            // descend into the lowest survivor of the current chunk at level d
            const int b = __ffsll((unsigned long long)M) - 1;
            M &= M - 1;
            lm = setl(lm, M, lane, d);
            const int64_t chunk = rl(lc, d) - (int64_t)CSTM_WAVE;
            const int srcd = d == 0 ? -1 : rl(ls, d);
            const int64_t at = chunk + b;
            const int32_t v = d == 0 ? (int32_t)at
                                     : (srcd < 0 ? ((const int32_t*)rlp(my_tadj, d))[at] : D->nt[srcd].adj[at]);
            const int32_t g = rl(my_need, d)
                                  ? (srcd < 0 ? ((const int32_t*)rlp(my_gid, d))[v] : D->nt[srcd].adj_gid[at])
                                  : 0;
            pl = setl(pl, v, lane, d);
            pg = setl(pg, g, lane, d);
            ++d;
            int64_t nlo, nhi;
            const int nsrc = pick_list(D, d, d - 1, v, pl, my_par, my_toff, my_nt, my_ntf, nlo, nhi);
            lc = setl(lc, nlo, lane, d);
            le = setl(le, nhi, lane, d);
            ls = setl(ls, (int32_t)nsrc, lane, d);
            lm = setl(lm, (uint64_t)0, lane, d);
        }
        if (lane == 0) atomicAdd(&A.qu->outstanding.v, ~0ull);
        t_busy += now_ticks() - w1;
    }
    if (cur_q >= 0 && cnt && lane == 0) atomicAdd(&A.counts[A.slot[cur_q]], (unsigned long long)cnt);
    if (A.stats && lane == 0) {
        atomicAdd(&A.stats[0], (unsigned long long)ntasks);
        atomicAdd(&A.stats[1], (unsigned long long)ndon);
        atomicAdd(&A.stats[2], (unsigned long long)nN);
        atomicAdd(&A.stats[3], (unsigned long long)nM);
        atomicAdd(&A.stats[4], (unsigned long long)nF);
        atomicAdd(&A.stats[5], (unsigned long long)t_wait);
        atomicAdd(&A.stats[6], (unsigned long long)t_busy);
        atomicAdd(&A.stats[7], (unsigned long long)nS);
        atomicAdd(&A.stats[8], (unsigned long long)nC);
    }
}

// Initial tasks: every seeding segment (a query and a run [lo, hi) of its
// root candidates) cut into tasks of chunk[i] root candidates.
__global__ void k_seed(GArgs A, const int64_t* __restrict__ first, const int64_t* __restrict__ seg_lo,
                       const int64_t* __restrict__ seg_hi, const int64_t* __restrict__ chunk,
                       const int32_t* __restrict__ seg_q, int ns, unsigned long long total) {
    unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long t = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        // segment i: the last with first[i] <= t
        int lo = 0, hi = ns - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if ((long long)t >= first[mid]) lo = mid;
            else hi = mid - 1;
        }
        const int i = lo;
        const int64_t r = (int64_t)t - first[i];
        GTask& T = A.tasks[t & A.qmask];
        T.q = seg_q[i];
        T.depth = 0;
        T.lo = seg_lo[i] + r * chunk[i];
        T.hi = T.lo + chunk[i] < seg_hi[i] ? T.lo + chunk[i] : seg_hi[i];
        for (int p = 0; p < CSTM_MAX_K; ++p) T.prefix[p] = 0;
        A.ready[t & A.qmask] = (unsigned int)((t >> A.qlog) + 1);
    }
}

// Clear n 32-bit words (a kernel rather than a memset node, so the same code
// serves callers that capture the stream).
__global__ void k_zero_words(uint32_t* __restrict__ p, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

void zero_words(void* p, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 4;
    if (!n) return;
    k_zero_words<<<cstm_blocks((int64_t)n, 256, 2048), 256, 0, s>>>((uint32_t*)p, n);
    HIP_TRY(hipGetLastError());
}

// Work counters of a launch (GArgs::stats).
constexpr int kWorkSlots = 9;

// Layout of a launch's workspace, every region 256-byte aligned and sized by
// sizeof(): ring | ready flags | queue state | work counters | descriptors |
// seed tables | count slots | limits | stop flags.
struct WsLayout {
    size_t off_ready, off_qu, off_work, off_desc, off_meta, off_slot, off_segq, off_lim, off_stop, need;
};
WsLayout ws_layout(unsigned long long qcap, int nq, int ns) {
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    WsLayout L;
    L.off_ready = up(qcap * sizeof(GTask));
    L.off_qu = up(L.off_ready + qcap * sizeof(unsigned int));
    L.off_work = up(L.off_qu + sizeof(GQueue));
    L.off_desc = up(L.off_work + kWorkSlots * sizeof(unsigned long long));
    L.off_meta = up(L.off_desc + (size_t)nq * sizeof(CstDev));
    L.off_slot = up(L.off_meta + (4 * (size_t)ns + 1) * sizeof(int64_t));
    L.off_segq = up(L.off_slot + (size_t)nq * sizeof(int32_t));
    L.off_lim = up(L.off_segq + (size_t)ns * sizeof(int32_t));
    L.off_stop = up(L.off_lim + (size_t)nq * sizeof(unsigned long long));
    L.need = up(L.off_stop + (size_t)nq * sizeof(unsigned int));
    return L;
}

// Task-ring size of launches in a caller's fixed workspace: 2^16 slots.
constexpr int kFixedQlog = 16;

}  // namespace

// Device bytes the context lends one HBM-mode launch of nq CSTs (its
// workspace, with the quarter of slack ws_acquire adds).
size_t cstm_hbm_workspace_bytes(int nq) {
    const size_t need = ws_layout(1ull << 20, nq, nq).need;
    return need + need / 4;
}

// Count (or list) the embeddings of nq CSTs in one launch, the CSTs read from
// HBM; counts go to counts_dev[slot[q]].
void cstm_enumerate_global_run(cstm_ctx* ctx, int nq, cstm_cst* const* csts, const int* slot, int list, int32_t* rows,
                               uint64_t cap, unsigned long long* counts_dev, unsigned long long* row_cursor,
                               const EnumOpts& o, cstm_enum_stats* st, hipStream_t s) {
    const bool fixed = o.fixed_ws != nullptr;
    const int qlog = fixed ? kFixedQlog : 20;
    const unsigned long long qcap = 1ull << qlog;
    // seeding order: as given, or (batch_order > 0) the heaviest queries
    // (largest W_CST, Section V-C) first, so the long searches start early
    std::vector<int32_t> perm(nq);
    for (int q = 0; q < nq; ++q) perm[q] = q;
    if (nq > 1 && ctx->tune.batch_order > 0) {
        std::vector<uint64_t> w(nq);
        for (int q = 0; q < nq; ++q) w[q] = cstm_cst_workload_run(csts[q]);
        std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return w[a] > w[b]; });
    }
    // seeding segments, in seeding order: all root candidates of each query,
    // or the caller's runs of them for a one-query call
    struct Seg {
        int32_t q;
        int64_t lo, hi;
    };
    std::vector<Seg> segs;
    if (nq == 1 && o.root_ranges) {
        const int64_t nr = csts[0]->empty ? 0 : csts[0]->host_desc.pos[0].n;
        for (int64_t i = 0; i < o.n_ranges; ++i) {
            const int64_t lo = o.root_ranges[2 * i], hi = o.root_ranges[2 * i + 1];
            CSTM_REQUIRE(0 <= lo && lo <= hi && hi <= nr, CSTM_EINVAL, "root range out of bounds");
            if (hi > lo) segs.push_back({0, lo, hi});
        }
    } else {
        for (int i = 0; i < nq; ++i) {
            const cstm_cst* c = csts[perm[i]];
            segs.push_back({perm[i], 0, c->empty ? 0 : (int64_t)c->host_desc.pos[0].n});
        }
    }
    const int ns = (int)segs.size();
    CSTM_REQUIRE(ns < (int)(qcap / 8), CSTM_EINVAL, "too many root ranges");
    // per segment: the first task and the roots per task (one root candidate
    // per task unless the batch would fill a quarter / half of the ring)
    const int64_t fill = o.root_ranges ? 4 : 2;
    std::vector<int64_t> first(ns + 1, 0), seg_lo(ns), seg_hi(ns), chunk(ns, 1);
    std::vector<int32_t> seg_q(ns);
    for (int i = 0; i < ns; ++i) {
        const int64_t len = segs[i].hi - segs[i].lo;
        const int64_t per = std::max<int64_t>(1, (len * fill * std::max(1, ns) + (int64_t)qcap - 1) / (int64_t)qcap);
        seg_lo[i] = segs[i].lo;
        seg_hi[i] = segs[i].hi;
        seg_q[i] = segs[i].q;
        chunk[i] = per;
        first[i + 1] = first[i] + (len + per - 1) / per;
    }
    const unsigned long long total = (unsigned long long)first[ns];
    CSTM_REQUIRE(total < qcap / 2, CSTM_EINVAL, "too many root candidates for the task ring");
    if (total == 0) return;
    // workspace lent by the context for this launch, every region 256-byte aligned and sized by sizeof():
    // ring | ready flags | queue state | work counters | descriptors | seed tables | count slots
    const WsLayout Lw = ws_layout(qcap, nq, ns);
    const size_t off_ready = Lw.off_ready, off_qu = Lw.off_qu, off_work = Lw.off_work, off_desc = Lw.off_desc;
    const size_t off_meta = Lw.off_meta, off_slot = Lw.off_slot, off_segq = Lw.off_segq, off_lim = Lw.off_lim;
    const size_t off_stop = Lw.off_stop, need = Lw.need;
    const size_t ready_b = qcap * sizeof(unsigned int);
    struct WsHold {
        cstm_ctx* ctx;
        void* p;
        ~WsHold() {
            if (p) ctx->ws_release(p);
        }
    } hold{ctx, nullptr};
    uint8_t* ws = nullptr;
    if (fixed) {
        CSTM_REQUIRE(need <= o.fixed_ws_bytes, CSTM_EINVAL,
                     "launch needs " + std::to_string(need) + " bytes of scratch, more than the " +
                         std::to_string(o.fixed_ws_bytes) + " available");
        ws = (uint8_t*)o.fixed_ws;
    } else {
        hold.p = ctx->ws_acquire(need);
        ws = (uint8_t*)hold.p;
    }
    GTask* tasks = (GTask*)ws;
    unsigned int* ready = (unsigned int*)(ws + off_ready);
    GQueue* qu = (GQueue*)(ws + off_qu);
    unsigned long long* work = (unsigned long long*)(ws + off_work);
    CstDev* descs = (CstDev*)(ws + off_desc);
    int64_t* meta = (int64_t*)(ws + off_meta);
    int32_t* dslot = (int32_t*)(ws + off_slot);
    int32_t* dsegq = (int32_t*)(ws + off_segq);
    unsigned long long* dlim = (unsigned long long*)(ws + off_lim);
    unsigned int* dstop = (unsigned int*)(ws + off_stop);
    bool any_limit = false;
    std::vector<unsigned long long> lim(nq, 0);
    if (o.limits)
        for (int q = 0; q < nq; ++q) {
            lim[q] = o.limits[slot[q]];
            any_limit |= lim[q] != 0;
        }
    if (any_limit) {
        HIP_TRY(hipMemcpyAsync(dlim, lim.data(), (size_t)nq * 8, hipMemcpyHostToDevice, s));
        zero_words(dstop, (size_t)nq * 4, s);
    }
    for (int q = 0; q < nq; ++q)
        HIP_TRY(hipMemcpyAsync(descs + q, &csts[q]->host_desc, sizeof(CstDev), hipMemcpyHostToDevice, s));
    zero_words(ready, ready_b, s);
    zero_words(work, kWorkSlots * sizeof(unsigned long long), s);
    GQueue init;
    std::memset(&init, 0, sizeof(init));
    init.tail.v = total;
    init.outstanding.v = total;
    HIP_TRY(hipMemcpyAsync(qu, &init, sizeof(init), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(meta, first.data(), (ns + 1) * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(meta + ns + 1, seg_lo.data(), ns * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(meta + 2 * ns + 1, seg_hi.data(), ns * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(meta + 3 * ns + 1, chunk.data(), ns * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(dslot, slot, nq * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(dsegq, seg_q.data(), ns * 4, hipMemcpyHostToDevice, s));
    GArgs A;
    A.descs = descs;
    A.slot = dslot;
    A.nq = nq;
    A.qu = qu;
    A.tasks = tasks;
    A.ready = ready;
    A.qmask = qcap - 1;
    A.qlog = qlog;
    // room kept free in the ring for pushes already decided (far more than the waves in flight)
    A.margin = fixed ? qcap / 4 : 1ull << 15;
    A.counts = counts_dev;
    A.list = list;
    A.rows = rows;
    A.cap = cap;
    A.row_cursor = row_cursor;
    A.stats = ctx->tune.collect_stats ? work : nullptr;
    A.idle_limit = 100ull * 1000 * (uint64_t)ctx->tune.hbm_idle_ms;  // at 100 MHz
    A.deadline = o.deadline_ms > 0 ? 100ull * 1000 * (uint64_t)o.deadline_ms : 0;
    int64_t longest = 0;
    for (int q = 0; q < nq; ++q) longest = std::max<int64_t>(longest, csts[q]->d_cst);
    A.small_lists = longest < (int64_t(1) << 23);
    A.limits = any_limit ? dlim : nullptr;
    A.qstop = any_limit ? dstop : nullptr;
    A.donate_period = ctx->tune.hbm_donate_period;
    A.donate_min = ctx->tune.hbm_donate_min > 0 ? ctx->tune.hbm_donate_min : 1;
    A.flat_max = ctx->tune.hbm_flat_max;  // negative: never flatten
    A.donate_last_min = ctx->tune.hbm_donate_last_min;
    A.last_sum = ctx->tune.last_level_sum;
    k_seed<<<cstm_blocks((int64_t)total, 256, 4096), 256, 0, s>>>(A, meta, meta + ns + 1, meta + 2 * ns + 1,
                                                                  meta + 3 * ns + 1, dsegq, ns, total);
    HIP_TRY(hipGetLastError());
    const unsigned grid = (unsigned)(ctx->num_cus * (o.wgs_per_cu > 0 ? o.wgs_per_cu : ctx->tune.hbm_wgs_per_cu));
    float kernel_ms = 0;
    if (fixed) {
        k_enumerate_global<<<grid, 256, 0, s>>>(A);
        HIP_TRY(hipGetLastError());
    } else {
        hipEvent_t ev[2];
        HIP_TRY(hipEventCreate(&ev[0]));
        HIP_TRY(hipEventCreate(&ev[1]));
        HIP_TRY(hipEventRecord(ev[0], s));
        k_enumerate_global<<<grid, 256, 0, s>>>(A);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipEventRecord(ev[1], s));
        HIP_TRY(hipEventSynchronize(ev[1]));
        HIP_TRY(hipEventElapsedTime(&kernel_ms, ev[0], ev[1]));
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
    }
    unsigned long long h[kWorkSlots];
    GQueue fin{};
    HIP_TRY(hipMemcpyAsync(h, work, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&fin, qu, sizeof(fin), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    st->kernel_ms += kernel_ms;
    st->mode = CSTM_MODE_HBM;
    st->launches += 1;
    st->images += h[0];
    st->image_bytes += h[1];
    st->extensions += h[2];
    st->edge_checks += h[3];
    st->pushed += h[4];
    st->busy_frac = (h[5] + h[6]) ? (double)h[6] / (double)(h[5] + h[6]) : 0.0;
    st->summed += h[7];
    st->chunks += h[8];
    {
        std::lock_guard<std::mutex> lk(ctx->ws_mu);
        ctx->last_enum = *st;  // kept even when the launch is reported as failed below
    }
    CSTM_REQUIRE(fin.abort.v != 2, CSTM_ETIMEOUT, "enumeration stopped at the deadline");
    CSTM_REQUIRE(fin.abort.v != 1, CSTM_EDEVICE,
                 "enumeration stopped: no wavefront made progress for " + std::to_string(ctx->tune.hbm_idle_ms) + " ms");
    CSTM_REQUIRE(fin.outstanding.v == 0, CSTM_EDEVICE, "enumeration work queue did not drain");
}

// ---------------------------------------------------------------- no-allocation entry point
//
// The task ring, queue state, descriptors and counts of cstm_enumerate_noalloc
// live in one file-scope device array.  In host code `scratch` names a host
// stand-in, not device memory: every host use goes through the address
// hipGetSymbolAddress returns for the current device, kept per device.
static __device__ __align__(256) unsigned char scratch[CSTM_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;                // guards g_scratch_ptr
void* g_scratch_ptr[kMaxDevices] = {};  // this device's copy of `scratch`
std::mutex g_call_mu[kMaxDevices];      // one no-allocation call at a time per device
}  // namespace

void cstm_noalloc_init(int device) {
    CSTM_REQUIRE(device >= 0 && device < kMaxDevices, CSTM_EINVAL, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    CSTM_REQUIRE(p != nullptr, CSTM_EDEVICE, "no device address for the scratch array");
    g_scratch_ptr[device] = p;
}

extern "C" cstm_status cstm_enumerate_noalloc(cstm_cst* cst, uint64_t limit, uint64_t* count_out, double deadline_s,
                                              void* stream) {
    uint64_t count = 0;
    cstm_status status = cstm_guard([&] {
        CSTM_REQUIRE(cst && count_out, CSTM_EINVAL, "NULL argument");
        CSTM_REQUIRE(deadline_s == deadline_s, CSTM_EINVAL, "deadline is NaN");
        cstm_ctx* ctx = cst->ctx;
        const int dev = ctx->device;
        HIP_TRY(hipSetDevice(dev));
        uint8_t* base = nullptr;
        {
            std::lock_guard<std::mutex> lk(g_scratch_mu);
            base = (uint8_t*)(dev >= 0 && dev < kMaxDevices ? g_scratch_ptr[dev] : nullptr);
        }
        CSTM_REQUIRE(base, CSTM_EDEVICE, "scratch array not set up on this device");
        if (cst->empty) return;
        hipStream_t s = stream ? (hipStream_t)stream : cst->stream;
        std::lock_guard<std::mutex> call(g_call_mu[dev]);
        // [0, 256): the count and the (unused) row cursor; the rest: the launch workspace
        unsigned long long* counts = (unsigned long long*)base;
        zero_words(counts, 2 * sizeof(unsigned long long), s);
        EnumOpts o;
        o.limits = limit ? &limit : nullptr;
        o.deadline_ms = deadline_s > 0 ? (int64_t)(deadline_s * 1e3) + 1 : ctx->tune.deadline_ms;
        o.fixed_ws = base + 256;
        o.fixed_ws_bytes = CSTM_NOALLOC_SCRATCH_BYTES - 256;
        cstm_cst* one[1] = {cst};
        const int slot0 = 0;
        cstm_enum_stats st{};
        cstm_enumerate_global_run(ctx, 1, one, &slot0, 0, nullptr, 0, counts, counts + 1, o, &st, s);
        unsigned long long h = 0;
        HIP_TRY(hipMemcpyAsync(&h, counts, sizeof(h), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        count = (limit && h > limit) ? limit : (uint64_t)h;
    });
    if (count_out) *count_out = count;
    return status;
}
