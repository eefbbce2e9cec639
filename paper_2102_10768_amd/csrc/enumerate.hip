// enumerate.hip -- embedding enumeration inside LDS-resident CST partitions
// (Section VI-A, Algorithms 4-8; buffer bound of Section VI-B).
//
// A persistent grid of workgroups pulls partition images from a device queue.
// Each workgroup copies one image from HBM into LDS with 16-byte loads and
// its wavefronts extend partial embeddings along the matching order, reading
// only LDS:
//   Generator        -- the candidates of the next position are the tree list
//                       of the parent's mapped candidate, taken 64 at a time,
//                       one extension per lane (at most N_o = 64 new partial
//                       results per level and round);
//   Visited check    -- the lane compares its data vertex with the mapped
//                       vertices of earlier positions that share its label
//                       (other labels can never collide);
//   Edge check       -- for each earlier non-tree neighbour, one bit test in
//                       the partition's bit row of that neighbour's candidate;
//   Synchronizer     -- a wavefront ballot keeps the survivors; at the last
//                       position they are counted (popcount) or written out,
//                       otherwise they become the next level's frontier.
// The deepest level with work is always expanded first, so each level holds
// at most one 64-wide chunk: the frontier is bounded by (k-1) * 64 entries
// and never leaves the chip.  Level state lives in the wavefront's own
// registers: lane d holds the state of level d and is read with v_readlane.
// Work inside a workgroup is shared at the granularity of (root, first child)
// pairs handed out 64 at a time from an LDS counter.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <exception>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace {

__device__ inline int lane_id() { return threadIdx.x & (CSTM_WAVE - 1); }

struct EnumArgs {
    const uint64_t* blobs;  // absolute image addresses
    const int32_t* qids;    // query slot per image (nullptr: slot 0)
    int64_t n_blobs;
    unsigned int* head;
    unsigned long long* counts;
    int list;
    int32_t* rows;
    uint64_t cap;
    unsigned long long* row_cursor;
    unsigned long long* stats;  // [images, bytes, N, M, F] or nullptr
    unsigned long long* stop;   // set to 2 once the deadline has passed
    uint64_t deadline;          // s_memrealtime ticks (100 MHz) after the start; 0 = none
    const unsigned long long* limits;  // per query slot: skip its images once its count reaches this
                                       // (0: none); nullptr: no limits
};

// Deadline check, the same answer in every lane of the wavefront: true once
// this launch has run past its deadline (any wavefront may have seen it first).
__device__ inline bool past_deadline(const EnumArgs& A, uint64_t t_end) {
    if (!A.deadline) return false;
    int stop = 0;
    if (lane_id() == 0) {
        if (__hip_atomic_load(A.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) stop = 1;
        else if (__builtin_amdgcn_s_memrealtime() > t_end) {
            atomicExch(A.stop, 2ull);
            stop = 1;
        }
    }
    return __shfl(stop, 0) != 0;
}

__device__ inline int mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

__device__ inline uint32_t rl(uint32_t x, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)x, l); }
__device__ inline int32_t rl(int32_t x, int l) { return __builtin_amdgcn_readlane(x, l); }
__device__ inline uint64_t rl64(uint64_t x, int l) {
    uint32_t lo = rl((uint32_t)x, l), hi = rl((uint32_t)(x >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

template <class T>
__device__ inline T setl(T cur, T val, int lane, int l) {
    return lane == l ? val : cur;
}

// Write complete embeddings of the lanes in `m`; row[u] = data vertex of query vertex u.
__device__ void emit_rows(const EnumArgs& A, uint64_t m, bool mine, int k, int lane, int32_t pg, uint32_t my_u,
                          int last_pos, int32_t g_last, int second_pos, int32_t g_second) {
    if (!m) return;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(A.row_cursor, (unsigned long long)__popcll(m));
    base = __shfl(base, 0);
    if (!mine) return;
    uint64_t idx = base + (uint64_t)mbcnt(m);
    if (idx >= A.cap) return;
    int32_t* row = A.rows + idx * (uint64_t)k;
    for (int i = 0; i < k; ++i) {
        int32_t val;
        if (i == last_pos) val = g_last;
        else if (i == second_pos) val = g_second;
        else val = rl(pg, i);
        row[rl(my_u, i)] = val;
    }
}

// Enumerate the image in LDS with one wavefront; returns the wavefront's count.
__device__ uint64_t enumerate_image(const uint8_t* img, unsigned int* s_next, const EnumArgs& A, uint64_t t_end,
                                    uint64_t& nN, uint64_t& nM, uint64_t& nF) {
    const int lane = lane_id();
    const BlobHdr* H = (const BlobHdr*)img;
    const int k = (int)H->k;
    const BlobPos* BP = (const BlobPos*)(img + sizeof(BlobHdr));
    const BlobNt* BN = (const BlobNt*)(img + sizeof(BlobHdr) + (size_t)k * sizeof(BlobPos));
    // lane d caches the record of position d
    uint32_t my_n = 0, my_gid = 0, my_toff = 0, my_tadj = 0, my_same = 0, my_nt = 0, my_ntf = 0, my_u = 0;
    int32_t my_par = -1;
    if (lane < k) {
        const BlobPos& P = BP[lane];
        my_n = P.n;
        my_gid = P.gid_off;
        my_toff = P.toff_off;
        my_tadj = P.tadj_off;
        my_same = P.same_mask;
        my_nt = P.nt_mask;
        my_ntf = P.u_nt_first & 0xFFFFu;
        my_u = P.u_nt_first >> 16;
        my_par = P.par;
    }
    const uint32_t n0 = rl(my_n, 0);
    const int32_t* gid0 = (const int32_t*)(img + rl(my_gid, 0));
    uint64_t cnt = 0;

    if (k == 1) {
        // every root candidate is an embedding; the first wavefront takes them
        if (threadIdx.x < CSTM_WAVE) {
            cnt = n0;
            if (A.list) {
                for (uint32_t j0 = 0; j0 < n0; j0 += CSTM_WAVE) {
                    bool ok = j0 + lane < n0;
                    uint64_t m = __ballot(ok);
                    int32_t g = ok ? gid0[j0 + lane] : 0;
                    emit_rows(A, m, ok, 1, lane, 0, my_u, 0, g, -1, 0);
                }
            }
        }
        return cnt;
    }

    const uint32_t* toff1 = (const uint32_t*)(img + rl(my_toff, 1));
    const uint16_t* tadj1 = (const uint16_t*)(img + rl(my_tadj, 1));
    const int32_t* gid1 = (const int32_t*)(img + rl(my_gid, 1));
    const uint32_t E1 = toff1[n0];
    const bool same01 = rl(my_same, 1) & 1u;

    // level state registers: lane d holds level d
    int32_t pl = 0, pg = 0;
    uint32_t lc = 0, le = 0;
    uint64_t lm = 0;

    uint32_t since_check = 0;
    for (;;) {
        if (past_deadline(A, t_end)) break;
        uint32_t t0 = 0;
        if (lane == 0) t0 = atomicAdd(s_next, (unsigned int)CSTM_WAVE);
        t0 = (uint32_t)__shfl((int)t0, 0);
        if (t0 >= E1) break;
        const uint32_t t = t0 + lane;
        const bool valid = t < E1;
        int32_t r = 0, v1 = 0, g0 = 0, g1 = 0;
        if (valid) {
            // root candidate owning list entry t: last r with toff1[r] <= t
            uint32_t lo = 0, hi = n0;
            while (lo < hi) {
                uint32_t mid = (lo + hi + 1) >> 1;
                if (toff1[mid] <= t) lo = mid;
                else hi = mid - 1;
            }
            r = (int32_t)lo;
            v1 = tadj1[t];
            g0 = gid0[r];
            g1 = gid1[v1];
        }
        const bool ok1 = valid && !(same01 && g0 == g1);
        uint64_t m1 = __ballot(ok1);
        nN += (uint64_t)__popcll(__ballot(valid));
        if (k == 2) {
            cnt += (uint64_t)__popcll(m1);
            if (A.list) emit_rows(A, m1, ok1, 2, lane, pg, my_u, 1, g1, 0, g0);
            continue;
        }
        nF += (uint64_t)__popcll(m1);
        while (m1) {
            const int b = __ffsll((unsigned long long)m1) - 1;
            m1 &= m1 - 1;
            const int32_t rb = __shfl(r, b), vb = __shfl(v1, b), g0b = __shfl(g0, b), g1b = __shfl(g1, b);
            pl = setl(pl, rb, lane, 0);
            pg = setl(pg, g0b, lane, 0);
            pl = setl(pl, vb, lane, 1);
            pg = setl(pg, g1b, lane, 1);
            // open level 2
            int d = 2;
            {
                const int p = rl(my_par, d);
                const uint32_t* toff = (const uint32_t*)(img + rl(my_toff, d));
                const int32_t x = rl(pl, p);
                lc = setl(lc, toff[x], lane, d);
                le = setl(le, toff[x + 1], lane, d);
                lm = setl(lm, (uint64_t)0, lane, d);
            }
            for (;;) {
                uint64_t M = rl64(lm, d);
                const uint32_t cur = rl(lc, d);
                const uint16_t* tadj = (const uint16_t*)(img + rl(my_tadj, d));
                if (M == 0) {
                    const uint32_t end = rl(le, d);
                    if (cur >= end) {
                        if (--d < 2) break;
                        continue;
                    }
                    if (++since_check >= 256u) {
                        since_check = 0;
                        if (past_deadline(A, t_end)) return cnt;
                    }
                    // Generator: one extension per lane
                    const uint32_t idx = cur + lane;
                    const bool val = idx < end;
                    const int32_t* gid = (const int32_t*)(img + rl(my_gid, d));
                    const int32_t v = val ? (int32_t)tadj[idx] : 0;
                    const int32_t g = gid[v];
                    bool ok = val;
                    // visited validation: earlier positions with the same label
                    uint32_t same = rl(my_same, d);
                    while (same) {
                        const int j = __ffs(same) - 1;
                        same &= same - 1;
                        ok = ok && g != rl(pg, j);
                    }
                    // edge validation: one bit per earlier non-tree neighbour
                    uint32_t ntm = rl(my_nt, d);
                    uint32_t e = rl(my_ntf, d);
                    while (ntm) {
                        const int j = __ffs(ntm) - 1;
                        ntm &= ntm - 1;
                        const BlobNt N = BN[e++];
                        const uint32_t* bits = (const uint32_t*)(img + N.bits_off);
                        const uint32_t row = (uint32_t)rl(pl, j);
                        const uint32_t word = bits[row * N.row_words + ((uint32_t)v >> 5)];
                        ok = ok && ((word >> (v & 31)) & 1u);
                    }
                    // Synchronizer
                    const uint64_t m = __ballot(ok);
                    {
                        const uint64_t nv = (uint64_t)__popcll(__ballot(val));
                        nN += nv;
                        nM += nv * (uint64_t)__popc(rl(my_nt, d));
                        if (d < k - 1) nF += (uint64_t)__popcll(m);
                    }
                    lc = setl(lc, cur + (uint32_t)CSTM_WAVE, lane, d);
                    if (d == k - 1) {
                        cnt += (uint64_t)__popcll(m);
                        if (A.list) emit_rows(A, m, ok, k, lane, pg, my_u, d, g, -1, 0);
                        continue;
                    }
                    if (!m) continue;
                    M = m;
                }
                // descend into the lowest surviving lane of the current chunk
                const int b = __ffsll((unsigned long long)M) - 1;
                M &= M - 1;
                lm = setl(lm, M, lane, d);
                const uint32_t chunk = rl(lc, d) - (uint32_t)CSTM_WAVE;
                const int32_t v = (int32_t)tadj[chunk + b];
                const int32_t* gid = (const int32_t*)(img + rl(my_gid, d));
                pl = setl(pl, v, lane, d);
                pg = setl(pg, gid[v], lane, d);
                ++d;
                const int p = rl(my_par, d);
                const uint32_t* toff = (const uint32_t*)(img + rl(my_toff, d));
                const int32_t x = rl(pl, p);
                lc = setl(lc, toff[x], lane, d);
                le = setl(le, toff[x + 1], lane, d);
                lm = setl(lm, (uint64_t)0, lane, d);
            }
        }
    }
    return cnt;
}

__global__ void k_enumerate(EnumArgs A) {
    extern __shared__ uint4 smem_u4[];
    uint8_t* img = (uint8_t*)smem_u4;
    __shared__ int64_t s_blob;
    __shared__ unsigned int s_next;
    __shared__ int s_skip;
    const int lane = lane_id();
    const uint64_t t_end = __builtin_amdgcn_s_memrealtime() + A.deadline;
    for (;;) {
        if (threadIdx.x == 0) {
            const bool stop = A.deadline && __hip_atomic_load(A.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int64_t nb = stop ? A.n_blobs : (int64_t)atomicAdd(A.head, 1u);
            // Counts grow only as images finish, so once a query's count has
            // reached its limit the result is min(total, limit) = limit
            // whatever its remaining images hold: they are skipped.
            int skip = 0;
            if (A.limits && nb < A.n_blobs) {
                const int q = A.qids ? A.qids[nb] : 0;
                const unsigned long long lim = A.limits[q];
                skip = lim && __hip_atomic_load(A.counts + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= lim;
            }
            s_blob = nb;
            s_skip = skip;
        }
        __syncthreads();
        const int64_t b = s_blob;
        if (b >= A.n_blobs) break;
        if (s_skip) {
            __syncthreads();  // every thread has read s_blob and s_skip before thread 0 writes them again
            continue;
        }
        const uint8_t* src = (const uint8_t*)A.blobs[b];
        const uint32_t bytes = ((const BlobHdr*)src)->bytes;
        for (uint32_t o = threadIdx.x * 16u; o < bytes; o += blockDim.x * 16u)
            *(uint4*)(img + o) = *(const uint4*)(src + o);
        if (threadIdx.x == 0) s_next = 0;
        __syncthreads();
        uint64_t nN = 0, nM = 0, nF = 0;
        const uint64_t c = enumerate_image(img, &s_next, A, t_end, nN, nM, nF);
        if (lane == 0 && c) atomicAdd(&A.counts[A.qids ? A.qids[b] : 0], (unsigned long long)c);
        if (A.stats && lane == 0) {
            if (threadIdx.x == 0) {
                atomicAdd(&A.stats[0], 1ull);
                atomicAdd(&A.stats[1], (unsigned long long)bytes);
            }
            atomicAdd(&A.stats[2], (unsigned long long)nN);
            atomicAdd(&A.stats[3], (unsigned long long)nM);
            atomicAdd(&A.stats[4], (unsigned long long)nF);
        }
        __syncthreads();
    }
}

}  // namespace

// One launch over the partition images of nq partitioned CSTs; counts go to counts_dev[slot[q]].
void cstm_enumerate_lds_run(cstm_ctx* ctx, int nq, cstm_cst* const* csts, const int* slot, int list, int32_t* rows,
                            uint64_t cap, unsigned long long* counts_dev, unsigned long long* row_cursor,
                            const EnumOpts& opt, cstm_enum_stats* st, hipStream_t s) {
    int64_t total = 0;
    uint64_t max_blob = 0;
    for (int q = 0; q < nq; ++q) {
        total += csts[q]->n_parts;
        max_blob = std::max<uint64_t>(max_blob, csts[q]->max_blob);
    }
    if (total == 0) return;
    CSTM_REQUIRE(total < ((int64_t)1 << 32) - 1, CSTM_EINVAL, "too many partitions for one launch");
    DevArena mem;
    mem.ctx = ctx;
    unsigned long long* work = mem.get_n<unsigned long long>(8);
    cstm_fill_words(work, 8 * sizeof(unsigned long long), 0u, s);  // a kernel, not a memset node
    uint64_t* bl = mem.get_n<uint64_t>(total);
    int32_t* qi = mem.get_n<int32_t>(total);
    std::vector<int32_t> hq(total);
    int64_t o = 0;
    for (int q = 0; q < nq; ++q) {
        int64_t n = csts[q]->n_parts;
        if (!n) continue;
        HIP_TRY(hipMemcpyAsync(bl + o, csts[q]->blob_off, n * 8, hipMemcpyDeviceToDevice, s));
        std::fill(hq.begin() + o, hq.begin() + o + n, slot[q]);
        o += n;
    }
    HIP_TRY(hipMemcpyAsync(qi, hq.data(), total * 4, hipMemcpyHostToDevice, s));
    EnumArgs A;
    A.blobs = bl;
    A.qids = qi;
    A.n_blobs = total;
    A.head = (unsigned int*)work;
    A.counts = counts_dev;
    A.list = list;
    A.rows = rows;
    A.cap = cap;
    A.row_cursor = row_cursor;
    A.stats = ctx->tune.collect_stats ? work + 1 : nullptr;
    A.stop = work + 6;
    A.deadline = opt.deadline_ms > 0 ? 100ull * 1000 * (uint64_t)opt.deadline_ms : 0;
    // per-slot limits (the caller's array is indexed by slot, as the counts are)
    std::vector<unsigned long long> hlim;
    A.limits = nullptr;
    if (opt.limits) {
        int32_t nslots = 0;
        for (int q = 0; q < nq; ++q) nslots = std::max(nslots, slot[q] + 1);
        hlim.assign(nslots, 0ull);
        bool any = false;
        for (int q = 0; q < nq; ++q) {
            hlim[slot[q]] = opt.limits[slot[q]];
            any |= hlim[slot[q]] != 0;
        }
        if (any) {
            unsigned long long* dlim = mem.get_n<unsigned long long>(nslots);
            HIP_TRY(hipMemcpyAsync(dlim, hlim.data(), (size_t)nslots * 8, hipMemcpyHostToDevice, s));
            A.limits = dlim;
        }
    }
    const int waves = ctx->tune.waves_per_wg;
    const size_t lds = (size_t)cstm_align16(max_blob);
    static std::once_flag attr_once;
    std::call_once(attr_once, [&] {
        (void)hipFuncSetAttribute((const void*)k_enumerate, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)ctx->lds_per_wg - 64);
        (void)hipGetLastError();
    });
    int64_t grid = (int64_t)ctx->num_cus * ctx->tune.wgs_per_cu;
    grid = std::min<int64_t>(grid, total);
    hipEvent_t ev[2];
    HIP_TRY(hipEventCreate(&ev[0]));
    HIP_TRY(hipEventCreate(&ev[1]));
    HIP_TRY(hipEventRecord(ev[0], s));
    k_enumerate<<<(unsigned)grid, waves * CSTM_WAVE, lds, s>>>(A);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(ev[1], s));
    HIP_TRY(hipEventSynchronize(ev[1]));
    float kernel_ms = 0;
    HIP_TRY(hipEventElapsedTime(&kernel_ms, ev[0], ev[1]));
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    unsigned long long h[7];
    HIP_TRY(hipMemcpyAsync(h, work, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    st->kernel_ms += kernel_ms;
    st->mode = CSTM_MODE_LDS;
    st->launches += 1;
    st->images += h[1];
    st->image_bytes += h[2];
    st->extensions += h[3];
    st->edge_checks += h[4];
    st->pushed += h[5];
    if (h[6]) {
        std::lock_guard<std::mutex> lk(ctx->ws_mu);
        ctx->last_enum = *st;
    }
    CSTM_REQUIRE(h[6] != 2, CSTM_ETIMEOUT, "enumeration stopped at the deadline");
}

// Partition, at the context's budget, the CSTs an LDS launch meets
// unpartitioned; fits[i] = 0 when the images of cut[i] would replicate it
// beyond max_replication (that CST stays in HBM).  Algorithm 2 runs on each
// CST's own stream, and its first round is a single workgroup, so several
// host threads cut different CSTs at once to keep the GPU busy.
static void partition_for_lds(cstm_ctx* ctx, cstm_cst* const* csts, const std::vector<int>& cut,
                              std::vector<char>& fits) {
    constexpr size_t kPartThreads = 8;
    const cstm_tune T = ctx->tune;
    fits.assign(cut.size(), 1);
    auto cut_one = [&](size_t i) {
        cstm_cst* c = csts[cut[i]];
        const uint64_t cap =
            T.max_replication > 0 ? (uint64_t)T.max_replication * std::max<uint64_t>(c->bytes, 4096) : 0;
        fits[i] = cstm_partition_run(c, 0, T.max_list_len, cap) ? 1 : 0;
    };
    const size_t n_threads = std::min(cut.size(), kPartThreads);
    if (n_threads <= 1) {
        for (size_t i = 0; i < cut.size(); ++i) cut_one(i);
        return;
    }
    std::atomic<size_t> next{0};
    std::mutex err_mu;
    std::exception_ptr err;
    auto worker = [&] {
        try {
            HIP_TRY(hipSetDevice(ctx->device));
            for (size_t i; (i = next.fetch_add(1)) < cut.size();) cut_one(i);
        } catch (...) {
            std::lock_guard<std::mutex> lk(err_mu);
            if (!err) err = std::current_exception();
            next.store(cut.size());  // the other threads take no further CST
        }
    };
    std::vector<std::thread> pool;
    try {
        for (size_t t = 0; t < n_threads; ++t) pool.emplace_back(worker);
    } catch (...) {
        next.store(cut.size());
        for (auto& th : pool) th.join();
        throw;
    }
    for (auto& th : pool) th.join();
    if (err) std::rethrow_exception(err);
}

// Enumerate nq CSTs: pick LDS images or the HBM-resident CST per the tuning,
// run at most one launch of each kind, and return per-CST counts.
void cstm_enumerate_run(cstm_ctx* ctx, int nq, cstm_cst* const* csts, int list, int32_t* rows, uint64_t cap,
                        uint64_t* counts_host, uint64_t* rows_written, const EnumOpts& o, hipStream_t s,
                        cstm_enum_stats* st_out) {
    const cstm_tune T = ctx->tune;
    std::vector<int> mode_of(nq, -1);  // -1: empty CST, nothing to launch
    std::vector<int> cut;              // LDS-mode CSTs still to partition, each CST once
    std::vector<int> cut_of(nq, -1);   // index into cut of the CST at q
    std::unordered_map<const cstm_cst*, int> seen;
    for (int q = 0; q < nq; ++q) {
        cstm_cst* c = csts[q];
        if (c->empty) continue;
        int mode = T.enum_mode;
        if (o.root_ranges || o.force_hbm) mode = CSTM_MODE_HBM;
        if (mode == CSTM_MODE_AUTO) {
            // partitions the caller asked for are enumerated on chip; otherwise the
            // CST stays in HBM, where the whole GPU shares one query's search
            mode = c->partitioned ? CSTM_MODE_LDS : CSTM_MODE_HBM;
        }
        if (mode == CSTM_MODE_LDS && !c->partitioned) {
            auto it = seen.emplace(c, (int)cut.size()).first;
            if (it->second == (int)cut.size()) cut.push_back(q);
            cut_of[q] = it->second;
        }
        mode_of[q] = mode;
    }
    if (!cut.empty()) {
        std::vector<char> fits;
        partition_for_lds(ctx, csts, cut, fits);
        for (int q = 0; q < nq; ++q)
            if (cut_of[q] >= 0 && !fits[cut_of[q]]) mode_of[q] = CSTM_MODE_HBM;
    }
    std::vector<cstm_cst*> lds_q, hbm_q;
    std::vector<int> lds_slot, hbm_slot;
    for (int q = 0; q < nq; ++q) {
        if (mode_of[q] < 0) continue;
        if (mode_of[q] == CSTM_MODE_LDS) {
            lds_q.push_back(csts[q]);
            lds_slot.push_back(q);
        } else {
            hbm_q.push_back(csts[q]);
            hbm_slot.push_back(q);
        }
    }
    DevArena mem;
    mem.ctx = ctx;
    unsigned long long* counts = mem.get_n<unsigned long long>(nq + 1);
    cstm_fill_words(counts, (nq + 1) * sizeof(unsigned long long), 0u, s);  // a kernel, not a memset node
    unsigned long long* row_cursor = counts + nq;
    cstm_enum_stats st{};
    if (!lds_q.empty())
        cstm_enumerate_lds_run(ctx, (int)lds_q.size(), lds_q.data(), lds_slot.data(), list, rows, cap, counts,
                               row_cursor, o, &st, s);
    if (!hbm_q.empty())
        cstm_enumerate_global_run(ctx, (int)hbm_q.size(), hbm_q.data(), hbm_slot.data(), list, rows, cap, counts,
                                  row_cursor, o, &st, s);
    std::vector<unsigned long long> h(nq + 1);
    HIP_TRY(hipMemcpyAsync(h.data(), counts, (nq + 1) * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    {
        std::lock_guard<std::mutex> lk(ctx->ws_mu);
        ctx->last_enum = st;
    }
    if (st_out) *st_out = st;
    for (int q = 0; q < nq; ++q) {
        counts_host[q] = h[q];
        // a launch passes a limit before it stops (an on-chip launch finishes every image it started)
        if (o.limits && o.limits[q] && counts_host[q] > o.limits[q]) counts_host[q] = o.limits[q];
    }
    if (rows_written) *rows_written = std::min<uint64_t>(h[nq], cap);
}

extern "C" cstm_status cstm_enumerate(cstm_cst* cst, int list, uint64_t limit, int32_t* rows, uint64_t cap,
                                      uint64_t* count_out, uint64_t* rows_written, double deadline_s, void* stream) {
    uint64_t count = 0;
    uint64_t written = 0;
    cstm_status st = cstm_guard([&] {
        CSTM_REQUIRE(cst, CSTM_EINVAL, "NULL cst");
        CSTM_REQUIRE(deadline_s == deadline_s, CSTM_EINVAL, "deadline is NaN");
        EnumOpts o;
        o.limits = limit ? &limit : nullptr;
        o.deadline_ms = deadline_s > 0 ? (int64_t)(deadline_s * 1e3) + 1 : cst->ctx->tune.deadline_ms;
        CSTM_REQUIRE(!list || rows || cap == 0, CSTM_EINVAL, "listing needs a row buffer");
        HIP_TRY(hipSetDevice(cst->ctx->device));
        hipStream_t s = stream ? (hipStream_t)stream : cst->stream;
        hipEvent_t a, b;
        HIP_TRY(hipEventCreate(&a));
        HIP_TRY(hipEventCreate(&b));
        HIP_TRY(hipEventRecord(a, s));
        cstm_cst* one[1] = {cst};
        cstm_enumerate_run(cst->ctx, 1, one, list, rows, cap, &count, &written, o, s);
        if (limit && written > limit) written = limit;
        HIP_TRY(hipEventRecord(b, s));
        HIP_TRY(hipEventSynchronize(b));
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, a, b));
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        cst->t_enum = ms;
    });
    if (count_out) *count_out = count;
    if (rows_written) *rows_written = written;
    if (st == CSTM_OK && list && count > cap) {
        cstm_set_error("row buffer smaller than the number of embeddings");
        return CSTM_EOVERFLOW;
    }
    return st;
}

extern "C" cstm_status cstm_batch_enumerate(cstm_ctx* ctx, int32_t nq, cstm_cst* const* csts, const uint64_t* limits,
                                            uint64_t* counts_out, void* stream) {
    return cstm_guard([&] {
        CSTM_REQUIRE(ctx && (nq == 0 || (csts && counts_out)), CSTM_EINVAL, "NULL argument");
        CSTM_REQUIRE(nq >= 0, CSTM_EINVAL, "negative query count");
        for (int q = 0; q < nq; ++q) CSTM_REQUIRE(csts[q] && csts[q]->ctx == ctx, CSTM_EINVAL, "bad CST handle");
        if (nq == 0) return;
        HIP_TRY(hipSetDevice(ctx->device));
        EnumOpts o;
        o.limits = limits;
        o.deadline_ms = ctx->tune.deadline_ms;
        cstm_enumerate_run(ctx, nq, csts, 0, nullptr, 0, counts_out, nullptr, o, (hipStream_t)stream);
    });
}
