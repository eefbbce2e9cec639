// partition.hip -- CST partition to the LDS budget (Section V-B, Algorithm 2).
//
// A partition is described by a Spec: index ranges over the candidate sets of
// some positions of the matching order.  Its candidate sets are obtained top
// down along the order: position 0 keeps the candidates in its range; every
// later position keeps the candidates its tree parent's kept candidates reach
// through the tree lists (and, if it has a range, only those inside it).  This
// is "pick the candidates that can reach the split part", read along the tree.
//
// One workgroup handles one Spec: it computes the restricted sets (bitmaps and
// sorted member lists in a private global scratch slot), the size of the
// on-chip image, and then either serialises the image (it fits) or emits
// k = ceil(max(size / delta_S, D / delta_D)) child Specs that split the
// candidates of the first splittable position into k contiguous, even parts.
// The host repeats the launch over the frontier of Specs until none is left.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / CSTM_WAVE;

enum : int { OVF_SPECS = 1, OVF_ARENA = 2, OVF_BLOBS = 4, OVERSIZE = 8 };

struct PartArgs {
    const CstDev* desc;
    const Spec* in;
    int64_t n_in;
    Spec* out;
    unsigned long long* n_out;
    int64_t out_cap;
    uint8_t* arena;
    unsigned long long* arena_used;
    uint64_t arena_cap;
    uint64_t* blob_off;
    unsigned long long* n_blobs;
    int64_t blob_cap;
    int32_t* scratch;
    int64_t slot_words;
    uint64_t budget;
    int32_t max_list;
    int* flags;
    unsigned int* max_blob;
};

__device__ inline int lane_id() { return threadIdx.x & (CSTM_WAVE - 1); }
__device__ inline int wave_id() { return threadIdx.x / CSTM_WAVE; }
__device__ inline int mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

// Exclusive scan of one int per thread over the block; returns the prefix, writes the total.
__device__ int block_exclusive_scan(int v, int* s_wave, int* total) {
    const int lane = lane_id(), w = wave_id();
    int x = v;
    for (int d = 1; d < CSTM_WAVE; d <<= 1) {
        int y = __shfl_up(x, d, CSTM_WAVE);
        if (lane >= d) x += y;
    }
    if (lane == CSTM_WAVE - 1) s_wave[w] = x;
    __syncthreads();
    int base = 0, tot = 0;
    for (int i = 0; i < kWaves; ++i) {
        if (i < w) base += s_wave[i];
        tot += s_wave[i];
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

__device__ inline int32_t lower_bound_i32(const int32_t* a, int64_t n, int32_t x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return (int32_t)lo;
}

__device__ inline uint64_t words_of(int64_t n) { return (uint64_t)((n + 31) >> 5); }

__global__ __launch_bounds__(kBlock) void k_partition(PartArgs A) {
    __shared__ Spec s_spec;
    __shared__ int64_t s_bm_off[CSTM_MAX_K], s_mem_off[CSTM_MAX_K];
    __shared__ int64_t s_tmp_off;
    __shared__ int64_t s_cnt[CSTM_MAX_K];
    __shared__ unsigned long long s_E[CSTM_MAX_K];
    __shared__ int s_maxlen;
    __shared__ int s_dead;
    __shared__ int s_wave[kWaves];
    __shared__ unsigned long long s_base;
    __shared__ uint32_t s_gid_off[CSTM_MAX_K], s_toff_off[CSTM_MAX_K], s_tadj_off[CSTM_MAX_K];
    __shared__ uint32_t s_bits_off[CSTM_MAX_NT];
    __shared__ uint64_t s_size;
    __shared__ int s_split;

    const CstDev& D = *A.desc;
    const int k = D.k;
    const int lane = lane_id(), w = wave_id();
    int32_t* slot = A.scratch + (int64_t)blockIdx.x * A.slot_words;

    if (threadIdx.x == 0) {
        int64_t off = 0;
        for (int i = 0; i < k; ++i) {
            s_bm_off[i] = off;
            off += (int64_t)words_of(D.pos[i].n);
        }
        for (int i = 0; i < k; ++i) {
            s_mem_off[i] = off;
            off += D.pos[i].n;
        }
        s_tmp_off = off;
    }
    __syncthreads();

    for (int64_t si = blockIdx.x; si < A.n_in; si += gridDim.x) {
        if (threadIdx.x == 0) {
            s_spec = A.in[si];
            s_dead = 0;
            s_maxlen = 0;
        }
        __syncthreads();
        // ---- restricted candidate sets, top-down along the order
        for (int i = 0; i < k; ++i) {
            const PosDesc& P = D.pos[i];
            const int32_t lo = s_spec.lo[i], hi = s_spec.hi[i];
            uint32_t* bm = (uint32_t*)(slot + s_bm_off[i]);
            int32_t* mem = slot + s_mem_off[i];
            if (i == 0) {
                for (int64_t j = threadIdx.x; j < hi - lo; j += kBlock) mem[j] = lo + (int32_t)j;
                // the root bitmap is only read by non-tree membership tests, never for position 0
                if (threadIdx.x == 0) {
                    s_cnt[0] = hi - lo;
                    s_E[0] = 0;
                }
                __syncthreads();
                if (s_cnt[0] <= 0) {
                    if (threadIdx.x == 0) s_dead = 1;
                    __syncthreads();
                    break;
                }
                continue;
            }
            const uint64_t W = words_of(P.n);
            for (uint64_t j = threadIdx.x; j < W; j += kBlock) bm[j] = 0u;
            if (threadIdx.x == 0) s_E[i] = 0;
            __syncthreads();
            const int p = P.par;
            const int32_t* mem_p = slot + s_mem_off[p];
            const int64_t cnt_p = s_cnt[p];
            unsigned long long E = 0;
            int maxlen = 0;
            for (int64_t x = w; x < cnt_p; x += kWaves) {
                const int32_t pv = mem_p[x];
                const int64_t b = P.toff[pv], e = P.toff[pv + 1];
                int c = 0;
                for (int64_t j = b + lane; j - lane < e; j += CSTM_WAVE) {
                    bool in = false;
                    if (j < e) {
                        int32_t v = P.tadj[j];
                        in = v >= lo && v < hi;
                        if (in) atomicOr(&bm[v >> 5], 1u << (v & 31));
                    }
                    c += __popcll(__ballot(in));
                }
                E += (unsigned long long)c;
                maxlen = c > maxlen ? c : maxlen;
            }
            if (lane == 0) {
                atomicAdd(&s_E[i], E);
                atomicMax(&s_maxlen, maxlen);
            }
            __syncthreads();
            // compact the bitmap into the sorted member list
            int64_t running = 0;
            for (uint64_t w0 = 0; w0 < W; w0 += kBlock) {
                uint64_t wi = w0 + threadIdx.x;
                uint32_t word = wi < W ? bm[wi] : 0u;
                int tot;
                int pre = block_exclusive_scan(__popc(word), s_wave, &tot);
                int64_t dst = running + pre;
                while (word) {
                    int b = __ffs(word) - 1;
                    word &= word - 1;
                    mem[dst++] = (int32_t)(wi * 32 + b);
                }
                running += tot;
            }
            if (threadIdx.x == 0) s_cnt[i] = running;
            __syncthreads();
            if (running == 0) {
                if (threadIdx.x == 0) s_dead = 1;
                __syncthreads();
                break;
            }
        }
        if (s_dead) {
            __syncthreads();
            continue;
        }
        // ---- D_CST over non-tree lists, only when a list-length limit is set
        if (A.max_list > 0) {
            for (int e = 0; e < D.n_nt; ++e) {
                const NtDesc& N = D.nt[e];
                const int32_t* mem_a = slot + s_mem_off[N.a];
                const uint32_t* bm_b = (const uint32_t*)(slot + s_bm_off[N.b]);
                int maxlen = 0;
                for (int64_t x = w; x < s_cnt[N.a]; x += kWaves) {
                    const int32_t av = mem_a[x];
                    const int64_t b = N.off[av], en = N.off[av + 1];
                    int c = 0;
                    for (int64_t j = b + lane; j - lane < en; j += CSTM_WAVE) {
                        bool in = false;
                        if (j < en) {
                            int32_t v = N.adj[j];
                            in = (bm_b[v >> 5] >> (v & 31)) & 1u;
                        }
                        c += __popcll(__ballot(in));
                    }
                    maxlen = c > maxlen ? c : maxlen;
                }
                if (lane == 0) atomicMax(&s_maxlen, maxlen);
            }
            __syncthreads();
        }
        // ---- size of the on-chip image
        if (threadIdx.x == 0) {
            uint64_t cur = blob_header_bytes(k, D.n_nt);
            for (int i = 0; i < k; ++i) {
                s_gid_off[i] = (uint32_t)cur;
                cur += 4ull * (uint64_t)s_cnt[i];
            }
            for (int i = 1; i < k; ++i) {
                s_toff_off[i] = (uint32_t)cur;
                cur += 4ull * (uint64_t)(s_cnt[D.pos[i].par] + 1);
                s_tadj_off[i] = (uint32_t)cur;
                cur += 4ull * ((s_E[i] + 1) / 2);
            }
            for (int e = 0; e < D.n_nt; ++e) {
                s_bits_off[e] = (uint32_t)(cur > 0xFFFFFFFFull ? 0xFFFFFFFFull : cur);
                cur += 4ull * (uint64_t)s_cnt[D.nt[e].a] * words_of(s_cnt[D.nt[e].b]);
            }
            s_size = cstm_align16(cur);
            bool fits = s_size <= A.budget && (A.max_list <= 0 || s_maxlen <= A.max_list);
            int split = -1;
            if (!fits) {
                for (int i = s_spec.uidx; i < k; ++i)
                    if (s_cnt[i] > 1) {
                        split = i;
                        break;
                    }
                if (split < 0) atomicOr(A.flags, OVERSIZE);
            }
            s_split = fits ? -1 : split;
            if (fits || split < 0) {
                unsigned long long off = atomicAdd(A.arena_used, (unsigned long long)s_size);
                unsigned long long bi = atomicAdd(A.n_blobs, 1ull);
                if (off + s_size > A.arena_cap) {
                    atomicOr(A.flags, OVF_ARENA);
                    s_split = -2;
                } else if ((int64_t)bi >= A.blob_cap) {
                    atomicOr(A.flags, OVF_BLOBS);
                    s_split = -2;
                } else {
                    A.blob_off[bi] = off;
                    s_base = off;
                    atomicMax(A.max_blob, (unsigned int)s_size);
                }
            }
        }
        __syncthreads();
        const int split = s_split;
        if (split == -2) {
            __syncthreads();
            continue;
        }
        if (split >= 0) {
            // ---- child specs: k contiguous even parts of the candidates at `split`
            const int64_t cnt_u = s_cnt[split];
            double f = (double)s_size / (double)A.budget;
            if (A.max_list > 0) {
                double fd = (double)s_maxlen / (double)A.max_list;
                f = fd > f ? fd : f;
            }
            int64_t kp = (int64_t)ceil(f);
            if (kp < 2) kp = 2;
            if (kp > cnt_u) kp = cnt_u;
            const int32_t* mem_u = slot + s_mem_off[split];
            const int64_t base = cnt_u / kp, extra = cnt_u % kp;
            for (int64_t j = threadIdx.x; j < kp; j += kBlock) {
                int64_t start = j * base + (j < extra ? j : extra);
                int64_t c = base + (j < extra ? 1 : 0);
                unsigned long long o = atomicAdd(A.n_out, 1ull);
                if ((int64_t)o >= A.out_cap) {
                    atomicOr(A.flags, OVF_SPECS);
                    continue;
                }
                Spec& S = A.out[o];
                S.qid = s_spec.qid;
                S.uidx = split;
                for (int i = 0; i < CSTM_MAX_K; ++i) {
                    S.lo[i] = s_spec.lo[i];
                    S.hi[i] = s_spec.hi[i];
                }
                S.lo[split] = mem_u[start];
                S.hi[split] = mem_u[start + c - 1] + 1;
            }
            __syncthreads();
            continue;
        }
        // ---- serialise the on-chip image
        uint8_t* img = A.arena + s_base;
        if (threadIdx.x == 0) {
            BlobHdr* H = (BlobHdr*)img;
            H->k = (uint32_t)k;
            H->n_nt = (uint32_t)D.n_nt;
            H->bytes = (uint32_t)s_size;
            H->qid = (uint32_t)s_spec.qid;
            for (int r = 0; r < 12; ++r) H->reserved[r] = 0;
            BlobPos* BP = (BlobPos*)(img + sizeof(BlobHdr));
            for (int i = 0; i < k; ++i) {
                const PosDesc& P = D.pos[i];
                BP[i].n = (uint32_t)s_cnt[i];
                BP[i].gid_off = s_gid_off[i];
                BP[i].par = P.par;
                BP[i].toff_off = i ? s_toff_off[i] : 0u;
                BP[i].tadj_off = i ? s_tadj_off[i] : 0u;
                BP[i].same_mask = P.same_mask;
                BP[i].nt_mask = P.nt_mask;
                BP[i].u_nt_first = ((uint32_t)P.u << 16) | ((uint32_t)(P.nt_first < 0 ? 0 : P.nt_first) & 0xFFFFu);
            }
            BlobNt* BN = (BlobNt*)(img + sizeof(BlobHdr) + (size_t)k * sizeof(BlobPos));
            for (int e = 0; e < D.n_nt; ++e) {
                BN[e].a = (uint32_t)D.nt[e].a;
                BN[e].b = (uint32_t)D.nt[e].b;
                BN[e].bits_off = s_bits_off[e];
                BN[e].row_words = (uint32_t)words_of(s_cnt[D.nt[e].b]);
            }
            // zero the header padding
            uint64_t hb = blob_header_bytes(k, D.n_nt);
            for (uint64_t o = sizeof(BlobHdr) + (uint64_t)k * sizeof(BlobPos) + (uint64_t)D.n_nt * sizeof(BlobNt);
                 o < hb; ++o)
                img[o] = 0;
            // zero the tail padding
            uint64_t last = 0;
            if (D.n_nt) {
                const NtDesc& N = D.nt[D.n_nt - 1];
                last = s_bits_off[D.n_nt - 1] + 4ull * (uint64_t)s_cnt[N.a] * words_of(s_cnt[N.b]);
            } else if (k > 1) {
                last = s_tadj_off[k - 1] + 4ull * ((s_E[k - 1] + 1) / 2);
            } else {
                last = s_gid_off[0] + 4ull * (uint64_t)s_cnt[0];
            }
            for (uint64_t o = last; o < s_size; ++o) img[o] = 0;
        }
        // data-vertex ids
        for (int i = 0; i < k; ++i) {
            const PosDesc& P = D.pos[i];
            const int32_t* mem = slot + s_mem_off[i];
            int32_t* gid = (int32_t*)(img + s_gid_off[i]);
            for (int64_t j = threadIdx.x; j < s_cnt[i]; j += kBlock) gid[j] = P.gid[mem[j]];
        }
        // tree lists, re-indexed into the partition's candidate lists
        int32_t* tmp = slot + s_tmp_off;
        for (int i = 1; i < k; ++i) {
            const PosDesc& P = D.pos[i];
            const int p = P.par;
            const int32_t* mem_p = slot + s_mem_off[p];
            const int32_t* mem_i = slot + s_mem_off[i];
            const int64_t cnt_p = s_cnt[p], cnt_i = s_cnt[i];
            const int32_t lo = s_spec.lo[i], hi = s_spec.hi[i];
            const bool full = lo == 0 && (int64_t)hi >= P.n;
            for (int64_t x = w; x < cnt_p; x += kWaves) {
                const int32_t pv = mem_p[x];
                const int64_t b = P.toff[pv], e = P.toff[pv + 1];
                int c = 0;
                if (full) c = (int)(e - b);
                else
                    for (int64_t j = b + lane; j - lane < e; j += CSTM_WAVE) {
                        bool in = false;
                        if (j < e) {
                            int32_t v = P.tadj[j];
                            in = v >= lo && v < hi;
                        }
                        c += __popcll(__ballot(in));
                    }
                if (lane == 0) tmp[x] = c;
            }
            __syncthreads();
            uint32_t* toff = (uint32_t*)(img + s_toff_off[i]);
            int running = 0;
            for (int64_t x0 = 0; x0 < cnt_p; x0 += kBlock) {
                int64_t x = x0 + threadIdx.x;
                int v = x < cnt_p ? tmp[x] : 0;
                int tot;
                int pre = block_exclusive_scan(v, s_wave, &tot);
                if (x < cnt_p) toff[x] = (uint32_t)(running + pre);
                running += tot;
            }
            if (threadIdx.x == 0) toff[cnt_p] = (uint32_t)running;
            __syncthreads();
            uint16_t* tadj = (uint16_t*)(img + s_tadj_off[i]);
            for (int64_t x = w; x < cnt_p; x += kWaves) {
                const int32_t pv = mem_p[x];
                const int64_t b = P.toff[pv], e = P.toff[pv + 1];
                uint32_t out = toff[x];
                for (int64_t j0 = b; j0 < e; j0 += CSTM_WAVE) {
                    int64_t j = j0 + lane;
                    bool in = false;
                    int32_t v = 0;
                    if (j < e) {
                        v = P.tadj[j];
                        in = v >= lo && v < hi;
                    }
                    uint64_t m = __ballot(in);
                    if (in) tadj[out + mbcnt(m)] = (uint16_t)lower_bound_i32(mem_i, cnt_i, v);
                    out += (uint32_t)__popcll(m);
                }
            }
            if (threadIdx.x == 0 && (s_E[i] & 1ull)) tadj[s_E[i]] = 0;
            __syncthreads();
        }
        // non-tree bit rows
        for (int e = 0; e < D.n_nt; ++e) {
            const NtDesc& N = D.nt[e];
            const int64_t cnt_a = s_cnt[N.a], cnt_b = s_cnt[N.b];
            const uint64_t rw = words_of(cnt_b);
            uint32_t* bits = (uint32_t*)(img + s_bits_off[e]);
            for (uint64_t j = threadIdx.x; j < (uint64_t)cnt_a * rw; j += kBlock) bits[j] = 0u;
            __syncthreads();
            const int32_t* mem_a = slot + s_mem_off[N.a];
            const int32_t* mem_b = slot + s_mem_off[N.b];
            const uint32_t* bm_b = (const uint32_t*)(slot + s_bm_off[N.b]);
            for (int64_t x = w; x < cnt_a; x += kWaves) {
                const int32_t av = mem_a[x];
                const int64_t b = N.off[av], en = N.off[av + 1];
                for (int64_t j = b + lane; j < en; j += CSTM_WAVE) {
                    int32_t v = N.adj[j];
                    if ((bm_b[v >> 5] >> (v & 31)) & 1u) {
                        int32_t nv = lower_bound_i32(mem_b, cnt_b, v);
                        atomicOr(&bits[(uint64_t)x * rw + (nv >> 5)], 1u << (nv & 31));
                    }
                }
            }
            __syncthreads();
        }
        __syncthreads();
    }
}

__global__ void k_to_ptrs(const uint64_t* __restrict__ off, int64_t n, uint64_t base, uint64_t* __restrict__ ptr) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) ptr[i] = base + off[i];
}

}  // namespace

// Smallest possible image: one candidate per position.
static uint64_t min_image_bytes(const cstm_cst* c) {
    uint64_t b = blob_header_bytes(c->k, (int)c->nt.size()) + 4ull * c->k;
    if (c->k > 1) b += (uint64_t)(c->k - 1) * (8 + 4);
    b += 4ull * c->nt.size();
    return cstm_align16(b);
}

bool cstm_partition_run(cstm_cst* c, uint64_t budget, int32_t max_list, uint64_t max_total_bytes) {
    cstm_ctx* ctx = c->ctx;
    hipStream_t s = c->stream;
    if (budget == 0) budget = ctx->tune.part_budget_bytes;
    if (max_list < 0) max_list = 0;
    const uint64_t lds_cap = (uint64_t)ctx->lds_per_wg - 256 - 64ull * 16;
    CSTM_REQUIRE(budget <= lds_cap, CSTM_EINVAL, "partition budget exceeds the LDS a workgroup can address");
    CSTM_REQUIRE(budget >= min_image_bytes(c), CSTM_EINVAL,
                 "partition budget is below the image size of a single-candidate partition");
    budget &= ~uint64_t(15);
    // drop earlier partitions
    if (c->blob_arena) c->mem.release(c->blob_arena);
    if (c->blob_off) c->mem.release(c->blob_off);
    c->blob_arena = nullptr;
    c->blob_off = nullptr;
    c->n_parts = 0;
    c->blob_bytes = 0;
    c->max_blob = 0;
    c->part_budget = budget;
    c->part_max_list = max_list;
    // marked partitioned only once every image is written: a run that throws
    // leaves the CST unpartitioned, never partitioned with missing images
    c->partitioned = c->empty;
    if (c->empty) return true;

    const int k = c->k;
    const CstDev& D = c->host_desc;
    int64_t slot_words = 1;
    {
        int64_t wsum = 0, nsum = 0, nmax = 0;
        for (int i = 0; i < k; ++i) {
            wsum += (D.pos[i].n + 31) / 32;
            nsum += D.pos[i].n;
            nmax = std::max(nmax, D.pos[i].n);
        }
        slot_words = wsum + nsum + nmax + 1;
    }
    // global scratch: one slot per resident workgroup, within ~2 GiB
    int64_t max_slots = std::max<int64_t>(1, ((int64_t)2 << 30) / (slot_words * 4));
    max_slots = std::min<int64_t>(max_slots, (int64_t)ctx->num_cus * 4);
    int32_t* scratch = c->mem.get_n<int32_t>((size_t)(max_slots * slot_words));

    int64_t spec_cap = 1 << 14;
    Spec* spec_a = c->mem.get_n<Spec>(spec_cap);
    Spec* spec_b = c->mem.get_n<Spec>(spec_cap);
    uint64_t arena_cap = std::max<uint64_t>(1ull << 24, 2 * c->bytes);
    uint8_t* arena = c->mem.get_n<uint8_t>(arena_cap);
    int64_t blob_cap = 1 << 14;
    uint64_t* blob_off = c->mem.get_n<uint64_t>(blob_cap);

    struct Counters {
        unsigned long long n_out, arena_used, n_blobs;
        int flags;
        unsigned int max_blob;
    };
    Counters* dc = c->mem.get_n<Counters>(1);
    Counters hc{0, 0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(dc, &hc, sizeof(hc), hipMemcpyHostToDevice, s));

    Spec root{};
    root.qid = 0;
    root.uidx = 0;
    for (int i = 0; i < CSTM_MAX_K; ++i) {
        root.lo[i] = 0;
        root.hi[i] = i < k ? (int32_t)D.pos[i].n : 0;
    }
    HIP_TRY(hipMemcpyAsync(spec_a, &root, sizeof(Spec), hipMemcpyHostToDevice, s));
    int64_t n_in = 1;
    int iter = 0;
    while (n_in > 0) {
        CSTM_REQUIRE(++iter < 100000, CSTM_EDEVICE, "partitioning did not converge");
        Counters before;
        HIP_TRY(hipMemcpyAsync(&before, dc, sizeof(before), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        before.n_out = 0;
        before.flags = 0;
        HIP_TRY(hipMemcpyAsync(dc, &before, sizeof(before), hipMemcpyHostToDevice, s));
        PartArgs A;
        A.desc = c->dev;
        A.in = spec_a;
        A.n_in = n_in;
        A.out = spec_b;
        A.n_out = &dc->n_out;
        A.out_cap = spec_cap;
        A.arena = arena;
        A.arena_used = &dc->arena_used;
        A.arena_cap = arena_cap;
        A.blob_off = blob_off;
        A.n_blobs = &dc->n_blobs;
        A.blob_cap = blob_cap;
        A.scratch = scratch;
        A.slot_words = slot_words;
        A.budget = budget;
        A.max_list = max_list;
        A.flags = &dc->flags;
        A.max_blob = &dc->max_blob;
        unsigned grid = (unsigned)std::min<int64_t>(n_in, max_slots);
        k_partition<<<grid, kBlock, 0, s>>>(A);
        HIP_TRY(hipGetLastError());
        Counters after;
        HIP_TRY(hipMemcpyAsync(&after, dc, sizeof(after), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        CSTM_REQUIRE(!(after.flags & OVERSIZE), CSTM_EDEVICE, "partition could not be split below the budget");
        if (after.flags & (OVF_SPECS | OVF_ARENA | OVF_BLOBS)) {
            // grow what overflowed and redo this round from the saved counters
            if (after.flags & OVF_SPECS) {
                int64_t want = std::max<int64_t>(spec_cap * 2, (int64_t)after.n_out + 1);
                c->mem.release(spec_b);
                spec_b = c->mem.get_n<Spec>(want);
                Spec* na = c->mem.get_n<Spec>(want);
                HIP_TRY(hipMemcpyAsync(na, spec_a, n_in * sizeof(Spec), hipMemcpyDeviceToDevice, s));
                HIP_TRY(hipStreamSynchronize(s));
                c->mem.release(spec_a);
                spec_a = na;
                spec_cap = want;
            }
            if (after.flags & OVF_ARENA) {
                uint64_t want = std::max<uint64_t>(arena_cap * 2, after.arena_used + (1ull << 20));
                uint8_t* na = c->mem.get_n<uint8_t>(want);
                if (before.arena_used)
                    HIP_TRY(hipMemcpyAsync(na, arena, before.arena_used, hipMemcpyDeviceToDevice, s));
                HIP_TRY(hipStreamSynchronize(s));
                c->mem.release(arena);
                arena = na;
                arena_cap = want;
            }
            if (after.flags & OVF_BLOBS) {
                int64_t want = std::max<int64_t>(blob_cap * 2, (int64_t)after.n_blobs + 1);
                uint64_t* nb = c->mem.get_n<uint64_t>(want);
                if (before.n_blobs)
                    HIP_TRY(hipMemcpyAsync(nb, blob_off, before.n_blobs * 8, hipMemcpyDeviceToDevice, s));
                HIP_TRY(hipStreamSynchronize(s));
                c->mem.release(blob_off);
                blob_off = nb;
                blob_cap = want;
            }
            before.flags = 0;
            before.n_out = 0;
            HIP_TRY(hipMemcpyAsync(dc, &before, sizeof(before), hipMemcpyHostToDevice, s));
            continue;
        }
        std::swap(spec_a, spec_b);
        n_in = (int64_t)after.n_out;
        if (n_in > spec_cap) n_in = spec_cap;
        if (max_total_bytes &&
            (after.arena_used > max_total_bytes || (uint64_t)n_in * 4096ull > max_total_bytes * 64ull)) {
            // the images replicate the CST beyond the caller's limit: give up
            c->mem.release(arena);
            c->mem.release(blob_off);
            c->mem.release(spec_a);
            c->mem.release(spec_b);
            c->mem.release(scratch);
            c->mem.release(dc);
            c->partitioned = false;
            return false;
        }
    }
    Counters fin;
    HIP_TRY(hipMemcpyAsync(&fin, dc, sizeof(fin), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    c->n_parts = (int64_t)fin.n_blobs;
    c->blob_bytes = fin.arena_used;
    c->max_blob = fin.max_blob;
    c->blob_arena = arena;
    c->blob_arena_cap = arena_cap;
    // absolute image addresses, for queues that mix partitions of several CSTs
    c->blob_off = c->mem.get_n<uint64_t>(c->n_parts ? c->n_parts : 1);
    if (c->n_parts) {
        k_to_ptrs<<<cstm_blocks(c->n_parts, 256, 4096), 256, 0, s>>>(blob_off, c->n_parts, (uint64_t)arena,
                                                                     c->blob_off);
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(s));
    c->mem.release(blob_off);
    c->mem.release(spec_a);
    c->mem.release(spec_b);
    c->mem.release(scratch);
    c->mem.release(dc);
    c->partitioned = true;
    return true;
}

extern "C" cstm_status cstm_cst_partition(cstm_cst* cst, uint64_t budget_bytes, int32_t max_list_len,
                                          uint64_t max_total_bytes, int64_t* n_parts_out) {
    return cstm_guard([&] {
        CSTM_REQUIRE(cst, CSTM_EINVAL, "NULL cst");
        HIP_TRY(hipSetDevice(cst->ctx->device));
        struct Events {
            hipEvent_t a = nullptr, b = nullptr;
            ~Events() {
                if (a) (void)hipEventDestroy(a);
                if (b) (void)hipEventDestroy(b);
            }
        } ev;
        HIP_TRY(hipEventCreate(&ev.a));
        HIP_TRY(hipEventCreate(&ev.b));
        HIP_TRY(hipEventRecord(ev.a, cst->stream));
        const bool done = cstm_partition_run(cst, budget_bytes, max_list_len, max_total_bytes);
        HIP_TRY(hipEventRecord(ev.b, cst->stream));
        HIP_TRY(hipEventSynchronize(ev.b));
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
        cst->t_part = ms;
        if (n_parts_out) *n_parts_out = done ? cst->n_parts : 0;
        CSTM_REQUIRE(done, CSTM_ENOMEM, "partition images would exceed max_total_bytes; the CST stays unpartitioned");
    });
}
