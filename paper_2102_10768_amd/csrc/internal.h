// internal.h -- shared definitions of the CST library (host and device side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "cstm.h"

#define CSTM_WAVE 64

// ---------------------------------------------------------------- errors

void cstm_set_error(const std::string& msg);

struct CstmError {
    cstm_status st;
    std::string msg;
};

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            throw CstmError{CSTM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define CSTM_REQUIRE(cond, status, msg)                       \
    do {                                                      \
        if (!(cond)) throw CstmError{(status), (msg)};        \
    } while (0)

// Run a body that may throw CstmError; convert to a status at the ABI.
template <class F>
cstm_status cstm_guard(F&& f) {
    try {
        f();
        return CSTM_OK;
    } catch (const CstmError& e) {
        cstm_set_error(e.msg);
        return e.st;
    } catch (const std::bad_alloc&) {
        cstm_set_error("host allocation failed");
        return CSTM_ENOMEM;
    } catch (...) {
        cstm_set_error("unexpected host exception");
        return CSTM_EDEVICE;
    }
}

// ---------------------------------------------------------------- context

struct cstm_ctx {
    int device = 0;
    cstm_alloc_fn alloc = nullptr;
    cstm_free_fn free_fn = nullptr;
    void* user = nullptr;
    cstm_tune tune{};
    int num_cus = 0;
    int64_t lds_per_wg = 0;
    cstm_enum_stats last_enum{};  // guarded by ws_mu
    // HBM-mode enumeration workspaces (task ring and queue state), reused
    // across launches; one per launch in flight, so launches on different
    // streams can run at the same time
    std::vector<std::pair<void*, size_t>> ws_free;
    std::vector<void*> ws_all;
    std::unordered_map<void*, size_t> ws_sizes;
    void* ws_acquire(size_t bytes);
    void ws_release(void* p);
    // cache of freed device blocks by power-of-two size class (hipMalloc path only)
    std::vector<std::vector<void*>> pool;
    std::unordered_map<void*, int> block_class;
    void release_pool();
    // A context may be used from several host threads (e.g. one building CSTs
    // while others enumerate on their own streams): the block cache and the
    // workspace list each have a lock.
    std::mutex pool_mu;
    std::mutex ws_mu;  // workspace list and last_enum

    void* dmalloc(size_t bytes);
    void dfree(void* p);
};

// A bag of device allocations released together.
struct DevArena {
    cstm_ctx* ctx = nullptr;
    std::vector<void*> blocks;
    std::vector<size_t> sizes;  // bytes requested for each block
    void* get(size_t bytes) {
        void* p = ctx->dmalloc(bytes ? bytes : 16);
        blocks.push_back(p);
        sizes.push_back(bytes ? bytes : 16);
        return p;
    }
    // bytes requested by the blocks held now
    uint64_t used() const {
        uint64_t t = 0;
        for (size_t b : sizes) t += b;
        return t;
    }
    template <class T>
    T* get_n(size_t n) {
        return static_cast<T*>(get(n * sizeof(T)));
    }
    void release(void* p);
    void clear();
    ~DevArena() { clear(); }
};

// ---------------------------------------------------------------- graph

struct cstm_graph {
    cstm_ctx* ctx = nullptr;
    int64_t n = 0, nnz = 0;
    const int64_t* row_ptr = nullptr;
    const int32_t* col = nullptr;
    const int32_t* label = nullptr;
    int32_t num_labels = 0;
    int64_t max_degree = 0;
    DevArena mem;
    // label index: vertices grouped by label, each group by (degree desc, id asc)
    int32_t* perm = nullptr;
    // per vertex: (label << key_shift) | rank inside its label group, packed
    // into 32 bits when the label and rank bits fit (key32), else 64 bits with
    // key_shift = 32 (key64); exactly one of the two is set
    uint32_t* key32 = nullptr;
    uint64_t* key64 = nullptr;
    int key_shift = 32;
    // label-grouped rows: lkey[row_ptr[v] + i] is the key of the i-th neighbour
    // of v in (label, id) order; the same width as the keys (one is set)
    uint32_t* lkey32 = nullptr;
    uint64_t* lkey64 = nullptr;
    std::vector<int64_t> label_ptr;  // host, num_labels + 1
    // host: count of vertices of label l with degree >= d, d = 0..CSTM_MAX_K
    std::vector<int64_t> deg_at_least;
    // host: prefix sums of degrees in label-index order (n + 1 entries)
    std::vector<int64_t> deg_prefix;

    // host: edges of G between each pair of labels (row entries (v, w) with
    // l(v) = a, l(w) = b at a * num_labels + b); empty above 128 labels
    std::vector<uint64_t> pair_count;

    // An upper bound on the row entries from label-a vertices to label-b
    // neighbours (~0 when unknown).
    uint64_t pair_bound(int32_t a, int32_t b) const {
        if (pair_count.empty() || a < 0 || b < 0 || a >= num_labels || b >= num_labels) return ~0ull;
        return pair_count[(size_t)a * num_labels + b];
    }

    int64_t count_ge(int32_t l, int32_t d) const {
        if (l < 0 || l >= num_labels) return 0;
        if (d > CSTM_MAX_K) d = CSTM_MAX_K;
        return deg_at_least[(size_t)l * (CSTM_MAX_K + 1) + (size_t)d];
    }
};

// ---------------------------------------------------------------- CST (device descriptors)

// One position i of the matching order O, as the partitioner sees the CST.
struct PosDesc {
    int32_t u;           // query vertex O[i]
    int32_t par;         // position of the tree parent (-1 at the root)
    int64_t n;           // #C(u)
    const int32_t* gid;  // C(u): data-vertex ids in candidate order
    const int64_t* toff; // tree list offsets over the parent's candidates (n_par + 1)
    const int32_t* tadj; // tree list entries: indices into C(u)
    uint32_t same_mask;  // earlier positions whose query label equals l(u)
    uint32_t nt_mask;    // earlier positions joined to i by a non-tree edge
    int32_t nt_first;    // first NtDesc whose later end is i
    int32_t label;
    int32_t need_gid;    // 1: checks at i read data-vertex ids (repeated label or non-tree edge)
    int32_t pad;
};

// A non-tree query edge between positions a < b, lists over C(O[a]) into C(O[b]).
struct NtDesc {
    int32_t a, b;
    const int64_t* off;
    const int32_t* adj;
    const int32_t* adj_gid;  // entries as data-vertex ids, ascending within each list
};

#define CSTM_MAX_NT (CSTM_MAX_K * (CSTM_MAX_K - 1) / 2)

struct CstDev {
    int32_t k;
    int32_t n_nt;
    int32_t qid;
    int32_t pad;
    PosDesc pos[CSTM_MAX_K];
    NtDesc nt[CSTM_MAX_NT];
};

// ---------------------------------------------------------------- on-chip image (partition blob)
//
// A partition is serialised as one self-contained image that the enumerator
// copies into LDS unchanged.  Layout (all offsets in bytes from the image
// start, every array 4-byte aligned, the image padded to 16 bytes):
//   BlobHdr, then k BlobPos, then n_nt BlobNt (padded to 16 bytes);
//   gid arrays of every position (int32 data-vertex ids);
//   per position i >= 1: tree offsets (uint32, n_par + 1) and tree entries
//     (uint16 candidate indices into position i, padded to 4 bytes);
//   per non-tree edge: n_a bit rows of row_words uint32 words over position b.
struct BlobHdr {
    uint32_t k;
    uint32_t n_nt;
    uint32_t bytes;
    uint32_t qid;
    uint32_t reserved[12];
};
struct BlobPos {
    uint32_t n;
    uint32_t gid_off;
    int32_t par;
    uint32_t toff_off;
    uint32_t tadj_off;
    uint32_t same_mask;
    uint32_t nt_mask;
    uint32_t u_nt_first;  // low 16 bits: nt_first, high 16 bits: query vertex u
};
struct BlobNt {
    uint32_t a, b;
    uint32_t bits_off;
    uint32_t row_words;
};
static_assert(sizeof(BlobHdr) == 64, "header size");
static_assert(sizeof(BlobPos) == 32, "position record size");
static_assert(sizeof(BlobNt) == 16, "non-tree record size");

__host__ __device__ inline uint64_t cstm_align16(uint64_t x) { return (x + 15) & ~uint64_t(15); }
__host__ __device__ inline uint64_t blob_header_bytes(int k, int n_nt) {
    return cstm_align16(sizeof(BlobHdr) + (uint64_t)k * sizeof(BlobPos) + (uint64_t)n_nt * sizeof(BlobNt));
}

// A partition request: the CST restricted by index ranges of some positions.
struct Spec {
    int32_t qid;
    int32_t uidx;  // first position that may be split
    int32_t lo[CSTM_MAX_K];
    int32_t hi[CSTM_MAX_K];
};

// ---------------------------------------------------------------- CST (host object)

struct EdgeLists {
    int32_t from = -1, to = -1;  // positions
    int64_t* off = nullptr;      // device, n_from + 1
    int32_t* adj = nullptr;      // device: indices into the later candidate set
    int32_t* adj_gid = nullptr;  // device, non-tree lists only: the same entries as data-vertex ids (ascending)
    int64_t entries = 0;
    int32_t max_len = 0;
};

struct cstm_cst {
    cstm_ctx* ctx = nullptr;
    const cstm_graph* g = nullptr;
    hipStream_t stream = nullptr;
    DevArena mem;
    int k = 0;
    int32_t qlabel[CSTM_MAX_K] = {};
    int32_t qdeg[CSTM_MAX_K] = {};
    uint32_t qadj[CSTM_MAX_K] = {};  // bitmask of query neighbours
    int root = 0;
    int parent[CSTM_MAX_K] = {};
    int bfs[CSTM_MAX_K] = {};
    int order[CSTM_MAX_K] = {};
    int pos_of[CSTM_MAX_K] = {};
    std::vector<std::pair<int, int>> nontree;  // (a, b) query ids, a < b
    int64_t cnt0[CSTM_MAX_K] = {};
    int64_t lb_lo[CSTM_MAX_K] = {};
    int64_t ncand[CSTM_MAX_K] = {};
    int32_t* cand[CSTM_MAX_K] = {};  // device gids, per query vertex
    EdgeLists tree[CSTM_MAX_K];      // indexed by child query vertex
    std::vector<EdgeLists> nt;       // one per non-tree edge, earlier -> later position
    CstDev* dev = nullptr;           // device copy of the descriptor
    CstDev host_desc{};
    uint64_t bytes = 0;
    int32_t d_cst = 0;
    // partitions
    bool partitioned = false;
    uint64_t part_budget = 0;
    int32_t part_max_list = 0;
    void* blob_arena = nullptr;
    uint64_t blob_arena_cap = 0;
    uint64_t blob_bytes = 0;
    uint64_t* blob_off = nullptr;  // device, n_parts
    int64_t n_parts = 0;
    uint64_t max_blob = 0;
    bool empty = false;  // some candidate set is empty: no embedding
    uint64_t mem_bytes = 0;  // device bytes the CST's arena holds after the build (bound-sized arrays included)
    double t_build = 0, t_part = 0, t_enum = 0;
    bool has_workload = false;     // W_CST computed (on first use)
    uint64_t workload = 0;         // W_CST of the workload DP (Section V-C), saturating at 2^64 - 1
    std::vector<uint64_t> root_w;  // c_root(v) for every root candidate, with workload
};

// ---------------------------------------------------------------- helpers shared across files

// Device-wide exclusive prefix sums (prims.hip): out[0..len) and out[len] =
// the total, where len = *n_dev when n_dev is given (n is then an upper bound
// that sizes the launch) and len = n otherwise; *total_out (may be NULL) also
// receives the total.  part: scratch of kScanPartSlots int64 (one scan at a
// time per buffer).  max_out (cstm_dscan_i64, may be NULL): raised by atomic
// maximum to the largest input (inputs below 2^31; the caller zeroes it).
// Nothing waits for the device.
constexpr int kScanPartSlots = 1025;
void cstm_dscan_i64(const int64_t* in, int64_t* out, const int64_t* n_dev, int64_t n, int64_t* total_out,
                    int64_t* part, hipStream_t s, int* max_out = nullptr);
void cstm_dscan_i32(const int32_t* in, int32_t* out, const int64_t* n_dev, int64_t n, int64_t* total_out,
                    int64_t* part, hipStream_t s);
void cstm_dscan_u32(const uint32_t* in, uint32_t* out, int64_t n, int64_t* part, hipStream_t s);
// Fill bytes / 4 words with value (a kernel, not a memset node).
void cstm_fill_words(void* p, size_t bytes, uint32_t value, hipStream_t s);
// Stable ascending sort of (keys, vals) by the low `bits` bits of the keys, in
// place (8-bit LSD passes); waits for the stream before returning.
void cstm_radix_sort_pairs(cstm_ctx* ctx, uint64_t* keys, int32_t* vals, int64_t n, int bits, hipStream_t s);

inline unsigned cstm_blocks(int64_t items, int per_block, unsigned cap = 1u << 20) {
    int64_t b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > (int64_t)cap) b = cap;
    return (unsigned)b;
}

// W_CST of the workload DP (Section V-C), cached in the CST.
uint64_t cstm_cst_workload_run(cstm_cst* c);

// Returns false (and leaves the CST unpartitioned) if the images would exceed max_total_bytes (0 = no limit).
bool cstm_partition_run(cstm_cst* cst, uint64_t budget, int32_t max_list, uint64_t max_total_bytes = 0);
// Per-call options of an enumeration launch.
struct EnumOpts {
    const uint64_t* limits = nullptr;  // per CST of the call: stop once it has this many embeddings (0: all)
    int64_t deadline_ms = 0;           // stop the launch after this long (0: no limit)
    // one-CST calls only: enumerate just these runs of root candidates, as
    // [lo, hi) index pairs (nullptr: all of them); forces the HBM-resident kernel
    const int64_t* root_ranges = nullptr;
    int64_t n_ranges = 0;
    // HBM-resident kernel only: run in this caller-provided workspace (a
    // smaller task ring, no allocation and no timing events) instead of one
    // lent by the context
    void* fixed_ws = nullptr;
    size_t fixed_ws_bytes = 0;
    // every CST of the call in device memory (no partitioning at launch), whatever tune.enum_mode says
    bool force_hbm = false;
    // HBM-resident kernel: workgroups per CU of the launch (0: tune.hbm_wgs_per_cu)
    int wgs_per_cu = 0;
};
// Device bytes the context lends one HBM-mode launch of nq CSTs.
size_t cstm_hbm_workspace_bytes(int nq);
// Look up this device's copy of the no-allocation scratch array (once per
// device, with the device current); cstm_ctx_create calls it.
void cstm_noalloc_init(int device);
void cstm_enumerate_lds_run(cstm_ctx* ctx, int nq, cstm_cst* const* csts, const int* slot, int list, int32_t* rows,
                            uint64_t cap, unsigned long long* counts_dev, unsigned long long* row_cursor,
                            const EnumOpts& o, cstm_enum_stats* st, hipStream_t s);
void cstm_enumerate_global_run(cstm_ctx* ctx, int nq, cstm_cst* const* csts, const int* slot, int list, int32_t* rows,
                               uint64_t cap, unsigned long long* counts_dev, unsigned long long* row_cursor,
                               const EnumOpts& o, cstm_enum_stats* st, hipStream_t s);
// *st_out (may be NULL) receives the launch statistics (also kept as the
// context's last ones).
void cstm_enumerate_run(cstm_ctx* ctx, int nq, cstm_cst* const* csts, int list, int32_t* rows, uint64_t cap,
                        uint64_t* counts_host, uint64_t* rows_written, const EnumOpts& o, hipStream_t s,
                        cstm_enum_stats* st_out = nullptr);
