/*
 * cstm.h -- C ABI of the CST subgraph-matching library (HIP, gfx950).
 *
 * The library enumerates or counts every embedding of a small connected query
 * graph q in a large vertex-labelled data graph G: every map f: V(q) -> V(G)
 * that is injective, keeps labels and maps each query edge onto an edge of G
 * (subgraph isomorphism, Section II-A, Definition 1; non-induced; automorphic
 * images count separately).  It follows the paper's system steps (Section IV):
 * build a candidate search tree (CST) for q (Section V-A, Algorithm 1),
 * partition it to an on-chip memory budget (Section V-B, Algorithm 2), and
 * extend partial embeddings inside each partition (Section VI-A,
 * Algorithms 4-8).
 *
 * Conventions for every call:
 *   - Every call returns a cstm_status; nothing throws across the ABI.  On an
 *     error, cstm_last_error() gives a message (thread-local, valid until the
 *     next call on the same thread).
 *   - "device" pointers are HIP device allocations on the context's device;
 *     "host" pointers are ordinary host memory.  The caller owns every array
 *     it passes in; the library never frees caller memory.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *     that return results to the host synchronise that stream before returning.
 *   - Threads: a context and a loaded graph may be shared by host threads.
 *     CST builds and enumeration launches from different threads may run at
 *     the same time on different streams (each launch borrows its own
 *     workspace).  A CST handle must not be used by two calls at once, and
 *     cstm_ctx_set_tune must not race with calls in flight on the context.
 *   - Vertex ids and labels are int32, CSR offsets int64, counts uint64.
 */
#ifndef CSTM_H
#define CSTM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CSTM_OK = 0,
    CSTM_EINVAL = 1,     /* bad argument, malformed graph or query          */
    CSTM_ENOMEM = 2,     /* an allocation failed                            */
    CSTM_EDEVICE = 3,    /* a HIP runtime call or kernel failed             */
    CSTM_ETIMEOUT = 4,   /* a deadline expired (no count is reported)       */
    CSTM_EOVERFLOW = 5,  /* listing buffer too small (the count is exact)   */
    CSTM_ECANCELLED = 6  /* reserved                                        */
} cstm_status;

#define CSTM_MAX_K 32

typedef struct cstm_ctx cstm_ctx;     /* device, allocator, tuning                  */
typedef struct cstm_graph cstm_graph; /* resident data graph G and its label index  */
typedef struct cstm_cst cstm_cst;     /* one query's CST and its partitions         */

/* Device allocator hooks (e.g. a framework's caching allocator).  NULL hooks
 * mean hipMalloc / hipFree.  alloc returns NULL on failure. */
typedef void* (*cstm_alloc_fn)(size_t bytes, void* user);
typedef void (*cstm_free_fn)(void* ptr, void* user);

/* Tuning knobs.  Zero fields take the defaults.
 *   part_budget_bytes  delta_S of Section V-B: the largest on-chip image a
 *                      partition may have (LDS bytes, at most the LDS a
 *                      workgroup can address minus the enumerator's state).
 *   max_list_len       delta_D of Section V-B: longest candidate list allowed
 *                      in a partition (0 = no limit).
 *   waves_per_wg       wavefronts sharing one partition image in LDS (1..16).
 *   wgs_per_cu         resident enumeration workgroups per compute unit.
 *   collect_stats      1: enumeration launches also count the work they do
 *                      (cstm_enum_stats); 0: they do not.
 *   enum_mode          where enumeration reads the CST from:
 *                        CSTM_MODE_LDS  partitions staged into LDS (the
 *                                       on-chip matcher of Section VI),
 *                        CSTM_MODE_HBM  the whole CST from device memory
 *                                       (L2-resident), with wavefronts sharing
 *                                       work through a device task queue,
 *                        CSTM_MODE_AUTO LDS for CSTs the caller partitioned
 *                                       (cstm_cst_partition), else HBM.
 *   max_replication    when a launch in LDS mode meets a CST the caller did
 *                      not partition, it partitions it at part_budget_bytes
 *                      unless the images would exceed max_replication times
 *                      the CST's bytes; such a CST is enumerated in HBM mode
 *                      instead (negative: no limit; default 16).
 *   deadline_ms        stop an enumeration launch after this many
 *                      milliseconds and return CSTM_ETIMEOUT, no count
 *                      reported (0 = no limit; both modes).
 *   hbm_wgs_per_cu     HBM mode: 256-thread workgroups per compute unit
 *                      (default 2).
 *   hbm_donate_period  HBM mode: longest interval, in chunks of 64
 *                      candidates, between a wavefront's checks for waiting
 *                      wavefronts (negative: never donate; default 64).
 *   hbm_donate_min     HBM mode: shortest such interval (default 16).  The
 *                      interval halves back to this after a donation and
 *                      doubles, up to hbm_donate_period, after a check that
 *                      finds no wavefront waiting.
 *   hbm_flat_max       HBM mode: the next level is expanded as one flat list
 *                      over all surviving parents of a chunk when their
 *                      candidate lists sum to at most this many entries, if it
 *                      is the last level, or the second-to-last while the last
 *                      is counted by list lengths (last_level_sum) (default
 *                      2048; negative: never).
 *   hbm_donate_last_min HBM mode: smallest remainder of the last level a
 *                      wavefront hands to a waiting one (default 4096).
 *   last_level_sum     HBM mode, counting only: when the last query vertex of
 *                      the matching order has no same-label predecessor and
 *                      no non-tree edge, every candidate in its tree list is an
 *                      embedding, so each surviving partial embedding one
 *                      level up adds the length of that list to the count
 *                      instead of visiting it (reported in
 *                      cstm_enum_stats.summed).  1 (default): on; negative:
 *                      off.  Listing always visits every candidate.
 *   batch_order        HBM mode, several CSTs in one launch: 0 (default)
 *                      or negative seeds them in the order given; positive
 *                      seeds the heaviest first by W_CST (cstm_cst_workload,
 *                      one workload DP per CST not yet weighed).
 *   hbm_idle_ms        HBM mode: a safety net.  Busy wavefronts refresh a
 *                      progress beat about once a millisecond; a launch in
 *                      which idle wavefronts see neither a task nor a beat for
 *                      this many milliseconds stops with CSTM_EDEVICE
 *                      (default 30000).  A deadline that passes first is
 *                      reported as CSTM_ETIMEOUT.
 *   order_rule         matching order of cstm_cst_build: 0 (default) the
 *                      path-based order of Section V-B (root-to-leaf paths
 *                      by their number of CST path embeddings); 1 constraint
 *                      first: after the root, repeatedly the vertex whose tree
 *                      parent is placed with the most placed query neighbours
 *                      (then the larger query degree, then the smaller id),
 *                      so that non-tree edges are checked early.  Any such
 *                      order gives the same embeddings (Section VII-C).
 *   serve_wgs_per_cu   cstm_server lanes: 256-thread workgroups per compute
 *                      unit of a launch made while CST builds are still
 *                      queued or running (default 2, which leaves room on
 *                      each CU for the build kernels); a launch with no build
 *                      in flight uses hbm_wgs_per_cu.                       */
#define CSTM_MODE_AUTO 0
#define CSTM_MODE_LDS 1
#define CSTM_MODE_HBM 2
typedef struct {
    uint64_t part_budget_bytes;
    int32_t max_list_len;
    int32_t waves_per_wg;
    int32_t wgs_per_cu;
    int32_t collect_stats;
    int32_t enum_mode;
    int32_t max_replication;
    int32_t deadline_ms;
    int32_t hbm_wgs_per_cu;
    int32_t hbm_donate_period;
    int32_t hbm_flat_max;
    int32_t hbm_donate_last_min;
    int32_t last_level_sum;
    int32_t hbm_donate_min;
    int32_t batch_order;
    int32_t hbm_idle_ms;
    int32_t order_rule;
    int32_t serve_wgs_per_cu;
} cstm_tune;

/* What the last enumeration launch on a context did (Section VI-B's counts).
 *   kernel_ms      duration of the enumeration kernel(s) alone (HIP events
 *                  on the stream, around each launch);
 *   images         LDS mode: partition images processed; HBM mode: tasks run;
 *   image_bytes    LDS mode: bytes staged from HBM into LDS; HBM mode: tasks
 *                  donated by busy wavefronts to idle ones;
 *   extensions     N: new partial results generated (one per lane per valid
 *                  candidate, all levels after the root);
 *   edge_checks    M: non-tree edge validations executed;
 *   pushed         F: surviving partial results that were extended further;
 *   summed         last-level extensions counted by list length, not
 *                  visited (tune.last_level_sum; included in extensions);
 *   chunks         HBM mode: 64-lane rounds that read candidates, so
 *                  (extensions - summed) / (64 * chunks) is the share of
 *                  lanes that held a candidate.
 * The work counters are zero unless tune.collect_stats was set. */
typedef struct {
    double kernel_ms;
    int32_t mode;        /* CSTM_MODE_LDS or CSTM_MODE_HBM (last launch)   */
    int32_t launches;
    uint64_t images;
    uint64_t image_bytes;
    uint64_t extensions;
    uint64_t edge_checks;
    uint64_t pushed;
    double busy_frac;    /* HBM mode: share of wavefront time spent expanding  */
    uint64_t summed;
    uint64_t chunks;
} cstm_enum_stats;

/* Facts about a built (and possibly partitioned) CST, for reports and tests. */
typedef struct {
    int32_t k;                       /* query vertices                              */
    int32_t root;                    /* root of the BFS tree t_q                    */
    int32_t parent[CSTM_MAX_K];      /* t_q parent per query vertex (-1 = root)     */
    int32_t order[CSTM_MAX_K];       /* matching order O (query ids)                */
    int64_t cand[CSTM_MAX_K];        /* #C(u) per query vertex                      */
    int64_t tree_entries;            /* total tree-list entries                     */
    int64_t nontree_entries;         /* total non-tree list entries (one direction) */
    uint64_t bytes;                  /* device bytes of the CST in HBM              */
    int32_t d_cst;                   /* longest list (D_CST)                        */
    int32_t n_nontree;               /* non-tree query edges                        */
    int64_t n_parts;                 /* partitions (0 before partitioning)          */
    uint64_t part_bytes;             /* total bytes of all partition images         */
    uint64_t max_part_bytes;         /* largest partition image                     */
} cstm_cst_info;

/* Create a context on HIP device `device`.  tune may be NULL (defaults). */
cstm_status cstm_ctx_create(int device, cstm_alloc_fn alloc, cstm_free_fn free_fn, void* user,
                            const cstm_tune* tune, cstm_ctx** out);
void cstm_ctx_destroy(cstm_ctx* ctx);
cstm_status cstm_ctx_get_tune(const cstm_ctx* ctx, cstm_tune* out);
cstm_status cstm_ctx_set_tune(cstm_ctx* ctx, const cstm_tune* tune);
/* LDS bytes one workgroup may address on this device. */
cstm_status cstm_ctx_lds_bytes(const cstm_ctx* ctx, int64_t* out);

/* Load G (Section II-A: undirected, vertex-labelled, simple) as CSR:
 *   row_ptr[n+1] int64, col[nnz] int32 (nnz = 2|E|, each row sorted ascending,
 *   no duplicates, no self-loops, symmetric), label[n] int32 >= 0.
 * on_device = 0: host arrays, copied to the device.  on_device = 1: device
 * arrays, borrowed (kept alive by the caller until cstm_graph_free).
 * A device kernel checks the CSR; violations give CSTM_EINVAL.  The call also
 * builds the label index: vertices grouped by label, each group ordered by
 * degree descending then id ascending, and a label-grouped copy of the rows
 * (each neighbour's packed label/rank key, every row ordered by label then
 * id; 4 bytes per entry, 8 when label and rank bits exceed 32), which CST
 * construction reads.  Building the copy sorts about 2^28 row entries at a
 * time (24 bytes of temporary device memory per entry); a chunk grows past
 * that only by its last row, and one of 2^31 entries or more (a row of more
 * than about 1.88 * 10^9 entries) gives CSTM_EINVAL.  n must be < 2^31 and
 * labels below 2^26; the label tables take about 280 bytes per label value
 * up to the largest one, on the host and (while loading) on the device, so
 * sparse label values are best renumbered densely first. */
cstm_status cstm_graph_load(cstm_ctx* ctx, int64_t n, int64_t nnz, const int64_t* row_ptr,
                            const int32_t* col, const int32_t* label, int on_device, void* stream,
                            cstm_graph** out);
void cstm_graph_free(cstm_graph* g);
cstm_status cstm_graph_info(const cstm_graph* g, int64_t* n, int64_t* nnz, int32_t* num_labels,
                            int64_t* max_degree);

/* Edges of G between each pair of labels, counted at load from the
 * label-grouped rows: out[a * num_labels + b] (host array of cap entries) is
 * the number of row entries (v, w) with l(v) = a and l(w) = b, so the table is
 * symmetric and sums to nnz.  CST construction sizes its per-edge buffers and
 * cstm_cst_estimate its bound with it.  *n_out (required) receives
 * num_labels^2, or 0 when the table was not made (more than 128 labels, or no
 * edges); at most cap entries are written. */
cstm_status cstm_graph_label_edges(const cstm_graph* g, uint64_t* out, int64_t cap, int64_t* n_out);

/* Build the CST of q (Section V-A, Algorithm 1) on the device.
 *   k in 1..32, qlabel[k] >= 0, qedges[2*m_q] (host arrays): undirected query
 *   edges as id pairs; q must be connected, with no self-loop or duplicate edge.
 * Candidates pass the label/degree filter; the BFS tree t_q is rooted at the
 * vertex minimising #candidates / query degree; the matching order follows
 * tune.order_rule (default: the path-based order of Section V-B). */
cstm_status cstm_cst_build(cstm_ctx* ctx, const cstm_graph* g, int32_t k, const int32_t* qlabel,
                           int32_t m_q, const int32_t* qedges, void* stream, cstm_cst** out);

/* As cstm_cst_build, with the caller's matching order (host, k entries: a
 * permutation of the query vertices that starts at the CST root and places
 * every vertex after its BFS-tree parent) instead of the path-based order of
 * Section V-B; NULL = the path-based order.  The order changes only the work
 * (Section VII-C studies its effect), never the embeddings.  CSTM_EINVAL for
 * an order that breaks these rules (the root is the vertex minimising
 * #C0(u)/d_q(u), see cstm_cst_info_get). */
cstm_status cstm_cst_build_ordered(cstm_ctx* ctx, const cstm_graph* g, int32_t k, const int32_t* qlabel,
                                   int32_t m_q, const int32_t* qedges, const int32_t* order, void* stream,
                                   cstm_cst** out);

/* Upper bound on the device bytes cstm_cst_build requests for the query
 * (k, qlabel, m_q, qedges as for cstm_cst_build): the CST of Section V-A plus
 * its build-time tables, from the label index alone.  #C(u) is at most the
 * number of vertices passing the label and degree filter, and a candidate edge
 * list holds each data edge at most once, so the summed degrees of either
 * endpoint's filtered candidates, and the edges between the two labels
 * (cstm_graph_label_edges), bound its entries.  Host-only: no device work,
 * no allocation.  The context's block cache rounds each request up to a power
 * of two (up to 256 MB), so device use can reach twice this figure.  Meant for
 * admission control before building.  CSTM_EINVAL on a malformed query. */
cstm_status cstm_cst_estimate(const cstm_graph* g, int32_t k, const int32_t* qlabel, int32_t m_q,
                              const int32_t* qedges, uint64_t* bytes_out);

/* Partition the CST (Section V-B, Algorithm 2) until every partition's
 * on-chip image is at most budget_bytes and its longest list at most
 * max_list_len (0 = no limit); budget_bytes = 0 takes the context's tuning.
 * Partitions are independent and together hold every embedding exactly once.
 * max_total_bytes (0 = no limit): give up with CSTM_ENOMEM, leaving the CST
 * unpartitioned, once the images together would exceed it (on hub-heavy
 * graphs the images can replicate the CST many times over).
 * *n_parts_out (may be NULL) receives the number of partitions. */
cstm_status cstm_cst_partition(cstm_cst* cst, uint64_t budget_bytes, int32_t max_list_len,
                               uint64_t max_total_bytes, int64_t* n_parts_out);

/* Workload estimate W_CST of Section V-C: with c_u(v) = product over u's tree
 * children u' of the sum of c_u'(v') over v's candidate list in C(u') (1 at
 * the leaves), W_CST = sum of c_root over the root's candidates.  It counts
 * the tree-shaped paths the CST holds: an upper bound on the embeddings, equal
 * to their number for tree queries with pairwise-distinct labels.  Computed on
 * the device in unsigned 64-bit integers that saturate: *w_out is exactly
 * min(W_CST, 2^64 - 1), and so is every c_root(v) the host share uses.
 * Cached in the CST; batched launches seed the heaviest queries first by it
 * when tune.batch_order > 0, and cstm_enumerate_shared splits work by it. */
cstm_status cstm_cst_workload(cstm_cst* cst, uint64_t* w_out);

cstm_status cstm_cst_info_get(const cstm_cst* cst, cstm_cst_info* out);

/* Copy C(u) (data-vertex ids, candidate order) of query vertex u to host
 * memory: cap entries at most; *n_out receives #C(u). */
cstm_status cstm_cst_candidates(const cstm_cst* cst, int32_t u, int32_t* out, int64_t cap, int64_t* n_out);

/* Enumerate the embeddings of one CST (Section VI-A; where the CST is read
 * from follows tune.enum_mode: partitions the caller made with
 * cstm_cst_partition are staged into LDS, otherwise the CST is read from
 * device memory).  list = 0 counts only; list = 1 also writes rows to the
 * DEVICE buffer rows[cap][k] (row[u] = data vertex of query vertex u, rows in
 * no particular order).
 *   limit        0: find every embedding.  > 0: *count_out is exactly
 *                min(total, limit), whatever order the search ran in; the
 *                search stops early once at least limit embeddings were
 *                found (over partition images: the images not yet started
 *                are skipped, every started one is counted in full).
 *   deadline_s   > 0: stop the launch after this many seconds and return
 *                CSTM_ETIMEOUT (nothing is reported); <= 0: the context's
 *                tune.deadline_ms applies.
 * *count_out receives the exact number of embeddings (or min(total, limit));
 * *rows_written min(that, cap).  Returns CSTM_EOVERFLOW when list = 1 and the
 * number exceeds cap (the count is still exact). */
cstm_status cstm_enumerate(cstm_cst* cst, int list, uint64_t limit, int32_t* rows, uint64_t cap,
                           uint64_t* count_out, uint64_t* rows_written, double deadline_s, void* stream);

/* Count the embeddings of many CSTs in one persistent launch that draws work
 * from a device queue (the batched form).  limits (host, may be NULL): per
 * CST, 0 = count all, > 0 = counts_out[i] is exactly min(total_i, limits[i])
 * (that CST's search stops once it has that many, as for cstm_enumerate).
 * counts_out[nq] is a host array. */
cstm_status cstm_batch_enumerate(cstm_ctx* ctx, int32_t nq, cstm_cst* const* csts, const uint64_t* limits,
                                 uint64_t* counts_out, void* stream);

/* Count the embeddings of one CST without allocating device memory: for
 * callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  It runs the HBM-resident kernel of
 * cstm_enumerate (whatever the context's enum_mode) with its task ring, queue
 * state, descriptor copy and count in a fixed array of
 * CSTM_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs
 * on until the process ends; the ring has 2^16 task slots (cstm_enumerate's
 * has 2^20).  It calls no allocator, no hipMalloc and no hipFree; the CST
 * must already be built.  limit and deadline_s as for cstm_enumerate;
 * *count_out receives the exact count, or min(total, limit).  Errors:
 * CSTM_EINVAL for NULL arguments or a launch needing more scratch than the
 * array holds; CSTM_ETIMEOUT / CSTM_EDEVICE as for cstm_enumerate.  Calls on
 * one device share the array (it keeps the last call's contents; each call
 * clears what must start at zero): the library serialises them with a lock
 * held until the count is back, so they never overlap within a process,
 * while a second process on the same device has its own copy. */
#define CSTM_NOALLOC_SCRATCH_BYTES (12u << 20)
cstm_status cstm_enumerate_noalloc(cstm_cst* cst, uint64_t limit, uint64_t* count_out, double deadline_s,
                                   void* stream);

/* ---------------------------------------------------------------- host share
 * Algorithm 3 (Section V-C): the root candidates of the CST are cut into
 * n_runs runs of consecutive candidates (0 = min(1024, #roots)), each weighed
 * by the sum of c_root(v) over it (the workload DP, see cstm_cst_workload).
 * In root order, a run goes to the host cores when W_C + W_run <
 * delta * (W_C + W_F + W_run), else to the GPU (W_C, W_F: the workload handed
 * to each so far), so the host's share of W_CST stays below delta.  The GPU
 * counts its runs with the HBM-resident kernel (whatever the context's
 * enum_mode) while host_threads threads (0 = the host's cores, at most 16)
 * count the others by backtracking over a host copy of the CST lists; the two
 * overlap.  *count_out = the total number of embeddings (host + GPU); st (may
 * be NULL) receives the split and its times.  delta = 0 gives everything to
 * the GPU.  Counts only (no listing, no limit); the context's deadline_ms
 * applies to the GPU part.  CSTM_EINVAL for delta outside [0, 1], negative
 * n_runs or host_threads outside [0, 256]. */
typedef struct cstm_share_stats {
    double delta;
    uint64_t w_host, w_device;       /* W_C and W_F after the last run (saturating at 2^64 - 1) */
    int64_t groups_host, groups_device;  /* runs each side received */
    uint64_t count_host, count_device;
    double copy_ms;                  /* until the host copy of the lists was complete */
    double host_ms;                  /* until the last host thread ended (0: no host runs) */
    double device_ms;                /* until the GPU's count was back */
    double wall_ms;                  /* both sides, from the split to the result */
    int32_t host_threads;
    int32_t reserved;
} cstm_share_stats;
cstm_status cstm_enumerate_shared(cstm_cst* cst, double delta, int64_t n_runs, int32_t host_threads,
                                  uint64_t* count_out, cstm_share_stats* st, void* stream);

/* ---------------------------------------------------------------- serving
 *
 * A request loop over one resident graph (the serving form of the method:
 * queries arrive one at a time and share the GPU).  The server admits
 * requests in arrival order while the device-memory bound of their CST
 * builds (cstm_cst_estimate, doubled for the block cache's rounding) fits
 * mem_budget (once a CST is built its charge drops to twice the device
 * bytes the CST holds, as the build's temporaries are freed); builds admitted
 * CSTs on `builders` threads, each with its own stream; and gives every
 * built CST to the next free enumeration lane, which
 * counts all CSTs built so far (up to max_batch) in one persistent launch on
 * its own stream, reading the CSTs from device memory whatever the context's
 * enum_mode (so no partition images exceed what admission charged).  Each
 * lane's launch workspace (its task ring) is charged to mem_budget once, when
 * the server is created.  Several lanes run launches at the same time.  A
 * request's count does not depend on which requests share its launch.  The
 * server is thread-safe; it uses the context's tuning (deadline_ms applies
 * per launch).
 * Zero or negative lanes / builders / max_batch take the defaults 2 / 2 / 256
 * (lanes + builders streams: HIP maps a process's streams onto a few
 * hardware queues, 4 by default, and streams sharing one queue run in
 * order, so a build queued behind a long enumeration launch would wait).
 * batch_wait_us: when a lane finds built CSTs while another lane is already
 * running a launch (the server is under load) and more requests are on their
 * way, it waits up to this long for more to join its launch; an idle server
 * launches at once (0: never wait).
 * Errors: CSTM_EINVAL for NULL arguments or a graph of another context;
 * CSTM_ENOMEM when mem_budget does not cover the lanes' task rings. */
typedef struct cstm_server cstm_server;
typedef struct {
    int32_t done;        /* 1: finished; the fields below are set                   */
    int32_t status;      /* the request's outcome: CSTM_OK; CSTM_ENOMEM when its CST
                            bound exceeds the whole budget; CSTM_EINVAL for a
                            malformed query; CSTM_ETIMEOUT / CSTM_EDEVICE from its
                            launch                                                   */
    uint64_t count;      /* number of embeddings (status CSTM_OK)                    */
    double submit_s;     /* server clock, seconds since creation, at submission     */
    double admit_s;      /* ... when it was admitted and its build began            */
    double built_s;      /* ... when its CST was built                               */
    double launch_s;     /* ... when its enumeration launch began                    */
    double done_s;       /* ... when the result became available                    */
    int32_t batch_size;  /* requests that shared its enumeration launch             */
    int32_t lane;        /* the lane that ran it                                    */
} cstm_request_result;
typedef struct {
    uint64_t submitted, completed, failed;
    uint64_t launches;   /* enumeration launches                                    */
    uint64_t batched;    /* requests over all launches                              */
    uint64_t peak_bytes; /* largest total charge of admitted requests               */
    uint64_t in_use_bytes;
    int32_t max_overlap; /* most lanes running launches at one time                 */
    int32_t reserved;
    uint64_t admission_bytes; /* what admission may charge: mem_budget less the lanes'
                                 task rings                                          */
    /* Summed over the enumeration launches that succeeded: kernel time (HIP
     * events on each lane's stream) and, when the context collects
     * statistics (cstm_tune.collect_stats), the work counters of
     * cstm_enum_stats.                                                          */
    double kernel_ms;
    uint64_t extensions, edge_checks, pushed, summed, chunks;
} cstm_server_stats;

cstm_status cstm_server_create(cstm_ctx* ctx, const cstm_graph* g, uint64_t mem_budget, int32_t lanes,
                               int32_t builders, int32_t max_batch, int32_t batch_wait_us, cstm_server** out);
/* Queue a query (copied; same arguments as cstm_cst_build); *ticket names it.
 * limit: 0 = count every embedding, > 0 = the result is min(total, limit)
 * and the search stops once it is reached.  Only the sizes are checked here:
 * a malformed query finishes with status CSTM_EINVAL. */
cstm_status cstm_server_submit(cstm_server* srv, int32_t k, const int32_t* qlabel, int32_t m_q,
                               const int32_t* qedges, uint64_t limit, uint64_t* ticket);
/* Non-blocking: out->done = 0 while the request runs.  A finished result is
 * handed out once; the ticket is unknown (CSTM_EINVAL) afterwards. */
cstm_status cstm_server_poll(cstm_server* srv, uint64_t ticket, cstm_request_result* out);
/* As poll, but waits up to timeout_s seconds (<= 0: until done). */
cstm_status cstm_server_wait(cstm_server* srv, uint64_t ticket, double timeout_s, cstm_request_result* out);
cstm_status cstm_server_get_stats(cstm_server* srv, cstm_server_stats* out);
/* Finishes every submitted request, then stops the threads and frees the server. */
void cstm_server_destroy(cstm_server* srv);

/* Statistics of the last enumeration launch (cstm_enumerate or
 * cstm_batch_enumerate) made with this context. */
cstm_status cstm_ctx_last_enum_stats(const cstm_ctx* ctx, cstm_enum_stats* out);

/* Milliseconds spent in the last build / partition / enumerate of this CST,
 * timed with HIP events on its stream (0 when not run). */
cstm_status cstm_cst_times(const cstm_cst* cst, double* build_ms, double* partition_ms, double* enumerate_ms);

void cstm_cst_free(cstm_cst* cst);

const char* cstm_last_error(void);
const char* cstm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CSTM_H */
