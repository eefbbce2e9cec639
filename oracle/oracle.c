/*
 * oracle.c -- plain CPU subgraph-isomorphism matcher.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load this library.  It shares no code with the HIP path and never sees a
 * candidate search tree: it works directly on the data graph G.
 *
 * What it computes (Section II-A, Definition 1 and the problem statement):
 * the set of all maps f: V(q) -> V(G) that are
 *   - injective,
 *   - label preserving:   l_G(f(u)) == l_q(u) for every query vertex u,
 *   - edge preserving:    (f(u), f(u')) in E(G) for every query edge (u, u'),
 * i.e. non-induced embeddings; every such map counts separately, so
 * automorphic images of one subgraph are distinct results.
 *
 * How: ordinary recursive backtracking, the textbook method the paper sets out
 * from (Sections I and III-A).  The order is chosen by the oracle itself and
 * is deliberately unrelated to the CST path order:
 *   pi_0 = a query vertex of maximum degree (smallest id on ties); then the
 *   unplaced vertex with the most placed neighbours (ties: larger query degree,
 *   then smaller id).  Each later vertex is extended from the adjacency list of
 *   its earliest-placed neighbour (the pivot) and checked against all its other
 *   placed neighbours by binary search in G's sorted rows.
 * Optionally the caller also passes G's rows regrouped by (label, id); then
 * the pivot's row is scanned only over the entries that carry u's label (a
 * binary search finds that range), which skips the entries the label test
 * would reject anyway and changes nothing else.
 * A degree test d_G(v) >= d_q(u) may prune candidates; it is sound because an
 * injective edge-preserving map sends the d_q(u) distinct neighbours of u to
 * distinct neighbours of f(u).  The tests check both settings agree.
 *
 * Root candidates are handed out to POSIX threads through an atomic counter;
 * per-thread counts are summed and per-thread rows concatenated and sorted.
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#include <unistd.h>

#define OR_OK 0
#define OR_EINVAL 1
#define OR_ENOMEM 2
#define OR_ETIMEOUT 4
#define OR_EOVERFLOW 5

#define OR_MAXK 32
#define FLUSH_MASK 0xFFFFull

typedef struct {
    int64_t n;
    const int64_t* rp;
    const int32_t* col;
    const int32_t* lab;
    const int32_t* lcol;      /* optional: rows regrouped by (label, id)       */
    int k;
    int32_t qlab[OR_MAXK];
    int32_t qdeg[OR_MAXK];
    int order[OR_MAXK];       /* order[i] = query vertex placed i-th            */
    int pivot[OR_MAXK];       /* position of the earliest placed neighbour      */
    int nchk[OR_MAXK];        /* number of other placed neighbours              */
    int chk[OR_MAXK][OR_MAXK];/* their positions                               */
    int degfilter;
    int mutate;
    int list;
    int64_t nroots;
    int32_t* roots;
    _Atomic int64_t next_root;
    _Atomic uint64_t nodes_total;
    _Atomic int stop;         /* 1 budget, 2 deadline, 3 out of memory, 4 limit */
    uint64_t limit;           /* > 0: stop once this many embeddings are found  */
    _Atomic uint64_t found;   /* embeddings published by the workers            */
    uint64_t node_budget;
    double deadline; /* absolute CLOCK_MONOTONIC seconds; 0 = none */
} ctx_t;

typedef struct {
    ctx_t* c;
    int32_t map[OR_MAXK];
    uint64_t count;
    uint64_t published;       /* part of count already added to c->found        */
    uint64_t nodes;
    uint64_t unflushed;
    int32_t* rows;
    uint64_t nrows, caprows;
    int oom;
} worker_t;

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static int has_edge(const ctx_t* c, int32_t a, int32_t b) {
    int64_t lo = c->rp[a], hi = c->rp[a + 1];
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        int32_t x = c->col[mid];
        if (x == b) return 1;
        if (x < b) lo = mid + 1; else hi = mid;
    }
    return 0;
}

static void flush_nodes(worker_t* w) {
    ctx_t* c = w->c;
    uint64_t tot = atomic_fetch_add(&c->nodes_total, w->unflushed) + w->unflushed;
    w->unflushed = 0;
    if (c->limit) {
        uint64_t f = atomic_fetch_add(&c->found, w->count - w->published) + (w->count - w->published);
        w->published = w->count;
        if (f >= c->limit) atomic_store(&c->stop, 4);
    }
    if (c->node_budget && tot > c->node_budget) atomic_store(&c->stop, 1);
    if (c->deadline > 0 && now_s() > c->deadline) atomic_store(&c->stop, 2);
}

static void emit(worker_t* w) {
    ctx_t* c = w->c;
    if (w->nrows == w->caprows) {
        uint64_t nc = w->caprows ? 2 * w->caprows : 1024;
        int32_t* p = (int32_t*)realloc(w->rows, nc * (uint64_t)c->k * sizeof(int32_t));
        if (!p) { w->oom = 1; atomic_store(&c->stop, 3); return; }
        w->rows = p;
        w->caprows = nc;
    }
    int32_t* row = w->rows + w->nrows * (uint64_t)c->k;
    /* rows are written in query-id order: row[u] = f(u) */
    for (int i = 0; i < c->k; ++i) {
        if (c->mutate == 6) row[i] = w->map[i];
        else row[c->order[i]] = w->map[i];
    }
    w->nrows++;
}

/* one more partial embedding: placed positions 0..depth-1 are in w->map */
static void visit(worker_t* w, int depth) {
    ctx_t* c = w->c;
    w->nodes++;
    if (++w->unflushed > FLUSH_MASK) flush_nodes(w);
    if (depth == c->k) {
        w->count++;
        if (c->list) emit(w);
        if (c->limit && w->count - w->published >= c->limit) flush_nodes(w);
        return;
    }
    const int u = c->order[depth];
    const int32_t pv = w->map[c->pivot[depth]];
    const int32_t* row = c->col;
    int64_t e0 = c->rp[pv], e1 = c->rp[pv + 1];
    if (c->lcol) {
        /* the entries of label qlab[u] form one run of the regrouped row */
        row = c->lcol;
        int64_t lo = e0, hi = e1;
        while (lo < hi) {
            int64_t mid = lo + ((hi - lo) >> 1);
            if (c->lab[row[mid]] < c->qlab[u]) lo = mid + 1; else hi = mid;
        }
        e0 = lo;
        hi = e1;
        while (lo < hi) {
            int64_t mid = lo + ((hi - lo) >> 1);
            if (c->lab[row[mid]] <= c->qlab[u]) lo = mid + 1; else hi = mid;
        }
        e1 = lo;
    }
    for (int64_t e = e0; e < e1; ++e) {
        if (atomic_load_explicit(&c->stop, memory_order_relaxed)) return;
        /* every scanned adjacency entry is work too, so a long fruitless scan still meets the budget */
        if (++w->unflushed > FLUSH_MASK) flush_nodes(w);
        const int32_t x = row[e];
        if (c->mutate != 3 && c->lab[x] != c->qlab[u]) continue;
        if (c->degfilter) {
            int64_t d = c->rp[x + 1] - c->rp[x];
            if (c->mutate == 5 ? d <= c->qdeg[u] : d < c->qdeg[u]) continue;
        }
        int dup = 0;
        if (c->mutate != 1)
            for (int j = 0; j < depth; ++j)
                if (w->map[j] == x) { dup = 1; break; }
        if (dup) continue;
        int ok = 1;
        if (c->mutate != 2)
            for (int t = 0; t < c->nchk[depth]; ++t)
                if (!has_edge(c, w->map[c->chk[depth][t]], x)) { ok = 0; break; }
        if (!ok) continue;
        w->map[depth] = x;
        visit(w, depth + 1);
    }
}

static void* worker_main(void* arg) {
    worker_t* w = (worker_t*)arg;
    ctx_t* c = w->c;
    for (;;) {
        if (atomic_load(&c->stop)) break;
        int64_t i = atomic_fetch_add(&c->next_root, 1);
        if (i >= c->nroots) break;
        w->map[0] = c->roots[i];
        visit(w, 1);
    }
    flush_nodes(w);
    return NULL;
}

static int row_cmp(const void* a, const void* b, void* kp) {
    const int32_t* x = (const int32_t*)a;
    const int32_t* y = (const int32_t*)b;
    const int kk = *(const int*)kp;
    for (int i = 0; i < kk; ++i) {
        if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
    }
    return 0;
}

int oracle_num_cores(void) {
    long n = sysconf(_SC_NPROCESSORS_ONLN);
    return n > 0 ? (int)n : 1;
}

/*
 * Count (and optionally list) all embeddings of q in G.
 *
 *   n, row_ptr[n+1], col[row_ptr[n]], label[n]: G as CSR, rows sorted, simple,
 *       symmetric (the caller guarantees this; it is not re-checked here).
 *   lcol (may be NULL): the same rows, each regrouped by (label, id); used
 *       only to find a pivot's neighbours of one label.
 *   k, qlabel[k], m_q, qedges[2*m_q]: q with query ids 0..k-1.
 *   degree_filter: 1 prunes candidates with d_G(v) < d_q(u).
 *   nthreads: worker threads, 0 = all online cores; the number used is written
 *       to *threads_used.
 *   limit (0: none): stop once at least limit embeddings were found; the call
 *       then returns OR_OK with *count_out = limit, which is min(total, limit)
 *       exactly (listing is not combined with a limit).
 *   deadline_s (<= 0: none) and node_budget (0: none): on expiry the call
 *       returns OR_ETIMEOUT and *count_out is a lower bound.  The budget caps
 *       the work done: partial embeddings visited (root level included) plus
 *       adjacency entries scanned.  That total is deterministic, so a budget
 *       screen accepts the same queries on any host; *nodes_out reports it.
 *   rows (may be NULL), cap: with list = 1, the first min(count, cap) rows of the
 *       lexicographically sorted result (row[u] = f(u)); OR_EOVERFLOW when
 *       count > cap (count still exact).
 *   mutate: 0 in every real use.  Non-zero values plant a deliberate mistake so
 *       that the tests can show their pins catch it.
 */
int oracle_match(int64_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* label,
                 const int32_t* lcol, int32_t k, const int32_t* qlabel, int32_t m_q, const int32_t* qedges,
                 int degree_filter, int nthreads, double deadline_s, uint64_t node_budget, uint64_t limit,
                 int list, int32_t* rows, uint64_t cap, int mutate,
                 uint64_t* count_out, uint64_t* nodes_out, uint64_t* rows_written, int* threads_used) {
    if (count_out) *count_out = 0;
    if (nodes_out) *nodes_out = 0;
    if (rows_written) *rows_written = 0;
    if (k < 1 || k > OR_MAXK || n < 0 || m_q < 0 || (limit && list)) return OR_EINVAL;
    ctx_t* c = (ctx_t*)calloc(1, sizeof(ctx_t));
    if (!c) return OR_ENOMEM;
    c->n = n; c->rp = row_ptr; c->col = col; c->lab = label; c->lcol = lcol; c->k = k;
    c->degfilter = degree_filter; c->mutate = mutate; c->list = list;
    c->node_budget = node_budget;
    c->limit = limit;
    c->deadline = deadline_s > 0 ? now_s() + deadline_s : 0;
    unsigned char adj[OR_MAXK][OR_MAXK];
    memset(adj, 0, sizeof(adj));
    for (int u = 0; u < k; ++u) {
        if (qlabel[u] < 0) { free(c); return OR_EINVAL; }
        c->qlab[u] = qlabel[u];
    }
    for (int e = 0; e < m_q; ++e) {
        int a = qedges[2 * e], b = qedges[2 * e + 1];
        if (a < 0 || b < 0 || a >= k || b >= k || a == b || adj[a][b]) { free(c); return OR_EINVAL; }
        adj[a][b] = adj[b][a] = 1;
        c->qdeg[a]++; c->qdeg[b]++;
    }
    /* connectivity of q */
    {
        int seen[OR_MAXK] = {0}, stack[OR_MAXK], sp = 0, cnt = 1;
        seen[0] = 1; stack[sp++] = 0;
        while (sp) {
            int x = stack[--sp];
            for (int y = 0; y < k; ++y)
                if (adj[x][y] && !seen[y]) { seen[y] = 1; cnt++; stack[sp++] = y; }
        }
        if (cnt != k) { free(c); return OR_EINVAL; }
    }
    /* the oracle's own order */
    int placed[OR_MAXK] = {0}, pos_of[OR_MAXK];
    int first = 0;
    for (int u = 1; u < k; ++u)
        if (c->qdeg[u] > c->qdeg[first]) first = u;
    c->order[0] = first; placed[first] = 1; pos_of[first] = 0;
    for (int i = 1; i < k; ++i) {
        int best = -1, best_np = -1;
        for (int u = 0; u < k; ++u) {
            if (placed[u]) continue;
            int np = 0;
            for (int t = 0; t < k; ++t) np += placed[t] && adj[u][t];
            if (np > best_np || (np == best_np && c->qdeg[u] > c->qdeg[best])) { best = u; best_np = np; }
        }
        c->order[i] = best; placed[best] = 1; pos_of[best] = i;
        int piv = -1;
        c->nchk[i] = 0;
        for (int j = 0; j < i; ++j) {
            if (!adj[best][c->order[j]]) continue;
            if (piv < 0) piv = j;
            else c->chk[i][c->nchk[i]++] = j;
        }
        c->pivot[i] = piv;
    }
    (void)pos_of;
    /* root candidates: every vertex with the first query vertex's label */
    int64_t nr = 0;
    int64_t scan_end = (mutate == 4 && n > 0) ? n - 1 : n;
    for (int64_t v = 0; v < scan_end; ++v)
        if (label[v] == c->qlab[first] && (!degree_filter || row_ptr[v + 1] - row_ptr[v] >= c->qdeg[first])) nr++;
    c->roots = (int32_t*)malloc((size_t)(nr ? nr : 1) * sizeof(int32_t));
    if (!c->roots) { free(c); return OR_ENOMEM; }
    nr = 0;
    for (int64_t v = 0; v < scan_end; ++v)
        if (label[v] == c->qlab[first] && (!degree_filter || row_ptr[v + 1] - row_ptr[v] >= c->qdeg[first]))
            c->roots[nr++] = (int32_t)v;
    c->nroots = nr;

    int nt = nthreads > 0 ? nthreads : oracle_num_cores();
    if (threads_used) *threads_used = nt;
    worker_t* ws = (worker_t*)calloc((size_t)nt, sizeof(worker_t));
    pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
    if (!ws || !th) { free(ws); free(th); free(c->roots); free(c); return OR_ENOMEM; }
    for (int t = 0; t < nt; ++t) {
        ws[t].c = c;
        if (nt == 1) worker_main(&ws[0]);
        else pthread_create(&th[t], NULL, worker_main, &ws[t]);
    }
    if (nt > 1)
        for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);

    uint64_t count = 0, total_rows = 0;
    int oom = 0;
    for (int t = 0; t < nt; ++t) {
        count += ws[t].count;
        total_rows += ws[t].nrows;
        oom |= ws[t].oom;
    }
    uint64_t nodes = atomic_load(&c->nodes_total);
    int status = OR_OK;
    if (oom) status = OR_ENOMEM;
    else if (limit && count >= limit) count = limit;  /* reached: min(total, limit) = limit */
    else if (atomic_load(&c->stop) || (node_budget && nodes > node_budget)) status = OR_ETIMEOUT;

    if (list && status == OR_OK && total_rows) {
        int32_t* all = (int32_t*)malloc(total_rows * (uint64_t)k * sizeof(int32_t));
        if (!all) status = OR_ENOMEM;
        else {
            uint64_t off = 0;
            for (int t = 0; t < nt; ++t) {
                if (!ws[t].nrows) continue;  /* a worker that found nothing holds no row buffer */
                memcpy(all + off * (uint64_t)k, ws[t].rows, ws[t].nrows * (uint64_t)k * sizeof(int32_t));
                off += ws[t].nrows;
            }
            int kk = k;
            qsort_r(all, total_rows, (size_t)k * sizeof(int32_t), row_cmp, &kk);
            uint64_t w = total_rows < cap ? total_rows : cap;
            if (rows && w) memcpy(rows, all, w * (uint64_t)k * sizeof(int32_t));
            if (rows_written) *rows_written = rows ? w : 0;
            if (total_rows > cap) status = OR_EOVERFLOW;
            free(all);
        }
    }
    for (int t = 0; t < nt; ++t) free(ws[t].rows);
    if (count_out) *count_out = count;
    if (nodes_out) *nodes_out = nodes;
    free(ws); free(th); free(c->roots); free(c);
    return status;
}

/* ------------------------------------------------------------------ label-grouped rows
 * The same rows as col, each reordered by (label of the entry, entry id): the
 * optional lcol argument of oracle_match.  Rows are split over nthreads POSIX
 * threads (0 = all online cores); each row is sorted on its own by a
 * comparison sort of (label, id) pairs, so the result does not depend on the
 * thread count.  Returns OR_OK or OR_ENOMEM. */
typedef struct {
    int64_t n;
    const int64_t* rp;
    const int32_t* col;
    const int32_t* lab;
    int32_t* out;
    _Atomic int64_t next;
    _Atomic int oom;
} group_t;

static int pair_cmp(const void* a, const void* b) {
    const int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static void* group_worker(void* arg) {
    group_t* G = (group_t*)arg;
    int64_t cap = 0;
    int64_t* buf = NULL;
    for (;;) {
        const int64_t v0 = atomic_fetch_add(&G->next, 4096);
        if (v0 >= G->n) break;
        const int64_t v1 = v0 + 4096 < G->n ? v0 + 4096 : G->n;
        for (int64_t v = v0; v < v1; ++v) {
            const int64_t e0 = G->rp[v], d = G->rp[v + 1] - e0;
            if (d > cap) {
                int64_t* nb = (int64_t*)realloc(buf, (size_t)d * sizeof(int64_t));
                if (!nb) { atomic_store(&G->oom, 1); free(buf); return NULL; }
                buf = nb;
                cap = d;
            }
            for (int64_t i = 0; i < d; ++i) {
                const int32_t x = G->col[e0 + i];
                buf[i] = ((int64_t)G->lab[x] << 32) | (int64_t)(uint32_t)x;
            }
            qsort(buf, (size_t)d, sizeof(int64_t), pair_cmp);
            for (int64_t i = 0; i < d; ++i) G->out[e0 + i] = (int32_t)(uint32_t)buf[i];
        }
    }
    free(buf);
    return NULL;
}

int oracle_label_group(int64_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* label, int32_t* out,
                       int nthreads) {
    group_t G;
    G.n = n; G.rp = row_ptr; G.col = col; G.lab = label; G.out = out;
    atomic_init(&G.next, 0);
    atomic_init(&G.oom, 0);
    int nt = nthreads > 0 ? nthreads : oracle_num_cores();
    pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
    if (!th) return OR_ENOMEM;
    for (int t = 0; t < nt; ++t) pthread_create(&th[t], NULL, group_worker, &G);
    for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
    free(th);
    return atomic_load(&G.oom) ? OR_ENOMEM : OR_OK;
}
