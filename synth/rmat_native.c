/*
 * rmat_native.c -- multithreaded R-MAT graph generator (input generation only).
 *
 * Builds the simple undirected CSR of an R-MAT graph (Graph500 style) with
 * 2^scale vertices from edge_factor * 2^scale samples: each sample descends
 * `scale` levels, picking a quadrant with probabilities a, b, c, d = 1-a-b-c
 * per level.  Self-loops are dropped, duplicates merged, vertex ids shuffled
 * by a seeded permutation, every edge stored in both directions and each row
 * sorted ascending.  It holds none of the matching method's arithmetic.
 *
 * Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014) applied to a
 * counter: draw j of sample i is mix(seed, i * 64 + j), so the graph does not
 * depend on the thread count.  The vertex permutation is a Fisher-Yates
 * shuffle driven by the same generator.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

static inline uint64_t draw(uint64_t seed, uint64_t ctr) { return splitmix64(seed ^ splitmix64(ctr)); }

typedef struct {
    int scale;
    uint64_t seed;
    uint64_t ta, tab, tabc;  /* quadrant thresholds scaled to 2^32 */
    const uint32_t* perm;
    uint64_t s0, s1;         /* sample range */
    uint64_t* out;           /* keys lo * n + hi, one per kept sample */
    uint64_t kept;
} gen_job;

static void* gen_worker(void* p) {
    gen_job* J = (gen_job*)p;
    const uint64_t n = 1ull << J->scale;
    uint64_t k = 0;
    for (uint64_t i = J->s0; i < J->s1; ++i) {
        uint64_t src = 0, dst = 0;
        for (int level = 0; level < J->scale; ++level) {
            /* two 32-bit uniforms per 64-bit draw */
            uint64_t r = draw(J->seed, i * 64 + (uint64_t)(level >> 1));
            uint64_t u = (level & 1) ? (r >> 32) : (r & 0xFFFFFFFFull);
            uint64_t sbit = u >= J->tab;
            uint64_t dbit = (u >= J->ta && u < J->tab) || u >= J->tabc;
            src |= sbit << level;
            dst |= dbit << level;
        }
        if (src == dst) continue;
        uint64_t a = J->perm[src], b = J->perm[dst];
        uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
        J->out[k++] = lo * n + hi;
    }
    J->kept = k;
    return NULL;
}

/* LSD radix sort of keys (bits below `bits`), 11 bits per pass, threads split the input. */
typedef struct {
    const uint64_t* in;
    uint64_t* out;
    uint64_t lo, hi;
    int shift;
    uint64_t* hist;  /* 2048 counters for this thread, then its start offsets */
    int phase;
} sort_job;

static void* sort_worker(void* p) {
    sort_job* S = (sort_job*)p;
    if (S->phase == 0) {
        memset(S->hist, 0, 2048 * sizeof(uint64_t));
        for (uint64_t i = S->lo; i < S->hi; ++i) S->hist[(S->in[i] >> S->shift) & 2047]++;
    } else {
        for (uint64_t i = S->lo; i < S->hi; ++i) {
            uint64_t d = (S->in[i] >> S->shift) & 2047;
            S->out[S->hist[d]++] = S->in[i];
        }
    }
    return NULL;
}

static int radix_sort(uint64_t* keys, uint64_t* tmp, uint64_t cnt, int bits, int nt) {
    sort_job* jobs = (sort_job*)calloc((size_t)nt, sizeof(sort_job));
    pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
    uint64_t* hist = (uint64_t*)calloc((size_t)nt * 2048, sizeof(uint64_t));
    if (!jobs || !th || !hist) { free(jobs); free(th); free(hist); return 1; }
    uint64_t* in = keys;
    uint64_t* out = tmp;
    int passes = 0;
    for (int shift = 0; shift < bits; shift += 11, ++passes) {
        for (int phase = 0; phase < 2; ++phase) {
            if (phase == 1) {
                uint64_t run = 0;
                for (int d = 0; d < 2048; ++d)
                    for (int t = 0; t < nt; ++t) {
                        uint64_t c = hist[(size_t)t * 2048 + d];
                        hist[(size_t)t * 2048 + d] = run;
                        run += c;
                    }
            }
            for (int t = 0; t < nt; ++t) {
                jobs[t].in = in;
                jobs[t].out = out;
                jobs[t].lo = cnt * (uint64_t)t / (uint64_t)nt;
                jobs[t].hi = cnt * (uint64_t)(t + 1) / (uint64_t)nt;
                jobs[t].shift = shift;
                jobs[t].hist = hist + (size_t)t * 2048;
                jobs[t].phase = phase;
                pthread_create(&th[t], NULL, sort_worker, &jobs[t]);
            }
            for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
        }
        uint64_t* x = in;
        in = out;
        out = x;
    }
    if (passes & 1) memcpy(keys, tmp, cnt * sizeof(uint64_t));
    free(jobs); free(th); free(hist);
    return 0;
}

/*
 * Returns 0 on success and fills *row_ptr_out (int64[n+1]) and *col_out
 * (int32[nnz]) with malloc'd arrays the caller releases with rmat_free.
 * Returns 1 on a bad argument, 2 when memory runs out.
 */
int rmat_csr(int scale, int edge_factor, double a, double b, double c, uint64_t seed, int nthreads,
             int64_t** row_ptr_out, int32_t** col_out, int64_t* nnz_out) {
    if (scale < 1 || scale > 30 || edge_factor < 1 || nthreads < 1 || nthreads > 256) return 1;
    if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return 1;
    const uint64_t n = 1ull << scale;
    const uint64_t samples = (uint64_t)edge_factor << scale;
    uint32_t* perm = (uint32_t*)malloc(n * sizeof(uint32_t));
    uint64_t* keys = (uint64_t*)malloc(samples * sizeof(uint64_t));
    if (!perm || !keys) { free(perm); free(keys); return 2; }
    for (uint64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    for (uint64_t i = n - 1; i > 0; --i) {
        uint64_t j = draw(seed ^ 0x5045524Dull, i) % (i + 1);
        uint32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
    /* samples, split over threads; each thread writes its own slice */
    gen_job* jobs = (gen_job*)calloc((size_t)nthreads, sizeof(gen_job));
    pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) { free(perm); free(keys); free(jobs); free(th); return 2; }
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].scale = scale;
        jobs[t].seed = seed;
        jobs[t].ta = (uint64_t)(a * 4294967296.0);
        jobs[t].tab = (uint64_t)((a + b) * 4294967296.0);
        jobs[t].tabc = (uint64_t)((a + b + c) * 4294967296.0);
        jobs[t].perm = perm;
        jobs[t].s0 = samples * (uint64_t)t / (uint64_t)nthreads;
        jobs[t].s1 = samples * (uint64_t)(t + 1) / (uint64_t)nthreads;
        jobs[t].out = keys + jobs[t].s0;
        pthread_create(&th[t], NULL, gen_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    uint64_t cnt = 0;
    for (int t = 0; t < nthreads; ++t) {
        memmove(keys + cnt, jobs[t].out, jobs[t].kept * sizeof(uint64_t));
        cnt += jobs[t].kept;
    }
    free(jobs); free(th); free(perm);
    /* sort and merge duplicates */
    uint64_t* tmp = (uint64_t*)malloc((cnt ? cnt : 1) * sizeof(uint64_t));
    if (!tmp) { free(keys); return 2; }
    if (radix_sort(keys, tmp, cnt, 2 * scale, nthreads)) { free(keys); free(tmp); return 2; }
    free(tmp);
    uint64_t m = 0;
    for (uint64_t i = 0; i < cnt; ++i)
        if (i == 0 || keys[i] != keys[i - 1]) keys[m++] = keys[i];
    /* CSR: degrees, offsets, then one pass in (lo, hi) order keeps every row sorted:
       for vertex v the entries lo < v arrive first (in ascending lo), then hi > v */
    int64_t* row_ptr = (int64_t*)calloc(n + 1, sizeof(int64_t));
    int32_t* col = (int32_t*)malloc((m ? 2 * m : 1) * sizeof(int32_t));
    if (!row_ptr || !col) { free(keys); free(row_ptr); free(col); return 2; }
    for (uint64_t i = 0; i < m; ++i) {
        row_ptr[keys[i] / n + 1]++;
        row_ptr[keys[i] % n + 1]++;
    }
    for (uint64_t v = 0; v < n; ++v) row_ptr[v + 1] += row_ptr[v];
    int64_t* pos = (int64_t*)malloc(n * sizeof(int64_t));
    if (!pos) { free(keys); free(row_ptr); free(col); return 2; }
    memcpy(pos, row_ptr, n * sizeof(int64_t));
    for (uint64_t i = 0; i < m; ++i) {
        uint64_t lo = keys[i] / n, hi = keys[i] % n;
        col[pos[lo]++] = (int32_t)hi;
        col[pos[hi]++] = (int32_t)lo;
    }
    free(pos);
    free(keys);
    *row_ptr_out = row_ptr;
    *col_out = col;
    *nnz_out = (int64_t)(2 * m);
    return 0;
}

void rmat_free(void* p) { free(p); }
