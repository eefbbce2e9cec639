/*
 * rmat_native.c -- multithreaded R-MAT and Chung-Lu graph generators (input
 * generation only).
 *
 * R-MAT: the simple undirected CSR of an R-MAT graph (Graph500 style) with
 * 2^scale vertices from edge_factor * 2^scale samples: each sample descends
 * `scale` levels, picking a quadrant with probabilities a, b, c, d = 1-a-b-c
 * per level.
 *
 * Chung-Lu: vertex i has weight (i + 1)^(-1 / (gamma - 1)); both endpoints
 * of a sample are drawn independently with probability proportional to
 * their weight (Walker's alias method, built by Vose's algorithm: M. D. Vose,
 * "A linear algorithm for generating random numbers with a given
 * distribution", IEEE TSE 1991); samples are drawn until m distinct non-loop
 * pairs were seen, and the first m distinct pairs in sample order are kept.
 *
 * For both, self-loops are dropped, duplicates merged, vertex ids shuffled by
 * a seeded permutation, every edge stored in both directions and each row
 * sorted ascending.  It holds none of the matching method's arithmetic.
 *
 * Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014) applied to a
 * counter: draw j of sample i is mix(seed, i * 64 + j), so the graph does not
 * depend on the thread count.  The vertex permutation is a Fisher-Yates
 * shuffle driven by the same generator.
 */
#include <math.h>
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

/* Sorts the (lo * n + hi) keys (2 * scale bits), merges duplicates and writes the
 * symmetric CSR; frees keys.  Returns 0, or 2 when memory runs out. */
static int keys_to_csr(uint64_t* keys, uint64_t cnt, int scale, int nthreads, int64_t** row_ptr_out,
                       int32_t** col_out, int64_t* nnz_out) {
    const uint64_t n = 1ull << scale;
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

/* A seeded Fisher-Yates permutation of 0..n-1. */
static uint32_t* seeded_perm(uint64_t n, uint64_t seed) {
    uint32_t* perm = (uint32_t*)malloc(n * sizeof(uint32_t));
    if (!perm) return NULL;
    for (uint64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    for (uint64_t i = n - 1; i > 0; --i) {
        uint64_t j = draw(seed ^ 0x5045524Dull, i) % (i + 1);
        uint32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
    return perm;
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
    uint32_t* perm = seeded_perm(n, seed);
    uint64_t* keys = (uint64_t*)malloc(samples * sizeof(uint64_t));
    if (!perm || !keys) { free(perm); free(keys); return 2; }
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
    return keys_to_csr(keys, cnt, scale, nthreads, row_ptr_out, col_out, nnz_out);
}

/* ------------------------------------------------------------------ Chung-Lu */

/* LSD radix sort of keys (bits below `bits`) carrying a 32-bit payload, 11
 * bits per pass, stable; threads split the input. */
typedef struct {
    const uint64_t* kin;
    const uint32_t* vin;
    uint64_t* kout;
    uint32_t* vout;
    uint64_t lo, hi;
    int shift, phase;
    uint64_t* hist;
} kv_job;

static void* kv_worker(void* p) {
    kv_job* S = (kv_job*)p;
    if (S->phase == 0) {
        memset(S->hist, 0, 2048 * sizeof(uint64_t));
        for (uint64_t i = S->lo; i < S->hi; ++i) S->hist[(S->kin[i] >> S->shift) & 2047]++;
    } else {
        for (uint64_t i = S->lo; i < S->hi; ++i) {
            uint64_t d = (S->kin[i] >> S->shift) & 2047;
            uint64_t o = S->hist[d]++;
            S->kout[o] = S->kin[i];
            S->vout[o] = S->vin[i];
        }
    }
    return NULL;
}

/* Sorts (k, v) in place, with (tk, tv) as scratch of the same sizes. */
static int radix_sort_kv(uint64_t* k, uint32_t* v, uint64_t* tk, uint32_t* tv, uint64_t cnt, int bits, int nt) {
    kv_job* jobs = (kv_job*)calloc((size_t)nt, sizeof(kv_job));
    pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
    uint64_t* hist = (uint64_t*)calloc((size_t)nt * 2048, sizeof(uint64_t));
    if (!jobs || !th || !hist) { free(jobs); free(th); free(hist); return 1; }
    uint64_t *ki = k, *ko = tk;
    uint32_t *vi = v, *vo = tv;
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
                jobs[t].kin = ki; jobs[t].vin = vi; jobs[t].kout = ko; jobs[t].vout = vo;
                jobs[t].lo = cnt * (uint64_t)t / (uint64_t)nt;
                jobs[t].hi = cnt * (uint64_t)(t + 1) / (uint64_t)nt;
                jobs[t].shift = shift;
                jobs[t].phase = phase;
                jobs[t].hist = hist + (size_t)t * 2048;
                pthread_create(&th[t], NULL, kv_worker, &jobs[t]);
            }
            for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
        }
        uint64_t* x = ki; ki = ko; ko = x;
        uint32_t* y = vi; vi = vo; vo = y;
    }
    if (passes & 1) {
        memcpy(k, tk, cnt * sizeof(uint64_t));
        memcpy(v, tv, cnt * sizeof(uint32_t));
    }
    free(jobs); free(th); free(hist);
    return 0;
}

/* Alias table of a discrete distribution over 0..n-1: draw i uniformly, keep
 * it with probability prob[i], else take alias[i]. */
typedef struct {
    double* prob;
    uint32_t* alias;
} alias_t;

static int alias_build(const double* w, uint64_t n, alias_t* A) {
    A->prob = (double*)malloc(n * sizeof(double));
    A->alias = (uint32_t*)malloc(n * sizeof(uint32_t));
    uint32_t* small = (uint32_t*)malloc(n * sizeof(uint32_t));
    uint32_t* large = (uint32_t*)malloc(n * sizeof(uint32_t));
    if (!A->prob || !A->alias || !small || !large) {
        free(A->prob); free(A->alias); free(small); free(large);
        return 2;
    }
    double total = 0.0;
    for (uint64_t i = 0; i < n; ++i) total += w[i];
    uint64_t ns = 0, nl = 0;
    for (uint64_t i = 0; i < n; ++i) {
        A->prob[i] = w[i] * (double)n / total;  /* scaled: mean 1 */
        A->alias[i] = (uint32_t)i;
        if (A->prob[i] < 1.0) small[ns++] = (uint32_t)i;
        else large[nl++] = (uint32_t)i;
    }
    while (ns && nl) {
        const uint32_t s = small[--ns], l = large[nl - 1];
        A->alias[s] = l;
        A->prob[l] -= 1.0 - A->prob[s];
        if (A->prob[l] < 1.0) {
            --nl;
            small[ns++] = l;
        }
    }
    while (nl) A->prob[large[--nl]] = 1.0;  /* rounding leftovers keep themselves */
    while (ns) A->prob[small[--ns]] = 1.0;
    free(small);
    free(large);
    return 0;
}

typedef struct {
    const alias_t* A;
    uint64_t n, seed, loop;
    uint64_t s0, s1;     /* sample range */
    uint64_t* key;       /* per sample: lo * n + hi, or `loop` for a self-loop */
    uint32_t* idx;       /* per sample: its index */
} cl_job;

static uint64_t cl_endpoint(const alias_t* A, uint64_t n, uint64_t r) {
    /* a 53-bit uniform u in [0, 1): column floor(u * n), kept with the column's probability */
    const double x = (double)(r >> 11) * 0x1.0p-53 * (double)n;
    uint64_t i = (uint64_t)x;
    if (i >= n) i = n - 1;
    return (x - (double)i) < A->prob[i] ? i : A->alias[i];
}

/* Sample s: one 64-bit draw per endpoint. */
static uint64_t cl_key(const alias_t* A, uint64_t n, uint64_t seed, uint64_t loop, uint64_t s) {
    const uint64_t a = cl_endpoint(A, n, draw(seed, 2 * s)), b = cl_endpoint(A, n, draw(seed, 2 * s + 1));
    return a == b ? loop : (a < b ? a * n + b : b * n + a);
}

static void* cl_worker(void* p) {
    cl_job* J = (cl_job*)p;
    for (uint64_t s = J->s0; s < J->s1; ++s) {
        J->key[s] = cl_key(J->A, J->n, J->seed, J->loop, s);
        J->idx[s] = (uint32_t)s;
    }
    return NULL;
}

/*
 * Chung-Lu CSR (see the file comment).  Returns 0 on success and fills
 * *row_ptr_out (int64[n+1]) and *col_out (int32[nnz]) with malloc'd arrays;
 * 1 on a bad argument, 2 when memory runs out.
 */
int chung_lu_csr(int64_t n_in, int64_t m_target, double gamma, uint64_t seed, int nthreads, int64_t** row_ptr_out,
                 int32_t** col_out, int64_t* nnz_out) {
    if (n_in < 2 || n_in > (1ll << 30) || m_target < 1 || gamma <= 1.0 || nthreads < 1 || nthreads > 256) return 1;
    const uint64_t n = (uint64_t)n_in, m = (uint64_t)m_target;
    if (m > n * (n - 1) / 2) return 1;
    int scale = 0;
    while ((1ull << scale) < n) ++scale;
    const uint64_t loop = 1ull << (2 * scale);  /* above every pair key */
    double* w = (double*)malloc(n * sizeof(double));
    if (!w) return 2;
    for (uint64_t i = 0; i < n; ++i) w[i] = pow((double)(i + 1), -1.0 / (gamma - 1.0));
    alias_t tab;
    if (alias_build(w, n, &tab)) { free(w); return 2; }
    free(w);
    const alias_t* table = &tab;
    uint64_t *K = NULL, *TK = NULL;
    uint32_t *I = NULL, *TI = NULL;
    uint64_t total = 0, distinct = 0, need = m;
    int status = 0;
    while (distinct < m) {
        const uint64_t batch = need + need / 3 + 4096;
        if (total + batch >= (1ull << 32)) { status = 1; break; }
        uint64_t* nk = (uint64_t*)realloc(K, (total + batch) * sizeof(uint64_t));
        if (nk) K = nk;
        uint32_t* ni = (uint32_t*)realloc(I, (total + batch) * sizeof(uint32_t));
        if (ni) I = ni;
        uint64_t* ntk = (uint64_t*)realloc(TK, (total + batch) * sizeof(uint64_t));
        if (ntk) TK = ntk;
        uint32_t* nti = (uint32_t*)realloc(TI, (total + batch) * sizeof(uint32_t));
        if (nti) TI = nti;
        if (!nk || !ni || !ntk || !nti) { status = 2; break; }
        /* new samples are appended after the sorted old ones; re-sorting all keeps stability by index */
        cl_job* jobs = (cl_job*)calloc((size_t)nthreads, sizeof(cl_job));
        pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
        if (!jobs || !th) { free(jobs); free(th); status = 2; break; }
        for (int t = 0; t < nthreads; ++t) {
            jobs[t].A = table; jobs[t].n = n; jobs[t].seed = seed; jobs[t].loop = loop;
            jobs[t].s0 = total + batch * (uint64_t)t / (uint64_t)nthreads;
            jobs[t].s1 = total + batch * (uint64_t)(t + 1) / (uint64_t)nthreads;
            jobs[t].key = K;
            jobs[t].idx = I;
            pthread_create(&th[t], NULL, cl_worker, &jobs[t]);
        }
        for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
        free(jobs); free(th);
        total += batch;
        /* the old samples are sorted by (key, index) and every new index is larger, so a
           stable sort by key leaves each key's first sample first */
        if (radix_sort_kv(K, I, TK, TI, total, 2 * scale + 1, nthreads)) { status = 2; break; }
        distinct = 0;
        for (uint64_t i = 0; i < total; ++i)
            if (K[i] != loop && (i == 0 || K[i] != K[i - 1])) distinct++;
        need = distinct < m ? m - distinct : 0;
    }
    free(TK); free(TI);
    if (status) { free(K); free(I); free(tab.prob); free(tab.alias); return status; }
    /* each distinct pair's first sample, then the m earliest of them */
    uint64_t* F = K;  /* reused in place: a head's slot is never read again */
    uint64_t nf = 0, prev = loop;
    for (uint64_t i = 0; i < total; ++i) {
        const uint64_t key = K[i];
        if (key != loop && (i == 0 || key != prev)) F[nf++] = I[i];
        prev = key;
    }
    free(I);
    uint64_t* tmp = (uint64_t*)malloc((nf ? nf : 1) * sizeof(uint64_t));
    if (!tmp) { free(K); free(tab.prob); free(tab.alias); return 2; }
    int sbits = 1;
    while (sbits < 64 && (total >> sbits)) ++sbits;
    if (radix_sort(F, tmp, nf, sbits, nthreads)) { free(tmp); free(K); free(tab.prob); free(tab.alias); return 2; }
    free(tmp);
    uint32_t* perm = seeded_perm(n, seed);
    uint64_t* out = (uint64_t*)malloc(m * sizeof(uint64_t));
    if (!perm || !out) { free(perm); free(out); free(K); free(tab.prob); free(tab.alias); return 2; }
    /* the kept samples' pairs, recomputed from their index, with shuffled ids */
    const uint64_t nn = 1ull << scale;
    for (uint64_t i = 0; i < m; ++i) {
        const uint64_t k = cl_key(table, n, seed, loop, F[i]);
        const uint64_t a = perm[k / n], b = perm[k % n];
        out[i] = a < b ? a * nn + b : b * nn + a;
    }
    free(perm); free(K); free(tab.prob); free(tab.alias);
    int64_t* rp = NULL;
    int st = keys_to_csr(out, m, scale, nthreads, &rp, col_out, nnz_out);
    if (st) return st;
    /* keys_to_csr laid out 2^scale rows; the graph has n (the rest are empty) */
    int64_t* row_ptr = (int64_t*)realloc(rp, (n + 1) * sizeof(int64_t));
    *row_ptr_out = row_ptr ? row_ptr : rp;
    return 0;
}

void rmat_free(void* p) { free(p); }
