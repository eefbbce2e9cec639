/*
 * Host-only driver for the AddressSanitizer / UndefinedBehaviorSanitizer build
 * of the CPU oracle (oracle/oracle.c) and the native R-MAT generator
 * (synth/rmat_native.c).  It runs both on small inputs whose answers are known
 * in closed form and exits non-zero on a wrong answer; the sanitizers abort on
 * any memory or undefined-behaviour error.  Built and run by
 * tests/test_sanitizers.py.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_match(int64_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* label, const int32_t* lcol,
                 int32_t k, const int32_t* qlabel, int32_t m_q, const int32_t* qedges, int degree_filter,
                 int nthreads, double deadline_s, uint64_t node_budget, uint64_t limit, int list, int32_t* rows,
                 uint64_t cap, int mutate, uint64_t* count_out, uint64_t* nodes_out, uint64_t* rows_written,
                 int* threads_used);
int oracle_label_group(int64_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* label, int32_t* out,
                       int nthreads);
int rmat_csr(int scale, int edge_factor, double a, double b, double c, uint64_t seed, int nthreads,
             int64_t** row_ptr_out, int32_t** col_out, int64_t* nnz_out);
int chung_lu_csr(int64_t n, int64_t m, double gamma, uint64_t seed, int nthreads, int64_t** row_ptr_out,
                 int32_t** col_out, int64_t* nnz_out);
void rmat_free(void* p);

static int fail(const char* what) {
    fprintf(stderr, "FAIL: %s\n", what);
    return 1;
}

int main(void) {
    /* K_n, one label: a connected k-vertex query has n!/(n-k)! embeddings */
    enum { N = 9 };
    int64_t rp[N + 1];
    int32_t col[N * (N - 1)], lab[N], lcol[N * (N - 1)];
    int64_t e = 0;
    for (int v = 0; v < N; ++v) {
        rp[v] = e;
        lab[v] = v % 2;
        for (int w = 0; w < N; ++w)
            if (w != v) col[e++] = w;
    }
    rp[N] = e;
    if (oracle_label_group(N, rp, col, lab, lcol, 3)) return fail("label grouping");
    /* a path u0-u1-u2-u3 with labels 0,1,0,1: 5 * 4 * 4 * 3 = 240 (five even, four odd vertices) */
    const int32_t ql[4] = {0, 1, 0, 1}, qe[6] = {0, 1, 1, 2, 2, 3};
    for (int threads = 1; threads <= 3; threads += 2) {
        for (int grouped = 0; grouped < 2; ++grouped) {
            uint64_t cnt = 0, nodes = 0, written = 0;
            int used = 0;
            int32_t rows[240 * 4];
            int st = oracle_match(N, rp, col, lab, grouped ? lcol : NULL, 4, ql, 3, qe, 1, threads, 0.0, 0, 0, 1,
                                  rows, 240, 0, &cnt, &nodes, &written, &used);
            if (st != 0 || cnt != 240 || written != 240) return fail("labelled path in K_9");
        }
    }
    /* a limit returns exactly min(total, limit) */
    {
        uint64_t cnt = 0, nodes = 0, written = 0;
        int used = 0;
        const int32_t tl[3] = {0, 0, 0}, te[6] = {0, 1, 1, 2, 0, 2};
        if (oracle_match(N, rp, col, lab, lcol, 3, tl, 3, te, 1, 2, 0.0, 0, 7, 0, NULL, 0, 0, &cnt, &nodes,
                         &written, &used) != 0 || cnt != 7)
            return fail("limit");
    }
    /* R-MAT and Chung-Lu: simple, symmetric, sorted rows; Chung-Lu with exactly m edges */
    for (int which = 0; which < 2; ++which) {
    int64_t* rrp = NULL;
    int32_t* rcol = NULL;
    int64_t nnz = 0;
    const int64_t n = which ? 1000 : 1 << 10;
    if (which == 0 && rmat_csr(10, 8, 0.57, 0.19, 0.19, 7, 3, &rrp, &rcol, &nnz)) return fail("rmat generation");
    if (which == 1 && (chung_lu_csr(n, 3000, 2.2, 9, 3, &rrp, &rcol, &nnz) || nnz != 6000))
        return fail("chung-lu generation");
    if (rrp[n] != nnz) return fail("row_ptr");
    for (int64_t v = 0; v < n; ++v)
        for (int64_t j = rrp[v]; j < rrp[v + 1]; ++j) {
            const int32_t w = rcol[j];
            if (w == v || (j > rrp[v] && rcol[j - 1] >= w)) return fail("row order");
            int found = 0;
            for (int64_t i = rrp[w]; i < rrp[w + 1]; ++i) found |= rcol[i] == (int32_t)v;
            if (!found) return fail("symmetry");
        }
    rmat_free(rrp);
    rmat_free(rcol);
    }
    printf("sanitized oracle and generator: ok\n");
    return 0;
}
