/*
 * Test driver for the sanitizer run of the CPU code (tests/test_sanitize.py):
 * the C oracle (oracle/orc.c, oracle/orc_dense.c) and the CPU-LR baseline
 * (baselines/cpu_lr.c) are built together with this file under
 * AddressSanitizer and UndefinedBehaviorSanitizer, run on a game read from a
 * file, and the results printed here are compared by the test with those of
 * the regular builds.  Host code only; nothing here touches a GPU.
 *
 * Input file (little endian): int64 n, int64 m, int64 offsets[n+1],
 * int32 targets[m], uint8 owner[n], int32 pri[n] (distinct), int32
 * pri_few[n] (a handful of repeated values).
 * Output: one "name value..." line per result.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n_major, n_valuations, n_even_switches, n_odd_switches;
} drv_stats;

int64_t orc_preprocess(int64_t n, const int64_t *off, const int32_t *tgt,
                       const uint8_t *owner, const int32_t *pri,
                       int64_t *off2, int32_t *tgt2, uint8_t *owner2,
                       int32_t *pri2, int32_t *dummy_of);
int orc_solve(int64_t n, const int64_t *off, const int32_t *tgt,
              const uint8_t *owner, const int32_t *pri, int method,
              int64_t max_major, int64_t max_inner, int reset,
              int32_t *sigma, int32_t *tau, int32_t *key, drv_stats *st,
              uint64_t *trace, int64_t trace_cap);
uint64_t orc_hash(int64_t len, const int32_t *a);
void orc_order_by_pri(int64_t n, const int32_t *pri, int32_t *by_pri);
int64_t orc_dense_preprocess(int64_t n, const int64_t *off,
                             const int32_t *tgt, const uint8_t *owner,
                             const int32_t *pri, int64_t *off2,
                             int32_t *tgt2, uint8_t *owner2, int32_t *pri2,
                             int32_t *dummy_of);
int64_t orc_dense_priorities(int64_t n, const int32_t *pri, int32_t *values,
                             int32_t *idx);
int orc_dense_solve(int64_t n, const int64_t *off, const int32_t *tgt,
                    const uint8_t *owner, const int32_t *pri,
                    int64_t max_major, int64_t max_inner, int br,
                    int32_t *sigma, int32_t *tau, int32_t *counts,
                    uint8_t *top, drv_stats *st, uint64_t *trace,
                    int64_t trace_cap);
int cl_valuation(int64_t n, const int32_t *succ, const int32_t *pri,
                 const int32_t *by_pri, const int32_t *by_signed,
                 int threads, int32_t *key, int64_t *n_finite);
int64_t cl_odd_switch(int64_t n, const int64_t *off, const int32_t *tgt,
                      const uint8_t *owner, const int32_t *key, int32_t *tau,
                      int threads);

static void *xmalloc(size_t bytes)
{
    void *p = malloc(bytes ? bytes : 1);
    if (!p) { fprintf(stderr, "out of memory\n"); exit(3); }
    return p;
}

static void rd(FILE *f, void *p, size_t size, size_t count)
{
    if (count && fread(p, size, count, f) != count) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
}

typedef struct {
    int64_t n, m;
    int64_t *off;
    int32_t *tgt, *pri;
    uint8_t *own;
} game;

/* signed-priority order: odd priorities descending, then even ascending */
static const int32_t *g_pri;
static int cmp_signed(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    int64_t ka = (g_pri[a] & 1) ? -(int64_t)g_pri[a]
                                : (int64_t)g_pri[a] + ((int64_t)1 << 40);
    int64_t kb = (g_pri[b] & 1) ? -(int64_t)g_pri[b]
                                : (int64_t)g_pri[b] + ((int64_t)1 << 40);
    return ka < kb ? -1 : (ka > kb ? 1 : 0);
}

int main(int argc, char **argv)
{
    if (argc != 2) { fprintf(stderr, "usage: %s game.bin\n", argv[0]); return 2; }
    FILE *f = fopen(argv[1], "rb");
    if (!f) { perror("open"); return 2; }
    game g;
    rd(f, &g.n, 8, 1);
    rd(f, &g.m, 8, 1);
    g.off = xmalloc(8 * (size_t)(g.n + 1));
    g.tgt = xmalloc(4 * (size_t)g.m);
    g.own = xmalloc((size_t)g.n);
    g.pri = xmalloc(4 * (size_t)g.n);
    int32_t *pri_few = xmalloc(4 * (size_t)g.n);
    rd(f, g.off, 8, (size_t)g.n + 1);
    rd(f, g.tgt, 4, (size_t)g.m);
    rd(f, g.own, 1, (size_t)g.n);
    rd(f, g.pri, 4, (size_t)g.n);
    rd(f, pri_few, 4, (size_t)g.n);
    fclose(f);

    /* the modified game (rank path), sized for 2n vertices, m + n edges */
    game a;
    a.off = xmalloc(8 * (size_t)(2 * g.n + 1));
    a.tgt = xmalloc(4 * (size_t)(g.m + g.n));
    a.own = xmalloc((size_t)(2 * g.n));
    a.pri = xmalloc(4 * (size_t)(2 * g.n));
    int32_t *dum = xmalloc(4 * (size_t)g.n);
    a.n = orc_preprocess(g.n, g.off, g.tgt, g.own, g.pri, a.off, a.tgt,
                         a.own, a.pri, dum);
    if (a.n < 0) { fprintf(stderr, "preprocess failed\n"); return 1; }
    a.m = a.off[a.n];
    printf("n_aug %lld %lld\n", (long long)a.n, (long long)a.m);

    int32_t *sigma = xmalloc(4 * (size_t)a.n), *tau = xmalloc(4 * (size_t)a.n);
    int32_t *key = xmalloc(4 * (size_t)(a.n + 1));
    uint64_t trace[4096];
    for (int method = 0; method < 2; ++method) {
        for (int64_t v = 0; v < a.n; ++v) {
            sigma[v] = -1;
            tau[v] = a.own[v] ? a.tgt[a.off[v]] : -1;
        }
        drv_stats st;
        memset(&st, 0, sizeof st);
        int rc = orc_solve(a.n, a.off, a.tgt, a.own, a.pri, method, 0, 0, 0,
                           sigma, tau, key, &st, trace, 4096);
        printf("solve%d %d %lld %lld %lld %lld %llu %llu %llu\n", method, rc,
               (long long)st.n_major, (long long)st.n_valuations,
               (long long)st.n_odd_switches, (long long)st.n_even_switches,
               (unsigned long long)orc_hash(a.n, sigma),
               (unsigned long long)orc_hash(a.n, tau),
               (unsigned long long)orc_hash(a.n + 1, key));
        printf("trace%d", method);
        for (int64_t i = 0; i < st.n_valuations && i < 4096; ++i)
            printf(" %llu", (unsigned long long)trace[i]);
        printf("\n");
    }

    /* CPU-LR: the first best response from the initial strategies */
    int32_t *by_pri = xmalloc(4 * (size_t)a.n), *by_signed = xmalloc(4 * (size_t)a.n);
    int32_t *succ = xmalloc(4 * (size_t)a.n);
    orc_order_by_pri(a.n, a.pri, by_pri);
    for (int64_t v = 0; v < a.n; ++v) by_signed[v] = (int32_t)v;
    g_pri = a.pri;
    qsort(by_signed, (size_t)a.n, sizeof(int32_t), cmp_signed);
    for (int64_t v = 0; v < a.n; ++v) {
        sigma[v] = -1;
        tau[v] = a.own[v] ? a.tgt[a.off[v]] : -1;
    }
    printf("cpulr");
    for (int it = 0; it < 64; ++it) {
        for (int64_t v = 0; v < a.n; ++v) succ[v] = a.own[v] ? tau[v] : sigma[v];
        int64_t nf = 0;
        int rc = cl_valuation(a.n, succ, a.pri, by_pri, by_signed, 2, key, &nf);
        if (rc) { printf(" rc%d", rc); break; }
        printf(" %llu", (unsigned long long)orc_hash(a.n + 1, key));
        if (cl_odd_switch(a.n, a.off, a.tgt, a.own, key, tau, 2) == 0) break;
    }
    printf("\n");

    /* count valuations on the few-priorities version of the game */
    game b;
    b.off = xmalloc(8 * (size_t)(2 * g.n + 1));
    b.tgt = xmalloc(4 * (size_t)(g.m + g.n));
    b.own = xmalloc((size_t)(2 * g.n));
    b.pri = xmalloc(4 * (size_t)(2 * g.n));
    b.n = orc_dense_preprocess(g.n, g.off, g.tgt, g.own, pri_few, b.off, b.tgt,
                               b.own, b.pri, dum);
    if (b.n < 0) { fprintf(stderr, "dense preprocess failed\n"); return 1; }
    int32_t *values = xmalloc(4 * (size_t)b.n);  /* room for n entries */
    int32_t *idx = xmalloc(4 * (size_t)b.n);
    int64_t d = orc_dense_priorities(b.n, b.pri, values, idx);
    int32_t *counts = xmalloc(4 * (size_t)((b.n + 1) * d));
    uint8_t *top = xmalloc((size_t)b.n);
    int32_t *sig2 = xmalloc(4 * (size_t)b.n), *tau2 = xmalloc(4 * (size_t)b.n);
    for (int br = 0; br < 3; ++br) {
        for (int64_t v = 0; v < b.n; ++v) {
            sig2[v] = -1;
            tau2[v] = b.own[v] ? b.tgt[b.off[v]] : -1;
        }
        drv_stats st;
        memset(&st, 0, sizeof st);
        int rc = orc_dense_solve(b.n, b.off, b.tgt, b.own, b.pri, 0, 0, br,
                                 sig2, tau2, counts, top, &st, NULL, 0);
        printf("dense%d %d %lld %lld %llu %llu\n", br, rc,
               (long long)st.n_major, (long long)st.n_valuations,
               (unsigned long long)orc_hash(b.n, sig2),
               (unsigned long long)orc_hash((b.n + 1) * d, counts));
    }
    free(g.off); free(g.tgt); free(g.own); free(g.pri); free(pri_few);
    free(a.off); free(a.tgt); free(a.own); free(a.pri); free(dum);
    free(sigma); free(tau); free(key); free(by_pri); free(by_signed); free(succ);
    free(b.off); free(b.tgt); free(b.own); free(b.pri); free(idx);
    free(counts); free(top); free(sig2); free(tau2); free(values);
    return 0;
}
