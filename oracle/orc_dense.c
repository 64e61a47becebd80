/*
 * Dense CPU oracle: greedy all-switches strategy improvement with the
 * paper's own valuation representation, for games whose priorities repeat.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  Plain single-threaded C99, built into the same
 * liborc.so as orc.c; it shares no code with the GPU path.
 *
 * Passages followed (Fearnley, "Efficient Parallel Strategy Improvement for
 * Parity Games"):
 *   - section 3, "Valuations": Val(v) is top when the play from v is
 *     infinite; otherwise it is L with L(p) = the number of vertices of
 *     priority p on the play v0 .. vk before the sink.  Two finite valuations
 *     are ordered by the largest priority p where their counts differ
 *     (Maxdiff): when p is even the larger count is the larger valuation,
 *     when p is odd the smaller count is.  Top is above every L.
 *   - section 3, "The algorithm" (sigma_init and the preprocessing) and
 *     "Switching rules" (greedy all-switches);
 *   - section 4, All_Odd and Algorithm 1;
 *   - section 4 (best responses as shortest paths) and section 6 (the
 *     best-response experiment): Bellman-Ford best responses, and SI-Reset,
 *     which starts every best response from the initial Odd strategy.
 *
 * The valuation is the natural sequential algorithm: follow each play until
 * the sink, a vertex whose valuation is already known, or a vertex of the
 * current walk (a cycle, so every vertex of the walk is top); then, back
 * along the walk, L(v) = L(succ v) plus one at pri(v).
 *
 * Priorities are handled through their sorted distinct values: values[j] is
 * the j-th smallest priority in use and counts hold one column per value, so
 * the largest differing column is Maxdiff and its value's parity decides.
 *
 * Preprocessing for this representation (a reading; the paper only asks for
 * "enough" dummy Even vertices): X, X' and the redirected edges as in orc.c,
 * but every dummy gets priority 0 and, when there is at least one dummy,
 * every original priority is raised by 2.  Order and parity of the original
 * priorities are kept and the dummies lie below all of them, so the largest
 * priority seen infinitely often on any play, hence every winner, is
 * unchanged, while the number of distinct priorities grows by at most one.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_SINK (-1)

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_EINADMISSIBLE = 2, ORC_EITERLIMIT = 3,
       ORC_ENOMEM = 4 };

/* orc.c */
int64_t orc_x_sets(int64_t n, const int64_t *off, const int32_t *tgt,
                   const uint8_t *owner, uint8_t *in_x, uint8_t *in_xp);
uint64_t orc_hash(int64_t len, const int32_t *a);

/* ------------------------------------------------------------------------ */
/* preprocessing                                                             */
/* ------------------------------------------------------------------------ */

/*
 * The modified game: n + |X'| vertices, m + |X'| edges (the caller sizes the
 * outputs for 2n vertices and m + n edges).  Dummy d_w of the i-th w in X'
 * (increasing w) has id n + i, the single row [w] and priority 0.  Returns
 * n + |X'|, or -1 on a priority overflow or an allocation failure.
 */
int64_t orc_dense_preprocess(int64_t n, const int64_t *off,
                             const int32_t *tgt, const uint8_t *owner,
                             const int32_t *pri, int64_t *off2,
                             int32_t *tgt2, uint8_t *owner2, int32_t *pri2,
                             int32_t *dummy_of)
{
    uint8_t *in_x = (uint8_t *)malloc((size_t)n);
    uint8_t *in_xp = (uint8_t *)malloc((size_t)n);
    int32_t *did = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t v, e, nxp, shift, m = off[n], i = 0;
    int bad = !in_x || !in_xp || !did;
    if (!bad) {
        nxp = orc_x_sets(n, off, tgt, owner, in_x, in_xp);
        bad = nxp < 0;
    }
    if (bad) { free(in_x); free(in_xp); free(did); return -1; }
    shift = nxp > 0 ? 2 : 0;
    for (v = 0; v < n; ++v) {
        did[v] = -1;
        if (in_xp[v]) { did[v] = (int32_t)(n + i); dummy_of[i] = (int32_t)v; ++i; }
        if ((int64_t)pri[v] + shift > 2147483647LL) bad = 1;
    }
    if (bad) { free(in_x); free(in_xp); free(did); return -1; }
    for (v = 0; v <= n; ++v) off2[v] = off[v];
    for (v = 0; v < n; ++v) {
        for (e = off[v]; e < off[v + 1]; ++e) {
            int32_t w = tgt[e];
            tgt2[e] = (in_x[v] && in_x[w]) ? did[w] : w;
        }
        owner2[v] = owner[v];
        pri2[v] = (int32_t)(pri[v] + shift);
    }
    for (v = 0; v < nxp; ++v) {
        off2[n + v + 1] = m + v + 1;
        tgt2[m + v] = dummy_of[v];
        owner2[n + v] = 0;
        pri2[n + v] = 0;
    }
    free(in_x); free(in_xp); free(did);
    return n + nxp;
}

/* ------------------------------------------------------------------------ */
/* priorities in use                                                         */
/* ------------------------------------------------------------------------ */

static int cmp_i32(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

/*
 * values[0..d) = the distinct priorities in increasing order (values needs
 * room for n entries); idx[v] = the position of pri[v] in values.  Returns d.
 */
int64_t orc_dense_priorities(int64_t n, const int32_t *pri, int32_t *values,
                             int32_t *idx)
{
    int64_t v, d = 0;
    memcpy(values, pri, sizeof(int32_t) * (size_t)n);
    qsort(values, (size_t)n, sizeof(int32_t), cmp_i32);
    for (v = 0; v < n; ++v)
        if (d == 0 || values[v] != values[d - 1]) values[d++] = values[v];
    for (v = 0; v < n; ++v) {
        int64_t lo = 0, hi = d - 1;
        while (lo < hi) {
            int64_t mid = (lo + hi) / 2;
            if (values[mid] < pri[v]) lo = mid + 1; else hi = mid;
        }
        idx[v] = (int32_t)lo;
    }
    return d;
}

/* ------------------------------------------------------------------------ */
/* valuation                                                                 */
/* ------------------------------------------------------------------------ */

/*
 * succ[v]: the successor under (sigma, tau), ORC_SINK for the sink.
 * counts: (n + 1) rows of d columns; row n is the sink (all zero), the rows
 * of top vertices are zero too.  top[v] = 1 when the play from v is infinite.
 * Returns ORC_EINADMISSIBLE when a cycle's largest priority is odd (sigma is
 * not admissible, section 3), else ORC_OK; the outputs are complete either
 * way.
 */
int orc_dense_valuation(int64_t n, const int32_t *succ, const int32_t *idx,
                        int64_t d, const int32_t *values, int32_t *counts,
                        uint8_t *top)
{
    uint8_t *state = (uint8_t *)calloc((size_t)(n ? n : 1), 1);
    int32_t *walk = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int64_t v, j;
    int rc = ORC_OK;
    if (!state || !walk) { free(state); free(walk); return ORC_ENOMEM; }
    memset(counts, 0, sizeof(int32_t) * (size_t)((n + 1) * d));
    for (v = 0; v < n; ++v) {
        int64_t len = 0;
        int32_t x = (int32_t)v;
        int is_top;
        const int32_t *base;
        if (state[v]) continue;
        /* state: 0 unseen, 1 on the current walk, 2 done */
        while (x != ORC_SINK && state[x] == 0) {
            state[x] = 1;
            walk[len++] = x;
            x = succ[x];
        }
        if (x == ORC_SINK) {
            is_top = 0;
            base = counts + n * d;
        } else if (state[x] == 2) {
            is_top = top[x];
            base = counts + (int64_t)x * d;
        } else {
            /* the walk closed a cycle: x .. walk[len-1] */
            int32_t mx = -1;
            int64_t i = len - 1;
            for (;;) {
                if (idx[walk[i]] > mx) mx = idx[walk[i]];
                if (walk[i] == x) break;
                --i;
            }
            if (values[mx] & 1) rc = ORC_EINADMISSIBLE;
            is_top = 1;
            base = NULL;
        }
        while (len > 0) {
            int32_t y = walk[--len];
            state[y] = 2;
            top[y] = (uint8_t)is_top;
            if (!is_top) {
                int32_t *row = counts + (int64_t)y * d;
                for (j = 0; j < d; ++j) row[j] = base[j];
                row[idx[y]] += 1;
                base = row;
            }
        }
    }
    free(state);
    free(walk);
    return rc;
}

/*
 * Compares Val(a) with Val(b) (a, b in [0, n], n being the sink): -1 when
 * Val(a) is strictly below, 0 when equal (top equals top), 1 when above.
 */
static int dense_cmp(int64_t n, int64_t d, const int32_t *values,
                     const int32_t *counts, const uint8_t *top, int64_t a,
                     int64_t b)
{
    int ta = a < n ? top[a] : 0, tb = b < n ? top[b] : 0;
    const int32_t *la, *lb;
    int64_t j;
    if (ta || tb) return ta == tb ? 0 : (ta ? 1 : -1);
    la = counts + a * d;
    lb = counts + b * d;
    for (j = d - 1; j >= 0; --j) {
        if (la[j] != lb[j]) {
            int even = (values[j] & 1) == 0;
            return ((la[j] < lb[j]) == even) ? -1 : 1;
        }
    }
    return 0;
}

/* three-way comparison exported for the tests */
int orc_dense_compare(int64_t n, int64_t d, const int32_t *values,
                      const int32_t *counts, const uint8_t *top, int64_t a,
                      int64_t b)
{
    return dense_cmp(n, d, values, counts, top, a, b);
}

/* ------------------------------------------------------------------------ */
/* switching                                                                 */
/* ------------------------------------------------------------------------ */

/* All_Odd: each Odd vertex takes the first successor of least valuation if
   that is strictly below its current choice.  Returns the switch count. */
int64_t orc_dense_odd_switch(int64_t n, const int64_t *off,
                             const int32_t *tgt, const uint8_t *owner,
                             int64_t d, const int32_t *values,
                             const int32_t *counts, const uint8_t *top,
                             int32_t *tau)
{
    int64_t v, e, count = 0;
    for (v = 0; v < n; ++v) {
        int32_t best;
        if (owner[v] != 1) continue;
        best = tgt[off[v]];
        for (e = off[v] + 1; e < off[v + 1]; ++e)
            if (dense_cmp(n, d, values, counts, top, tgt[e], best) < 0)
                best = tgt[e];
        if (dense_cmp(n, d, values, counts, top, best, tau[v]) < 0) {
            tau[v] = best;
            ++count;
        }
    }
    return count;
}

/* All_Even: options are the sink, then the row; the first greatest
   valuation wins if it is strictly above the current choice. */
int64_t orc_dense_even_switch(int64_t n, const int64_t *off,
                              const int32_t *tgt, const uint8_t *owner,
                              int64_t d, const int32_t *values,
                              const int32_t *counts, const uint8_t *top,
                              int32_t *sigma)
{
    int64_t v, e, count = 0;
    for (v = 0; v < n; ++v) {
        int64_t best = n, cur;
        if (owner[v] != 0) continue;
        for (e = off[v]; e < off[v + 1]; ++e)
            if (dense_cmp(n, d, values, counts, top, tgt[e], best) > 0)
                best = tgt[e];
        cur = sigma[v] < 0 ? n : sigma[v];
        if (dense_cmp(n, d, values, counts, top, best, cur) > 0) {
            sigma[v] = best == n ? ORC_SINK : (int32_t)best;
            ++count;
        }
    }
    return count;
}

/*
 * Bellman-Ford best response against sigma (section 4: with sigma
 * admissible, a best response is a shortest path to the sink for each vertex
 * under the valuation order, odd priorities acting as negative weights).
 * Labels are count vectors; a vertex without a path to the sink yet has no
 * label, which compares as top.  Jacobi rounds: every vertex recomputes its
 * label from the previous round's labels -- an Even vertex from sigma(v), an
 * Odd vertex from the least labelled successor -- plus one at pri(v), until
 * a round changes nothing (that round is counted).  Then tau(v) is the first
 * row position of least final label, counts/top hold the labels as
 * valuations (no label = top), and the number of rounds is returned.
 */
int64_t orc_dense_bellman_ford(int64_t n, const int64_t *off,
                               const int32_t *tgt, const uint8_t *owner,
                               const int32_t *idx, int64_t d,
                               const int32_t *values, const int32_t *sigma,
                               int32_t *tau, int32_t *counts, uint8_t *top)
{
    size_t rows = (size_t)(n + 1) * (size_t)(d ? d : 1);
    int32_t *nl = (int32_t *)calloc(rows, sizeof(int32_t));
    uint8_t *ntop = (uint8_t *)malloc((size_t)(n ? n : 1));
    int64_t v, e, j, rounds = 0;
    int changed = 1;
    if (!nl || !ntop) { free(nl); free(ntop); return -1; }
    memset(counts, 0, sizeof(int32_t) * rows);
    for (v = 0; v < n; ++v) top[v] = 1;
    while (changed) {
        changed = 0;
        ++rounds;
        for (v = 0; v < n; ++v) {
            int64_t best = -1;
            int32_t *row = nl + v * d;
            if (owner[v] == 0) {
                best = sigma[v] < 0 ? n : sigma[v];
                if (best < n && top[best]) best = -1;
            } else {
                for (e = off[v]; e < off[v + 1]; ++e) {
                    int64_t u = tgt[e];
                    if (top[u]) continue;
                    if (best < 0 ||
                        dense_cmp(n, d, values, counts, top, u, best) < 0)
                        best = u;
                }
            }
            ntop[v] = best < 0;
            for (j = 0; j < d; ++j)
                row[j] = best < 0 ? 0 : counts[best * d + j];
            if (best >= 0) row[idx[v]] += 1;
        }
        for (v = 0; v < n; ++v) {
            if (ntop[v] != top[v]) changed = 1;
            for (j = 0; j < d && !changed; ++j)
                if (nl[v * d + j] != counts[v * d + j]) changed = 1;
        }
        for (v = 0; v < n; ++v) {
            top[v] = ntop[v];
            for (j = 0; j < d; ++j) counts[v * d + j] = nl[v * d + j];
        }
    }
    for (v = 0; v < n; ++v) {
        int32_t best;
        if (owner[v] != 1) continue;
        best = tgt[off[v]];
        for (e = off[v] + 1; e < off[v + 1]; ++e)
            if (dense_cmp(n, d, values, counts, top, tgt[e], best) < 0)
                best = tgt[e];
        tau[v] = best;
    }
    free(nl); free(ntop);
    return rounds;
}

typedef struct {
    int64_t n_major;
    int64_t n_valuations;
    int64_t n_even_switches;
    int64_t n_odd_switches;
} orc_dense_stats;

enum { ORC_BR_SI = 0, ORC_BR_SI_RESET = 1, ORC_BR_BELLMAN_FORD = 2 };

/*
 * Algorithm 1 on the (already modified) game, as orc_solve but with count
 * valuations.  sigma/tau are in-out (the caller passes the initial
 * strategies); counts[(n+1)*d] and top[n] receive the last valuation
 * (d = number of distinct priorities, values[] as orc_dense_priorities
 * returns them).  trace (nullable, capacity trace_cap) receives, per
 * valuation, the hash of its counts followed by the hash of its top flags.
 * br selects the best response: ORC_BR_SI (Algorithm 1), ORC_BR_SI_RESET
 * (each best response starts from the initial Odd strategy) or
 * ORC_BR_BELLMAN_FORD (orc_dense_bellman_ford; n_valuations then counts its
 * rounds and nothing is traced).
 */
int orc_dense_solve(int64_t n, const int64_t *off, const int32_t *tgt,
                    const uint8_t *owner, const int32_t *pri,
                    int64_t max_major, int64_t max_inner, int br,
                    int32_t *sigma, int32_t *tau, int32_t *counts,
                    uint8_t *top, orc_dense_stats *st, uint64_t *trace,
                    int64_t trace_cap)
{
    size_t nn = (size_t)(n ? n : 1);
    int32_t *succ = (int32_t *)malloc(sizeof(int32_t) * nn);
    int32_t *values = (int32_t *)malloc(sizeof(int32_t) * nn);
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * nn);
    int32_t *top32 = (int32_t *)malloc(sizeof(int32_t) * nn);
    int64_t v, d, nval = 0, nmaj = 0, ev = 0, od = 0;
    int rc = ORC_OK;
    if (!succ || !values || !idx || !top32) {
        free(succ); free(values); free(idx); free(top32);
        return ORC_ENOMEM;
    }
    d = orc_dense_priorities(n, pri, values, idx);
    for (;;) {
        int64_t inner = 0, c;
        if (max_major > 0 && nmaj >= max_major) { rc = ORC_EITERLIMIT; break; }
        ++nmaj;
        if (br == ORC_BR_SI_RESET)
            for (v = 0; v < n; ++v)
                if (owner[v]) tau[v] = tgt[off[v]];
        if (br == ORC_BR_BELLMAN_FORD) {
            int64_t r = orc_dense_bellman_ford(n, off, tgt, owner, idx, d,
                                               values, sigma, tau, counts, top);
            if (r < 0) { rc = ORC_ENOMEM; break; }
            nval += r;
        } else
        for (;;) {
            if (max_inner > 0 && inner >= max_inner) { rc = ORC_EITERLIMIT; break; }
            for (v = 0; v < n; ++v) succ[v] = owner[v] ? tau[v] : sigma[v];
            rc = orc_dense_valuation(n, succ, idx, d, values, counts, top);
            if (trace && 2 * nval + 1 < trace_cap) {
                for (v = 0; v < n; ++v) top32[v] = top[v];
                trace[2 * nval] = orc_hash((n + 1) * d, counts);
                trace[2 * nval + 1] = orc_hash(n, top32);
            }
            ++nval; ++inner;
            if (rc != ORC_OK) break;
            c = orc_dense_odd_switch(n, off, tgt, owner, d, values, counts,
                                     top, tau);
            od += c;
            if (c == 0) break;
        }
        if (rc != ORC_OK) break;
        c = orc_dense_even_switch(n, off, tgt, owner, d, values, counts, top,
                                  sigma);
        ev += c;
        if (c == 0) break;
    }
    if (st) { st->n_major = nmaj; st->n_valuations = nval;
              st->n_even_switches = ev; st->n_odd_switches = od; }
    free(succ); free(values); free(idx); free(top32);
    return rc;
}
