/*
 * Scalable CPU oracle for greedy all-switches strategy improvement on parity
 * games with pairwise distinct priorities.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  Plain single-threaded C99, written for a reader
 * who has the paper (Fearnley, "Efficient Parallel Strategy Improvement for
 * Parity Games") at hand; it shares no code with the GPU path.
 *
 * What it computes, passage by passage:
 *   - preprocessing (section 3, "The algorithm"): dummy Even vertices so that
 *     Odd cannot close an Odd-only cycle against sigma_init;
 *   - Algorithm 1 (section 4): the outer loop switches Even by greedy
 *     all-switches (section 3, "Switching rules"), the inner loop computes a
 *     best response by one-player SI switching All_Odd (section 4);
 *   - valuations (section 3, "Valuations"): top for an infinite play, else
 *     the multiset of priorities on the path to the sink, ordered by Maxdiff.
 *
 * Valuation representation.  Priorities are pairwise distinct, so a finite
 * valuation is the set of priorities on a simple path to the sink and two
 * such sets differ exactly on the vertices of the tree path between the two
 * starting vertices (the common part above their meeting point cancels).
 * Maxdiff is the largest priority on that tree path.  The oracle stores, for
 * every vertex, its rank among all finite vertices (the sink included, with
 * the zero valuation) and KEY_TOP for top; comparing ranks is comparing
 * valuations.  Two independent constructions of the rank are provided:
 *
 *   ORC_RANK_PATHSORT  a comparison sort whose comparator walks both tree
 *                      paths up to their meeting point and applies the
 *                      Maxdiff rule to the largest priority it met -- the
 *                      definition written out (cost grows with tree depth);
 *   ORC_RANK_KRUSKAL   merging tree edges (x, succ x) in increasing pri(x)
 *                      with union-find; each merge makes a node whose two
 *                      sides are ordered by the parity of pri(x).  When the
 *                      edge of x merges two parts, every pair split by it
 *                      has x as the largest vertex of its tree path, on the
 *                      side of the vertex whose subtree holds x; Maxdiff says
 *                      that side is larger iff pri(x) is even.
 *
 * Readings where the paper is open (also in the design notes): see
 * oracle/literal.py; this file follows the same ones.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_SINK (-1)
#define ORC_KEY_TOP 2147483647

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_EINADMISSIBLE = 2, ORC_EITERLIMIT = 3,
       ORC_ENOMEM = 4 };
enum { ORC_RANK_KRUSKAL = 0, ORC_RANK_PATHSORT = 1 };

/* ------------------------------------------------------------------------ */
/* preprocessing                                                             */
/* ------------------------------------------------------------------------ */

/*
 * X  = largest set of Odd vertices each having a successor in X;
 * X' = members of X with a predecessor in X.
 * Writes in_x[n] and in_xp[n]; returns |X'|.
 */
int64_t orc_x_sets(int64_t n, const int64_t *off, const int32_t *tgt,
                   const uint8_t *owner, uint8_t *in_x, uint8_t *in_xp)
{
    int64_t m = off[n];
    int64_t *cnt = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    int64_t *poff = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *pred = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    int64_t *fill = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int64_t qh = 0, qt = 0, v, e, nxp = 0;
    if (!cnt || !poff || !pred || !fill || !queue) {
        free(cnt); free(poff); free(pred); free(fill); free(queue);
        return -1;
    }
    for (v = 0; v < n; ++v) in_x[v] = owner[v] == 1;
    /* predecessor lists */
    for (e = 0; e < m; ++e) poff[tgt[e] + 1]++;
    for (v = 0; v < n; ++v) poff[v + 1] += poff[v];
    for (v = 0; v < n; ++v)
        for (e = off[v]; e < off[v + 1]; ++e)
            pred[poff[tgt[e]] + fill[tgt[e]]++] = (int32_t)v;
    /* count successors in X; drop Odd vertices whose count reaches zero */
    for (v = 0; v < n; ++v) {
        if (!in_x[v]) continue;
        for (e = off[v]; e < off[v + 1]; ++e) cnt[v] += in_x[tgt[e]];
    }
    for (v = 0; v < n; ++v)
        if (in_x[v] && cnt[v] == 0) { in_x[v] = 0; queue[qt++] = (int32_t)v; }
    while (qh < qt) {
        int32_t w = queue[qh++];
        for (e = poff[w]; e < poff[w + 1]; ++e) {
            int32_t u = pred[e];
            if (!in_x[u]) continue;
            if (--cnt[u] == 0) { in_x[u] = 0; queue[qt++] = u; }
        }
    }
    memset(in_xp, 0, (size_t)n);
    for (v = 0; v < n; ++v) {
        if (!in_x[v]) continue;
        for (e = off[v]; e < off[v + 1]; ++e)
            if (in_x[tgt[e]]) in_xp[tgt[e]] = 1;
    }
    for (v = 0; v < n; ++v) nxp += in_xp[v];
    free(cnt); free(poff); free(pred); free(fill); free(queue);
    return nxp;
}

/*
 * Build the modified game.  Output buffers must hold n + |X'| vertices and
 * m + |X'| edges.  Dummy d_w (for the i-th w of X' in increasing order) has
 * id n + i, owner Even, priority i and the single row [w]; edges (u, w) with
 * u, w in X are redirected to d_w; original priorities are shifted by K =
 * |X'| rounded up to even.  Returns n_aug, or -1 on overflow of int32
 * priorities / allocation failure.
 */
int64_t orc_preprocess(int64_t n, const int64_t *off, const int32_t *tgt,
                       const uint8_t *owner, const int32_t *pri,
                       int64_t *off2, int32_t *tgt2, uint8_t *owner2,
                       int32_t *pri2, int32_t *dummy_of)
{
    uint8_t *in_x = (uint8_t *)malloc((size_t)n);
    uint8_t *in_xp = (uint8_t *)malloc((size_t)n);
    int32_t *did = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t v, e, nxp, k, m = off[n];
    if (!in_x || !in_xp || !did) { free(in_x); free(in_xp); free(did); return -1; }
    nxp = orc_x_sets(n, off, tgt, owner, in_x, in_xp);
    if (nxp < 0) { free(in_x); free(in_xp); free(did); return -1; }
    k = nxp + (nxp & 1);
    {
        int64_t i = 0;
        for (v = 0; v < n; ++v) {
            did[v] = -1;
            if (in_xp[v]) { did[v] = (int32_t)(n + i); dummy_of[i] = (int32_t)v; ++i; }
        }
    }
    for (v = 0; v < n; ++v) {
        if ((int64_t)pri[v] + k > 2147483647LL) {
            free(in_x); free(in_xp); free(did); return -1;
        }
    }
    for (v = 0; v <= n; ++v) off2[v] = off[v];
    for (v = 0; v < n; ++v) {
        for (e = off[v]; e < off[v + 1]; ++e) {
            int32_t w = tgt[e];
            tgt2[e] = (in_x[v] && in_x[w]) ? did[w] : w;
        }
        owner2[v] = owner[v];
        pri2[v] = (int32_t)(pri[v] + k);
    }
    for (v = 0; v < nxp; ++v) {
        off2[n + v + 1] = m + v + 1;
        tgt2[m + v] = dummy_of[v];
        owner2[n + v] = 0;
        pri2[n + v] = (int32_t)v;
    }
    free(in_x); free(in_xp); free(did);
    return n + nxp;
}

/* ------------------------------------------------------------------------ */
/* valuation                                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    const int32_t *succ; /* successor or ORC_SINK */
    const int32_t *pri;
    const int32_t *depth; /* tree depth (sink = 0) */
} path_ctx;

static path_ctx g_ctx; /* the comparator's context (single-threaded) */

/* -1 if Val(a) is below Val(b), +1 if above; a, b finite, n means the sink */
static int path_cmp(int32_t a, int32_t b)
{
    const path_ctx *c = &g_ctx;
    int32_t best = -1, best_side = 0; /* side 1 = a, 2 = b */
    int32_t da, db;
    if (a == b) return 0;
    da = (a == c->n) ? 0 : c->depth[a];
    db = (b == c->n) ? 0 : c->depth[b];
    while (da > db) {
        if (best < 0 || c->pri[a] > c->pri[best]) { best = a; best_side = 1; }
        a = c->succ[a] < 0 ? (int32_t)c->n : c->succ[a];
        --da;
    }
    while (db > da) {
        if (best < 0 || c->pri[b] > c->pri[best]) { best = b; best_side = 2; }
        b = c->succ[b] < 0 ? (int32_t)c->n : c->succ[b];
        --db;
    }
    while (a != b) {
        if (best < 0 || c->pri[a] > c->pri[best]) { best = a; best_side = 1; }
        if (c->pri[b] > c->pri[best]) { best = b; best_side = 2; }
        a = c->succ[a] < 0 ? (int32_t)c->n : c->succ[a];
        b = c->succ[b] < 0 ? (int32_t)c->n : c->succ[b];
    }
    /* Maxdiff = pri(best); it occurs once, on best_side's path only */
    if (c->pri[best] % 2 == 0) return best_side == 1 ? 1 : -1;
    return best_side == 1 ? -1 : 1;
}

static int path_qsort_cmp(const void *x, const void *y)
{
    return path_cmp(*(const int32_t *)x, *(const int32_t *)y);
}

static int64_t uf_find(int64_t *par, int64_t x)
{
    int64_t r = x, t;
    while (par[r] != r) r = par[r];
    while (par[x] != r) { t = par[x]; par[x] = r; x = t; }
    return r;
}

/*
 * Val^{sigma,tau} as ranks.  succ[v] is the play successor (ORC_SINK for the
 * sink).  by_pri lists the vertices in increasing priority (only used by the
 * Kruskal method; may be NULL for the path sort).  key[n+1] receives ranks,
 * ORC_KEY_TOP for an infinite play, and the sink's rank at key[n].
 * Returns ORC_OK, or ORC_EINADMISSIBLE when some cycle has an odd largest
 * priority (an inadmissible sigma, section 3 "Admissible strategies").
 * n_finite (nullable) receives the number of finite vertices (sink included).
 */
int orc_valuation(int64_t n, const int32_t *succ, const int32_t *pri,
                  const int32_t *by_pri, int method, int32_t *key,
                  int64_t *n_finite)
{
    /* state: 0 unseen, 1 on the current walk, 2 finite, 3 top */
    uint8_t *state = (uint8_t *)calloc((size_t)n, 1);
    int32_t *depth = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int32_t *walk = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int64_t v, nf = 1;
    int rc = ORC_OK;
    if (!state || !depth || !walk) { free(state); free(depth); free(walk); return ORC_ENOMEM; }
    for (v = 0; v < n; ++v) {
        int64_t len = 0, i;
        int32_t u = (int32_t)v;
        int32_t base_depth;
        uint8_t fate;
        if (state[v]) continue;
        while (u != ORC_SINK && state[u] == 0) {
            state[u] = 1;
            walk[len++] = u;
            u = succ[u];
        }
        if (u == ORC_SINK) { fate = 2; base_depth = 0; }
        else if (state[u] == 2) { fate = 2; base_depth = depth[u]; }
        else if (state[u] == 3) { fate = 3; base_depth = 0; }
        else {
            /* state 1: the walk closed a cycle at u; its largest priority
               must be even for an admissible sigma */
            int32_t mx = -1;
            for (i = len - 1; i >= 0; --i) {
                if (pri[walk[i]] > mx) mx = pri[walk[i]];
                if (walk[i] == u) break;
            }
            if (mx % 2 != 0) rc = ORC_EINADMISSIBLE;
            fate = 3; base_depth = 0;
        }
        for (i = len - 1; i >= 0; --i) {
            state[walk[i]] = fate;
            if (fate == 2) depth[walk[i]] = base_depth + (int32_t)(len - i);
        }
    }
    for (v = 0; v < n; ++v) {
        key[v] = ORC_KEY_TOP;
        if (state[v] == 2) ++nf;
    }
    if (method == ORC_RANK_PATHSORT) {
        int32_t *items = (int32_t *)malloc(sizeof(int32_t) * (size_t)nf);
        int64_t k = 0;
        for (v = 0; v < n; ++v) if (state[v] == 2) items[k++] = (int32_t)v;
        items[k++] = (int32_t)n;
        g_ctx.n = n; g_ctx.succ = succ; g_ctx.pri = pri; g_ctx.depth = depth;
        qsort(items, (size_t)nf, sizeof(int32_t), path_qsort_cmp);
        for (k = 0; k < nf; ++k) key[items[k]] = (int32_t)k;
        free(items);
    } else {
        /* leaves 0..n (n = the sink); internal nodes n+1 .. */
        int64_t nodes = n + 1 + (nf - 1);
        int64_t *par = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
        int64_t *top = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
        int64_t *lc = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nodes - n));
        int64_t *rc2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nodes - n));
        int64_t *stack = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nodes + 1));
        int64_t next = n + 1, i, sp = 0, rank = 0;
        for (v = 0; v <= n; ++v) { par[v] = v; top[v] = v; }
        for (i = 0; i < n; ++i) {
            int32_t x = by_pri[i];
            int64_t a, b, s;
            if (state[x] != 2) continue;
            s = succ[x] < 0 ? n : succ[x];
            a = uf_find(par, x);
            b = uf_find(par, s);
            if (pri[x] % 2 == 0) { lc[next - n - 1] = top[b]; rc2[next - n - 1] = top[a]; }
            else { lc[next - n - 1] = top[a]; rc2[next - n - 1] = top[b]; }
            par[a] = b;
            top[b] = next++;
        }
        /* in-order over the leaves: iterative, right child pushed first */
        stack[sp++] = top[uf_find(par, n)];
        while (sp) {
            int64_t x = stack[--sp];
            if (x <= n) { key[x] = (int32_t)rank++; continue; }
            stack[sp++] = rc2[x - n - 1];
            stack[sp++] = lc[x - n - 1];
        }
        free(par); free(top); free(lc); free(rc2); free(stack);
    }
    if (n_finite) *n_finite = nf;
    free(state); free(depth); free(walk);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* switching                                                                 */
/* ------------------------------------------------------------------------ */

/* All_Odd: each Odd vertex takes the first successor of least key if that is
   strictly below its current choice.  Returns the number of switches. */
int64_t orc_odd_switch(int64_t n, const int64_t *off, const int32_t *tgt,
                       const uint8_t *owner, const int32_t *key, int32_t *tau)
{
    int64_t v, e, count = 0;
    for (v = 0; v < n; ++v) {
        int32_t best;
        if (owner[v] != 1) continue;
        best = tgt[off[v]];
        for (e = off[v] + 1; e < off[v + 1]; ++e)
            if (key[tgt[e]] < key[best]) best = tgt[e];
        if (key[best] < key[tau[v]]) { tau[v] = best; ++count; }
    }
    return count;
}

/* All_Even: options are the sink, then the row; the first greatest key wins
   if it is strictly above the current choice. */
int64_t orc_even_switch(int64_t n, const int64_t *off, const int32_t *tgt,
                        const uint8_t *owner, const int32_t *key, int32_t *sigma)
{
    int64_t v, e, count = 0;
    for (v = 0; v < n; ++v) {
        int32_t best = ORC_SINK, kb, kc;
        if (owner[v] != 0) continue;
        kb = key[n];
        for (e = off[v]; e < off[v + 1]; ++e)
            if (key[tgt[e]] > kb) { best = tgt[e]; kb = key[tgt[e]]; }
        kc = sigma[v] < 0 ? key[n] : key[sigma[v]];
        if (kb > kc) { sigma[v] = best; ++count; }
    }
    return count;
}

/* polynomial hash of an int32 array (for compact traces) */
uint64_t orc_hash(int64_t len, const int32_t *a)
{
    uint64_t h = 0;
    int64_t i;
    for (i = 0; i < len; ++i)
        h = h * 1099511628211ULL + (uint64_t)(uint32_t)a[i] + 1ULL;
    return h;
}

static int cmp_pri_ctx(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    int32_t pa = g_ctx.pri[a], pb = g_ctx.pri[b];
    return (pa > pb) - (pa < pb);
}

/* vertices in increasing priority */
void orc_order_by_pri(int64_t n, const int32_t *pri, int32_t *by_pri)
{
    int64_t v;
    for (v = 0; v < n; ++v) by_pri[v] = (int32_t)v;
    g_ctx.pri = pri;
    qsort(by_pri, (size_t)n, sizeof(int32_t), cmp_pri_ctx);
}

typedef struct {
    int64_t n_major;
    int64_t n_valuations;
    int64_t n_even_switches;
    int64_t n_odd_switches;
} orc_stats;

/*
 * Algorithm 1 on the (already modified) game.  sigma/tau are in-out (the
 * caller passes the initial strategies).  key[n+1] receives the last
 * valuation.  trace (nullable, capacity trace_cap) receives the hash of every
 * valuation's key array, in order.  reset != 0 is SI-Reset (section 6, the
 * best-response experiment): every best response starts again from the
 * initial Odd strategy (the first entry of each row) instead of the previous
 * best response.  Returns a status code.
 */
int orc_solve(int64_t n, const int64_t *off, const int32_t *tgt,
              const uint8_t *owner, const int32_t *pri, int method,
              int64_t max_major, int64_t max_inner, int reset,
              int32_t *sigma, int32_t *tau, int32_t *key,
              orc_stats *st, uint64_t *trace, int64_t trace_cap)
{
    int32_t *succ = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int32_t *by_pri = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int64_t v, nval = 0, nmaj = 0, ev = 0, od = 0;
    int rc = ORC_OK;
    if (!succ || !by_pri) { free(succ); free(by_pri); return ORC_ENOMEM; }
    orc_order_by_pri(n, pri, by_pri);
    for (;;) {
        int64_t inner = 0, c;
        if (max_major > 0 && nmaj >= max_major) { rc = ORC_EITERLIMIT; break; }
        ++nmaj;
        if (reset)
            for (v = 0; v < n; ++v)
                if (owner[v]) tau[v] = tgt[off[v]];
        for (;;) {
            if (max_inner > 0 && inner >= max_inner) { rc = ORC_EITERLIMIT; break; }
            for (v = 0; v < n; ++v) succ[v] = owner[v] ? tau[v] : sigma[v];
            rc = orc_valuation(n, succ, pri, by_pri, method, key, NULL);
            if (trace && nval < trace_cap) trace[nval] = orc_hash(n + 1, key);
            ++nval; ++inner;
            if (rc != ORC_OK) break;
            c = orc_odd_switch(n, off, tgt, owner, key, tau);
            od += c;
            if (c == 0) break;
        }
        if (rc != ORC_OK) break;
        c = orc_even_switch(n, off, tgt, owner, key, sigma);
        ev += c;
        if (c == 0) break;
    }
    if (st) { st->n_major = nmaj; st->n_valuations = nval;
              st->n_even_switches = ev; st->n_odd_switches = od; }
    free(succ); free(by_pri);
    return rc;
}
