/*
 * Multi-core CPU baseline of a best-response iteration with parallel list
 * ranking: the paper's CPU-LR implementation (section 6, "Implementation":
 * the valuation's list ranking spread over the CPU's threads).  It is a
 * baseline to time next to the single-threaded oracle and the device
 * library; neither of them uses it.
 *
 * The valuation is the one of rank keys for distinct priorities: the key of
 * a finite vertex is its position in the in-order of the nearest-greater
 * tree rooted at the sink (children of odd priority by decreasing priority,
 * then the node, then children of even priority by increasing priority);
 * a vertex whose play reaches a cycle gets KEY_TOP.  Steps:
 *   1. ng(v), the nearest vertex after v on its play with a larger
 *      priority (the sink, or TOP when the play closes a cycle first),
 *      all vertices in parallel, handed out in increasing priority order:
 *      a walk jumps over a smaller vertex u straight to ng(u) when that is
 *      known already, and steps to u's successor otherwise;
 *   2. fates (finite or top) in parallel, in decreasing priority order;
 *   3. children grouped by parent, siblings in signed-priority order
 *      (group sizes counted in parallel; the sink's children compacted from
 *      the signed order; the other groups filled by atomic slots and sorted
 *      by signed position);
 *   4. the Euler list of the tree (section 5, "Formal reduction"), built in
 *      parallel: enter and leave elements per vertex, each vertex's
 *      in-order point marked on one element;
 *   5. list ranking by sublists (section 5, "List ranking"): splitters at a
 *      fixed element stride, sublists summed in parallel, the reduced list
 *      ranked by one thread, the sublists walked again in parallel to emit
 *      the keys.
 * The Odd switch step (section 4, All_Odd) runs in parallel over vertices.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define KEY_TOP 2147483647
#define STRIDE 64

enum { CL_OK = 0, CL_ENOMEM = 1, CL_EINADMISSIBLE = 2, CL_EINTERNAL = 3 };

static int cmp_u64(const void *a, const void *b) {
  const uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return x < y ? -1 : x > y;
}

/*
 * succ[v]: successor of v (-1: the sink); pri: distinct priorities;
 * by_pri: the vertices in increasing priority; by_signed: the vertices in
 * signed-priority order (odd priorities descending, then even ascending).
 * key[n + 1] receives the keys (key[n]: the sink).  threads <= 0: OpenMP's
 * default.  Returns a CL_ status.
 */
int cl_valuation(int64_t n, const int32_t *succ, const int32_t *pri,
                 const int32_t *by_pri, const int32_t *by_signed,
                 int threads, int32_t *key, int64_t *n_finite) {
  const int32_t N = (int32_t)n, TOP = (int32_t)n + 1;
  if (threads > 0) omp_set_num_threads(threads);
  int32_t *ng = malloc(sizeof(int32_t) * (size_t)(n + 1));
  uint8_t *fin = malloc((size_t)n + 1);
  int64_t *cnt = calloc((size_t)n + 2, sizeof(int64_t));
  int32_t *kids = malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t *pos = malloc(sizeof(int32_t) * (size_t)(n + 1));
  int64_t *fill = malloc(sizeof(int64_t) * (size_t)(n + 1));
  int st = CL_OK;
  if (!ng || !fin || !cnt || !kids || !pos || !fill) {
    st = CL_ENOMEM;
    goto out0;
  }
  /* 1. ng, every vertex in parallel, taken in increasing priority order:
     a walk jumps over a smaller vertex u straight to ng(u) when ng(u) is
     already known (everything between u and ng(u) is smaller than u), and
     steps to u's successor otherwise.  More than n steps mean the walk
     circles vertices all smaller than v: nothing larger follows (TOP). */
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) ng[v] = -1;
  int bad1 = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(| : bad1)
  for (int64_t k = 0; k < n; ++k) {
    const int32_t v = by_pri[k];
    const int32_t pv = pri[v];
    int32_t u = succ[v] < 0 ? N : succ[v];
    int32_t r;
    for (int64_t steps = 0;; ++steps) {
      if (u == N) { r = N; break; }
      if (u == v) {            /* v is the largest of its cycle */
        if (pv & 1) bad1 = 1;
        r = TOP;
        break;
      }
      if (pri[u] > pv) { r = u; break; }
      if (steps > n) { r = TOP; break; }
      const int32_t j = __atomic_load_n(&ng[u], __ATOMIC_RELAXED);
      if (j == N || j == TOP) { r = j; break; }
      u = j >= 0 ? j : (succ[u] < 0 ? N : succ[u]);
    }
    __atomic_store_n(&ng[v], r, __ATOMIC_RELAXED);
  }
  if (bad1) { st = CL_EINADMISSIBLE; goto out0; }
  /* 2. fates, in parallel in decreasing priority order: a vertex takes the
     fate of its parent ng(v) (a larger vertex, so mostly known already),
     following the ng chain while it is not */
  fin[N] = 1;
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) fin[v] = 2;   /* unknown */
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t k = n - 1; k >= 0; --k) {
    const int32_t v = by_pri[k];
    int32_t p = ng[v];
    uint8_t f;
    for (;;) {
      if (p == N) { f = 1; break; }
      if (p == TOP) { f = 0; break; }
      const uint8_t q = __atomic_load_n(&fin[p], __ATOMIC_RELAXED);
      if (q != 2) { f = q; break; }
      p = ng[p];
    }
    __atomic_store_n(&fin[v], f, __ATOMIC_RELAXED);
  }
  /* 3. children by parent, siblings in signed order.  Counts per parent
     (atomic), their scan; the sink's children (the largest group) taken
     from the signed order by a per-thread-chunk compaction; every other
     vertex placed by an atomic slot in its parent's group, each group then
     sorted by signed position (groups are small) */
  int64_t nf = 0;
  {
    uint64_t *tmp = malloc(sizeof(uint64_t) * (size_t)(n + 1));
    int32_t *sr = malloc(sizeof(int32_t) * (size_t)(n + 1));
    const int T = omp_get_max_threads();
    int64_t *chunk = calloc((size_t)T + 1, sizeof(int64_t));
    if (!tmp || !sr || !chunk) {
      free(tmp);
      free(sr);
      free(chunk);
      st = CL_ENOMEM;
      goto out0;
    }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) sr[by_signed[k]] = (int32_t)k;
    int64_t sink_kids = 0;   /* counted apart: one shared counter would
                                serialise most of the increments */
#pragma omp parallel for schedule(static) reduction(+ : sink_kids)
    for (int64_t v = 0; v < n; ++v) {
      if (!fin[v]) continue;
      if (ng[v] == N) ++sink_kids;
      else __atomic_fetch_add(&cnt[ng[v] + 1], 1, __ATOMIC_RELAXED);
    }
    cnt[N + 1] = sink_kids;
    for (int64_t q = 0; q <= n; ++q) cnt[q + 1] += cnt[q];
    nf = cnt[n + 1];
    /* the sink's children in signed order */
#pragma omp parallel
    {
      const int nt = omp_get_num_threads();
      for (int t = omp_get_thread_num(); t < T; t += nt) {
        int64_t c = 0;
        for (int64_t k = n * t / T; k < n * (t + 1) / T; ++k) {
          const int32_t v = by_signed[k];
          c += fin[v] && ng[v] == N;
        }
        chunk[t + 1] = c;
      }
    }
    for (int t = 0; t < T; ++t) chunk[t + 1] += chunk[t];
#pragma omp parallel
    {
      const int nt = omp_get_num_threads();
      for (int t = omp_get_thread_num(); t < T; t += nt) {
        int64_t i = cnt[N] + chunk[t];
        for (int64_t k = n * t / T; k < n * (t + 1) / T; ++k) {
          const int32_t v = by_signed[k];
          if (fin[v] && ng[v] == N) tmp[i++] = ((uint64_t)k << 32) | (uint32_t)v;
        }
      }
    }
    /* the other groups: a slot each, then each group sorted */
    memcpy(fill, cnt, sizeof(int64_t) * (size_t)(n + 1));
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; ++v) {
      if (!fin[v] || ng[v] == N) continue;
      const int64_t i = __atomic_fetch_add(&fill[ng[v]], 1, __ATOMIC_RELAXED);
      tmp[i] = ((uint64_t)(uint32_t)sr[v] << 32) | (uint32_t)v;
    }
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t q = 0; q < n; ++q) {
      const int64_t a = cnt[q], b = cnt[q + 1];
      if (b - a > 32) {
        qsort(tmp + a, (size_t)(b - a), sizeof(uint64_t), cmp_u64);
      } else {
        for (int64_t i = a + 1; i < b; ++i) {   /* insertion sort */
          const uint64_t x = tmp[i];
          int64_t j = i - 1;
          while (j >= a && tmp[j] > x) { tmp[j + 1] = tmp[j]; --j; }
          tmp[j + 1] = x;
        }
      }
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nf; ++i) {
      const int32_t v = (int32_t)(uint32_t)tmp[i];
      kids[i] = v;
      pos[v] = (int32_t)i;
    }
    free(tmp);
    free(sr);
    free(chunk);
  }
  /* 4. the Euler list: 0/1 enter/leave the sink, 2i+2/2i+3 enter/leave
     kids[i]; y = node | (weight << 31) */
  const int64_t L = 2 * nf + 2;
  int32_t *nx = malloc(sizeof(int32_t) * (size_t)L);
  int32_t *ny = malloc(sizeof(int32_t) * (size_t)L);
  if (!nx || !ny) { st = CL_ENOMEM; goto out1; }
  {
    const int64_t s0 = cnt[N], s1 = cnt[N + 1];
    const int has = s1 > s0;
    const int last_even = has && !(pri[kids[s1 - 1]] & 1);
    nx[0] = has ? (int32_t)(2 * s0 + 2) : 1;
    ny[0] = N;
    nx[1] = -1;
    ny[1] = N | ((!last_even) ? (int32_t)0x80000000 : 0);
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nf; ++i) {
    const int32_t c = kids[i];
    const int32_t p = ng[c];
    const int64_t ps = cnt[p], pe = cnt[p + 1];   /* parent's children */
    const int ev = !(pri[c] & 1);
    const int wd = ev && (i == ps || (pri[kids[i - 1]] & 1));
    const int64_t cs = cnt[c], ce = cnt[c + 1];   /* c's children */
    const int has = ce > cs;
    const int wu = !has || (pri[kids[ce - 1]] & 1);
    nx[2 * i + 2] = has ? (int32_t)(2 * cs + 2) : (int32_t)(2 * i + 3);
    ny[2 * i + 2] = p | (wd ? (int32_t)0x80000000 : 0);
    nx[2 * i + 3] = i + 1 < pe ? (int32_t)(2 * i + 4)
                               : (p == N ? 1 : 2 * pos[p] + 3);
    ny[2 * i + 3] = c | (wu ? (int32_t)0x80000000 : 0);
  }
  /* 5. list ranking by sublists */
  {
    const int64_t ns = (L + STRIDE - 1) / STRIDE;
    int32_t *ssum = malloc(sizeof(int32_t) * (size_t)ns);
    int32_t *snext = malloc(sizeof(int32_t) * (size_t)ns);
    int32_t *sbase = malloc(sizeof(int32_t) * (size_t)ns);
    int bad = 0;
    if (!ssum || !snext || !sbase) {
      st = CL_ENOMEM;
    } else {
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
      for (int64_t j = 0; j < ns; ++j) {
        int64_t e = j * STRIDE, steps = 0;
        int32_t acc = 0;
        for (;;) {
          acc += (int32_t)((uint32_t)ny[e] >> 31);
          e = nx[e];
          if (e < 0 || e % STRIDE == 0) break;
          if (++steps > L) { bad = 1; e = -1; break; }
        }
        ssum[j] = acc;
        snext[j] = e < 0 ? -1 : (int32_t)(e / STRIDE);
      }
      /* the reduced list from the head (splitter 0) */
      int64_t acc = 0, steps = 0;
      for (int64_t j = 0; j >= 0 && !bad; j = snext[j]) {
        if (++steps > ns) { bad = 1; break; }
        sbase[j] = (int32_t)acc;
        acc += ssum[j];
      }
      if (acc != nf + 1) bad = 1;
      if (!bad) {
#pragma omp parallel for schedule(static)
        for (int64_t v = 0; v < n; ++v)
          if (!fin[v]) key[v] = KEY_TOP;
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t j = 0; j < ns; ++j) {
          int64_t e = j * STRIDE;
          int32_t b = sbase[j];
          for (int64_t steps2 = 0; steps2 <= L; ++steps2) {
            if (ny[e] < 0) key[ny[e] & 0x7fffffff] = b++;
            e = nx[e];
            if (e < 0 || e % STRIDE == 0) break;
          }
        }
      }
      if (bad) st = CL_EINTERNAL;
    }
    free(ssum);
    free(snext);
    free(sbase);
  }
  if (n_finite) *n_finite = nf + 1;
out1:
  free(nx);
  free(ny);
out0:
  free(ng);
  free(fin);
  free(cnt);
  free(kids);
  free(pos);
  free(fill);
  return st;
}

/* All_Odd (section 4): the first row entry of least key replaces tau(v)
   when strictly below the current choice.  Returns the switch count. */
int64_t cl_odd_switch(int64_t n, const int64_t *off, const int32_t *tgt,
                      const uint8_t *owner, const int32_t *key, int32_t *tau,
                      int threads) {
  if (threads > 0) omp_set_num_threads(threads);
  int64_t count = 0;
#pragma omp parallel for schedule(static) reduction(+ : count)
  for (int64_t v = 0; v < n; ++v) {
    if (owner[v] != 1) continue;
    int32_t best = tgt[off[v]];
    for (int64_t e = off[v] + 1; e < off[v + 1]; ++e)
      if (key[tgt[e]] < key[best]) best = tgt[e];
    if (key[best] < key[tau[v]]) {
      tau[v] = best;
      ++count;
    }
  }
  return count;
}

int cl_max_threads(void) { return omp_get_max_threads(); }
