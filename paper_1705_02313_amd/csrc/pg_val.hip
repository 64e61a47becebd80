// Valuation of the play graph and the switching rules.
//
// The play graph of (sigma, tau) gives every vertex one successor (section 5,
// "Pseudoforests and Euler tours"): the vertices whose play reaches the sink
// form a tree rooted at the sink, the others lie on or lead into cycles and
// have valuation top.  With pairwise distinct priorities a finite valuation is
// the set of priorities on the tree path to the sink, and two such sets
// differ exactly on the tree path between their vertices, so Maxdiff (section
// 3, "Valuations") is the largest priority on that path.  Let ng(v) be the
// nearest vertex after v on its play with a larger priority (the sink counts
// as larger than everything).  Ordering the children of every node of the ng
// tree by signed priority -- odd priorities descending, then even priorities
// ascending -- and listing the tree in order (odd children, the node, even
// children) lists the finite vertices in increasing valuation.  The rank of a
// vertex in that order is its key.
//
// Steps, one kernel (or a few) each:
//   ng      bounded walks along the play with shortcuts through the ng values
//           and walk candidates other threads have already published; a
//           vertex that walks back to itself is the largest of its cycle and
//           gets ng = TOP (its priority must be even, else sigma is not
//           admissible, section 3)
//   root    walks along the ng chain to the sink or to TOP: finite or top
//   sort    stable radix sort of the finite vertices (taken in signed-priority
//           order) by ng: each node's children end up contiguous and ordered
//   euler   the Euler-tour list of the ng tree (section 5, "Formal
//           reduction"): enter/leave elements per node, one weighted element
//           per node marking its in-order point
//   rank    list ranking by sublists (section 5, "List ranking"): splitters
//           at fixed element strides, every sublist summed by one thread, the
//           reduced list ranked recursively and finally in LDS by pointer
//           jumping, then each sublist is walked again to emit keys
#include "pg_common.h"

namespace pgk {

__device__ __forceinline__ int ld_relaxed(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// wave-aggregated counter increment: one atomic per wave
__device__ __forceinline__ void count_wave(int32_t *ctr, bool pred) {
  uint64_t b = __ballot(pred);
  if (b && (threadIdx.x & (kWave - 1)) == (unsigned)(__ffsll((long long)b) - 1))
    atomicAdd(ctr, (int)__popcll(b));
}

// ---------------------------------------------------------------------------
// ng: nearest greater vertex along the play
// ---------------------------------------------------------------------------
// N = n_aug (the sink's id), TOP id = N + 1.  cand[v] of an unresolved v is
// the next vertex of v's play not yet compared with v; every vertex strictly
// between v and cand[v] has a smaller priority than v.
__global__ __launch_bounds__(kBlock) void k_ng_walk(
    int32_t N, const int2 *__restrict__ sp, int32_t *ng, int32_t *cand,
    const int32_t *wl_in, int32_t wl_len, int32_t *wl_out, int32_t *ctr,
    int wl_ctr, int steps) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t v;
  int32_t u;
  bool live;
  if (wl_in) {
    live = i < wl_len;
    v = live ? wl_in[i] : 0;
    u = live ? cand[v] : 0;
  } else {
    live = i < N;
    v = live ? (int32_t)i : 0;
    u = live ? sp[v].x : 0;
  }
  bool pending = false;
  if (live) {
    const int pv = sp[v].y;
    int32_t res = -1;
    for (int s = 0; s < steps; ++s) {
      if (u == N) { res = N; break; }
      if (u == v) {
        // v returned to itself: it has the largest priority of its cycle
        res = N + 1;
        if (pv & 1) atomicOr(&ctr[C_ERR], ERR_INADMISSIBLE);
        break;
      }
      const int2 su = sp[u];
      if (su.y > pv) { res = u; break; }
      const int32_t r = ld_relaxed(&ng[u]);
      if (r >= 0) {
        if (r >= N) { res = r; break; }  // nothing larger after u
        u = r;
        continue;
      }
      const int32_t c = ld_relaxed(&cand[u]);
      u = (c >= 0) ? c : su.x;
    }
    if (res >= 0) {
      __hip_atomic_store(&ng[v], res, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __hip_atomic_store(&cand[v], u, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      pending = true;
    }
  }
  if (pending) wl_out[atomicAdd(&ctr[wl_ctr], 1)] = v;
}

// ---------------------------------------------------------------------------
// root: does the ng chain end at the sink (finite) or at TOP?
// rs[v]: 0 unknown, 1 finite, 2 top.  Top vertices get key TOP and ng TOP.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_root_walk(
    int32_t N, int32_t *ng, uint8_t *rs, int32_t *cand, int32_t *key,
    const int32_t *wl_in, int32_t wl_len, int32_t *wl_out, int32_t *ctr,
    int wl_ctr, int steps) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t v = 0, r = 0;
  bool live;
  if (wl_in) {
    live = i < wl_len;
    if (live) { v = wl_in[i]; r = cand[v]; }
  } else {
    live = i < N;
    if (live) { v = (int32_t)i; r = ng[v]; }
  }
  int fate = 0;
  bool pending = false;
  if (live) {
    for (int s = 0; s < steps; ++s) {
      if (r == N) { fate = 1; break; }
      if (r == N + 1) { fate = 2; break; }
      const int known = __hip_atomic_load(&rs[r], __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
      if (known) { fate = known; break; }
      const int32_t c = wl_in ? ld_relaxed(&cand[r]) : -1;
      // in the first pass follow ng; in later rounds jump over the
      // candidates published by other unresolved vertices
      r = (c >= 0 && wl_in) ? c : ld_relaxed(&ng[r]);
    }
    if (fate) {
      __hip_atomic_store(&rs[v], (uint8_t)fate, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      if (fate == 2) key[v] = PG_KEY_TOP;
    } else {
      __hip_atomic_store(&cand[v], r, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      pending = true;
    }
  }
  count_wave(&ctr[C_NFIN], fate == 1);
  if (pending) wl_out[atomicAdd(&ctr[wl_ctr], 1)] = v;
}

// sort keys in signed-priority order: the parent for finite vertices, N + 1
// (after every parent) for top vertices
__global__ __launch_bounds__(kBlock) void k_sort_keys(
    int32_t N, const int32_t *__restrict__ perm, const int32_t *__restrict__ ng,
    const uint8_t *__restrict__ rs, uint32_t *sk, uint32_t *sv) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int32_t v = perm[i];
  sk[i] = (rs[v] == 1) ? (uint32_t)ng[v] : (uint32_t)(N + 1);
  sv[i] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// Euler list of the ng tree
// ---------------------------------------------------------------------------
// Sorted position i (0 <= i < nF) holds vertex kids[i] with parent skS[i].
// Elements: 0 enters the root (the sink), 1 leaves it; 2i+2 enters kids[i],
// 2i+3 leaves it.
__global__ __launch_bounds__(kBlock) void k_link_info(
    int32_t N, int32_t nF, int32_t n_oddpri, const uint32_t *__restrict__ skS,
    const uint32_t *__restrict__ svS, const int32_t *__restrict__ perm,
    int32_t *kids, int32_t *pos, int32_t *first, uint8_t *haseven) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nF) return;
  const uint32_t p = skS[i];
  const uint32_t r = svS[i];
  const int32_t c = perm[r];
  kids[i] = c;
  pos[c] = (int32_t)i;
  if (i == 0 || skS[i - 1] != p) first[p] = (int32_t)i;
  if (i == nF - 1 || skS[i + 1] != p) haseven[p] = (r >= (uint32_t)n_oddpri);
}

__global__ __launch_bounds__(kBlock) void k_link_build(
    int32_t N, int32_t nF, int32_t n_oddpri, const uint32_t *__restrict__ skS,
    const uint32_t *__restrict__ svS, const int32_t *__restrict__ kids,
    const int32_t *__restrict__ pos, const int32_t *__restrict__ first,
    const uint8_t *__restrict__ haseven, int2 *elem) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    const int32_t f = first[N];
    elem[0] = make_int2(f >= 0 ? 2 * f + 2 : 1, N);
    const int w = (f < 0 || !haseven[N]) ? 1 : 0;
    elem[1] = make_int2(-1, N | (w << 31));
  }
  if (i >= nF) return;
  const int32_t c = kids[i];
  const uint32_t p = skS[i];
  const bool ev = svS[i] >= (uint32_t)n_oddpri;
  const bool seg_start = (i == 0) || (skS[i - 1] != p);
  const bool seg_end = (i == nF - 1) || (skS[i + 1] != p);
  const int32_t fc = first[c];
  // enter c: first child of c, or straight to leaving c.  It carries the
  // parent's in-order point when c is the parent's first even child.
  const bool wd = ev && (seg_start || svS[i - 1] < (uint32_t)n_oddpri);
  elem[2 * i + 2] =
      make_int2(fc >= 0 ? 2 * fc + 2 : (int32_t)(2 * i + 3),
                (int32_t)p | ((int32_t)wd << 31));
  // leave c: next sibling, else leave the parent.  It carries c's own
  // in-order point when c has no even child.
  const bool wu = (fc < 0) || !haseven[c];
  int32_t nx;
  if (!seg_end) nx = (int32_t)(2 * i + 4);
  else nx = (p == (uint32_t)N) ? 1 : 2 * pos[p] + 3;
  elem[2 * i + 3] = make_int2(nx, c | ((int32_t)wu << 31));
}

// ---------------------------------------------------------------------------
// list ranking by sublists
// ---------------------------------------------------------------------------
// Level 1 walks the Euler list (weights are the top bits of elem[].y); higher
// levels walk the reduced lists (int weights).  Splitters are the elements
// whose index is a multiple of the stride; element 0 (the list head) is one.
__global__ __launch_bounds__(kBlock) void k_lr_sum1(
    const int2 *__restrict__ elem, int64_t L, int stride, int64_t nsplit,
    int per_thread, int32_t *sum, int32_t *next, int32_t *ctr) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  for (int k = 0; k < per_thread; ++k) {
    const int64_t j = t + (int64_t)k * nthreads;
    if (j >= nsplit) break;
    int64_t e = j * stride;
    int32_t acc = 0;
    int64_t steps = 0;
    for (;;) {
      const int2 el = elem[e];
      acc += (int32_t)((uint32_t)el.y >> 31);
      e = el.x;
      if (e < 0 || e % stride == 0) break;
      if (++steps > L) { atomicOr(&ctr[C_ERR], ERR_LISTWALK); e = -1; break; }
    }
    sum[j] = acc;
    next[j] = e < 0 ? -1 : (int32_t)(e / stride);
  }
}

__global__ __launch_bounds__(kBlock) void k_lr_sumk(
    const int32_t *__restrict__ lnext, const int32_t *__restrict__ lw,
    int64_t L, int stride, int64_t nsplit, int32_t *sum, int32_t *next,
    int32_t *ctr) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nsplit) return;
  int64_t e = j * stride;
  int32_t acc = 0;
  int64_t steps = 0;
  for (;;) {
    acc += lw[e];
    e = lnext[e];
    if (e < 0 || e % stride == 0) break;
    if (++steps > L) { atomicOr(&ctr[C_ERR], ERR_LISTWALK); e = -1; break; }
  }
  sum[j] = acc;
  next[j] = e < 0 ? -1 : (int32_t)(e / stride);
}

// Ranks a list of at most kTopMax elements (head = 0) inside one block by
// pointer jumping: suffix sums, then base = total - suffix.
constexpr int kTopMax = 4096;
constexpr int kTopThreads = 1024;

__global__ __launch_bounds__(kTopThreads) void k_lr_top(
    const int32_t *__restrict__ lnext, const int32_t *__restrict__ lw,
    int32_t L, int32_t *base, int32_t expect_total, int32_t *ctr) {
  __shared__ int32_t nx[kTopMax];
  __shared__ int32_t sm[kTopMax];
  constexpr int per = kTopMax / kTopThreads;
  for (int k = 0; k < per; ++k) {
    const int i = threadIdx.x + k * kTopThreads;
    nx[i] = (i < L) ? lnext[i] : -1;
    sm[i] = (i < L) ? lw[i] : 0;
  }
  __syncthreads();
  for (int round = 0; (1 << round) < L; ++round) {
    int32_t nn[per], ss[per];
    for (int k = 0; k < per; ++k) {
      const int i = threadIdx.x + k * kTopThreads;
      const int p = nx[i];
      nn[k] = (p >= 0) ? nx[p] : -1;
      ss[k] = (p >= 0) ? sm[i] + sm[p] : sm[i];
    }
    __syncthreads();
    for (int k = 0; k < per; ++k) {
      const int i = threadIdx.x + k * kTopThreads;
      nx[i] = nn[k];
      sm[i] = ss[k];
    }
    __syncthreads();
  }
  const int32_t total = sm[0];
  for (int k = 0; k < per; ++k) {
    const int i = threadIdx.x + k * kTopThreads;
    if (i < L) base[i] = total - sm[i];
  }
  if (threadIdx.x == 0 && expect_total >= 0 && total != expect_total)
    atomicOr(&ctr[C_ERR], ERR_RANKCOUNT);
}

// Hands each element of a level-k sublist its exclusive rank.
__global__ __launch_bounds__(kBlock) void k_lr_distk(
    const int32_t *__restrict__ lnext, const int32_t *__restrict__ lw,
    int stride, int64_t nsplit, const int32_t *__restrict__ sbase,
    int32_t *lbase) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nsplit) return;
  int64_t e = j * stride;
  int32_t b = sbase[j];
  for (;;) {
    lbase[e] = b;
    b += lw[e];
    e = lnext[e];
    if (e < 0 || e % stride == 0) break;
  }
}

// Final pass over the Euler list: every weighted element emits the key of
// its node.
__global__ __launch_bounds__(kBlock) void k_lr_emit1(
    const int2 *__restrict__ elem, int stride, int64_t nsplit, int per_thread,
    const int32_t *__restrict__ sbase, int32_t *key) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  for (int k = 0; k < per_thread; ++k) {
    const int64_t j = t + (int64_t)k * nthreads;
    if (j >= nsplit) break;
    int64_t e = j * stride;
    int32_t b = sbase[j];
    for (;;) {
      const int2 el = elem[e];
      if (el.y < 0) key[el.y & 0x7fffffff] = b++;
      e = el.x;
      if (e < 0 || e % stride == 0) break;
    }
  }
}

// ---------------------------------------------------------------------------
// switching rules
// ---------------------------------------------------------------------------
// All_Odd (section 4): the first successor of least key, if strictly below
// the current choice.  All decisions read the same valuation.
__global__ __launch_bounds__(kBlock) void k_odd_switch(
    int32_t N, const int64_t *__restrict__ off, const int32_t *__restrict__ tgt,
    const uint8_t *__restrict__ owner, const int32_t *__restrict__ key,
    int2 *sp, int32_t *ctr) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool sw = false;
  if (v < N && owner[v] == 1) {
    int64_t e = off[v];
    const int64_t end = off[v + 1];
    int32_t best = tgt[e];
    int32_t kb = key[best];
    for (++e; e < end; ++e) {
      const int32_t u = tgt[e];
      const int32_t ku = key[u];
      if (ku < kb) { kb = ku; best = u; }
    }
    const int32_t cur = sp[v].x;
    if (kb < key[cur]) {
      sp[v].x = best;
      sw = true;
    }
  }
  count_wave(&ctr[C_SWITCH], sw);
}

// All_Even, greedy all-switches (section 3): options are the sink (first),
// then the row; the first option of greatest key, if strictly above the
// current choice.
__global__ __launch_bounds__(kBlock) void k_even_switch(
    int32_t N, const int64_t *__restrict__ off, const int32_t *__restrict__ tgt,
    const uint8_t *__restrict__ owner, const int32_t *__restrict__ key,
    int2 *sp, int32_t *ctr) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool sw = false;
  if (v < N && owner[v] == 0) {
    int32_t best = N;
    int32_t kb = key[N];
    for (int64_t e = off[v], end = off[v + 1]; e < end; ++e) {
      const int32_t u = tgt[e];
      const int32_t ku = key[u];
      if (ku > kb) { kb = ku; best = u; }
    }
    const int32_t cur = sp[v].x;
    if (kb > key[cur]) {
      sp[v].x = best;
      sw = true;
    }
  }
  count_wave(&ctr[C_SWITCH], sw);
}

}  // namespace pgk

// ===========================================================================
// host side of the valuation
// ===========================================================================
namespace pgk {

constexpr int kWalkSteps = 256;     // bounded walks before the jump rounds
constexpr int kMaxRounds = 64;      // jump rounds before giving up
constexpr int kStride1 = 32;        // level-1 splitter stride
constexpr int kStrideK = 32;        // higher-level splitter stride
constexpr int kPerThread1 = 4;      // level-1 sublists per thread

static pg_status read_ctr(pg_game *g, hipStream_t s) {
  PG_HIP(hipMemcpyAsync(g->hctr, g->ctr, sizeof(int32_t) * C_COUNT,
                        hipMemcpyDeviceToHost, s));
  PG_HIP(hipStreamSynchronize(s));
  if (g->prof.on) g->prof.flush();
  return PG_OK;
}

static void zero_ctr(pg_game *g, hipStream_t s, int which) {
  fill_i32(g->ctr + which, 0, 1, s, &g->prof);
}

// Plans the sublist levels for a level-1 list of L elements.
static void plan_levels(pg_game *g, int64_t L) {
  int k = 0;
  int64_t size = L;
  int stride = kStride1;
  // level 0 always walks the Euler list; further levels until the reduced
  // list fits the LDS ranking
  while ((k == 0 || size > kTopMax) && k < 7) {
    g->lv[k].size = size;
    g->lv[k].stride = stride;
    g->lv[k].nsplit = (size + stride - 1) / stride;
    size = g->lv[k].nsplit;
    stride = kStrideK;
    ++k;
  }
  g->lv[k].size = size;
  g->lv[k].stride = 0;
  g->lv[k].nsplit = 0;
  g->nlevels = k;  // levels that walk; level k is ranked in LDS
}

pg_status valuation_device(pg_game *g, hipStream_t s, int64_t *n_finite_out) {
  const int32_t N = (int32_t)g->n_aug;
  // --- ng ---------------------------------------------------------------
  Prof *pf = &g->prof;
  fill_i32(g->ng, -1, N, s, pf);
  fill_i32(g->cand, -1, N, s, pf);
  fill_i32(g->ctr, 0, C_COUNT, s, pf);
  PG_LAUNCH(pf, K_NG_WALK, 20.0 * N, k_ng_walk, dim3(grid_for(N)),
            dim3(kBlock), 0, s, N, g->sp, g->ng, g->cand,
            (const int32_t *)nullptr, 0, g->wl0, g->ctr, (int)C_WL_NG,
            kWalkSteps);
  pg_status st = read_ctr(g, s);
  if (st != PG_OK) return st;
  int32_t pending = g->hctr[C_WL_NG];
  int32_t *wa = g->wl0, *wb = g->wl1;
  for (int round = 0; pending > 0; ++round) {
    if (round >= kMaxRounds)
      return pg_fail(PG_EINTERNAL, "ng resolution did not converge");
    zero_ctr(g, s, C_WL_NG);
    PG_LAUNCH(pf, K_NG_ROUND, 24.0 * pending, k_ng_walk,
              dim3(grid_for(pending)), dim3(kBlock), 0, s, N, g->sp, g->ng,
              g->cand, (const int32_t *)wa, pending, wb, g->ctr, (int)C_WL_NG,
              kWalkSteps);
    st = read_ctr(g, s);
    if (st != PG_OK) return st;
    pending = g->hctr[C_WL_NG];
    int32_t *t = wa; wa = wb; wb = t;
  }
  if (g->hctr[C_ERR] & ERR_INADMISSIBLE)
    return pg_fail(PG_EINADMISSIBLE,
                   "the play graph has a cycle whose largest priority is odd");
  // --- root: finite or top ---------------------------------------------
  fill_u8(g->rs, 0, (int64_t)N + 1, s, pf);
  fill_i32(g->cand, -1, N, s, pf);
  PG_LAUNCH(pf, K_ROOT_WALK, 10.0 * N, k_root_walk, dim3(grid_for(N)),
            dim3(kBlock), 0, s, N, g->ng, g->rs, g->cand, g->key,
            (const int32_t *)nullptr, 0, g->wl0, g->ctr, (int)C_WL_ROOT,
            kWalkSteps);
  st = read_ctr(g, s);
  if (st != PG_OK) return st;
  pending = g->hctr[C_WL_ROOT];
  wa = g->wl0; wb = g->wl1;
  for (int round = 0; pending > 0; ++round) {
    if (round >= kMaxRounds)
      return pg_fail(PG_EINTERNAL, "root resolution did not converge");
    zero_ctr(g, s, C_WL_ROOT);
    PG_LAUNCH(pf, K_ROOT_ROUND, 14.0 * pending, k_root_walk,
              dim3(grid_for(pending)), dim3(kBlock), 0, s, N, g->ng, g->rs,
              g->cand, g->key, (const int32_t *)wa, pending, wb, g->ctr,
              (int)C_WL_ROOT, kWalkSteps);
    st = read_ctr(g, s);
    if (st != PG_OK) return st;
    pending = g->hctr[C_WL_ROOT];
    int32_t *t = wa; wa = wb; wb = t;
  }
  const int32_t nF = g->hctr[C_NFIN];
  // --- sort finite vertices by (parent, signed priority) -------------------
  PG_LAUNCH(pf, K_SORT_KEYS, 17.0 * N, k_sort_keys, dim3(grid_for(N)),
            dim3(kBlock), 0, s, N, g->perm, g->ng, g->rs, g->sk0, g->sv0);
  int which = radix_sort(g->sk0, g->sv0, g->sk1, g->sv1, N, g->sort_bits,
                         g->tile_cnt, g->scan_tmp, s, pf);
  const uint32_t *skS = which ? g->sk1 : g->sk0;
  const uint32_t *svS = which ? g->sv1 : g->sv0;
  // --- Euler list ----------------------------------------------------------
  fill_i32(g->first, -1, (int64_t)N + 1, s, pf);
  fill_u8(g->haseven, 0, (int64_t)N + 1, s, pf);
  if (nF > 0)
    PG_LAUNCH(pf, K_LINK_INFO, 24.0 * nF, k_link_info, dim3(grid_for(nF)),
              dim3(kBlock), 0, s, N, nF, g->n_oddpri, skS, svS, g->perm,
              g->kids, g->pos, g->first, g->haseven);
  PG_LAUNCH(pf, K_LINK_BUILD, 41.0 * nF, k_link_build,
            dim3(grid_for(nF > 0 ? nF : 1)), dim3(kBlock), 0, s, N, nF,
            g->n_oddpri, skS, svS, g->kids, g->pos, g->first, g->haseven,
            g->elem);
  // --- list ranking -----------------------------------------------------
  const int64_t L = 2 * (int64_t)nF + 2;
  plan_levels(g, L);
  const int nl = g->nlevels;
  const int32_t expect = nF + 1;
  // level 0 is the Euler list itself
  {
    RankLevel &l0 = g->lv[0];
    const int64_t threads = (l0.nsplit + kPerThread1 - 1) / kPerThread1;
    PG_LAUNCH(pf, K_LR_SUM1, 8.0 * L + 8.0 * l0.nsplit, k_lr_sum1,
              dim3(grid_for(threads)), dim3(kBlock), 0, s, g->elem, L,
              l0.stride, l0.nsplit, kPerThread1, l0.sum, l0.next, g->ctr);
  }
  for (int k = 1; k < nl; ++k) {
    RankLevel &lp = g->lv[k - 1];
    RankLevel &lk = g->lv[k];
    PG_LAUNCH(pf, K_LR_SUMK, 8.0 * lk.size + 8.0 * lk.nsplit, k_lr_sumk,
              dim3(grid_for(lk.nsplit)), dim3(kBlock), 0, s, lp.next, lp.sum,
              lk.size, lk.stride, lk.nsplit, lk.sum, lk.next, g->ctr);
  }
  {
    RankLevel &lt = g->lv[nl - 1];
    PG_LAUNCH(pf, K_LR_TOP, 12.0 * lt.nsplit, k_lr_top, dim3(1),
              dim3(kTopThreads), 0, s, lt.next, lt.sum, (int32_t)lt.nsplit,
              lt.base, expect, g->ctr);
  }
  for (int k = nl - 1; k >= 1; --k) {
    RankLevel &lp = g->lv[k - 1];
    RankLevel &lk = g->lv[k];
    PG_LAUNCH(pf, K_LR_DISTK, 12.0 * lk.size + 4.0 * lk.nsplit, k_lr_distk,
              dim3(grid_for(lk.nsplit)), dim3(kBlock), 0, s, lp.next, lp.sum,
              lk.stride, lk.nsplit, lk.base, lp.base);
  }
  {
    RankLevel &l0 = g->lv[0];
    const int64_t threads = (l0.nsplit + kPerThread1 - 1) / kPerThread1;
    PG_LAUNCH(pf, K_LR_EMIT1, 8.0 * L + 4.0 * l0.nsplit + 4.0 * (nF + 1),
              k_lr_emit1, dim3(grid_for(threads)), dim3(kBlock), 0, s,
              g->elem, l0.stride, l0.nsplit, kPerThread1, l0.base, g->key);
  }
  if (n_finite_out) *n_finite_out = (int64_t)nF + 1;
  return PG_OK;
}

pg_status switch_device(pg_game *g, bool odd, hipStream_t s, int32_t *count) {
  const int32_t N = (int32_t)g->n_aug;
  zero_ctr(g, s, C_SWITCH);
  Prof *pf = &g->prof;
  // offsets (8 B per row) and owners for every vertex; for the player's own
  // rows the targets and the key of each target (8 B per edge), the current
  // choice and its key (12 B per vertex)
  if (odd)
    PG_LAUNCH(pf, K_ODD_SWITCH,
              9.0 * N + 8.0 + 8.0 * g->m_odd + 12.0 * g->n_odd, k_odd_switch,
              dim3(grid_for(N)), dim3(kBlock), 0, s, N, g->off, g->tgt,
              g->owner, g->key, g->sp, g->ctr);
  else
    PG_LAUNCH(pf, K_EVEN_SWITCH,
              9.0 * N + 8.0 + 8.0 * (g->m_aug - g->m_odd) +
                  12.0 * (N - g->n_odd),
              k_even_switch, dim3(grid_for(N)), dim3(kBlock), 0, s, N, g->off,
              g->tgt, g->owner, g->key, g->sp, g->ctr);
  pg_status st = read_ctr(g, s);
  if (st != PG_OK) return st;
  if (g->hctr[C_ERR] & ERR_LISTWALK)
    return pg_fail(PG_EINTERNAL, "list ranking walk exceeded its bound");
  if (g->hctr[C_ERR] & ERR_RANKCOUNT)
    return pg_fail(PG_EINTERNAL, "list ranking lost elements");
  *count = g->hctr[C_SWITCH];
  return PG_OK;
}

}  // namespace pgk
