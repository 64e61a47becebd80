// Count valuations for games whose priorities repeat: the paper's own
// representation (section 3, "Valuations": a finite valuation counts how
// often each priority occurs on the play to the sink) computed the paper's
// way (section 5, "Formal reduction to list ranking"): one list ranking over
// the Euler tour of the tree of finite vertices rooted at the sink, with the
// weight +1 at pri(v) on the edge entering v and -1 on the edge leaving it,
// and vector addition as the operator.  The exclusive prefix at the edge
// leaving v is Val(v).
//
// Steps per valuation (after the walks of pg_val.hip have classified every
// vertex as finite or top):
//   1. compaction: finite vertex v gets position f; element 0 is the sink's
//      list head, 2f+1 the edge entering v, 2f+2 the edge leaving it.  An
//      element is {next, v | bit 31 on the edge leaving v, column of
//      pri(v)}: 16 bytes, so one load per list step brings its weight (a
//      random access costs a whole cache line either way); top vertices get
//      -1 in the first count column, so a comparison reads one row;
//   2. the list by the atomic-exchange construction (section 5,
//      "Constructing the list ranking instance in parallel"): start(x) is
//      the end of x's list so far; every finite v swaps the edge leaving v
//      into start(parent) and links the previous end to the edge entering v;
//      a last pass links the end of every list to the edge leaving its
//      vertex.  The sink's children are the exception: early on most Even
//      vertices choose the sink, and millions of exchanges on its one
//      pointer serialise.  They are chained instead in position order from a
//      scan of "my parent is the sink" flags (any order of the children
//      gives an Euler tour, and this one keeps the sink's part of the tour
//      in increasing memory order); the last of them ends the tour;
//   3. list ranking by sublists (section 5, "List ranking") with count
//      vectors of dw ints as weights: level-1 sums, recursive levels, the top
//      level by pointer jumping in LDS, bases handed back down.  The level-1
//      walk leaves at the edge leaving v the prefix within its sublist in
//      v's count row, with the sublist's number in the row's last column
//      when the priorities leave it free (else in the element's spare
//      word), so that one coalesced pass over the positions adds each
//      sublist's base instead of a second walk.
// Switching compares count rows by Maxdiff (the largest column that differs
// decides by the parity of its priority); top is above every count vector.
#include <algorithm>

#include "pg_common.h"

namespace pgk {

constexpr int kVTopThreads = 1024;
constexpr int kVTopInts = 8192;   // LDS ints holding the top level's sums

__host__ __device__ constexpr int vtop_max(int D) { return kVTopInts / D; }

// ---------------------------------------------------------------------------
// set-up: distinct priorities and each vertex's column
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t decode_signed(uint32_t k) {
  // inverse of the signed-priority key (odd descending, then even ascending)
  return k < 0x80000000u ? (int32_t)(0x7fffffffu - k)
                         : (int32_t)(k - 0x80000000u);
}

__global__ void k_cnt_count_distinct(const uint32_t *skS, int64_t n,
                                     int32_t *ctr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool first = i < n && (i == 0 || skS[i] != skS[i - 1]);
  count_block(&ctr[C_DIST_MISC], first);
}

// only launched once at most kCountMax distinct keys are known to exist
__global__ void k_cnt_write_distinct(const uint32_t *skS, int64_t n,
                                     int32_t *vals, int32_t *ctr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || (i > 0 && skS[i] == skS[i - 1])) return;
  const int slot = atomicAdd(&ctr[C_MISC], 1);
  if (slot < kCountMax) vals[slot] = decode_signed(skS[i]);
}

__global__ void k_cnt_pidx(const int32_t *pri, int64_t n,
                           const int32_t *__restrict__ vals, int d,
                           uint8_t *pidx) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t p = pri[v];
  int lo = 0, hi = d - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (vals[mid] < p) lo = mid + 1;
    else hi = mid;
  }
  pidx[v] = (uint8_t)lo;
}

// ---------------------------------------------------------------------------
// the Euler list of the tree of finite vertices
// ---------------------------------------------------------------------------
__global__ void k_cnt_flags(int32_t N, const uint8_t *rs, uint32_t *f,
                            const int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < N) f[v] = rs[v] == 1;
}

// Positions of the finite vertices, the payloads of their two elements and
// the initial list ends; the top marker in the count rows of top vertices.
template <int D>
__global__ void k_cnt_compact(int32_t N, const uint8_t *__restrict__ rs,
                              const uint32_t *__restrict__ fscan,
                              const uint8_t *__restrict__ pidx, int32_t *fpos,
                              int32_t *fvert, int32_t *start, int4 *elem,
                              int32_t *cnt, int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  const int32_t nF = ctr[C_NFIN];
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v == 0) elem[0] = make_int4(-1, N, 0, 0);  // the head: no weight
  if (v >= N) return;
  const uint8_t st = rs[v];
  if (st == 2) cnt[v * D] = -1;
  if (st != 1) return;
  const int32_t f = (int32_t)fscan[v];
  if (f >= nF) {  // the finite count and the compaction disagree
    atomicOr(&ctr[C_ERR], ERR_RANKCOUNT);
    return;
  }
  fpos[v] = f;
  fvert[f] = (int32_t)v;
  start[f] = 2 * f + 1;
  // whole 16-byte elements (the links are filled in by the next kernels)
  const int32_t col = pidx[v];
  elem[2 * f + 1] = make_int4(-1, (int32_t)v, col, 0);
  elem[2 * f + 2] = make_int4(-1, (int32_t)v | (int32_t)0x80000000, col, 0);
}

// Every finite v whose parent is not the sink appends the tour of its
// subtree to its parent's list; the others raise their flag for the scan.
__global__ void k_cnt_link(int32_t N, const int32_t *__restrict__ fvert,
                           const int2 *__restrict__ sp,
                           const int32_t *__restrict__ fpos, int32_t *start,
                           int4 *elem, uint32_t *sink_flag,
                           const int32_t *ctr) {
  if (ctr[C_ABORT] || (ctr[C_ERR] & ERR_RANKCOUNT)) return;
  const int32_t nF = ctr[C_NFIN];
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nF) return;
  const int32_t v = fvert[f];
  const int32_t u = sp[v].x;                 // finite or the sink
  sink_flag[f] = u == N;
  if (u == N) return;
  const int32_t old = atomicExch(&start[fpos[u]], (int32_t)(2 * f + 2));
  elem[old].x = (int32_t)(2 * f + 1);
}

// The end of every finite vertex's list leads to the edge leaving it; the
// sink's children are listed by their rank among them.
__global__ void k_cnt_close(const int32_t *__restrict__ start,
                            const uint32_t *__restrict__ sink_flag,
                            const uint32_t *__restrict__ sink_rank,
                            int32_t *sink_kids, int4 *elem,
                            const int32_t *ctr) {
  if (ctr[C_ABORT] || (ctr[C_ERR] & ERR_RANKCOUNT)) return;
  const int32_t nF = ctr[C_NFIN];
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nF) return;
  elem[start[f]].x = (int32_t)(2 * f + 2);
  if (sink_flag[f]) sink_kids[sink_rank[f]] = (int32_t)f;
}

// The sink's list: head -> tour(c0) -> tour(c1) -> ... -> end, c_r being
// its r-th child in position order.
__global__ void k_cnt_sink_chain(const uint32_t *__restrict__ sink_flag,
                                 const uint32_t *__restrict__ sink_rank,
                                 const int32_t *__restrict__ sink_kids,
                                 int4 *elem, const int32_t *ctr) {
  if (ctr[C_ABORT] || (ctr[C_ERR] & ERR_RANKCOUNT)) return;
  const int32_t nF = ctr[C_NFIN];
  const int64_t S =
      nF > 0 ? (int64_t)sink_rank[nF - 1] + sink_flag[nF - 1] : 0;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r == 0) elem[0].x = S > 0 ? 2 * sink_kids[0] + 1 : -1;
  if (r >= S) return;
  elem[2 * sink_kids[r] + 2].x = (r + 1 < S) ? 2 * sink_kids[r + 1] + 1 : -1;
}

// ---------------------------------------------------------------------------
// vector list ranking
// ---------------------------------------------------------------------------
// adds s at column col without indexing a register array at run time
template <int D>
__device__ __forceinline__ void add_unit(int32_t (&a)[D], int col,
                                         int32_t s) {
#pragma unroll
  for (int i = 0; i < D; ++i) a[i] += (i == col) ? s : 0;
}

template <int D>
__device__ __forceinline__ void load_vec(const int32_t *p, int32_t (&a)[D]) {
  const int4 *q = reinterpret_cast<const int4 *>(p);
#pragma unroll
  for (int i = 0; i < D / 4; ++i) {
    const int4 x = q[i];
    a[4 * i] = x.x;
    a[4 * i + 1] = x.y;
    a[4 * i + 2] = x.z;
    a[4 * i + 3] = x.w;
  }
}

template <int D>
__device__ __forceinline__ void store_vec(int32_t *p, const int32_t (&a)[D]) {
  int4 *q = reinterpret_cast<int4 *>(p);
#pragma unroll
  for (int i = 0; i < D / 4; ++i)
    q[i] = make_int4(a[4 * i], a[4 * i + 1], a[4 * i + 2], a[4 * i + 3]);
}

// Level 1: each splitter (element index a multiple of the stride s0, a
// power of two; element 0, the head, is one) sums the weights of its
// sublist.  At the edge leaving v it writes the sum so far (v's prefix
// within the sublist) to v's count row, and the sublist's number to the
// row's last column when `spare` (fewer distinct priorities than columns:
// that column is zero in every count vector), else to the element's fourth
// word (only this walk touches the element).
template <int D>
__global__ __launch_bounds__(kBlock) void k_vlr_sum1(
    int32_t N, int4 *elem, int per_thread, int s0, int spare, int32_t *vsum,
    int32_t *next, int32_t *cnt, int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  const int64_t L = 2 * (int64_t)ctr[C_NFIN] + 1;
  const int64_t nsplit = level_size(L, 1, s0);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  for (int k = 0; k < per_thread; ++k) {
    const int64_t j = t + (int64_t)k * nthreads;
    if (j >= nsplit) break;
    int64_t e = j * s0;
    int32_t acc[D] = {};
    int64_t steps = 0;
    for (;;) {
      const int4 el = elem[e];
      const int32_t x = el.y & 0x7fffffff;
      if (x < N) {
        if (el.y < 0) {
          int32_t r[D];
#pragma unroll
          for (int i = 0; i < D; ++i) r[i] = acc[i];
          if (spare) r[D - 1] = (int32_t)j;
          else reinterpret_cast<int32_t *>(elem)[4 * e + 3] = (int32_t)j;
          store_vec<D>(cnt + (int64_t)x * D, r);
        }
        add_unit<D>(acc, el.z, el.y < 0 ? -1 : 1);
      }
      e = el.x;
      if (e < 0 || (e & (s0 - 1)) == 0) break;
      if (++steps > L) {
        atomicOr(&ctr[C_ERR], ERR_LISTWALK);
        e = -1;
        break;
      }
    }
    store_vec<D>(vsum + j * D, acc);
    next[j] = e < 0 ? -1 : (int32_t)(e / s0);
  }
}

// Level k >= 2: the same over the list of level-(k-1) splitters.
template <int D>
__global__ __launch_bounds__(kBlock) void k_vlr_sumk(
    const int32_t *__restrict__ lnext, const int32_t *__restrict__ lw,
    int level, int s0, int32_t *vsum, int32_t *next, int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  const int64_t L = 2 * (int64_t)ctr[C_NFIN] + 1;
  const int64_t size = level_size(L, level, s0);
  const int64_t nsplit = level_size(L, level + 1, s0);
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nsplit) return;
  int64_t e = j * kStrideUp;
  int32_t acc[D] = {};
  int64_t steps = 0;
  for (;;) {
    int32_t w[D];
    load_vec<D>(lw + e * D, w);
#pragma unroll
    for (int i = 0; i < D; ++i) acc[i] += w[i];
    e = lnext[e];
    if (e < 0 || e % kStrideUp == 0) break;
    if (++steps > size) {
      atomicOr(&ctr[C_ERR], ERR_LISTWALK);
      e = -1;
      break;
    }
  }
  store_vec<D>(vsum + j * D, acc);
  next[j] = e < 0 ? -1 : (int32_t)(e / kStrideUp);
}

// The top level (at most vtop_max(D) nodes, head = 0) in one block: suffix
// sums by pointer jumping in LDS, then base = total - suffix.  The whole tour
// sums to the zero vector (every vertex is entered and left once).
template <int D>
__global__ __launch_bounds__(kVTopThreads) void k_vlr_top(
    const int32_t *__restrict__ lnext, const int32_t *__restrict__ lw,
    int level, int s0, int32_t *base, int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  constexpr int TM = vtop_max(D);
  constexpr int per = (TM + kVTopThreads - 1) / kVTopThreads;
  __shared__ int32_t nx[TM];
  __shared__ int32_t sm[TM * D];
  const int64_t L0 = 2 * (int64_t)ctr[C_NFIN] + 1;
  const int32_t T = (int32_t)level_size(L0, level, s0);
  if (T > TM) {
    if (threadIdx.x == 0) atomicOr(&ctr[C_ERR], ERR_LISTWALK);
    return;
  }
  for (int k = 0; k < per; ++k) {
    const int i = threadIdx.x + k * kVTopThreads;
    if (i >= TM) break;
    nx[i] = (i < T) ? lnext[i] : -1;
#pragma unroll
    for (int c = 0; c < D; ++c) sm[i * D + c] = (i < T) ? lw[i * D + c] : 0;
  }
  __syncthreads();
  for (int round = 0; (1 << round) < T; ++round) {
    int32_t nn[per], ss[per][D];
    for (int k = 0; k < per; ++k) {
      const int i = threadIdx.x + k * kVTopThreads;
      if (i >= TM) break;
      const int p = nx[i];
      nn[k] = (p >= 0) ? nx[p] : -1;
#pragma unroll
      for (int c = 0; c < D; ++c)
        ss[k][c] = sm[i * D + c] + ((p >= 0) ? sm[p * D + c] : 0);
    }
    __syncthreads();
    for (int k = 0; k < per; ++k) {
      const int i = threadIdx.x + k * kVTopThreads;
      if (i >= TM) break;
      nx[i] = nn[k];
#pragma unroll
      for (int c = 0; c < D; ++c) sm[i * D + c] = ss[k][c];
    }
    __syncthreads();
  }
  for (int k = 0; k < per; ++k) {
    const int i = threadIdx.x + k * kVTopThreads;
    if (i >= T) break;
#pragma unroll
    for (int c = 0; c < D; ++c) base[i * D + c] = sm[c] - sm[i * D + c];
  }
  if (threadIdx.x < D && sm[threadIdx.x] != 0)
    atomicOr(&ctr[C_ERR], ERR_RANKCOUNT);
}

// Hands each node of a level-k sublist its exclusive prefix vector.
template <int D>
__global__ __launch_bounds__(kBlock) void k_vlr_distk(
    const int32_t *__restrict__ lnext, const int32_t *__restrict__ lw,
    int level, int s0, const int32_t *__restrict__ sbase, int32_t *lbase,
    const int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  const int64_t L = 2 * (int64_t)ctr[C_NFIN] + 1;
  const int64_t size = level_size(L, level, s0);
  const int64_t nsplit = level_size(L, level + 1, s0);
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nsplit) return;
  int64_t e = j * kStrideUp;
  int32_t b[D];
  load_vec<D>(sbase + j * D, b);
  for (int64_t steps = 0; steps <= size; ++steps) {
    store_vec<D>(lbase + e * D, b);
    int32_t w[D];
    load_vec<D>(lw + e * D, w);
#pragma unroll
    for (int i = 0; i < D; ++i) b[i] += w[i];
    e = lnext[e];
    if (e < 0 || e % kStrideUp == 0) break;
  }
}

// Val(v) for the finite vertex v = fvert[f] at position f: the exclusive
// prefix at the edge leaving v, i.e. the base of its level-1 sublist plus
// the prefix within the sublist that the level-1 walk left in v's row.
// Positions follow vertex order, so the rows are read and written in order.
// (A list the set-up flagged as inconsistent is not read: its elements need
// not all have been written.)
template <int D>
__global__ __launch_bounds__(kBlock) void k_vlr_emit1(
    int32_t N, const int32_t *__restrict__ fvert, const int4 *__restrict__ elem,
    int spare, const int32_t *__restrict__ sbase, int64_t nbase, int32_t *cnt,
    const int32_t *ctr) {
  if (ctr[C_ABORT] || (ctr[C_ERR] & ERR_RANKCOUNT)) return;
  const int64_t nF = ctr[C_NFIN];
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nF) return;
  const int32_t x = fvert[f];
  if ((uint32_t)x >= (uint32_t)N) return;
  int32_t a[D], b[D];
  load_vec<D>(cnt + (int64_t)x * D, a);
  int32_t sj;
  if (spare) {
    sj = a[D - 1];
    a[D - 1] = 0;
  } else {
    sj = elem[2 * f + 2].w;
  }
  if ((uint32_t)sj >= (uint64_t)nbase) return;
  load_vec<D>(sbase + (int64_t)sj * D, b);
#pragma unroll
  for (int i = 0; i < D; ++i) a[i] += b[i];
  store_vec<D>(cnt + (int64_t)x * D, a);
}

// ---------------------------------------------------------------------------
// switching on count valuations
// ---------------------------------------------------------------------------
// -1: a below b, 0: equal, 1: above.  Top equals top and is above every
// count vector; otherwise the largest differing column decides: a larger
// count is better at an even priority, worse at an odd one.
template <int D>
__device__ __forceinline__ int vcmp(bool ta, const int32_t (&a)[D], bool tb,
                                    const int32_t (&b)[D], uint32_t odd_cols) {
  if (ta || tb) return ta == tb ? 0 : (ta ? 1 : -1);
  int r = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    if (a[i] != b[i]) {
      const bool even = !((odd_cols >> i) & 1u);
      r = ((a[i] < b[i]) == even) ? -1 : 1;
    }
  }
  return r;
}

// the valuation of vertex u (u == N: the sink, the zero vector); returns
// whether it is top (the marker -1 in the first column)
template <int D>
__device__ __forceinline__ bool load_val(const int32_t *cnt, int32_t u,
                                         int32_t (&a)[D]) {
  load_vec<D>(cnt + (int64_t)u * D, a);
  return a[0] < 0;
}

// All_Odd (section 4): the first successor of least valuation, if strictly
// below the current choice.
template <int D>
__global__ __launch_bounds__(kBlock) void k_cnt_odd_switch(
    int32_t N, int64_t count, const int32_t *__restrict__ ids,
    const int64_t *__restrict__ off, const int32_t *__restrict__ tgt,
    const int32_t *__restrict__ cnt, uint32_t odd_cols,
    const int32_t *__restrict__ pri, int2 *sp,
    int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool sw = false;
  const int2 me = t < count ? sp[ids[t]] : make_int2(0, kTopMark);
  // a vertex known to stay top has only top successors: no switch
  if (me.y != kTopMark) {
    const int32_t v = ids[t];
    const int64_t e0 = off[v], e1 = off[v + 1];
    // the current choice is normally in the row: its valuation comes with
    // the row's loads (a strategy given at the C ABI may name another vertex)
    const int32_t cur = me.x;
    int32_t cv[D];
    bool ct = false, have_c = false;
    int32_t best = tgt[e0];
    int32_t bv[D];
    bool bt = load_val<D>(cnt, best, bv);
    if (best == cur) {
      ct = bt;
      have_c = true;
#pragma unroll
      for (int i = 0; i < D; ++i) cv[i] = bv[i];
    }
    for (int64_t e = e0 + 1; e < e1; ++e) {
      const int32_t u = tgt[e];
      int32_t uv[D];
      const bool ut = load_val<D>(cnt, u, uv);
      if (u == cur) {
        ct = ut;
        have_c = true;
#pragma unroll
        for (int i = 0; i < D; ++i) cv[i] = uv[i];
      }
      if (vcmp<D>(ut, uv, bt, bv, odd_cols) < 0) {
        best = u;
        bt = ut;
#pragma unroll
        for (int i = 0; i < D; ++i) bv[i] = uv[i];
      }
    }
    if (!have_c) ct = load_val<D>(cnt, cur, cv);
    if (vcmp<D>(bt, bv, ct, cv, odd_cols) < 0) {
      sp[v] = make_int2(best, pri[best]);
      sw = true;
    }
  }
  count_block(&ctr[C_DIST_SW], sw);
}

// All_Even, greedy all-switches (section 3): the sink first, then the row;
// the first option of greatest valuation, if strictly above the current one.
template <int D>
__global__ __launch_bounds__(kBlock) void k_cnt_even_switch(
    int32_t N, int64_t count, const int32_t *__restrict__ ids,
    const int64_t *__restrict__ off, const int32_t *__restrict__ tgt,
    const int32_t *__restrict__ cnt, uint32_t odd_cols,
    const int32_t *__restrict__ pri, int2 *sp,
    int32_t *ctr) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool sw = false;
  const int2 me = t < count ? sp[ids[t]] : make_int2(0, kTopMark);
  // a vertex known to stay top keeps its choice
  if (me.y != kTopMark) {
    const int32_t v = ids[t];
    const int64_t e0 = off[v], e1 = off[v + 1];
    // the current choice is the sink (the zero vector) or normally in the
    // row (see All_Odd)
    const int32_t cur = me.x;
    int32_t cv[D] = {};
    bool ct = false, have_c = cur == N;
    int32_t best = N;
    int32_t bv[D] = {};
    bool bt = false;
    for (int64_t e = e0; e < e1; ++e) {
      const int32_t u = tgt[e];
      int32_t uv[D];
      const bool ut = load_val<D>(cnt, u, uv);
      if (u == cur) {
        ct = ut;
        have_c = true;
#pragma unroll
        for (int i = 0; i < D; ++i) cv[i] = uv[i];
      }
      if (vcmp<D>(ut, uv, bt, bv, odd_cols) > 0) {
        best = u;
        bt = ut;
#pragma unroll
        for (int i = 0; i < D; ++i) bv[i] = uv[i];
      }
    }
    if (!have_c) ct = load_val<D>(cnt, cur, cv);
    if (vcmp<D>(bt, bv, ct, cv, odd_cols) > 0) {
      sp[v] = make_int2(best, best == N ? 2147483647 : pri[best]);
      sw = true;
    }
  }
  count_block(&ctr[C_DIST_SW], sw);
}

// ---------------------------------------------------------------------------
// Bellman-Ford best responses (section 4: shortest paths to the sink under
// the valuation order; section 6 compares them with one-player SI).  Labels
// are count rows; a vertex without a path to the sink yet carries the top
// marker.  Jacobi rounds read one buffer and write the other.
// ---------------------------------------------------------------------------
template <int D>
__global__ void k_bf_init(int32_t N, int32_t *lab) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v > N) return;
  int32_t z[D] = {};
  if (v < N) z[0] = -1;   // no label yet; the sink's row stays zero
  store_vec<D>(lab + v * D, z);
}

// An Even vertex takes sigma(v)'s label, an Odd vertex its least successor
// label (top when none has a label), plus one at pri(v).  Counts the
// vertices whose label changed.
template <int D>
__global__ __launch_bounds__(kBlock) void k_bf_round(
    int32_t N, const int64_t *__restrict__ off,
    const int32_t *__restrict__ tgt, const uint8_t *__restrict__ owner,
    const uint8_t *__restrict__ pidx, const int2 *__restrict__ sp,
    const int32_t *__restrict__ old, int32_t *nw, uint32_t odd_cols,
    int32_t *ctr) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool changed = false;
  if (v < N) {
    int32_t bv[D];
    bool bt;
    if (owner[v] == 0) {
      bt = load_val<D>(old, sp[v].x, bv);
    } else {
      const int64_t e0 = off[v], e1 = off[v + 1];
      bt = load_val<D>(old, tgt[e0], bv);
      for (int64_t e = e0 + 1; e < e1; ++e) {
        int32_t uv[D];
        const bool ut = load_val<D>(old, tgt[e], uv);
        if (vcmp<D>(ut, uv, bt, bv, odd_cols) < 0) {
          bt = ut;
#pragma unroll
          for (int i = 0; i < D; ++i) bv[i] = uv[i];
        }
      }
    }
    if (bt) {
#pragma unroll
      for (int i = 0; i < D; ++i) bv[i] = i == 0 ? -1 : 0;
    } else {
      add_unit<D>(bv, pidx[v], 1);
    }
    int32_t ov[D];
    load_vec<D>(old + v * D, ov);
#pragma unroll
    for (int i = 0; i < D; ++i) changed |= ov[i] != bv[i];
    store_vec<D>(nw + v * D, bv);
  }
  count_block(&ctr[C_DIST_SW], changed);
}

// At the fixpoint: tau(v) = the first row position of least label, and the
// finite/top classification the winners are read from.
template <int D>
__global__ __launch_bounds__(kBlock) void k_bf_finish(
    int32_t N, const int64_t *__restrict__ off,
    const int32_t *__restrict__ tgt, const uint8_t *__restrict__ owner,
    const int32_t *__restrict__ lab, uint32_t odd_cols,
    const int32_t *__restrict__ pri, int2 *sp, uint8_t *rs) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  rs[v] = lab[v * D] < 0 ? 2 : 1;
  if (owner[v] != 1) return;
  const int64_t e0 = off[v], e1 = off[v + 1];
  int32_t best = tgt[e0];
  int32_t bv[D];
  bool bt = load_val<D>(lab, best, bv);
  for (int64_t e = e0 + 1; e < e1; ++e) {
    const int32_t u = tgt[e];
    int32_t uv[D];
    const bool ut = load_val<D>(lab, u, uv);
    if (vcmp<D>(ut, uv, bt, bv, odd_cols) < 0) {
      best = u;
      bt = ut;
#pragma unroll
      for (int i = 0; i < D; ++i) bv[i] = uv[i];
    }
  }
  sp[v] = make_int2(best, pri[best]);
}

// counts out[(N+1) * d] (rows of top vertices zero) and top[N]
template <int D>
__global__ void k_cnt_export(int32_t N, int d, const uint8_t *rs,
                             const int32_t *cnt, int32_t *out, uint8_t *top) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v > N) return;
  const bool tp = v < N && rs[v] == 2;
  if (v < N && top) top[v] = tp;
  for (int j = 0; j < d; ++j) out[v * d + j] = tp ? 0 : cnt[v * D + j];
}

}  // namespace pgk

// ===========================================================================
// host side
// ===========================================================================
namespace pgk {

constexpr int kVPerThread1 = 1;   // level-1 sublists per thread (1 measured best)

// Level-0 stride of the count valuation's list ranking: shorter sublists
// keep more walks in flight, longer ones keep the levels above small.  On
// the 4-priority games per valuation: 1M vertices 0.689 ms at 32, 0.600 at
// 16, 0.567 at 8; 10M vertices 3.47 ms at 32, 3.35 at 16, 3.39 at 8.
int count_stride(int64_t n_aug) { return n_aug >= (int64_t(1) << 22) ? 16 : 8; }

int count_levels(int64_t n_aug, int dw) {
  const int64_t Lmax = 2 * n_aug + 1;
  const int s0 = count_stride(n_aug);
  int k = 1;
  while (level_size(Lmax, k, s0) > vtop_max(dw)) ++k;
  return k;
}

pg_status count_setup(pg_game *g, hipStream_t s) {
  const int64_t N = g->n_aug;
  // the distinct priorities, from the signed-priority order
  hipLaunchKernelGGL(k_rv_keys, dim3(grid_for(N)), dim3(kBlock), 0, s, g->pri,
                     g->sk0, g->sv0, N);
  const int w = radix_sort(g->sk0, g->sv0, g->sk1, g->sv1, N, 32, g->tile_cnt,
                           g->scan_tmp, s);
  const uint32_t *skS = w ? g->sk1 : g->sk0;
  fill_i32(g->ctr, 0, C_TOTAL, s);
  hipLaunchKernelGGL(k_cnt_count_distinct, dim3(grid_for(N)), dim3(kBlock), 0,
                     s, skS, N, g->ctr);
  sum_dist(g->ctr, C_DIST_MISC, C_MISC, s);
  PG_TRY(sync_ctr(g, s));
  const int d = g->hctr[C_MISC];
  if (d < 1 || d > kCountMax)
    return pg_fail(PG_EINVAL,
                   "count valuations support at most 32 distinct priorities "
                   "(after preprocessing); this game uses " +
                       std::to_string(d));
  PG_TRY(dev_alloc(&g->cvals, kCountMax));
  fill_i32(g->ctr + C_MISC, 0, 1, s);
  hipLaunchKernelGGL(k_cnt_write_distinct, dim3(grid_for(N)), dim3(kBlock), 0,
                     s, skS, N, g->cvals, g->ctr);
  PG_HIP(hipMemcpyAsync(g->values, g->cvals, sizeof(int32_t) * d,
                        hipMemcpyDeviceToHost, s));
  PG_HIP(hipStreamSynchronize(s));
  std::sort(g->values, g->values + d);
  PG_HIP(hipMemcpyAsync(g->cvals, g->values, sizeof(int32_t) * d,
                        hipMemcpyHostToDevice, s));
  g->d = d;
  g->dw = d <= 4 ? 4 : d <= 8 ? 8 : d <= 16 ? 16 : 32;
  g->odd_cols = 0;
  for (int j = 0; j < d; ++j)
    if (g->values[j] & 1) g->odd_cols |= 1u << j;
  PG_TRY(dev_alloc(&g->pidx, N));
  PG_TRY(dev_alloc(&g->elem4, 2 * N + 2));
  hipLaunchKernelGGL(k_cnt_pidx, dim3(grid_for(N)), dim3(kBlock), 0, s, g->pri,
                     N, g->cvals, d, g->pidx);
  // count rows; the sink's row stays zero
  PG_TRY(dev_alloc(&g->cnt, (N + 1) * g->dw));
  fill_i32(g->cnt, 0, (N + 1) * g->dw, s);
  PG_TRY(dev_alloc(&g->cnt2, (N + 1) * g->dw));
  fill_i32(g->cnt2, 0, (N + 1) * g->dw, s);
  for (int k = 0; k < kMaxLevels; ++k) {
    const int64_t ns = level_size(2 * N + 1, k + 1, count_stride(N));
    PG_TRY(dev_alloc(&g->vsum[k], ns * g->dw));
    PG_TRY(dev_alloc(&g->vbase[k], ns * g->dw));
    if (ns <= 1) break;
  }
  PG_HIP(hipStreamSynchronize(s));
  return PG_OK;
}

template <int D>
static void enqueue_count_t(pg_game *g, hipStream_t s) {
  const int32_t N = (int32_t)g->n_aug;
  Prof *pf = &g->prof;
  const int32_t *gate = g->ctr + C_ABORT;
  uint32_t *flags = g->sk0, *fscan = g->sk1;
  int32_t *start = reinterpret_cast<int32_t *>(g->fh);
  // rs 1, flag 4; then the scan
  PG_LAUNCH(pf, K_LINK_INFO, 5.0 * N, k_cnt_flags, dim3(grid_for(N)),
            dim3(kBlock), 0, s, N, g->rs, flags, g->ctr);
  scan_excl_u32(flags, fscan, N, g->scan_tmp, s, pf, gate);
  // rs 1, scan 4 per vertex; column 1, fpos, fvert, start 12 and two
  // payloads 16 per finite vertex
  PG_LAUNCH(pf, K_LINK_INFO, 5.0 * N, k_cnt_compact<D>, dim3(grid_for(N)),
            dim3(kBlock), 0, s, N, g->rs, fscan, g->pidx, g->pos, g->kids,
            start, g->elem4, g->cnt, g->ctr);
  // fvert 4, play-graph record 8, flag 4, fpos 4, exchange 8, link 4
  uint32_t *sink_flag = g->sk0, *sink_rank = g->sk1;
  int32_t *sink_kids = reinterpret_cast<int32_t *>(g->sv0);
  PG_LAUNCH_NF(pf, K_LINK_BUILD, 32.0, k_cnt_link, dim3(grid_for(N)),
               dim3(kBlock), 0, s, N, g->kids, g->sp, g->pos, start,
               g->elem4, sink_flag, g->ctr);
  scan_excl_u32(sink_flag, sink_rank, N, g->scan_tmp, s, pf, gate);
  // start 4, link 4, flag and rank 8, then the sink's chain (about 12 per
  // child of the sink)
  PG_LAUNCH_NF(pf, K_LINK_BUILD, 16.0, k_cnt_close, dim3(grid_for(N)),
               dim3(kBlock), 0, s, start, sink_flag, sink_rank, sink_kids,
               g->elem4, g->ctr);
  PG_LAUNCH(pf, K_LINK_BUILD, 0.0, k_cnt_sink_chain, dim3(grid_for(N)),
            dim3(kBlock), 0, s, sink_flag, sink_rank, sink_kids, g->elem4,
            g->ctr);
  const int nl = g->nlevels;
  const int s0 = count_stride(N);
  const int64_t Lmax = 2 * (int64_t)N + 1;
  const int64_t ns1 = level_size(Lmax, 1, s0);
  const int64_t thr1 = (ns1 + kVPerThread1 - 1) / kVPerThread1;
  // a free last column of the count rows carries the sublist's number
  const int spare = g->d < D;
  // two elements (16 B each) and a count row per finite vertex
  PG_LAUNCH_NF(pf, K_LR_SUM1, 32.0 + 4.0 * D, k_vlr_sum1<D>,
               dim3(grid_for(thr1)), dim3(kBlock), 0, s, N, g->elem4,
               kVPerThread1, s0, spare, g->vsum[0], g->lv[0].next, g->cnt,
               g->ctr);
  for (int k = 1; k < nl; ++k) {
    const int64_t nsk = level_size(Lmax, k + 1, s0);
    PG_LAUNCH_NF(pf, K_LR_SUMK,
                 (4.0 * D + 4.0) * 2.0 * (double)level_size(Lmax, k, s0) /
                     (double)Lmax,
                 k_vlr_sumk<D>, dim3(grid_for(nsk)), dim3(kBlock), 0, s,
                 g->lv[k - 1].next, g->vsum[k - 1], k, s0, g->vsum[k],
                 g->lv[k].next, g->ctr);
  }
  PG_LAUNCH(pf, K_LR_TOP, (8.0 * D + 4.0) * level_size(Lmax, nl, s0),
            k_vlr_top<D>, dim3(1), dim3(kVTopThreads), 0, s,
            g->lv[nl - 1].next, g->vsum[nl - 1], nl, s0, g->vbase[nl - 1],
            g->ctr);
  for (int k = nl - 1; k >= 1; --k) {
    const int64_t nsk = level_size(Lmax, k + 1, s0);
    PG_LAUNCH_NF(pf, K_LR_DISTK,
                 (8.0 * D + 4.0) * 2.0 * (double)level_size(Lmax, k, s0) /
                     (double)Lmax,
                 k_vlr_distk<D>, dim3(grid_for(nsk)), dim3(kBlock), 0, s,
                 g->lv[k - 1].next, g->vsum[k - 1], k, s0, g->vbase[k],
                 g->vbase[k - 1], g->ctr);
  }
  // a position's vertex, its row read and written and a base row read
  PG_LAUNCH_NF(pf, K_LR_EMIT1, 4.0 + 12.0 * D, k_vlr_emit1<D>,
               dim3(grid_for(N)), dim3(kBlock), 0, s, N, g->kids, g->elem4,
               spare, g->vbase[0], ns1, g->cnt, g->ctr);
}

void enqueue_count(pg_game *g, hipStream_t s) {
  switch (g->dw) {
    case 4: enqueue_count_t<4>(g, s); break;
    case 8: enqueue_count_t<8>(g, s); break;
    case 16: enqueue_count_t<16>(g, s); break;
    default: enqueue_count_t<32>(g, s); break;
  }
}

template <int D>
static void enqueue_count_switch_t(pg_game *g, bool odd, hipStream_t s,
                                   bool fresh) {
  const int32_t N = (int32_t)g->n_aug;
  Prof *pf = &g->prof;
  if (!fresh) fill_i32(g->ctr + C_DIST_SW, 0, kDistSlots * kDistStride, s, pf);
  // per vertex: id 4, two offsets 16, current choice 8 (its row is one of
  // the row's); per edge: target 4, its top flag 1 and its count row 4 D
  if (odd) {
    const int64_t cnt = g->n_odd;
    if (cnt > 0)
      PG_LAUNCH(pf, K_ODD_SWITCH,
                28.0 * cnt + (5.0 + 4.0 * D) * g->m_odd,
                k_cnt_odd_switch<D>, dim3(grid_for(cnt)), dim3(kBlock), 0, s,
                N, cnt, g->odd_ids, g->off, g->tgt, g->cnt,
                g->odd_cols, g->pri, g->sp, g->ctr);
  } else {
    const int64_t cnt = N - g->n_odd;
    if (cnt > 0)
      PG_LAUNCH(pf, K_EVEN_SWITCH,
                28.0 * cnt +
                    (5.0 + 4.0 * D) * (g->m_aug - g->m_odd),
                k_cnt_even_switch<D>, dim3(grid_for(cnt)), dim3(kBlock), 0, s,
                N, cnt, g->even_ids, g->off, g->tgt, g->cnt,
                g->odd_cols, g->pri, g->sp, g->ctr);
  }
  // the host sums the switch count's slots when it reads the counters
}

void enqueue_count_switch(pg_game *g, bool odd, hipStream_t s, bool fresh) {
  switch (g->dw) {
    case 4: enqueue_count_switch_t<4>(g, odd, s, fresh); break;
    case 8: enqueue_count_switch_t<8>(g, odd, s, fresh); break;
    case 16: enqueue_count_switch_t<16>(g, odd, s, fresh); break;
    default: enqueue_count_switch_t<32>(g, odd, s, fresh); break;
  }
}

template <int D>
static pg_status bf_best_response_t(pg_game *g, hipStream_t s,
                                    int64_t *rounds) {
  const int32_t N = (int32_t)g->n_aug;
  Prof *pf = &g->prof;
  hipLaunchKernelGGL(k_bf_init<D>, dim3(grid_for(N + 1)), dim3(kBlock), 0, s,
                     N, g->cnt);
  int64_t r = 0;
  for (;;) {
    if (r > (int64_t)N + 2)
      return pg_fail(PG_EINTERNAL, "Bellman-Ford did not reach a fixpoint");
    fill_i32(g->ctr + C_DIST_SW, 0, kDistSlots * kDistStride, s, pf);
    // every vertex: its label and its row's labels; Odd rows dominate
    PG_LAUNCH(pf, K_ODD_SWITCH, (16.0 + 8.0 * D) * N + (4.0 + 4.0 * D) *
                                    g->m_aug,
              k_bf_round<D>, dim3(grid_for(N)), dim3(kBlock), 0, s, N, g->off,
              g->tgt, g->owner, g->pidx, g->sp, g->cnt, g->cnt2, g->odd_cols,
              g->ctr);
    PG_HIP(hipMemcpyAsync(g->hctr, g->ctr, sizeof(int32_t) * C_COUNT,
                          hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    fold_switches(g->hctr);
    if (g->prof.on) g->prof.flush();
    std::swap(g->cnt, g->cnt2);
    ++r;
    if (g->hctr[C_SWITCH] == 0) break;
  }
  hipLaunchKernelGGL(k_bf_finish<D>, dim3(grid_for(N)), dim3(kBlock), 0, s, N,
                     g->off, g->tgt, g->owner, g->cnt, g->odd_cols, g->pri,
                     g->sp, g->rs);
  *rounds = r;
  return PG_OK;
}

pg_status bf_best_response(pg_game *g, hipStream_t s, int64_t *rounds) {
  switch (g->dw) {
    case 4: return bf_best_response_t<4>(g, s, rounds);
    case 8: return bf_best_response_t<8>(g, s, rounds);
    case 16: return bf_best_response_t<16>(g, s, rounds);
    default: return bf_best_response_t<32>(g, s, rounds);
  }
}

pg_status export_counts(pg_game *g, int32_t *counts, uint8_t *top, bool dev,
                        hipStream_t s) {
  const int64_t N = g->n_aug;
  const int64_t nc = (N + 1) * g->d;
  int32_t *dc = counts;
  uint8_t *dt = top;
  // temporaries go back to where they came from (the game cache while a
  // call holds it) once the stream has drained
  struct Tmp {
    void *p[2] = {nullptr, nullptr};
    hipStream_t s = nullptr;
    ~Tmp() {
      if (p[0] || p[1]) (void)hipStreamSynchronize(s);
      for (void *x : p) dev_free(x);
    }
  } tmp;
  tmp.s = s;
  if (!dev) {
    PG_TRY(dev_alloc(&dc, nc));
    tmp.p[0] = dc;
    if (top) {
      PG_TRY(dev_alloc(&dt, N));
      tmp.p[1] = dt;
    }
  }
  const unsigned grid = grid_for(N + 1);
  switch (g->dw) {
    case 4: hipLaunchKernelGGL(k_cnt_export<4>, dim3(grid), dim3(kBlock), 0, s,
                               (int32_t)N, g->d, g->rs, g->cnt, dc, dt); break;
    case 8: hipLaunchKernelGGL(k_cnt_export<8>, dim3(grid), dim3(kBlock), 0, s,
                               (int32_t)N, g->d, g->rs, g->cnt, dc, dt); break;
    case 16: hipLaunchKernelGGL(k_cnt_export<16>, dim3(grid), dim3(kBlock), 0,
                                s, (int32_t)N, g->d, g->rs, g->cnt, dc, dt);
      break;
    default: hipLaunchKernelGGL(k_cnt_export<32>, dim3(grid), dim3(kBlock), 0,
                                s, (int32_t)N, g->d, g->rs, g->cnt, dc, dt);
      break;
  }
  if (!dev) {
    PG_TRY(copy_out(counts, dc, sizeof(int32_t) * nc, false, s));
    if (top) PG_TRY(copy_out(top, dt, N, false, s));
  }
  PG_HIP(hipStreamSynchronize(s));
  return PG_OK;
}

}  // namespace pgk
