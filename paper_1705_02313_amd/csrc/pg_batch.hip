// Many games solved together: an arena holding the disjoint union of the live
// games, each game running its own copy of Algorithm 1 (section 4).
//
// Every submitted game is validated and preprocessed on its own, exactly as
// pg_load_csr would (its modified game is therefore the solo one).  The arena
// concatenates the live modified games: vertex v of game s becomes vb_s + v,
// all games share one sink, and game s's priorities are raised by an even
// offset so that the priority ranges of different games are disjoint.  Within
// a game, order and parity of priorities are unchanged and its plays never
// leave it, so every valuation of the arena orders a game's vertices (and the
// sink) exactly as the solo valuation does; the switching rules compare keys
// within one row only.  Hence each game takes the same switches, valuation
// counts and winners as when solved alone.
//
// A step advances every live game by one best-response iteration: one
// valuation of the arena, All_Odd on the games' Odd vertices, and, for games
// whose All_Odd switched nothing, All_Even.  A game whose All_Even switched
// nothing is finished: its results are copied out and it leaves the arena at
// the next rebuild.  Rebuilds happen when queued games fit (admission by the
// arena's vertex and edge capacity, first come first served) or when finished
// games hold a quarter of the arena.
//
// A rebuild sorts nothing: every game's signed-priority order (odd
// priorities descending, then even ascending) is computed once at submission,
// and since the games' priority ranges are disjoint and grow with the slot,
// the arena's order is the games' odd parts in decreasing slot order followed
// by their even parts in increasing slot order.  Games leaving the arena are
// freed at the next rebuild, once the step that used them has finished, so a
// rebuild never waits for the device.
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "pg_common.h"

namespace pgk {

struct GameDesc {
  // the game in its own signed-priority order (local id = position)
  const int64_t *off;
  const int32_t *tgt;
  const uint8_t *owner;
  const int32_t *pri;
  int2 *saved;        // [n_aug] strategies in local ids
  uint8_t *res_winner;
  int32_t *res_sigma, *res_tau;
  const int32_t *rvperm;  // [n_aug] local id -> the caller's vertex id
  int64_t odd_pos;    // arena id of the game's first odd-priority vertex
  int64_t even_pos;   // arena id of its first even-priority vertex
  int64_t odd_eb;     // arena edge of the first row of its odd part
  int64_t even_eb;    // arena edge of the first row of its even part
  int64_t e_split;    // local edge of the first row of its even part
  int32_t n_aug, n_orig;
  int64_t m_aug;
  int32_t n_oddpri;   // vertices of odd priority (local ids 0..n_oddpri-1)
  int32_t poff;       // priority offset (even)
  int32_t init;       // 1: start from the initial strategies
};

// Arena ids are positions in the arena's signed-priority order: the games'
// odd-priority parts in decreasing slot order (higher slots hold the larger
// priorities), then their even parts in increasing slot order; each part is
// a run of the game's local ids.  Rows follow in the same order, so the
// arena is one CSR made of 2 G segments.
__device__ __forceinline__ int32_t to_arena(const GameDesc &g, int32_t t) {
  return (int32_t)(t < g.n_oddpri ? g.odd_pos + t
                                  : g.even_pos + (t - g.n_oddpri));
}
__device__ __forceinline__ int32_t to_local(const GameDesc &g, int64_t x,
                                            int64_t odd_total) {
  return (int32_t)(x < odd_total ? x - g.odd_pos
                                 : g.n_oddpri + (x - g.even_pos));
}

// index of the segment whose range [start[j], start[j+1]) holds x (empty
// segments share their start with the next one and are never returned)
__device__ __forceinline__ int find_seg(const int64_t *start, int S,
                                        int64_t x) {
  int lo = 0, hi = S - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// segment j < G: the odd part of slot G - 1 - j; else the even part of j - G
__device__ __forceinline__ int seg_game(int j, int G, bool *odd) {
  *odd = j < G;
  return j < G ? G - 1 - j : j - G;
}

__global__ void k_arena_vertices(const GameDesc *__restrict__ d,
                                  const int64_t *__restrict__ vstart, int G,
                                  int32_t N, int64_t M, int64_t *off,
                                  uint8_t *owner, int32_t *pri, int32_t *gid,
                                  uint32_t *oddf, int2 *sp) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v == 0) off[N] = M;
  if (v >= N) return;
  bool oddp;
  const int s = seg_game(find_seg(vstart, 2 * G, v), G, &oddp);
  const GameDesc &g = d[s];
  const int64_t lv = oddp ? v - g.odd_pos : g.n_oddpri + (v - g.even_pos);
  off[v] = (oddp ? g.odd_eb : g.even_eb - g.e_split) + g.off[lv];
  const uint8_t ow = g.owner[lv];
  owner[v] = ow;
  oddf[v] = ow == 1;
  pri[v] = g.pri[lv] + g.poff;
  gid[v] = s;
  int32_t x;
  if (g.init) {
    x = ow ? to_arena(g, g.tgt[g.off[lv]]) : N;
  } else {
    const int32_t l = g.saved[lv].x;
    x = (l == g.n_aug) ? N : to_arena(g, l);
  }
  sp[v].x = x;
}

__global__ void k_arena_edges(const GameDesc *__restrict__ d,
                              const int64_t *__restrict__ estart, int G,
                              int64_t M, int32_t *tgt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M) return;
  bool oddp;
  const int s = seg_game(find_seg(estart, 2 * G, e), G, &oddp);
  const GameDesc &g = d[s];
  const int64_t le = oddp ? e - g.odd_eb : g.e_split + (e - g.even_eb);
  tgt[e] = to_arena(g, g.tgt[le]);
}

// the priority of each vertex's successor (second half of sp)
__global__ void k_arena_sp_pri(const int32_t *pri, int2 *sp, int32_t N) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v == 0) sp[N] = make_int2(N, 2147483647);
  if (v >= N) return;
  const int32_t x = sp[v].x;
  sp[v].y = (x == N) ? 2147483647 : pri[x];
}

// strategies of the arena back into each live game's local ids
__global__ void k_arena_save(const GameDesc *__restrict__ d,
                             const int32_t *__restrict__ gid, const int2 *sp,
                             int32_t N, int64_t odd_total) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const GameDesc &g = d[gid[v]];
  const int32_t x = sp[v].x;
  g.saved[to_local(g, v, odd_total)].x =
      (x == N) ? g.n_aug : to_local(g, x, odd_total);
}

// results of the games that finished in this step, in the caller's ids
// (Theorem 1: W_Even is the set of top keys), as pg_solve gives them
// (all kernels after the valuation return at once when its bounded walks
// left vertices open: the host then redoes the step on the careful path)
__global__ void k_arena_export(const GameDesc *__restrict__ d,
                               const int32_t *__restrict__ gid,
                               const uint8_t *__restrict__ newly_done,
                               const int2 *sp, const int32_t *key,
                               const uint8_t *owner, int32_t N,
                               int64_t odd_total, const int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const int s = gid[v];
  if (!newly_done[s]) return;
  const GameDesc &g = d[s];
  const int32_t c = g.rvperm[to_local(g, v, odd_total)];
  const int32_t x = sp[v].x;
  const bool even = owner[v] == 0;
  int32_t cx = PG_SINK;
  if (x != N) {
    const int32_t lx = to_local(g, x, odd_total);
    cx = g.rvperm[lx];
    // an Odd choice of a dummy d_w is reported as w, the only entry of the
    // dummy's row (as pg_solve reports it)
    if (!even && cx >= g.n_orig) cx = g.rvperm[g.tgt[g.off[lx]]];
  }
  g.res_sigma[c] = even ? cx : PG_SINK;
  g.res_tau[c] = even ? PG_SINK : cx;
  if (c < g.n_orig) g.res_winner[c] = key[v] == PG_KEY_TOP ? 0 : 1;
}

// first edge of the even-priority rows of a game stored in signed order
__global__ void k_part_edge(const int64_t *off, const int32_t *ctr,
                            int64_t *out) {
  out[0] = off[ctr[C_MISC]];
}

// Odd vertices of a game (into the distributed counter C_DIST_NF)
__global__ void k_count_owner_odd(const uint8_t *owner, int64_t n,
                                  int32_t *ctr) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  count_block(&ctr[C_DIST_NF], v < n && owner[v] == 1);
}

// counts one per switching lane into cnt[game]; one atomic per wave when the
// wave's lanes all belong to the same game
__device__ __forceinline__ void count_game(int32_t *cnt, int s, bool sw) {
  const int lane = threadIdx.x & (kWave - 1);
  const int s0 = __shfl(s, 0, kWave);
  const bool same = __all(s == s0);
  const uint64_t b = __ballot(sw);
  if (same) {
    if (lane == 0 && b) atomicAdd(&cnt[s0], (int)__popcll(b));
  } else if (sw) {
    atomicAdd(&cnt[s], 1);
  }
}

constexpr int kRowBatchB = 4;

__global__ __launch_bounds__(kBlock) void k_batch_odd(
    int64_t count, const int32_t *__restrict__ ids,
    const int64_t *__restrict__ off, const int32_t *__restrict__ tgt,
    const int32_t *__restrict__ key, const int32_t *__restrict__ pri, int2 *sp,
    const int32_t *__restrict__ gid, const uint8_t *__restrict__ run,
    int32_t *cnt, const int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool sw = false;
  int s = 0;
  if (t < count) {
    const int32_t v = ids[t];
    s = gid[v];
    const int2 me = sp[v];
    // a vertex known to stay top has only top successors: no switch
    if (run[s] && me.y != kTopMark) {
      const int64_t e0 = off[v], e1 = off[v + 1];
      // the current choice's key comes with the row's gathers when it is in
      // the row (it always is in a batch: strategies start from the rows)
      const int32_t cur = me.x;
      int32_t kc = 0;
      bool have_kc = false;
      int32_t best = -1, kb = 0;
      for (int64_t b = e0; b < e1; b += kRowBatchB) {
        int32_t u[kRowBatchB], k[kRowBatchB];
#pragma unroll
        for (int j = 0; j < kRowBatchB; ++j)
          u[j] = (b + j < e1) ? tgt[b + j] : -1;
#pragma unroll
        for (int j = 0; j < kRowBatchB; ++j) k[j] = (u[j] >= 0) ? key[u[j]] : 0;
#pragma unroll
        for (int j = 0; j < kRowBatchB; ++j) {
          if (u[j] >= 0 && (best < 0 || k[j] < kb)) { kb = k[j]; best = u[j]; }
          if (u[j] == cur) { kc = k[j]; have_kc = true; }
        }
      }
      if (!have_kc) kc = key[cur];
      if (kb < kc) {
        sp[v] = make_int2(best, pri[best]);
        sw = true;
      }
    }
  }
  count_game(cnt, s, sw);
}

__global__ __launch_bounds__(kBlock) void k_batch_even(
    int32_t N, int64_t count, const int32_t *__restrict__ ids,
    const int64_t *__restrict__ off, const int32_t *__restrict__ tgt,
    const int32_t *__restrict__ key, const int32_t *__restrict__ pri, int2 *sp,
    const int32_t *__restrict__ gid, const uint8_t *__restrict__ pending,
    int32_t *cnt, const int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool sw = false;
  int s = 0;
  if (t < count) {
    const int32_t v = ids[t];
    s = gid[v];
    const int2 me = sp[v];
    // a vertex known to stay top keeps its choice
    if (pending[s] && me.y != kTopMark) {
      const int64_t e0 = off[v], e1 = off[v + 1];
      // the current choice is the sink or in the row (see k_batch_odd)
      const int32_t cur = me.x;
      int32_t best = N, kb = key[N];
      int32_t kc = kb;
      bool have_kc = cur == N;
      for (int64_t b = e0; b < e1; b += kRowBatchB) {
        int32_t u[kRowBatchB], k[kRowBatchB];
#pragma unroll
        for (int j = 0; j < kRowBatchB; ++j)
          u[j] = (b + j < e1) ? tgt[b + j] : -1;
#pragma unroll
        for (int j = 0; j < kRowBatchB; ++j) k[j] = (u[j] >= 0) ? key[u[j]] : 0;
#pragma unroll
        for (int j = 0; j < kRowBatchB; ++j) {
          if (u[j] >= 0 && k[j] > kb) { kb = k[j]; best = u[j]; }
          if (u[j] == cur) { kc = k[j]; have_kc = true; }
        }
      }
      if (!have_kc) kc = key[cur];
      if (kb > kc) {
        sp[v] = make_int2(best, best == N ? 2147483647 : pri[best]);
        sw = true;
      }
    }
  }
  count_game(cnt, s, sw);
}

// Per game, after All_Odd: one more valuation; no Odd switch ends the inner
// loop and starts an All_Even step (one more outer iteration).
__global__ void k_batch_ctl1(int G, const uint8_t *run, const int32_t *cnt_odd,
                             uint8_t *pending, int32_t *n_val,
                             int32_t *n_major, const int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= G) return;
  pending[s] = 0;
  if (!run[s]) return;
  n_val[s] += 1;
  if (cnt_odd[s] == 0) {
    pending[s] = 1;
    n_major[s] += 1;
  }
}

// The games whose inner loop ended this step (a best response) mark their
// top vertices, as a single solve does (see k_mark_top): later walks stop
// at them.  A rebuild writes the successor records afresh (no marks).
__global__ void k_batch_mark(int32_t N, const int32_t *__restrict__ gid,
                             const uint8_t *__restrict__ pending,
                             uint8_t *rs, int2 *sp, const int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N || !pending[gid[v]]) return;
  if (rs[v] == 2) sp[v].y = kTopMark;
  // the game's next inner loop starts after its Even switches: its
  // fates are found afresh (a valuation keeps only the finite fates of
  // the previous one of the same inner loop)
  rs[v] = 0;
}

// Per game, after All_Even: no Even switch finishes the game.
__global__ void k_batch_ctl2(int G, uint8_t *run, uint8_t *pending,
                             int32_t *cnt_odd, int32_t *cnt_even,
                             int64_t *sw_odd, int64_t *sw_even,
                             uint8_t *newly_done, const int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= G) return;
  newly_done[s] = 0;
  if (run[s]) {
    sw_odd[s] += cnt_odd[s];
    if (pending[s]) {
      sw_even[s] += cnt_even[s];
      if (cnt_even[s] == 0) {
        newly_done[s] = 1;
        run[s] = 0;
      }
    }
  }
  cnt_odd[s] = 0;
  cnt_even[s] = 0;
}


// ---------------------------------------------------------------------------
// Submissions in bulk: the games of one pg_batch_submit_many call are
// validated and preprocessed together over their disjoint union.  Game g's
// vertices are union ids vs[g] .. vs[g+1]-1 and its edges es[g] .. es[g+1]-1;
// its modified game (originals, then its dummies) takes ids ab[g] ..
// ab[g+1]-1 and edges aeb[g] .. aeb[g+1]-1.  Every kernel below works per
// vertex or per edge and writes what the single-game path writes for that
// game, in its own ids.
// ---------------------------------------------------------------------------
// the last g with starts[g] <= x (starts increasing, count >= 1)
__device__ __forceinline__ int bm_game(const int64_t *starts, int count,
                                       int64_t x) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (starts[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// per-game sums: one atomic per wave for the lanes of the wave's first game
// (games are contiguous, so that is nearly every lane), one per lane for the
// others.  Every lane of the wave must call it.
__device__ __forceinline__ void bm_add(unsigned long long *sum, int g,
                                       unsigned long long x) {
  const int g0 = __shfl(g, 0);
  unsigned long long part = g == g0 ? x : 0ull;
  for (int o = kWave / 2; o > 0; o >>= 1) part += __shfl_xor(part, o);
  if ((threadIdx.x & (kWave - 1)) == 0 && part) atomicAdd(&sum[g0], part);
  if (g != g0 && x) atomicAdd(&sum[g], x);
}

__device__ __forceinline__ void bm_max(int32_t *mx, int g, int32_t x) {
  const int g0 = __shfl(g, 0);
  int32_t part = g == g0 ? x : -1;
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const int32_t y = __shfl_xor(part, o);
    part = y > part ? y : part;
  }
  if ((threadIdx.x & (kWave - 1)) == 0 && part >= 0) atomicMax(&mx[g0], part);
  if (g != g0 && x >= 0) atomicMax(&mx[g], x);
}

// offsets: raw holds each game's n_g + 1 entries from ostart[g] on
template <typename OffT>
__global__ void k_bm_offsets(const OffT *raw, const int64_t *ostart,
                             const int64_t *vs, const int64_t *es, int count,
                             int64_t *uoff, int32_t *err) {
  const int64_t R = ostart[count];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= R) return;
  const int g = bm_game(ostart, count, j);
  const int64_t i = j - ostart[g];
  const int64_t ng = vs[g + 1] - vs[g], mg = es[g + 1] - es[g];
  const int64_t x = (int64_t)raw[j];
  bool bad = i == 0 && x != 0;
  if (i == ng) {
    bad |= x != mg;
  } else {
    bad |= (int64_t)raw[j + 1] <= x;
    uoff[vs[g] + i] = es[g] + x;
  }
  if (j == R - 1) uoff[vs[count]] = es[count];
  if (bad) atomicOr(&err[g], ERR_OFFSETS);
}

// targets to union ids (in place)
__global__ void k_bm_targets(int32_t *tgt, const int64_t *vs,
                             const int64_t *es, int count, int32_t *err) {
  const int64_t M = es[count];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M) return;
  const int g = bm_game(es, count, e);
  const int32_t t = tgt[e];
  if (t < 0 || (int64_t)t >= vs[g + 1] - vs[g]) {
    atomicOr(&err[g], ERR_INVAL);
    tgt[e] = (int32_t)vs[g];
  } else {
    tgt[e] = (int32_t)(vs[g] + t);
  }
}

__global__ void k_bm_vertices(const uint8_t *owner, const int32_t *pri,
                              const int64_t *vs, int count, int32_t *gid,
                              int32_t *err) {
  const int64_t N = vs[count];
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const int g = bm_game(vs, count, v);
  gid[v] = g;
  if (owner[v] > 1 || pri[v] < 0) atomicOr(&err[g], ERR_INVAL);
}

// dummies per game and the union rank of each game's first one
__global__ void k_bm_dummies(const int64_t *vs, int count,
                             const uint32_t *did, const uint32_t *xp,
                             int64_t *nxp, uint32_t *dbase) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= count) return;
  const int64_t a = vs[g], z = vs[g + 1] - 1;
  dbase[g] = did[a];
  nxp[g] = (int64_t)did[z] + xp[z] - did[a];
}

// the modified games (as k_aug_build for rank valuations): originals keep
// their rows, an edge between members of X goes to the dummy of its
// target, the dummy of the j-th member w of X' (in increasing w) is the
// game's vertex n_g + j: Even, priority j, row [w]; originals raised by K[g]
__global__ void k_bm_aug(int64_t N, const int64_t *uoff, const int32_t *utgt,
                         const uint8_t *uown, const int32_t *upri,
                         const uint8_t *inx, const uint32_t *xp,
                         const uint32_t *did, const int32_t *gid,
                         const int64_t *vs, const int64_t *es,
                         const int64_t *K, const int64_t *ab,
                         const int64_t *aeb, const uint32_t *dbase, int count,
                         int64_t *aoff, int32_t *atgt, uint8_t *aown,
                         int32_t *apri, int32_t *agid, int32_t *err) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const int g = gid[v];
  const int64_t i = v - vs[g];
  const int64_t ng = vs[g + 1] - vs[g], mg = es[g + 1] - es[g];
  const int64_t a = ab[g] + i;
  const int64_t eb = aeb[g] - es[g];   // union edge -> modified union edge
  aoff[a] = uoff[v] + eb;
  const bool vx = inx[v] != 0;
  for (int64_t e = uoff[v], end = uoff[v + 1]; e < end; ++e) {
    const int32_t w = utgt[e];
    const int64_t t = (vx && inx[w]) ? ng + (int64_t)(did[w] - dbase[g])
                                     : (int64_t)w - vs[g];
    atgt[e + eb] = (int32_t)(ab[g] + t);
  }
  aown[a] = uown[v];
  const int64_t p = (int64_t)upri[v] + K[g];
  if (p > 2147483647LL) atomicOr(&err[g], ERR_INVAL);
  apri[a] = (int32_t)p;
  agid[a] = g;
  if (xp[v]) {
    const int64_t j = (int64_t)(did[v] - dbase[g]);
    const int64_t d = ab[g] + ng + j;
    aown[d] = 0;
    apri[d] = (int32_t)j;
    atgt[aeb[g] + mg + j] = (int32_t)a;
    aoff[d] = aeb[g] + mg + j;
    agid[d] = g;
  }
  if (v == N - 1) aoff[ab[count]] = aeb[count];
}

__device__ __forceinline__ uint32_t bm_signed_key(int32_t pri) {
  const uint32_t p = (uint32_t)pri;
  return (p & 1u) ? (0x7fffffffu - p) : (0x80000000u + p);
}

// the game of each vertex of the sorted order, as the key of the stable sort
// that groups the games
__global__ void k_bm_gidkeys(const uint32_t *sv, const int32_t *agid,
                             uint32_t *k, int64_t n) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) k[p] = (uint32_t)agid[sv[p]];
}

struct BmOut {
  int64_t *off;
  int32_t *tgt;
  uint8_t *owner;
  int32_t *pri;
  int32_t *rvperm;
};

// position p of the grouped signed order holds vertex a of game g at rank
// p - ab[g]: the game's perm and the union's rank map, each row's length,
// the repeat check and the odd-priority count
__global__ void k_bm_rank(int64_t NA, const uint32_t *sv, const int32_t *agid,
                          const int32_t *apri, const int64_t *aoff,
                          const int64_t *ab, const BmOut *out, int32_t *urank,
                          int64_t *len, unsigned long long *n_oddpri,
                          int32_t *err) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int g = 0;
  unsigned long long odd = 0;
  if (p < NA) {
    const int32_t a = (int32_t)sv[p];
    g = agid[a];
    const int64_t r = p - ab[g];
    if (out[g].rvperm) out[g].rvperm[r] = (int32_t)(a - ab[g]);
    urank[a] = (int32_t)r;
    len[p] = aoff[a + 1] - aoff[a];
    const uint32_t key = bm_signed_key(apri[a]);
    odd = key < 0x80000000u;
    if (r > 0 && bm_signed_key(apri[sv[p - 1]]) == key)
      atomicOr(&err[g], ERR_DUPPRI);
    if (p == NA - 1) len[NA] = 0;
  } else {
    g = agid[sv[NA - 1]];
  }
  bm_add(n_oddpri, g, odd);
}

// each game stored in its signed order (rows keep their edge order), with
// its largest priority, Odd vertices and the edges of their rows
__global__ void k_bm_relabel(int64_t NA, const uint32_t *sv,
                             const int32_t *agid, const int64_t *aoff,
                             const int32_t *atgt, const uint8_t *aown,
                             const int32_t *apri, const int32_t *urank,
                             const int64_t *lscan, const int64_t *ab,
                             const int64_t *aeb, const BmOut *out,
                             int32_t *maxpri, unsigned long long *n_odd,
                             unsigned long long *m_odd) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int g = 0;
  int32_t pr = -1;
  unsigned long long odd = 0, oe = 0;
  if (p < NA) {
    const int32_t a = (int32_t)sv[p];
    g = agid[a];
    const int64_t r = p - ab[g];
    const BmOut o = out[g];
    const int64_t e0 = aoff[a], e1 = aoff[a + 1];
    pr = apri[a];
    odd = aown[a] == 1;
    oe = odd ? (unsigned long long)(e1 - e0) : 0ull;
    if (o.off) {
      const int64_t at = lscan[p] - aeb[g];
      o.off[r] = at;
      if (p + 1 == ab[g + 1]) o.off[r + 1] = at + (e1 - e0);
      for (int64_t e = e0; e < e1; ++e) o.tgt[at + (e - e0)] = urank[atgt[e]];
      o.owner[r] = aown[a];
      o.pri[r] = pr;
    }
  } else {
    g = agid[sv[NA - 1]];
  }
  bm_max(maxpri, g, pr);
  bm_add(n_odd, g, odd);
  bm_add(m_odd, g, oe);
}

// the first edge of each game's even-priority rows
__global__ void k_bm_split(const BmOut *out, const unsigned long long *n_oddpri,
                           int count, int64_t *e_split) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= count) return;
  e_split[g] = out[g].off ? out[g].off[n_oddpri[g]] : 0;
}


}  // namespace pgk

using namespace pgk;

namespace {

enum BState { B_QUEUED = 0, B_LIVE = 1, B_DONE = 2 };

struct BGame {
  int64_t ticket = 0;
  pg_game *g = nullptr;     // the modified game (no valuation state)
  int state = B_QUEUED;
  int slot = -1;            // index in the current arena build
  bool started = false;     // has been in an arena before
  int32_t maxpri = 0;
  int2 *saved = nullptr;
  uint8_t *res_winner = nullptr;
  int32_t *res_sigma = nullptr, *res_tau = nullptr;
  // the game's signed order: position -> the caller's id, and back (the
  // game is stored in that order from submission on)
  int32_t *rvperm = nullptr, *rvrank = nullptr;
  int64_t n_oddpri = 0, n_odd = 0, m_odd = 0;
  int64_t e_split = 0;      // first edge of the even-priority rows
  pg_stats st{};
  bool in_arena = false;    // still occupies arena vertices
  bool polled = false;      // results handed out; free once out of the arena
};

// (call with the batch's pool set, see PoolScope)
void free_bgame(BGame *b) {
  if (!b) return;
  dev_free(b->saved);
  dev_free(b->res_winner);
  dev_free(b->res_sigma);
  dev_free(b->res_tau);
  dev_free(b->rvperm);
  dev_free(b->rvrank);
  free_game(b->g);
  delete b;
}

}  // namespace

struct pg_batch {
  int device = 0;
  hipStream_t stream = nullptr;
  // Submissions may run on another thread while steps run: they preprocess
  // on a stream of their own, in memory of their own (the pool is
  // thread-safe), and take `mu` only to queue the finished game; steps,
  // polls and queries hold `mu` throughout.
  hipStream_t sub_stream = nullptr;
  std::mutex mu;
  int64_t cap_v = 0, cap_e = 0;
  int max_games = 0;
  pg_game *arena = nullptr;
  int64_t next_ticket = 1;
  std::map<int64_t, BGame *> games;
  std::deque<BGame *> queue;
  std::vector<BGame *> built;      // games of the current arena, by slot
  std::vector<BGame *> grave;      // left the arena; freed at the next rebuild
  DevPool pool;                    // memory of the submitted games
  int64_t done_vertices = 0;       // arena vertices of finished games
  int64_t queued_steps = 0;        // steps taken while a fitting game waited
  // per-slot device state
  GameDesc *d_desc = nullptr;
  // [2 G] first arena vertex / edge of each segment (odd parts by
  // decreasing slot, then even parts by increasing slot)
  int64_t *d_pstart = nullptr, *d_estart = nullptr;
  int32_t *d_gid = nullptr;
  uint8_t *d_run = nullptr, *d_pending = nullptr, *d_newly = nullptr;
  int32_t *d_cnt_odd = nullptr, *d_cnt_even = nullptr;
  int32_t *d_nval = nullptr, *d_nmaj = nullptr;
  int64_t *d_sw_odd = nullptr, *d_sw_even = nullptr;
  int32_t *d_i32 = nullptr;        // scratch
  // a step (walks, valuation, switches, control, export, the results to
  // h_res) captured per arena layout; dropped at rebuild
  hipGraphExec_t step_exec = nullptr;
  bool use_graph = true;
  // steps since the last rebuild: a layout is captured only once it has
  // served kEagerSteps steps (admissions under a steady stream rebuild
  // every few steps, and a capture costs about as much as a step)
  int64_t steps_in_layout = 0;
  // pinned: per slot newly finished (G bytes, then padding to 8), n_val,
  // n_major (4 G each), Odd and Even switches (8 G each)
  uint8_t *h_res = nullptr;
  // host mirrors and staging
  std::vector<GameDesc> h_desc;
  std::vector<int64_t> h_pstart, h_estart;
  std::vector<uint8_t> h_newly;
  std::vector<int32_t> h_nval, h_nmaj;
  std::vector<int64_t> h_sw_odd, h_sw_even;
};

namespace {

// the pinned result block of a step (see pg_batch::h_res)
size_t res_off_nval(int G) { return ((size_t)G + 7) & ~size_t(7); }
size_t res_off_nmaj(int G) { return res_off_nval(G) + 4 * (size_t)G; }
size_t res_off_swodd(int G) {
  return (res_off_nmaj(G) + 4 * (size_t)G + 7) & ~size_t(7);
}
size_t res_off_sweven(int G) { return res_off_swodd(G) + 8 * (size_t)G; }
size_t res_bytes(int G) { return res_off_sweven(G) + 8 * (size_t)G; }

void drop_step_graphs(pg_batch *b) {
  if (b->step_exec) {
    (void)hipGraphExecDestroy(b->step_exec);
    b->step_exec = nullptr;
  }
}

pg_status batch_alloc(pg_batch *b) {
  pg_game *a = new (std::nothrow) pg_game();
  if (!a) return pg_fail(PG_ENOMEM, "host allocation failed");
  b->arena = a;
  a->device = b->device;
  a->relabeled = true;   // arena ids are signed-order positions
  PG_HIP(hipStreamCreateWithFlags(&b->sub_stream, hipStreamNonBlocking));
  PG_HIP(hipHostMalloc((void **)&a->hctr, sizeof(int32_t) * C_COUNT,
                       hipHostMallocDefault));
  PG_TRY(dev_alloc(&a->ctr, C_TOTAL));
  PG_TRY(dev_alloc(&a->off, b->cap_v + 1));
  PG_TRY(dev_alloc(&a->tgt, b->cap_e));
  PG_TRY(dev_alloc(&a->owner, b->cap_v));
  PG_TRY(dev_alloc(&a->pri, b->cap_v));
  PG_TRY(alloc_state(a, b->cap_v));
  const int G = b->max_games;
  PG_TRY(dev_alloc(&b->d_desc, G));
  PG_TRY(dev_alloc(&b->d_estart, 2 * (int64_t)G));
  PG_TRY(dev_alloc(&b->d_pstart, 2 * (int64_t)G));
  PG_TRY(dev_alloc(&b->d_gid, b->cap_v));
  PG_TRY(dev_alloc(&b->d_run, G));
  PG_TRY(dev_alloc(&b->d_pending, G));
  PG_TRY(dev_alloc(&b->d_newly, G));
  PG_TRY(dev_alloc(&b->d_cnt_odd, G));
  PG_TRY(dev_alloc(&b->d_cnt_even, G));
  PG_TRY(dev_alloc(&b->d_nval, G));
  PG_TRY(dev_alloc(&b->d_nmaj, G));
  PG_TRY(dev_alloc(&b->d_sw_odd, G));
  PG_TRY(dev_alloc(&b->d_sw_even, G));
  PG_TRY(dev_alloc(&b->d_i32, 4));
  b->h_newly.resize(G);
  b->h_nval.resize(G);
  b->h_nmaj.resize(G);
  b->h_sw_odd.resize(G);
  b->h_sw_even.resize(G);
  PG_HIP(hipHostMalloc((void **)&b->h_res, res_bytes(G), hipHostMallocDefault));
  return PG_OK;
}

void batch_release(pg_batch *b) {
  if (!b) return;
  if (b->sub_stream) {
    (void)hipStreamSynchronize(b->sub_stream);
    (void)hipStreamDestroy(b->sub_stream);
  }
  {
    PoolScope ps(&b->pool);
    for (auto &kv : b->games) free_bgame(kv.second);
    for (BGame *g : b->grave) free_bgame(g);
  }
  b->pool.clear();
  drop_step_graphs(b);
  if (b->h_res) (void)hipHostFree(b->h_res);
  free_game(b->arena);
  void *ptrs[] = {b->d_desc,    b->d_estart,  b->d_pstart,
                  b->d_gid,
                  b->d_run,     b->d_pending, b->d_newly,   b->d_cnt_odd,
                  b->d_cnt_even, b->d_nval,   b->d_nmaj,    b->d_sw_odd,
                  b->d_sw_even, b->d_i32};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete b;
}

// Copies the live games' strategies out of the arena, then lays out the
// arena again with the live games plus queued games that fit.  Nothing here
// waits for the device: games that leave are freed at the next rebuild, after
// the step that last used them has been synchronised.
pg_status rebuild(pg_batch *b, bool *built_any) {
  hipStream_t s = b->stream;
  pg_game *a = b->arena;
  drop_step_graphs(b);   // the arena's sizes and slots change
  b->steps_in_layout = 0;
  {
    PoolScope ps(&b->pool);
    for (BGame *g : b->grave) free_bgame(g);
  }
  b->grave.clear();
  // save strategies of games still running
  if (!b->built.empty() && a->n_aug > 0)
    hipLaunchKernelGGL(k_arena_save, dim3(grid_for(a->n_aug)), dim3(kBlock), 0,
                       s, b->d_desc, b->d_gid, a->sp, (int32_t)a->n_aug,
                       (int64_t)a->n_oddpri);
  std::vector<BGame *> next;
  int64_t nv = 0, ne = 0;
  for (BGame *g : b->built)
    if (g->state == B_LIVE) {
      next.push_back(g);
      nv += g->g->n_aug;
      ne += g->g->m_aug;
    } else {
      g->in_arena = false;
      if (g->polled) {
        b->games.erase(g->ticket);
        b->grave.push_back(g);
      }
    }
  while (!b->queue.empty()) {
    BGame *g = b->queue.front();
    if (nv + g->g->n_aug > b->cap_v || ne + g->g->m_aug > b->cap_e ||
        (int)next.size() >= b->max_games)
      break;  // first come, first served
    b->queue.pop_front();
    g->state = B_LIVE;
    next.push_back(g);
    nv += g->g->n_aug;
    ne += g->g->m_aug;
  }
  const int G = (int)next.size();
  // host staging that lives until the copies below have run (the next
  // synchronisation of the stream happens at the end of the step)
  b->h_desc.resize(G);
  b->h_pstart.resize(2 * (size_t)G);
  b->h_estart.resize(2 * (size_t)G);
  b->h_nval.assign(G, 0);
  b->h_nmaj.assign(G, 0);
  b->h_sw_odd.assign(G, 0);
  b->h_sw_even.assign(G, 0);
  int64_t n_odd = 0, m_odd = 0, poff = 0;
  for (BGame *g : next) {
    n_odd += g->n_odd;
    m_odd += g->m_odd;
  }
  for (int i = 0; i < G; ++i) {
    BGame *g = next[i];
    GameDesc &d = b->h_desc[i];
    d.off = g->g->off;
    d.tgt = g->g->tgt;
    d.owner = g->g->owner;
    d.pri = g->g->pri;
    d.saved = g->saved;
    d.res_winner = g->res_winner;
    d.res_sigma = g->res_sigma;
    d.res_tau = g->res_tau;
    d.rvperm = g->rvperm;
    d.e_split = g->e_split;
    d.n_aug = (int32_t)g->g->n_aug;
    d.n_orig = (int32_t)g->g->n;
    d.m_aug = g->g->m_aug;
    d.n_oddpri = (int32_t)g->n_oddpri;
    d.poff = (int32_t)poff;
    d.init = g->started ? 0 : 1;
    b->h_nval[i] = (int32_t)g->st.n_valuations;
    b->h_nmaj[i] = (int32_t)g->st.n_major;
    b->h_sw_odd[i] = g->st.n_odd_switches;
    b->h_sw_even[i] = g->st.n_even_switches;
    poff += (int64_t)g->maxpri + 1;
    poff += poff & 1;
    if (poff > 2000000000LL)
      return pg_fail(PG_ENOMEM, "batch: priority space of the arena exhausted");
    g->slot = i;
    g->started = true;
    g->in_arena = true;
  }
  // the 2 G segments in arena order: odd parts by decreasing slot (higher
  // slots hold the larger priorities, which come first), then even parts
  int64_t vb = 0, eb = 0;
  for (int j = 0; j < 2 * G; ++j) {
    const bool oddp = j < G;
    const int i = oddp ? G - 1 - j : j - G;
    BGame *g = next[i];
    GameDesc &d = b->h_desc[i];
    b->h_pstart[j] = vb;
    b->h_estart[j] = eb;
    if (oddp) {
      d.odd_pos = vb;
      d.odd_eb = eb;
      vb += g->n_oddpri;
      eb += g->e_split;
    } else {
      d.even_pos = vb;
      d.even_eb = eb;
      vb += g->g->n_aug - g->n_oddpri;
      eb += g->g->m_aug - g->e_split;
    }
  }
  int64_t odd_total = 0;
  for (BGame *g : next) odd_total += g->n_oddpri;
  b->built = next;
  b->done_vertices = 0;
  *built_any = G > 0;
  a->n = a->n_aug = vb;
  a->m = a->m_aug = eb;
  if (G == 0) return PG_OK;
  // the launch and walk parameters of the arena's size class
  a->tune = tuning_for(vb);
  PG_HIP(hipMemcpyAsync(b->d_desc, b->h_desc.data(), sizeof(GameDesc) * G,
                        hipMemcpyHostToDevice, s));
  PG_HIP(hipMemcpyAsync(b->d_pstart, b->h_pstart.data(),
                        sizeof(int64_t) * 2 * G, hipMemcpyHostToDevice, s));
  PG_HIP(hipMemcpyAsync(b->d_estart, b->h_estart.data(),
                        sizeof(int64_t) * 2 * G, hipMemcpyHostToDevice, s));
  const int32_t N = (int32_t)vb;
  uint32_t *oddf = a->sk0, *oscan = a->sk1;
  hipLaunchKernelGGL(k_arena_vertices, dim3(grid_for(N)), dim3(kBlock), 0, s,
                     b->d_desc, b->d_pstart, G, N, eb, a->off, a->owner,
                     a->pri, b->d_gid, oddf, a->sp);
  hipLaunchKernelGGL(k_arena_edges, dim3(grid_for(eb)), dim3(kBlock), 0, s,
                     b->d_desc, b->d_estart, G, eb, a->tgt);
  hipLaunchKernelGGL(k_arena_sp_pri, dim3(grid_for(N)), dim3(kBlock), 0, s,
                     a->pri, a->sp, N);
  // the two players' vertex lists (their sizes are known on the host)
  scan_excl_u32(oddf, oscan, N, a->scan_tmp, s);
  hipLaunchKernelGGL(k_split_players, dim3(grid_for(N)), dim3(kBlock), 0, s,
                     a->owner, oscan, a->odd_ids, a->even_ids, N);
  int bits = 1;
  while ((int64_t(1) << bits) <= (int64_t)N + 1) ++bits;
  a->sort_bits = bits;
  a->n_oddpri = (int32_t)odd_total;
  a->n_odd = n_odd;
  a->m_odd = m_odd;
  fill_i32(a->ctr, 0, C_TOTAL, s);
  fill_u8(b->d_run, 1, G, s);
  fill_u8(b->d_pending, 0, G, s);
  fill_u8(b->d_newly, 0, G, s);
  fill_i32(b->d_cnt_odd, 0, G, s);
  fill_i32(b->d_cnt_even, 0, G, s);
  PG_HIP(hipMemcpyAsync(b->d_nval, b->h_nval.data(), 4 * (size_t)G,
                        hipMemcpyHostToDevice, s));
  PG_HIP(hipMemcpyAsync(b->d_nmaj, b->h_nmaj.data(), 4 * (size_t)G,
                        hipMemcpyHostToDevice, s));
  PG_HIP(hipMemcpyAsync(b->d_sw_odd, b->h_sw_odd.data(), 8 * (size_t)G,
                        hipMemcpyHostToDevice, s));
  PG_HIP(hipMemcpyAsync(b->d_sw_even, b->h_sw_even.data(), 8 * (size_t)G,
                        hipMemcpyHostToDevice, s));
  valuation_reset(a, s);
  return PG_OK;
}

// The kernels of a step after the valuation: All_Odd of every live game,
// the inner-loop control, All_Even of the games whose All_Odd switched
// nothing, the outer-loop control, the results of games that finished, and
// the per-slot counts and the counters to the host (h_res, hctr).
void enqueue_step_rest(pg_batch *b, hipStream_t s) {
  pg_game *a = b->arena;
  const int G = (int)b->built.size();
  const int32_t N = (int32_t)a->n_aug;
  if (a->n_odd > 0)
    hipLaunchKernelGGL(k_batch_odd, dim3(grid_for(a->n_odd)), dim3(kBlock), 0,
                       s, a->n_odd, a->odd_ids, a->off, a->tgt, a->key,
                       a->pri, a->sp, b->d_gid, b->d_run, b->d_cnt_odd,
                       a->ctr);
  hipLaunchKernelGGL(k_batch_ctl1, dim3(grid_for(G)), dim3(kBlock), 0, s, G,
                     b->d_run, b->d_cnt_odd, b->d_pending, b->d_nval,
                     b->d_nmaj, a->ctr);
  if (N > 0)
    hipLaunchKernelGGL(k_batch_mark, dim3(grid_for(N)), dim3(kBlock), 0, s, N,
                       b->d_gid, b->d_pending, a->rs, a->sp, a->ctr);
  const int64_t ne = N - a->n_odd;
  if (ne > 0)
    hipLaunchKernelGGL(k_batch_even, dim3(grid_for(ne)), dim3(kBlock), 0, s,
                       N, ne, a->even_ids, a->off, a->tgt, a->key, a->pri,
                       a->sp, b->d_gid, b->d_pending, b->d_cnt_even, a->ctr);
  hipLaunchKernelGGL(k_batch_ctl2, dim3(grid_for(G)), dim3(kBlock), 0, s, G,
                     b->d_run, b->d_pending, b->d_cnt_odd, b->d_cnt_even,
                     b->d_sw_odd, b->d_sw_even, b->d_newly, a->ctr);
  hipLaunchKernelGGL(k_arena_export, dim3(grid_for(N)), dim3(kBlock), 0, s,
                     b->d_desc, b->d_gid, b->d_newly, a->sp, a->key, a->owner,
                     N, (int64_t)a->n_oddpri, a->ctr);
  uint8_t *r = b->h_res;
  (void)hipMemcpyAsync(r, b->d_newly, G, hipMemcpyDeviceToHost, s);
  (void)hipMemcpyAsync(r + res_off_nval(G), b->d_nval, 4 * (size_t)G,
                       hipMemcpyDeviceToHost, s);
  (void)hipMemcpyAsync(r + res_off_nmaj(G), b->d_nmaj, 4 * (size_t)G,
                       hipMemcpyDeviceToHost, s);
  (void)hipMemcpyAsync(r + res_off_swodd(G), b->d_sw_odd, 8 * (size_t)G,
                       hipMemcpyDeviceToHost, s);
  (void)hipMemcpyAsync(r + res_off_sweven(G), b->d_sw_even, 8 * (size_t)G,
                       hipMemcpyDeviceToHost, s);
  (void)hipMemcpyAsync(a->hctr, a->ctr, sizeof(int32_t) * C_COUNT,
                       hipMemcpyDeviceToHost, s);
}

// One step of every live game: replayed from the graph of the current
// layout (captured at first use after each rebuild), else
// launched one kernel at a time; one host synchronisation.  When the bounded
// walks left vertices open, the careful walks, the valuation and the rest
// of the step run again (the gated kernels did nothing).
constexpr int64_t kEagerSteps = 2;

pg_status step_device(pg_batch *b, hipStream_t s) {
  pg_game *a = b->arena;
  bool ran = false;
  if (b->use_graph && b->steps_in_layout++ >= kEagerSteps) {
    hipGraphExec_t &ex = b->step_exec;
    if (!ex) {
      if (!a->cap_stream &&
          hipStreamCreateWithFlags(&a->cap_stream, hipStreamNonBlocking) !=
              hipSuccess) {
        a->cap_stream = nullptr;
        b->use_graph = false;
      }
      hipStream_t cs = a->cap_stream;
      hipError_t e = cs ? hipStreamBeginCapture(
                              cs, hipStreamCaptureModeThreadLocal)
                        : hipErrorInvalidValue;
      if (e == hipSuccess) {
        enqueue_valuation(a, cs);
        enqueue_step_rest(b, cs);
        hipGraph_t gr = nullptr;
        e = hipStreamEndCapture(cs, &gr);
        if (e == hipSuccess)
          e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        if (gr) (void)hipGraphDestroy(gr);
      }
      if (e != hipSuccess) {   // capture refused: launch eagerly from now on
        ex = nullptr;
        b->use_graph = false;
        (void)hipGetLastError();
      }
    }
    if (ex) {
      PG_HIP(hipGraphLaunch(ex, s));
      ran = true;
    }
  }
  if (!ran) {
    enqueue_valuation(a, s);
    enqueue_step_rest(b, s);
  }
  PG_HIP(hipStreamSynchronize(s));
  if (a->hctr[C_ABORT]) {
    PG_TRY(redo_valuation(a, s));
    enqueue_step_rest(b, s);
    PG_HIP(hipStreamSynchronize(s));
  }
  return valuation_status(a);
}

// pg_batch_submit_many's work on the games `idx` (indices into the call's
// arrays), all of whose arguments passed the host checks.  Games the device
// checks reject get their status and are left out; the call then runs again
// on the others (the union must hold valid games only).
pg_status submit_union(pg_batch *b, const std::vector<int> &idx,
                       const int64_t *n, const int64_t *m,
                       const void *const *offsets,
                       const int32_t *const *targets,
                       const uint8_t *const *owner,
                       const int32_t *const *priority, uint32_t flags,
                       int64_t *tickets, pg_status *status) {
  const int count = (int)idx.size();
  if (count == 0) return PG_OK;
  hipStream_t s = b->sub_stream;
  const bool dev = flags & PG_PTR_DEVICE;
  const bool i32 = flags & PG_OFFSETS_I32;
  std::vector<int64_t> hv(count + 1, 0), he(count + 1, 0), ho(count + 1, 0);
  for (int k = 0; k < count; ++k) {
    hv[k + 1] = hv[k] + n[idx[k]];
    he[k + 1] = he[k] + m[idx[k]];
    ho[k + 1] = ho[k] + n[idx[k]] + 1;
  }
  const int64_t N = hv[count], M = he[count], R = ho[count];
  // temporaries: returned to the batch's pool once the stream has drained
  struct Tmp {
    hipStream_t s;
    std::vector<void *> p;
    ~Tmp() {
      if (!p.empty()) (void)hipStreamSynchronize(s);
      for (void *x : p) dev_free(x);
    }
  } tmp{s, {}};
  auto alloc = [&](auto **ptr, int64_t c) -> pg_status {
    PG_TRY(dev_alloc(ptr, c));
    tmp.p.push_back((void *)*ptr);
    return PG_OK;
  };
  // game tables: vs, es, ostart (count + 1 each), later K, ab, aeb
  int64_t *tab = nullptr;
  PG_TRY(alloc(&tab, 6 * (int64_t)(count + 1)));
  int64_t *d_vs = tab, *d_es = tab + (count + 1), *d_os = tab + 2 * (count + 1);
  int64_t *d_K = tab + 3 * (count + 1), *d_ab = tab + 4 * (count + 1);
  int64_t *d_aeb = tab + 5 * (count + 1);
  std::vector<int64_t> htab(6 * (size_t)(count + 1), 0);
  std::copy(hv.begin(), hv.end(), htab.begin());
  std::copy(he.begin(), he.end(), htab.begin() + (count + 1));
  std::copy(ho.begin(), ho.end(), htab.begin() + 2 * (count + 1));
  PG_HIP(hipMemcpyAsync(tab, htab.data(), sizeof(int64_t) * 3 * (count + 1),
                        hipMemcpyHostToDevice, s));
  // the inputs, one slice per game
  void *raw = nullptr;
  int64_t *uoff = nullptr;
  int32_t *utgt = nullptr, *upri = nullptr, *gid = nullptr, *err = nullptr;
  uint8_t *uown = nullptr;
  if (i32) PG_TRY(alloc((int32_t **)&raw, R));
  else PG_TRY(alloc((int64_t **)&raw, R));
  PG_TRY(alloc(&uoff, N + 1));
  PG_TRY(alloc(&utgt, M));
  PG_TRY(alloc(&uown, N));
  PG_TRY(alloc(&upri, N));
  PG_TRY(alloc(&gid, N));
  PG_TRY(alloc(&err, count));
  const size_t ob = i32 ? 4 : 8;
  for (int k = 0; k < count; ++k) {
    const int q = idx[k];
    PG_TRY(copy_in((uint8_t *)raw + ob * ho[k], offsets[q],
                   ob * (n[q] + 1), dev, s));
    PG_TRY(copy_in(utgt + he[k], targets[q], sizeof(int32_t) * m[q], dev, s));
    PG_TRY(copy_in(uown + hv[k], owner[q], n[q], dev, s));
    PG_TRY(copy_in(upri + hv[k], priority[q], sizeof(int32_t) * n[q], dev,
                   s));
  }
  fill_i32(err, 0, count, s);
  if (i32)
    hipLaunchKernelGGL(k_bm_offsets<int32_t>, dim3(grid_for(R)),
                       dim3(kBlock), 0, s, (const int32_t *)raw, d_os, d_vs,
                       d_es, count, uoff, err);
  else
    hipLaunchKernelGGL(k_bm_offsets<int64_t>, dim3(grid_for(R)),
                       dim3(kBlock), 0, s, (const int64_t *)raw, d_os, d_vs,
                       d_es, count, uoff, err);
  hipLaunchKernelGGL(k_bm_targets, dim3(grid_for(M)), dim3(kBlock), 0, s,
                     utgt, d_vs, d_es, count, err);
  hipLaunchKernelGGL(k_bm_vertices, dim3(grid_for(N)), dim3(kBlock), 0, s,
                     uown, upri, d_vs, count, gid, err);
  std::vector<int32_t> herr(count);
  PG_HIP(hipMemcpyAsync(herr.data(), err, sizeof(int32_t) * count,
                        hipMemcpyDeviceToHost, s));
  PG_HIP(hipStreamSynchronize(s));
  {
    std::vector<int> ok;
    for (int k = 0; k < count; ++k) {
      if (herr[k] & ERR_OFFSETS)
        status[idx[k]] = pg_fail(PG_EINVAL,
                                 "offsets must start at 0, end at m and give "
                                 "every vertex a non-empty row");
      else if (herr[k])
        status[idx[k]] = pg_fail(PG_EINVAL,
                                 "targets must lie in [0, n), owners in "
                                 "{0, 1} and priorities be >= 0");
      else
        ok.push_back(idx[k]);
    }
    if ((int)ok.size() < count)
      return submit_union(b, ok, n, m, offsets, targets, owner, priority,
                          flags, tickets, status);
  }

  // X and its members with a predecessor in X (section 3, "The algorithm")
  uint8_t *inx = nullptr;
  uint32_t *wit = nullptr, *did = nullptr;
  int32_t *ctr = nullptr;
  PG_TRY(alloc(&inx, N));
  PG_TRY(alloc(&wit, N));
  PG_TRY(alloc(&did, N));
  PG_TRY(alloc(&ctr, C_COUNT));
  int32_t hflag = 0;
  hipLaunchKernelGGL(k_x_init, dim3(grid_for(N)), dim3(kBlock), 0, s, uown,
                     inx, N);
  fill_i32((int32_t *)wit, 0, N, s);
  for (int64_t round = 0;; round += 4) {
    if (round > 4 * N + 64)
      return pg_fail(PG_EINTERNAL, "preprocessing did not converge");
    fill_i32(ctr, 0, C_COUNT, s);
    for (int k = 0; k < 4; ++k)
      hipLaunchKernelGGL(k_x_round, dim3(grid_for(N)), dim3(kBlock), 0, s,
                         uoff, utgt, inx, wit, N, ctr);
    PG_HIP(hipMemcpyAsync(&hflag, ctr + C_MISC, sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    if (hflag == 0) break;
  }
  uint32_t *xp = wit;   // the witnesses are done with
  fill_i32((int32_t *)xp, 0, N, s);
  hipLaunchKernelGGL(k_xp_mark, dim3(grid_for(N)), dim3(kBlock), 0, s, uoff,
                     utgt, inx, xp, N);
  {
    void *stmp = nullptr;
    const size_t need = scan_excl_u32(nullptr, nullptr, N, nullptr, s);
    PG_TRY(alloc((uint8_t **)&stmp, (int64_t)need + 16));
    scan_excl_u32(xp, did, N, stmp, s);
  }
  int64_t *nxp = nullptr;
  uint32_t *dbase = nullptr;
  PG_TRY(alloc(&nxp, count));
  PG_TRY(alloc(&dbase, count));
  hipLaunchKernelGGL(k_bm_dummies, dim3(grid_for(count)), dim3(kBlock), 0, s,
                     d_vs, count, did, xp, nxp, dbase);
  std::vector<int64_t> hnxp(count);
  PG_HIP(hipMemcpyAsync(hnxp.data(), nxp, sizeof(int64_t) * count,
                        hipMemcpyDeviceToHost, s));
  PG_HIP(hipStreamSynchronize(s));

  // the modified games' sizes, places and priority shifts; games that do not
  // fit the arena are refused here (their rows are still built, not kept)
  std::vector<char> keep(count, 1);
  int64_t *hK = htab.data() + 3 * (count + 1);
  int64_t *hab = htab.data() + 4 * (count + 1);
  int64_t *haeb = htab.data() + 5 * (count + 1);
  for (int k = 0; k < count; ++k) {
    const int q = idx[k];
    const int64_t na = n[q] + hnxp[k], ma = m[q] + hnxp[k];
    hK[k] = hnxp[k] + (hnxp[k] & 1);
    hab[k + 1] = hab[k] + na;
    haeb[k + 1] = haeb[k] + ma;
    if (na > kMaxVertices) {
      status[q] = pg_fail(PG_EINVAL, "too many vertices after preprocessing");
      keep[k] = 0;
    } else if (na > b->cap_v || ma > b->cap_e) {
      status[q] = pg_fail(PG_ENOMEM, "game larger than the batch capacity");
      keep[k] = 0;
    }
  }
  const int64_t NA = hab[count], MA = haeb[count];
  if (NA > kMaxVertices)
    return pg_fail(PG_EINTERNAL, "submission union too large");
  PG_HIP(hipMemcpyAsync(d_K, hK, sizeof(int64_t) * 3 * (count + 1),
                        hipMemcpyHostToDevice, s));
  int64_t *aoff = nullptr;
  int32_t *atgt = nullptr, *apri = nullptr, *agid = nullptr;
  uint8_t *aown = nullptr;
  PG_TRY(alloc(&aoff, NA + 1));
  PG_TRY(alloc(&atgt, MA));
  PG_TRY(alloc(&aown, NA));
  PG_TRY(alloc(&apri, NA));
  PG_TRY(alloc(&agid, NA));
  hipLaunchKernelGGL(k_bm_aug, dim3(grid_for(N)), dim3(kBlock), 0, s, N, uoff,
                     utgt, uown, upri, inx, xp, did, gid, d_vs, d_es, d_K,
                     d_ab, d_aeb, dbase, count, aoff, atgt, aown, apri, agid,
                     err);

  // each game's signed-priority order: sort by the signed key, then stably
  // by game
  uint32_t *k0 = nullptr, *v0 = nullptr, *k1 = nullptr, *v1 = nullptr;
  uint32_t *tc = nullptr;
  uint8_t *rtmp = nullptr;
  PG_TRY(alloc(&k0, NA));
  PG_TRY(alloc(&v0, NA));
  PG_TRY(alloc(&k1, NA));
  PG_TRY(alloc(&v1, NA));
  PG_TRY(alloc(&tc, 256 * radix_tiles(NA)));
  PG_TRY(alloc(&rtmp, (int64_t)radix_scan_tmp_bytes(NA) + 16));
  hipLaunchKernelGGL(k_rv_keys, dim3(grid_for(NA)), dim3(kBlock), 0, s, apri,
                     k0, v0, NA);
  int w = radix_sort(k0, v0, k1, v1, NA, 32, tc, rtmp, s);
  uint32_t *svs = w ? v1 : v0, *kx = w ? k0 : k1, *vx = w ? v0 : v1;
  uint32_t *kg = w ? k1 : k0;
  hipLaunchKernelGGL(k_bm_gidkeys, dim3(grid_for(NA)), dim3(kBlock), 0, s,
                     svs, agid, kg, NA);
  int gbits = 1;
  while ((int64_t(1) << gbits) < count) ++gbits;
  const int w2 = radix_sort(kg, svs, kx, vx, NA, gbits, tc, rtmp, s);
  const uint32_t *sv = w2 ? vx : svs;

  // the games' own arrays (kept games only) and their pointer table
  std::vector<BGame *> made(count, nullptr);
  struct Made {
    hipStream_t s;
    std::vector<BGame *> *v;
    ~Made() {
      bool any = false;
      for (BGame *g : *v) any |= g != nullptr;
      if (!any) return;
      (void)hipStreamSynchronize(s);   // no kernel may still write them
      for (BGame *g : *v) free_bgame(g);
    }
  } made_guard{s, &made};
  std::vector<BmOut> hout(count, BmOut{nullptr, nullptr, nullptr, nullptr,
                                       nullptr});
  for (int k = 0; k < count; ++k) {
    if (!keep[k]) continue;
    const int q = idx[k];
    const int64_t na = hab[k + 1] - hab[k], ma = haeb[k + 1] - haeb[k];
    BGame *bg = new (std::nothrow) BGame();
    if (!bg) return pg_fail(PG_ENOMEM, "host allocation failed");
    made[k] = bg;
    bg->g = new (std::nothrow) pg_game();
    if (!bg->g) return pg_fail(PG_ENOMEM, "host allocation failed");
    pg_game *gg = bg->g;
    gg->device = b->device;
    gg->n = n[q];
    gg->m = m[q];
    gg->n_aug = na;
    gg->m_aug = ma;
    gg->relabeled = true;
    PG_TRY(dev_alloc(&gg->off, na + 1));
    PG_TRY(dev_alloc(&gg->tgt, ma));
    PG_TRY(dev_alloc(&gg->owner, na));
    PG_TRY(dev_alloc(&gg->pri, na));
    PG_TRY(dev_alloc(&bg->rvperm, na));
    PG_TRY(dev_alloc(&bg->saved, na));
    PG_TRY(dev_alloc(&bg->res_winner, n[q]));
    PG_TRY(dev_alloc(&bg->res_sigma, na));
    PG_TRY(dev_alloc(&bg->res_tau, na));
    hout[k] = BmOut{gg->off, gg->tgt, gg->owner, gg->pri, bg->rvperm};
  }
  BmOut *dout = nullptr;
  PG_TRY(alloc((uint8_t **)&dout, (int64_t)sizeof(BmOut) * count));
  PG_HIP(hipMemcpyAsync(dout, hout.data(), sizeof(BmOut) * count,
                        hipMemcpyHostToDevice, s));
  int32_t *urank = nullptr, *maxpri = nullptr;
  int64_t *len = nullptr, *lscan = nullptr, *esplit = nullptr;
  unsigned long long *cnt = nullptr;   // [3 count] odd priorities, Odd, edges
  PG_TRY(alloc(&urank, NA));
  PG_TRY(alloc(&len, NA + 1));
  PG_TRY(alloc(&lscan, NA + 1));
  PG_TRY(alloc(&maxpri, count));
  PG_TRY(alloc(&esplit, count));
  PG_TRY(alloc(&cnt, 3 * (int64_t)count));
  fill_i32((int32_t *)cnt, 0, 6 * (int64_t)count, s);
  fill_i32(maxpri, -1, count, s);
  hipLaunchKernelGGL(k_bm_rank, dim3(grid_for(NA)), dim3(kBlock), 0, s, NA,
                     sv, agid, apri, aoff, d_ab, dout, urank, len, cnt, err);
  {
    void *stmp = nullptr;
    const size_t need = scan_excl_i64(nullptr, nullptr, NA + 1, nullptr, s);
    PG_TRY(alloc((uint8_t **)&stmp, (int64_t)need + 16));
    scan_excl_i64(len, lscan, NA + 1, stmp, s);
  }
  hipLaunchKernelGGL(k_bm_relabel, dim3(grid_for(NA)), dim3(kBlock), 0, s,
                     NA, sv, agid, aoff, atgt, aown, apri, urank, lscan, d_ab,
                     d_aeb, dout, maxpri, cnt + count, cnt + 2 * count);
  hipLaunchKernelGGL(k_bm_split, dim3(grid_for(count)), dim3(kBlock), 0, s,
                     dout, cnt, count, esplit);
  std::vector<int32_t> hmax(count);
  std::vector<unsigned long long> hcnt(3 * (size_t)count);
  std::vector<int64_t> hsplit(count);
  PG_HIP(hipMemcpyAsync(herr.data(), err, sizeof(int32_t) * count,
                        hipMemcpyDeviceToHost, s));
  PG_HIP(hipMemcpyAsync(hmax.data(), maxpri, sizeof(int32_t) * count,
                        hipMemcpyDeviceToHost, s));
  PG_HIP(hipMemcpyAsync(hcnt.data(), cnt, sizeof(uint64_t) * 3 * count,
                        hipMemcpyDeviceToHost, s));
  PG_HIP(hipMemcpyAsync(hsplit.data(), esplit, sizeof(int64_t) * count,
                        hipMemcpyDeviceToHost, s));
  PG_HIP(hipStreamSynchronize(s));

  std::lock_guard<std::mutex> lock(b->mu);
  for (int k = 0; k < count; ++k) {
    BGame *bg = made[k];
    if (!bg) continue;
    const int q = idx[k];
    if (herr[k] & ERR_INVAL) {
      status[q] = pg_fail(PG_EINVAL,
                          "a priority exceeds INT32_MAX after preprocessing");
      continue;
    }
    if (herr[k] & ERR_DUPPRI) {
      status[q] = pg_fail(PG_EINVAL, "priorities must be pairwise distinct");
      continue;
    }
    bg->maxpri = hmax[k];
    bg->n_oddpri = (int64_t)hcnt[k];
    bg->n_odd = (int64_t)hcnt[count + k];
    bg->m_odd = (int64_t)hcnt[2 * count + k];
    bg->e_split = hsplit[k];
    bg->st.n = n[q];
    bg->st.m = m[q];
    bg->st.n_aug = bg->g->n_aug;
    bg->st.m_aug = bg->g->m_aug;
    bg->ticket = b->next_ticket++;
    b->games[bg->ticket] = bg;
    b->queue.push_back(bg);
    tickets[q] = bg->ticket;
    status[q] = PG_OK;
    made[k] = nullptr;   // the batch owns it now
  }
  return PG_OK;
}

}  // namespace

extern "C" {

pg_status pg_batch_create(int64_t max_vertices, int64_t max_edges,
                          int32_t max_games, void *hip_stream,
                          pg_batch **out) {
  if (!out) return pg_fail(PG_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_vertices < 1 || max_edges < 1 || max_vertices > kMaxVertices ||
      max_games < 1)
    return pg_fail(PG_EINVAL, "bad batch capacity");
  pg_batch *b = new (std::nothrow) pg_batch();
  if (!b) return pg_fail(PG_ENOMEM, "host allocation failed");
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return pg_fail(PG_EDEVICE, "no HIP device");
  }
  b->stream = (hipStream_t)hip_stream;
  b->cap_v = max_vertices;
  b->cap_e = max_edges;
  b->max_games = max_games;
  pg_status st = batch_alloc(b);
  if (st != PG_OK) {
    batch_release(b);
    return st;
  }
  *out = b;
  return PG_OK;
}

pg_status pg_batch_submit(pg_batch *b, int64_t n, int64_t m,
                          const void *offsets, const int32_t *targets,
                          const uint8_t *owner, const int32_t *priority,
                          uint32_t flags, int64_t *ticket) {
  if (!b || !ticket) return pg_fail(PG_EINVAL, "NULL argument");
  if (n < 1 || m < n) return pg_fail(PG_EINVAL, "need n >= 1 and m >= n");
  if (flags & PG_ODD_REGION)
    return pg_fail(PG_EINVAL, "a batch does not take PG_ODD_REGION games");
  hipStream_t s = b->sub_stream;
  PoolScope ps(&b->pool);   // the game's memory comes from the batch's pool
  BGame *bg = new (std::nothrow) BGame();
  if (!bg) return pg_fail(PG_ENOMEM, "host allocation failed");
  bg->g = new (std::nothrow) pg_game();
  if (!bg->g) {
    delete bg;
    return pg_fail(PG_ENOMEM, "host allocation failed");
  }
  bg->g->device = b->device;
  pg_status st = load_modified(n, m, offsets, targets, owner, priority, flags,
                               s, bg->g, kLoadRank);
  if (st == PG_OK && (bg->g->n_aug > b->cap_v || bg->g->m_aug > b->cap_e))
    st = pg_fail(PG_ENOMEM, "game larger than the batch capacity");
  if (st == PG_OK) st = dev_alloc(&bg->saved, bg->g->n_aug);
  if (st == PG_OK) st = dev_alloc(&bg->res_winner, n);
  if (st == PG_OK) st = dev_alloc(&bg->res_sigma, bg->g->n_aug);
  if (st == PG_OK) st = dev_alloc(&bg->res_tau, bg->g->n_aug);
  if (st == PG_OK) st = dev_alloc(&bg->rvperm, bg->g->n_aug);
  if (st == PG_OK) st = dev_alloc(&bg->rvrank, bg->g->n_aug);
  // the submission's own scratch (steps may be using the arena's)
  struct Scratch {
    uint32_t *k0 = nullptr, *v0 = nullptr, *k1 = nullptr, *v1 = nullptr;
    uint32_t *tc = nullptr;
    uint8_t *st = nullptr;
    int64_t *i64 = nullptr;   // [3] max priority, Odd-row edges, even split
    ~Scratch() {
      for (void *p : {(void *)k0, (void *)v0, (void *)k1, (void *)v1,
                      (void *)tc, (void *)st, (void *)i64})
        dev_free(p);
    }
  } sc;
  if (st == PG_OK) {
    const int64_t N = bg->g->n_aug;
    st = dev_alloc(&sc.k0, N);
    if (st == PG_OK) st = dev_alloc(&sc.v0, N);
    if (st == PG_OK) st = dev_alloc(&sc.k1, N);
    if (st == PG_OK) st = dev_alloc(&sc.v1, N);
    if (st == PG_OK) st = dev_alloc(&sc.tc, 256 * radix_tiles(N));
    if (st == PG_OK)
      st = dev_alloc(&sc.st, (int64_t)radix_scan_tmp_bytes(N) + 16);
    if (st == PG_OK) st = dev_alloc(&sc.i64, 3);
  }
  if (st == PG_OK) {
    // the largest priority (for the arena offsets), the game's own
    // signed-priority order (a repeated priority is an error), and its Odd
    // vertex and edge counts
    pg_game *gg = bg->g;
    const int64_t N = gg->n_aug;
    int32_t *d_max = (int32_t *)sc.i64;
    unsigned long long *d_me = (unsigned long long *)(sc.i64 + 1);
    int64_t *d_es = sc.i64 + 2;
    // every counter but the error bits (the preprocessing's priority
    // overflow is read with the rest below)
    fill_i32(gg->ctr + 1, 0, C_TOTAL - 1, s);
    fill_i32((int32_t *)sc.i64, 0, 6, s);
    fill_i32(d_max, -1, 1, s);
    hipLaunchKernelGGL(k_max_i32, dim3(256), dim3(kBlock), 0, s, gg->pri, N,
                       d_max);
    hipLaunchKernelGGL(k_rv_keys, dim3(grid_for(N)), dim3(kBlock), 0, s,
                       gg->pri, sc.k0, sc.v0, N);
    const int w = radix_sort(sc.k0, sc.v0, sc.k1, sc.v1, N, 32, sc.tc, sc.st,
                             s);
    hipLaunchKernelGGL(k_rv_finish, dim3(grid_for(N)), dim3(kBlock), 0, s,
                       w ? sc.k1 : sc.k0, w ? sc.v1 : sc.v0, bg->rvperm,
                       bg->rvrank, N, 1, gg->ctr);
    sum_dist(gg->ctr, C_DIST_MISC, C_MISC, s);
    hipLaunchKernelGGL(k_count_owner_odd, dim3(grid_for(N)), dim3(kBlock), 0,
                       s, gg->owner, N, gg->ctr);
    sum_dist(gg->ctr, C_DIST_NF, C_NFIN, s);
    hipLaunchKernelGGL(k_count_odd_edges, dim3(256), dim3(kBlock), 0, s,
                       gg->off, gg->owner, N, d_me);
    // the game is stored in its signed order from here on (its rows keep
    // their edge order); the even-priority rows start at off[n_oddpri]
    int64_t *off2 = nullptr;
    int32_t *tgt2 = nullptr, *pri2 = nullptr;
    uint8_t *own2 = nullptr;
    // without a drain: the batch's pool is reused in this stream's order
    // (submissions run on it; steps only return memory to the pool)
    st = relabel_game(gg->off, gg->tgt, gg->owner, gg->pri, bg->rvperm,
                      bg->rvrank, N, gg->m_aug, &off2, &tgt2, &own2, &pri2, s,
                      false);
    dev_free(st == PG_OK ? gg->off : off2);
    dev_free(st == PG_OK ? (void *)gg->tgt : (void *)tgt2);
    dev_free(st == PG_OK ? gg->owner : own2);
    dev_free(st == PG_OK ? gg->pri : pri2);
    if (st == PG_OK) {
      gg->off = off2;
      gg->tgt = tgt2;
      gg->owner = own2;
      gg->pri = pri2;
      gg->relabeled = true;
      hipLaunchKernelGGL(k_part_edge, dim3(1), dim3(1), 0, s, gg->off,
                         gg->ctr, d_es);
    }
    int32_t mx = 0;
    unsigned long long me = 0;
    int64_t es = 0;
    hipError_t e = hipMemcpyAsync(&mx, d_max, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(&me, d_me, sizeof(me), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(&es, d_es, sizeof(es), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess && st == PG_OK)
      st = pg_fail(PG_EDEVICE, hipGetErrorString(e));
    if (st == PG_OK) st = sync_ctr(gg, s);
    if (st == PG_OK && (gg->hctr[C_ERR] & ERR_INVAL))
      st = pg_fail(PG_EINVAL,
                   "a priority exceeds INT32_MAX after preprocessing");
    if (st == PG_OK && (gg->hctr[C_ERR] & ERR_DUPPRI))
      st = pg_fail(PG_EINVAL, "priorities must be pairwise distinct");
    bg->maxpri = mx;
    bg->n_oddpri = gg->hctr[C_MISC];
    bg->n_odd = gg->hctr[C_NFIN];
    bg->m_odd = (int64_t)me;
    bg->e_split = es;
  }
  if (st != PG_OK) {
    (void)hipStreamSynchronize(s);
    free_bgame(bg);
    return st;
  }
  bg->st.n = n;
  bg->st.m = m;
  bg->st.n_aug = bg->g->n_aug;
  bg->st.m_aug = bg->g->m_aug;
  std::lock_guard<std::mutex> lock(b->mu);
  bg->ticket = b->next_ticket++;
  b->games[bg->ticket] = bg;
  b->queue.push_back(bg);
  *ticket = bg->ticket;
  return PG_OK;
}

pg_status pg_batch_submit_many(pg_batch *b, int32_t count, const int64_t *n,
                               const int64_t *m, const void *const *offsets,
                               const int32_t *const *targets,
                               const uint8_t *const *owner,
                               const int32_t *const *priority, uint32_t flags,
                               int64_t *tickets, pg_status *status) {
  if (!b || count < 0) return pg_fail(PG_EINVAL, "bad batch or count");
  if (count == 0) return PG_OK;
  if (!n || !m || !offsets || !targets || !owner || !priority || !tickets ||
      !status)
    return pg_fail(PG_EINVAL, "NULL argument");
  if (flags & PG_ODD_REGION)
    return pg_fail(PG_EINVAL, "a batch does not take PG_ODD_REGION games");
  std::vector<int> idx;
  for (int32_t q = 0; q < count; ++q) {
    tickets[q] = -1;
    status[q] = PG_OK;
    if (n[q] < 1 || m[q] < n[q])
      status[q] = pg_fail(PG_EINVAL, "need n >= 1 and m >= n");
    else if (n[q] > kMaxVertices / 2)
      status[q] = pg_fail(PG_EINVAL, "game too large for a batch");
    else if (!offsets[q] || !targets[q] || !owner[q] || !priority[q])
      status[q] = pg_fail(PG_EINVAL, "a game array is NULL");
    else if ((flags & PG_OFFSETS_I32) && m[q] > 0x7fffffffLL)
      status[q] = pg_fail(PG_EINVAL, "int32 offsets cannot address m edges");
    if (status[q] == PG_OK) idx.push_back(q);
  }
  PoolScope ps(&b->pool);   // the games' memory comes from the batch's pool
  // chunks of at most 2^28 vertices, so that a chunk's modified games
  // (at most twice its vertices) keep 32-bit ids
  size_t at = 0;
  pg_status st = PG_OK;
  while (at < idx.size() && st == PG_OK) {
    std::vector<int> part;
    int64_t nv = 0;
    while (at < idx.size() &&
           (part.empty() || nv + n[idx[at]] <= (int64_t(1) << 28))) {
      nv += n[idx[at]];
      part.push_back(idx[at++]);
    }
    st = submit_union(b, part, n, m, offsets, targets, owner, priority, flags,
                      tickets, status);
  }
  if (st != PG_OK) {
    (void)hipStreamSynchronize(b->sub_stream);
    // what was not queued carries the call's error
    for (int q : idx)
      if (tickets[q] < 0 && status[q] == PG_OK) status[q] = st;
  }
  return st;
}

pg_status pg_batch_step(pg_batch *b, int32_t *n_live, int32_t *n_queued,
                        int32_t *n_finished) {
  if (!b) return pg_fail(PG_EINVAL, "batch is NULL");
  std::lock_guard<std::mutex> lock(b->mu);
  hipStream_t s = b->stream;
  pg_game *a = b->arena;
  // Rebuild when finished games hold a quarter of the arena, or to admit
  // queued games: once those that fit (first come, first served) add up to
  // an eighth of the arena's vertices, once a fitting game has waited
  // kAdmitSteps steps, or when nothing is live.  A rebuild costs about a
  // step, so admitting one small game per step would double the steps'
  // cost under a steady stream of arrivals.
  constexpr int64_t kAdmitSteps = 8;
  int64_t live_v = 0, live_e = 0;
  int running = 0;
  for (BGame *g : b->built)
    if (g->state == B_LIVE) {
      live_v += g->g->n_aug;
      live_e += g->g->m_aug;
      ++running;
    }
  bool admit = false;
  if (!b->queue.empty()) {
    int64_t v = live_v, e = live_e, add_v = 0;
    int fit = 0;
    for (BGame *q : b->queue) {
      if (v + q->g->n_aug > b->cap_v || e + q->g->m_aug > b->cap_e ||
          running + fit >= b->max_games)
        break;
      v += q->g->n_aug;
      e += q->g->m_aug;
      add_v += q->g->n_aug;
      ++fit;
    }
    if (fit > 0) {
      admit = 8 * add_v >= b->cap_v || b->queued_steps >= kAdmitSteps ||
              running == 0;
      if (!admit) ++b->queued_steps;
    }
  }
  const bool shrink = a->n_aug > 0 && 4 * b->done_vertices >= a->n_aug;
  const bool empty = live_v == 0;
  if (admit || shrink || (empty && !b->built.empty())) {
    bool any = false;
    PG_TRY(rebuild(b, &any));
    b->queued_steps = 0;
  }
  int32_t finished = 0;
  const int G = (int)b->built.size();
  bool live = false;
  for (BGame *g : b->built) live |= g->state == B_LIVE;
  if (live) {
    PG_TRY(step_device(b, s));
    const uint8_t *r = b->h_res;
    for (int i = 0; i < G; ++i) {
      b->h_newly[i] = r[i];
      b->h_nval[i] = ((const int32_t *)(r + res_off_nval(G)))[i];
      b->h_nmaj[i] = ((const int32_t *)(r + res_off_nmaj(G)))[i];
      b->h_sw_odd[i] = ((const int64_t *)(r + res_off_swodd(G)))[i];
      b->h_sw_even[i] = ((const int64_t *)(r + res_off_sweven(G)))[i];
    }
    for (int i = 0; i < G; ++i) {
      BGame *g = b->built[i];
      if (g->state != B_LIVE) continue;
      g->st.n_valuations = b->h_nval[i];
      g->st.n_major = b->h_nmaj[i];
      g->st.n_odd_switches = b->h_sw_odd[i];
      g->st.n_even_switches = b->h_sw_even[i];
      if (b->h_newly[i]) {
        g->state = B_DONE;
        b->done_vertices += g->g->n_aug;
        ++finished;
      }
    }
  }
  if (n_live) {
    int32_t c = 0;
    for (BGame *g : b->built) c += g->state == B_LIVE;
    *n_live = c;
  }
  if (n_queued) *n_queued = (int32_t)b->queue.size();
  if (n_finished) *n_finished = finished;
  return PG_OK;
}

pg_status pg_batch_poll_many(pg_batch *b, int32_t count,
                             const int64_t *tickets, int32_t *done,
                             uint8_t *const *winner, int32_t *const *sigma,
                             int32_t *const *tau, pg_stats *stats,
                             uint32_t flags) {
  if (!b || count < 0 || (count > 0 && (!tickets || !done)))
    return pg_fail(PG_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lock(b->mu);
  std::vector<BGame *> gs((size_t)count);
  for (int32_t i = 0; i < count; ++i) {
    auto it = b->games.find(tickets[i]);
    if (it == b->games.end()) return pg_fail(PG_EINVAL, "unknown ticket");
    gs[i] = it->second;
  }
  hipStream_t s = b->stream;
  const bool dev = flags & PG_PTR_DEVICE;
  // what each finished game hands out (nothing: a query that keeps it)
  auto sizes = [&](int32_t i, size_t *wb, size_t *sb, size_t *tb) {
    const BGame *g = gs[i];
    *wb = winner && winner[i] ? (size_t)g->g->n : 0;
    *sb = sigma && sigma[i] ? sizeof(int32_t) * (size_t)g->g->n_aug : 0;
    *tb = tau && tau[i] ? sizeof(int32_t) * (size_t)g->g->n_aug : 0;
  };
  for (int32_t i = 0; i < count; ++i) {
    done[i] = gs[i]->state == B_DONE;
    if (stats) stats[i] = gs[i]->st;
  }
  // every copy on the batch's stream, then one wait
  for (int32_t i = 0; i < count; ++i) {
    if (!done[i]) continue;
    const BGame *g = gs[i];
    size_t wb, sb, tb;
    sizes(i, &wb, &sb, &tb);
    if (wb) PG_TRY(copy_out(winner[i], g->res_winner, wb, dev, s));
    if (sb) PG_TRY(copy_out(sigma[i], g->res_sigma, sb, dev, s));
    if (tb) PG_TRY(copy_out(tau[i], g->res_tau, tb, dev, s));
  }
  PG_HIP(hipStreamSynchronize(s));
  for (int32_t i = 0; i < count; ++i) {
    if (!done[i]) continue;
    BGame *g = gs[i];
    size_t wb, sb, tb;
    sizes(i, &wb, &sb, &tb);
    if (wb + sb + tb == 0) continue;   // a query: the ticket stays
    g->polled = true;
    if (!g->in_arena) {
      b->games.erase(g->ticket);
      PoolScope ps(&b->pool);
      free_bgame(g);
    }  // else: still laid out in the arena; released at the next rebuild
  }
  return PG_OK;
}

pg_status pg_batch_poll(pg_batch *b, int64_t ticket, int32_t *done,
                        uint8_t *winner, int32_t *sigma, int32_t *tau,
                        pg_stats *stats, uint32_t flags) {
  if (!b || !done) return pg_fail(PG_EINVAL, "NULL argument");
  return pg_batch_poll_many(b, 1, &ticket, done, &winner, &sigma, &tau,
                            stats, flags);
}

pg_status pg_batch_finished(const pg_batch *b, int64_t *tickets,
                            int32_t capacity, int32_t *count) {
  if (!b || !count) return pg_fail(PG_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lock(const_cast<pg_batch *>(b)->mu);
  int32_t c = 0;
  for (const auto &kv : b->games) {
    const BGame *g = kv.second;
    if (g->state == B_DONE && !g->polled) {
      if (tickets && c < capacity) tickets[c] = g->ticket;
      ++c;
    }
  }
  *count = c;
  return PG_OK;
}

pg_status pg_batch_info(const pg_batch *b, int32_t *n_live,
                        int32_t *n_queued, int64_t *arena_vertices,
                        int64_t *arena_edges) {
  if (!b) return pg_fail(PG_EINVAL, "batch is NULL");
  std::lock_guard<std::mutex> lock(const_cast<pg_batch *>(b)->mu);
  int32_t c = 0;
  for (BGame *g : b->built) c += g->state == B_LIVE;
  if (n_live) *n_live = c;
  if (n_queued) *n_queued = (int32_t)b->queue.size();
  if (arena_vertices) *arena_vertices = b->arena->n_aug;
  if (arena_edges) *arena_edges = b->arena->m_aug;
  return PG_OK;
}

pg_status pg_batch_free(pg_batch *b) {
  if (!b) return PG_OK;
  (void)hipStreamSynchronize(b->stream);
  batch_release(b);
  return PG_OK;
}

}  // extern "C"
