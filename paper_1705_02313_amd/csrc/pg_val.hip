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
//           reduction"): enter/leave elements per inner node, one element
//           per leaf; each node's in-order point is marked on one element
//   rank    list ranking by sublists (section 5, "List ranking"): splitters
//           at fixed element strides, every sublist summed by one thread, the
//           reduced list ranked recursively and finally in LDS by pointer
//           jumping, then each sublist is walked again to emit keys
#include "pg_common.h"

namespace pgk {


// ---------------------------------------------------------------------------
// ng: nearest greater vertex along the play
// ---------------------------------------------------------------------------
// "Greater" orders vertices by priority, then by id.  With pairwise distinct
// priorities (rank valuations) the id never decides.  Count valuations use
// the ng chains only for the fates and for the parity of each cycle's
// largest priority (the largest vertex of a cycle in this order carries the
// cycle's largest priority), and for those the order need only be total:
// with a handful of repeated priorities a strict priority comparison would
// send every vertex of the largest priority on a walk to the sink or round
// its cycle, while the id breaks ties about at random on a random game and
// keeps the chains short.
// N = n_aug (the sink's id), TOP id = N + 1.  cand[v] of an unresolved v is
// the next vertex of v's play not yet compared with v; every vertex strictly
// between v and cand[v] has a smaller priority than v.  Returns ng(v), or -1
// with *u holding the candidate when the step budget runs out.
__device__ __forceinline__ int32_t ng_walk(int32_t N, const int2 *sp,
                                           const int32_t *pri,
                                           const int32_t *ng,
                                           const int32_t *cand, int32_t v,
                                           int32_t *u_io, int steps,
                                           int32_t *ctr) {
  const int pv = pri[v];
  int32_t u = *u_io;
  for (int s = 0; s < steps; ++s) {
    if (u == N) return N;
    if (u == v) {
      // v came back to itself: it has the largest priority of its cycle,
      // which must be even for an admissible sigma (section 3)
      if (pv & 1) atomicOr(&ctr[C_ERR], ERR_INADMISSIBLE);
      return N + 1;
    }
    const int pu = pri[u];
    if (pu > pv || (pu == pv && u > v)) return u;   // ties: by id
    const int32_t r = ld_relaxed(&ng[u]);
    if (r >= 0) {
      if (r >= N) return r;  // nothing larger than u (hence v) after u
      u = r;
      continue;
    }
    const int32_t c = ld_relaxed(&cand[u]);
    if (c >= 0) {
      u = c;
    } else {
      const int2 su = sp[u];
      if (su.y == kTopMark) return N + 1;   // on into a known top part
      u = su.x;
    }
  }
  *u_io = u;
  return -1;
}

// Full pass: a plain walk along the play (one 8-byte load per step, no
// reads of other threads' results).  A vertex that runs out of steps keeps
// ng = -1 and records where its walk stopped in cand; the rounds pick it up.
// Also resets the fates it does not keep.  With `dist`, the unresolved
// vertices are counted there; with `wl`, they are listed there for the
// rounds (every thread of the block takes part in either).
__global__ __launch_bounds__(kBlock) void k_ng_full(
    int32_t N, const int2 *__restrict__ sp, const int32_t *__restrict__ pri,
    int32_t *ng, int32_t *cand, int32_t *ctr, int steps, uint8_t *rs,
    int32_t *dist, int32_t *wl, int64_t wl_cap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool pending = false;
  if (i < N) {
    const int32_t v = (int32_t)i;
    // a vertex finite in the previous valuation of the same inner loop is
    // finite now (Odd's switches only lower valuations, section 4): its
    // fate stays; every other fate is found again
    // (rcand needs no clearing: the root pass writes it for every vertex
    // it leaves undecided, and the rounds read it for those only)
    if (rs[v] != 1) rs[v] = 0;
    // sp[x] = {successor of x, priority of that successor}: the first
    // comparison needs no gather, each further step one
    const int pv = pri[v];
    const int2 me = sp[v];
    int32_t u = me.x;
    int pu = me.y;
    int32_t res = -1;
    // Brent's cycle detection: a walk that meets its checkpoint again
    // circles a cycle without v whose vertices are all below v, so
    // nothing after v is larger (ng = TOP)
    int32_t mark = v;
    int lam = 1, power = 1;
    for (int st = 0; st < steps; ++st) {
      if (u == N) { res = N; break; }
      // the successor is known to stay top (a solve marks those after each
      // best response, Theorem 1): so is every play through it
      if (pu == kTopMark) { res = N + 1; break; }
      if (u == v) {
        // back at v: v has the largest priority of its cycle, which must be
        // even for an admissible sigma (section 3)
        if (pv & 1) atomicOr(&ctr[C_ERR], ERR_INADMISSIBLE);
        res = N + 1;
        break;
      }
      if (pu > pv || (pu == pv && u > v)) { res = u; break; }   // ties: by id
      if (u == mark) { res = N + 1; break; }
      if (lam == power) {
        mark = u;
        power <<= 1;
        lam = 0;
      }
      ++lam;
      const int2 su = sp[u];
      u = su.x;
      pu = su.y;
    }
    // every ng entry is written (-1: open), so no valuation clears them;
    // a candidate is read only while its vertex's ng is open
    ng[v] = res;
    if (res < 0) cand[v] = u;
    pending = res < 0;
  }
  if (dist) count_block(dist, pending);
  if (wl) append_block(&ctr[C_DIST_WLNG], wl, wl_cap, pending, (int32_t)i);
}

// A round over every vertex whose ng is still open: its walk continues from
// its candidate and jumps over other vertices' results and candidates
// (pointer jumping).  A dense pass (one coalesced read of ng per vertex),
// for the host-driven rounds that count the open vertices; the bounded
// rounds walk the full pass's lists (k_ng_round_list).  `last`: a vertex
// still open raises C_ABORT.
__global__ __launch_bounds__(kBlock) void k_ng_round(
    int32_t N, const int2 *__restrict__ sp, const int32_t *__restrict__ pri,
    int32_t *ng, int32_t *cand, int32_t *ctr, int last, int steps,
    int32_t *dist) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool pending = false;
  if (i < N) {
    const int32_t v = (int32_t)i;
    if (ld_relaxed(&ng[v]) < 0) {
      int32_t u = ld_relaxed(&cand[v]);
      const int32_t res = ng_walk(N, sp, pri, ng, cand, v, &u, steps, ctr);
      if (res >= 0) st_relaxed(&ng[v], res);
      else st_relaxed(&cand[v], u);
      pending = res < 0;
    }
  }
  if (last && __ballot(pending) && (threadIdx.x & (kWave - 1)) == 0)
    atomicOr(&ctr[C_ABORT], 1);
  if (dist) count_block(dist, pending);
}

// The same round over the vertices the full pass listed: on most
// valuations a few thousand of 10^7 vertices are open after the full pass,
// and a dense round would read every ng.  The grid holds the same number of
// blocks for each of the first min(grid, kDistSlots) lists (list_grid);
// each block takes every parts-th stretch of blockDim entries of its list.
constexpr int kListBlocks = 32;   // blocks per list at most
struct ListPart {
  int slot, part, parts;
};
__device__ __forceinline__ ListPart list_part() {
  const int nslots = gridDim.x < kDistSlots ? (int)gridDim.x : kDistSlots;
  return {(int)(blockIdx.x % nslots), (int)(blockIdx.x / nslots),
          (int)(gridDim.x / nslots)};
}

__global__ __launch_bounds__(kBlock) void k_ng_round_list(
    int32_t N, const int2 *__restrict__ sp, const int32_t *__restrict__ pri,
    int32_t *ng, int32_t *cand, int32_t *ctr, int last, int steps,
    const int32_t *__restrict__ wl, int64_t wl_cap) {
  const ListPart lp = list_part();
  const int32_t len = ctr[C_DIST_WLNG + lp.slot * kDistStride];
  const int32_t *lst = wl + (int64_t)lp.slot * wl_cap;
  bool open = false;
  for (int64_t k = (int64_t)lp.part * blockDim.x + threadIdx.x; k < len;
       k += (int64_t)lp.parts * blockDim.x) {
    const int32_t v = lst[k];
    if (ld_relaxed(&ng[v]) < 0) {
      int32_t u = ld_relaxed(&cand[v]);
      const int32_t res = ng_walk(N, sp, pri, ng, cand, v, &u, steps, ctr);
      if (res >= 0) st_relaxed(&ng[v], res);
      else st_relaxed(&cand[v], u);
      open |= res < 0;
    }
  }
  if (last && open) atomicOr(&ctr[C_ABORT], 1);
}

// ---------------------------------------------------------------------------
// root: does the ng chain end at the sink (finite) or at TOP?
// rs[v]: 0 unknown, 1 finite, 2 top.  Top vertices get key TOP.
// ---------------------------------------------------------------------------
// Follows the chain from *r_io; returns the fate, or 0 with *r_io at the
// first vertex not yet decided (-2 when ng of v itself is unresolved).
__device__ __forceinline__ int root_walk(int32_t N, const int32_t *ng,
                                         const uint8_t *rs,
                                         const int32_t *rcand, int32_t v,
                                         int32_t *r_io, int steps) {
  int32_t r = *r_io;
  if (r == -2) r = ld_relaxed(&ng[v]);
  if (r < 0) {
    *r_io = -2;
    return 0;
  }
  for (int s = 0; s < steps; ++s) {
    if (r == N) return 1;
    if (r == N + 1) return 2;
    const int known = __hip_atomic_load(&rs[r], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
    if (known) return known;
    int32_t nx = ld_relaxed(&rcand[r]);
    if (nx < 0) nx = ld_relaxed(&ng[r]);
    if (nx < 0) break;  // ng of r not resolved yet
    r = nx;
  }
  *r_io = r;
  return 0;
}

// Full pass: a plain walk along the ng chain (one load per step).  Writes
// the vertex's sort key at its signed-priority position rvpos[v], or at v
// when rvpos is null (a relabeled game): its parent when finite, N + 1 when
// top.  Also clears this valuation's Euler-list per-vertex state.  An
// undecided vertex keeps rs = 0 and records where its walk stopped in rcand
// (-2: its own ng is still open).  With `dist`, undecided vertices are
// counted there; with `wl`, listed there for the rounds.
__global__ __launch_bounds__(kBlock) void k_root_full(
    int32_t N, const int32_t *ng, uint8_t *rs, int32_t *rcand, int32_t *key,
    int32_t *ctr, int steps,
    uint2 *fh, const int32_t *__restrict__ rvpos, uint32_t *sk,
    int32_t *dist, int32_t *wl, int64_t wl_cap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) fh[N] = make_uint2(0u, 0u);
  int fate = 0;
  if (i < N) {
    const int32_t v = (int32_t)i;
    fh[v] = make_uint2(0u, 0u);
    const int32_t p = ng[v];
    int32_t r = p;
    if (r < 0) {
      r = -2;                       // ng(v) itself is not resolved yet
    } else if (rs[v] == 1 && r <= N) {
      r = N;                        // known finite: no walk to the root
    } else {
      for (int st = 0; st < steps; ++st) {
        if (r >= N) break;
        const int32_t nx = ng[r];
        if (nx < 0) break;          // ng of r not resolved yet
        r = nx;
      }
    }
    if (r == N) fate = 1;
    else if (r == N + 1) fate = 2;
    if (fate) {
      rs[v] = (uint8_t)fate;
      sk[rvpos ? rvpos[v] : v] = fate == 1 ? (uint32_t)p : (uint32_t)(N + 1);
      if (fate == 2) key[v] = PG_KEY_TOP;
    } else {
      rcand[v] = r;
    }
  }
  count_block(&ctr[C_DIST_NF], fate == 1);
  if (dist) count_block(dist, i < N && fate == 0);
  if (wl)
    append_block(&ctr[C_DIST_WLRT], wl, wl_cap, i < N && fate == 0,
                 (int32_t)i);
}

// A round over every undecided vertex (dense, like k_ng_round).
__global__ __launch_bounds__(kBlock) void k_root_round(
    int32_t N, const int32_t *ng, uint8_t *rs, int32_t *rcand, int32_t *key,
    int32_t *ctr, int last, int steps, const int32_t *__restrict__ rvpos,
    uint32_t *sk, int32_t *dist) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int fate = 0;
  bool pending = false;
  if (i < N) {
    const int32_t v = (int32_t)i;
    if (rs[v] == 0) {
      int32_t r = ld_relaxed(&rcand[v]);
      fate = root_walk(N, ng, rs, rcand, v, &r, steps);
      if (fate) {
        __hip_atomic_store(&rs[v], (uint8_t)fate, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        sk[rvpos ? rvpos[v] : v] =
            fate == 1 ? (uint32_t)ng[v] : (uint32_t)(N + 1);
        if (fate == 2) key[v] = PG_KEY_TOP;
      } else {
        st_relaxed(&rcand[v], r);
        pending = true;
      }
    }
  }
  if (last && __ballot(pending) && (threadIdx.x & (kWave - 1)) == 0)
    atomicOr(&ctr[C_ABORT], 1);
  count_block(&ctr[C_DIST_NF], fate == 1);
  if (dist) count_block(dist, pending);
}

// The same round over the vertices the full pass listed (as
// k_ng_round_list).
__global__ __launch_bounds__(kBlock) void k_root_round_list(
    int32_t N, const int32_t *ng, uint8_t *rs, int32_t *rcand, int32_t *key,
    int32_t *ctr, int last, int steps, const int32_t *__restrict__ rvpos,
    uint32_t *sk, const int32_t *__restrict__ wl, int64_t wl_cap) {
  const ListPart lp = list_part();
  const int32_t len = ctr[C_DIST_WLRT + lp.slot * kDistStride];
  const int32_t *lst = wl + (int64_t)lp.slot * wl_cap;
  bool open = false;
  int32_t nfin = 0;
  for (int64_t k = (int64_t)lp.part * blockDim.x + threadIdx.x; k < len;
       k += (int64_t)lp.parts * blockDim.x) {
    const int32_t v = lst[k];
    if (rs[v] == 0) {
      int32_t r = ld_relaxed(&rcand[v]);
      const int fate = root_walk(N, ng, rs, rcand, v, &r, steps);
      if (fate) {
        __hip_atomic_store(&rs[v], (uint8_t)fate, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        sk[rvpos ? rvpos[v] : v] =
            fate == 1 ? (uint32_t)ng[v] : (uint32_t)(N + 1);
        if (fate == 2) key[v] = PG_KEY_TOP;
        nfin += fate == 1;
      } else {
        st_relaxed(&rcand[v], r);
        open = true;
      }
    }
  }
  if (last && open) atomicOr(&ctr[C_ABORT], 1);
  add_block(&ctr[C_DIST_NF], nfin);
}

// ---------------------------------------------------------------------------
// Euler list of the ng tree
// ---------------------------------------------------------------------------
// Sorted position i (0 <= i < nF) holds the vertex at signed-order position
// svS[i] (the vertex itself in a relabeled game) with parent skS[i]: as the
// parent sort leaves them, i < ni holds an inner parent, the rest are the
// sink's children, their positions stored reversed at the top of svS.
// Splitters of the list ranking sit at even element indices (multiples of
// the stride): every even index from 2 on is the element of a position.
__device__ __forceinline__ uint32_t ps_key(const uint32_t *skS, int64_t i,
                                           int64_t ni, int32_t N) {
  return i < ni ? skS[i] : (uint32_t)N;
}
__device__ __forceinline__ uint32_t ps_val(const uint32_t *svS, int64_t i,
                                           int64_t ni, int64_t nF) {
  return svS[i < ni ? i : ni + nF - 1 - i];
}

// fh[p] = {first, last} sorted position of p's children, + 1 each, for
// every inner parent p (a vertex with children; the sink's children are the
// positions from ni on).  The root walks clear fh to {0, 0}, so a vertex
// whose fh.x is 0 is a leaf.  Plain stores: the first and the last position
// of a segment write different words.
__global__ __launch_bounds__(kBlock) void k_link_info(
    int32_t N, const uint32_t *__restrict__ skS,
    const uint32_t *__restrict__ n_inner, uint2 *fh, int32_t *ctr) {
  if (ctr[C_ABORT] || (ctr[C_ERR] & ERR_RANKCOUNT)) return;
  const int64_t ni = *n_inner;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ni) return;
  const uint32_t p = skS[i];
  if (p >= (uint32_t)N) {  // inner parents are vertices
    atomicOr(&ctr[C_ERR], ERR_RANKCOUNT);
    return;
  }
  uint32_t *f = reinterpret_cast<uint32_t *>(fh);
  if (i == 0 || skS[i - 1] != p) f[2 * p] = (uint32_t)(i + 1);
  if (i == ni - 1 || skS[i + 1] != p) f[2 * p + 1] = (uint32_t)(i + 1);
}

// Elements: 0 enters the root (the sink), 1 leaves it; 2i+2 enters the
// vertex at sorted position i (a leaf: visits it); 2i+3, when i is the last
// child of an inner parent p, leaves p.  So the last child links to its
// parent's leave element next door, and the parent's own position, which
// knows where its children end (fh), links that element onward: no vertex
// needs its own sorted position.  Each node's in-order point is marked on
// one element: the enter element of its first even child, or its leave
// element when no child is even.  A leaf -- most vertices of the tree on
// random games -- is visited by one element, which carries the parent's
// point (bit 30, when the leaf is the parent's first even child) and its own
// (bit 31).
__global__ __launch_bounds__(kBlock) void k_link_build(
    int32_t N, int32_t n_oddpri, const uint32_t *__restrict__ skS,
    const uint32_t *__restrict__ svS, const uint32_t *__restrict__ n_inner,
    const int32_t *__restrict__ perm, const uint2 *__restrict__ fh,
    int2 *elem, int32_t *ctr) {
  if (ctr[C_ABORT] || (ctr[C_ERR] & ERR_RANKCOUNT)) return;
  const int64_t nF = ctr[C_NFIN], ni = *n_inner;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t *el = reinterpret_cast<int32_t *>(elem);   // .x at 2e, .y at 2e+1
  if (nF == 0) {   // the sink alone: its point on its leave element
    if (i == 0) {
      elem[0] = make_int2(1, N);
      elem[1] = make_int2(-1, N | (int32_t)0x80000000);
    }
    return;
  }
  if (i >= nF) return;
  const uint32_t p = ps_key(skS, i, ni, N);
  const uint32_t r = ps_val(svS, i, ni, nF);
  const int32_t c = perm ? perm[r] : (int32_t)r;
  const bool ev = r >= (uint32_t)n_oddpri;
  const bool seg_start = (i == 0) || (ps_key(skS, i - 1, ni, N) != p);
  const bool seg_end = (i == nF - 1) || (ps_key(skS, i + 1, ni, N) != p);
  // c is the parent's first even child: the parent's in-order point comes
  // just before c's subtree
  const bool wd = ev && (seg_start || ps_val(svS, i - 1, ni, nF) <
                                          (uint32_t)n_oddpri);
  // after c's subtree: the next sibling, else leave the parent
  const int32_t nx = !seg_end ? (int32_t)(2 * i + 4)
                              : (p == (uint32_t)N ? 1 : (int32_t)(2 * i + 3));
  if (p == (uint32_t)N && seg_start) elem[0] = make_int2((int32_t)(2 * i + 2), N);
  if (seg_end) {
    // leave the parent: it carries the parent's point when c, its last
    // child, is odd (then no child is even)
    const int32_t w = ev ? 0 : (int32_t)0x80000000;
    if (p == (uint32_t)N) elem[1] = make_int2(-1, N | w);
    else el[2 * (2 * i + 3) + 1] = (int32_t)p | w;
  }
  const uint2 f = fh[c];
  // a leaf: one element visits it, carrying the parent's point (bit 30)
  // and then its own (bit 31); else enter c: its first child, carrying the
  // parent's point when wd
  const int2 e0 =
      f.x == 0
          ? make_int2(nx, c | (int32_t)0x80000000 | ((int32_t)wd << 30))
          : make_int2((int32_t)(2 * f.x), (int32_t)p | ((int32_t)wd << 31));
  if (seg_end && p != (uint32_t)N) {
    elem[2 * i + 2] = e0;   // 2i+3 leaves p: written above and by p
  } else {
    // 2i+3 is unused: one 16-byte store covers the pair (partly written
    // sectors cost a read-modify-write when they leave the cache)
    *reinterpret_cast<int4 *>(&elem[2 * i + 2]) =
        make_int4(e0.x, e0.y, 0, 0);
  }
  // leave c, next to its last child: on to c's continuation
  if (f.x != 0) el[2 * (2 * (int64_t)f.y + 1)] = nx;
}

// ---------------------------------------------------------------------------
// list ranking by sublists
// ---------------------------------------------------------------------------
// Level 0 walks the Euler list (weights are bits 31 and 30 of elem[].y, the
// second only on leaves that carry their parent's point); level k
// walks the list of level-(k-1) splitters (int weights).  Splitters are the
// elements whose index is a multiple of the stride; element 0 (the list head)
// is one.  Every size comes from the finite count on the device.
// Also records, for every element that carries a point, its sublist and
// the sublist's weight before it (aux), so that the keys can be emitted by
// one pass over sorted positions instead of a second walk.  The records are
// kept by sorted position (aux_slot), so that a run of leaf siblings fills
// whole sectors.
__device__ __forceinline__ int64_t aux_slot(int64_t e, int64_t N) {
  // 2i+2 -> i; 2i+3 -> N + i; 1 (leave the sink) -> 2N
  return (e & 1) ? (e == 1 ? 2 * N : N + (e - 3) / 2) : (e - 2) / 2;
}

constexpr int kSum1Batch = 16;

__global__ __launch_bounds__(kBlock) void k_lr_sum1(
    int32_t N, const int2 *__restrict__ elem, int per_thread, int s0,
    int32_t *sum, int32_t *next, int2 *aux, int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  const int64_t L = 2 * (int64_t)ctr[C_NFIN] + 2;
  const int64_t nsplit = level_size(L, 1, s0);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  for (int k = 0; k < per_thread; ++k) {
    const int64_t j = t + (int64_t)k * nthreads;
    if (j >= nsplit) break;
    int64_t e = j * s0;
    int32_t acc = 0;
    int64_t steps = 0;
    bool done = false;
    // A store issued inside the walk would hold up the next step's load
    // (vector loads and stores retire through one in-order counter), so
    // the records of kSum1Batch steps wait in registers (fixed indices: the
    // block of steps is unrolled) and go out together.
    while (!done) {
      int32_t slot[kSum1Batch], before[kSum1Batch];
#pragma unroll
      for (int b = 0; b < kSum1Batch; ++b) {
        slot[b] = -1;
        if (done) continue;
        const int2 el = elem[e];
        const int32_t w =
            (int32_t)((uint32_t)el.y >> 31) + ((el.y >> 30) & 1);
        if (w) {
          slot[b] = (int32_t)aux_slot(e, N);
          before[b] = acc;
        }
        acc += w;
        e = el.x;
        if (e < 0 || e % s0 == 0) {
          done = true;
        } else if (++steps > L) {
          atomicOr(&ctr[C_ERR], ERR_LISTWALK);
          e = -1;
          done = true;
        }
      }
#pragma unroll
      for (int b = 0; b < kSum1Batch; ++b)
        if (slot[b] >= 0) aux[slot[b]] = make_int2((int32_t)j, before[b]);
    }
    sum[j] = acc;
    next[j] = e < 0 ? -1 : (int32_t)(e / s0);
  }
}

__global__ __launch_bounds__(kBlock) void k_lr_sumk(
    const int32_t *__restrict__ lnext, const int32_t *__restrict__ lw,
    int level, int s0, int32_t *sum, int32_t *next, int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  const int64_t L = 2 * (int64_t)ctr[C_NFIN] + 2;
  const int64_t size = level_size(L, level, s0);
  const int64_t nsplit = level_size(L, level + 1, s0);
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nsplit) return;
  int64_t e = j * kStrideUp;
  int32_t acc = 0;
  int64_t steps = 0;
  for (;;) {
    acc += lw[e];
    e = lnext[e];
    if (e < 0 || e % kStrideUp == 0) break;
    if (++steps > size) {
      atomicOr(&ctr[C_ERR], ERR_LISTWALK);
      e = -1;
      break;
    }
  }
  sum[j] = acc;
  next[j] = e < 0 ? -1 : (int32_t)(e / kStrideUp);
}

// Ranks the top list (at most kTopMax elements, head = 0) inside one block
// by pointer jumping: suffix sums, then base = total - suffix.
constexpr int kTopMax = 4096;
constexpr int kTopThreads = 1024;

__global__ __launch_bounds__(kTopThreads) void k_lr_top(
    const int32_t *__restrict__ lnext, const int32_t *__restrict__ lw,
    int level, int s0, int32_t *base, int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  const int32_t nF = ctr[C_NFIN];
  const int64_t L0 = 2 * (int64_t)nF + 2;
  const int32_t L = (int32_t)level_size(L0, level, s0);
  __shared__ int32_t nx[kTopMax];
  __shared__ int32_t sm[kTopMax];
  constexpr int per = kTopMax / kTopThreads;
  if (L > kTopMax) {
    if (threadIdx.x == 0) atomicOr(&ctr[C_ERR], ERR_LISTWALK);
    return;
  }
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
  if (threadIdx.x == 0 && total != nF + 1)
    atomicOr(&ctr[C_ERR], ERR_RANKCOUNT);
}

// Hands each element of a level-k sublist its exclusive rank.
__global__ __launch_bounds__(kBlock) void k_lr_distk(
    const int32_t *__restrict__ lnext, const int32_t *__restrict__ lw,
    int level, int s0, const int32_t *__restrict__ sbase, int32_t *lbase,
    const int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  const int64_t L = 2 * (int64_t)ctr[C_NFIN] + 2;
  const int64_t size = level_size(L, level, s0);
  const int64_t nsplit = level_size(L, level + 1, s0);
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nsplit) return;
  int64_t e = j * kStrideUp;
  int32_t b = sbase[j];
  int64_t steps = 0;
  bool done = false;
  // the bases wait in registers and go out together (see k_lr_sum1)
  while (!done) {
    int64_t at[kStrideUp];
    int32_t val[kStrideUp];
#pragma unroll
    for (int q = 0; q < kStrideUp; ++q) {
      at[q] = -1;
      if (done) continue;
      at[q] = e;
      val[q] = b;
      b += lw[e];
      e = lnext[e];
      if (e < 0 || e % kStrideUp == 0 || ++steps > size) done = true;
    }
#pragma unroll
    for (int q = 0; q < kStrideUp; ++q)
      if (at[q] >= 0) lbase[at[q]] = val[q];
  }
}

// Keys, one sorted position per thread: each element of the position that
// carries a point emits the key of its node, the rank of its sublist's
// start plus the weight before it in the sublist (aux); a leaf with bit 30
// first its parent's, then its own.  Position nF - 1 (the sink's last
// child) also takes the sink's leave element.
__global__ __launch_bounds__(kBlock) void k_lr_emit1(
    int32_t N, const int2 *__restrict__ elem, const int2 *__restrict__ aux,
    const uint32_t *__restrict__ skS, const uint32_t *__restrict__ n_inner,
    const int32_t *__restrict__ sbase, int32_t *key, const int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  const int64_t nF = ctr[C_NFIN], ni = *n_inner;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > nF || (i == nF && nF > 0)) return;
  if (i == (nF > 0 ? nF - 1 : 0)) {
    const int2 el = elem[1];
    if (el.y < 0) {
      const int2 a = aux[2 * (int64_t)N];
      key[N] = sbase[a.x] + a.y;
    }
    if (nF == 0) return;
  }
  const uint32_t p = ps_key(skS, i, ni, N);
  const int2 el = elem[2 * i + 2];
  if (el.y & (int32_t)0xC0000000) {
    const int2 a = aux[i];
    int32_t b = sbase[a.x] + a.y;
    if (el.y & 0x40000000) key[p] = b++;          // a leaf's parent
    if (el.y < 0) key[el.y & 0x3fffffff] = b;
  }
  if (p != (uint32_t)N &&
      (i == nF - 1 || ps_key(skS, i + 1, ni, N) != p)) {
    const int2 lv = elem[2 * i + 3];               // leaves p
    if (lv.y < 0) {
      const int2 a = aux[N + i];
      key[lv.y & 0x3fffffff] = sbase[a.x] + a.y;
    }
  }
}

// ---------------------------------------------------------------------------
// switching rules
// ---------------------------------------------------------------------------
// Each thread takes one vertex of the player from a compacted list and reads
// its row four targets at a time, so that four key gathers are in flight.
// After a best response (Algorithm 1, the inner loop ended with no Odd
// switch) a vertex whose valuation is top stays top for the rest of the
// solve: Even's switches only raise valuations (Theorem 1, second item) and
// every later valuation is at least the best response's (section 3, "Best
// responses").  Its successor is then top too (for an Odd vertex every
// successor is, or Odd would have a better one; an Even vertex never
// switches away from top), so marking sp[v].y lets a later walk stop as
// soon as it reaches such a vertex.
__global__ void k_mark_top(int32_t N, const uint8_t *__restrict__ rs,
                           int2 *sp) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < N && rs[v] == 2) sp[v].y = kTopMark;
}

constexpr int kRowBatch = 4;

// All_Odd (section 4): the first successor of least key, if strictly below
// the current choice.  All decisions read the same valuation.  A vertex that
// switches also records its new successor's priority in the play graph.
__global__ __launch_bounds__(kBlock) void k_odd_switch(
    int32_t N, int64_t count, const int32_t *__restrict__ ids,
    const int64_t *__restrict__ off, const int32_t *__restrict__ tgt,
    const int32_t *__restrict__ key, const int32_t *__restrict__ pri, int2 *sp,
    int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool sw = false;
  const int2 me = t < count ? sp[ids[t]] : make_int2(0, kTopMark);
  // a vertex known to stay top has only top successors: no switch
  if (me.y != kTopMark) {
    const int32_t v = ids[t];
    const int64_t e0 = off[v], e1 = off[v + 1];
    const int32_t cur = me.x;
    // the current choice is normally in the row: its key comes with the
    // row's gathers (a strategy given at the C ABI may name another vertex)
    int32_t kc = 0;
    bool have_kc = false;
    int32_t best = -1;
    int32_t kb = 0;
    for (int64_t b = e0; b < e1; b += kRowBatch) {
      int32_t u[kRowBatch], k[kRowBatch];
#pragma unroll
      for (int j = 0; j < kRowBatch; ++j) u[j] = (b + j < e1) ? tgt[b + j] : -1;
#pragma unroll
      for (int j = 0; j < kRowBatch; ++j) k[j] = (u[j] >= 0) ? key[u[j]] : 0;
#pragma unroll
      for (int j = 0; j < kRowBatch; ++j) {
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
  count_block(&ctr[C_DIST_SW], sw);
}

// All_Even, greedy all-switches (section 3): options are the sink (first),
// then the row; the first option of greatest key, if strictly above the
// current choice.
__global__ __launch_bounds__(kBlock) void k_even_switch(
    int32_t N, int64_t count, const int32_t *__restrict__ ids,
    const int64_t *__restrict__ off, const int32_t *__restrict__ tgt,
    const int32_t *__restrict__ key, const int32_t *__restrict__ pri, int2 *sp,
    int32_t *ctr) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool sw = false;
  const int2 me = t < count ? sp[ids[t]] : make_int2(0, kTopMark);
  // a vertex known to stay top keeps its choice (nothing is above top)
  if (me.y != kTopMark) {
    const int32_t v = ids[t];
    const int64_t e0 = off[v], e1 = off[v + 1];
    const int32_t cur = me.x;
    // the current choice is the sink or normally in the row (see All_Odd)
    int32_t best = N;
    int32_t kb = key[N];
    int32_t kc = kb;
    bool have_kc = cur == N;
    for (int64_t b = e0; b < e1; b += kRowBatch) {
      int32_t u[kRowBatch], k[kRowBatch];
#pragma unroll
      for (int j = 0; j < kRowBatch; ++j) u[j] = (b + j < e1) ? tgt[b + j] : -1;
#pragma unroll
      for (int j = 0; j < kRowBatch; ++j) k[j] = (u[j] >= 0) ? key[u[j]] : 0;
#pragma unroll
      for (int j = 0; j < kRowBatch; ++j) {
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
  count_block(&ctr[C_DIST_SW], sw);
}

}  // namespace pgk

// ===========================================================================
// host side
// ===========================================================================
namespace pgk {

// A wave lasts as long as its longest walk, so the full passes stop early and
// leave long walks to rounds (which also take shortcuts).  Rank games
// take their budgets from the game's tuning (per size class, measured).
// Count games keep fixed ones: with ties broken by id their chains are about
// as short as with distinct priorities (on the 10M-vertex game with 4
// priorities the walks went from 773 to 369 us per valuation; before the
// tie rule, many cheap rounds served best: {4, 32, 4}).
struct WalkBudget {
  int full;    // plain-walk steps of the full passes
  int walk;    // shortcut-walk steps of one round
  int rounds;  // rounds enqueued without looking back
};
constexpr WalkBudget kCountWalks = {32, 32, 2};
static WalkBudget walk_budget(const pg_game *g) {
  if (g->dense) return kCountWalks;
  return {g->tune.walk_full, g->tune.walk_round, g->tune.walk_rounds};
}
// threads per block of the full ng and root passes
static int walk_block(const pg_game *g) {
  return g->dense ? kBlock : g->tune.walk_block;
}
constexpr int kMaxRounds = 64;    // rounds of the careful path before failing

static pg_status read_ctr(pg_game *g, hipStream_t s) {
  PG_HIP(hipMemcpyAsync(g->hctr, g->ctr, sizeof(int32_t) * C_COUNT,
                        hipMemcpyDeviceToHost, s));
  PG_HIP(hipStreamSynchronize(s));
  fold_switches(g->hctr);
  if (g->prof.on) {
    g->prof.nf = (double)g->hctr[C_NFIN];
    g->prof.ni = (double)g->hctr[C_NINNER];
    g->prof.flush();
  }
  return PG_OK;
}

// number of walking levels of the sublist ranking for the longest list
static int plan_levels(int64_t N, int s0) {
  const int64_t Lmax = 2 * N + 2;
  int k = 1;
  while (level_size(Lmax, k, s0) > kTopMax) ++k;
  return k;
}

void fates_reset(pg_game *g, hipStream_t s) {
  fill_u8(g->rs, 0, g->n_aug + 1, s, &g->prof);
}

void valuation_reset(pg_game *g, hipStream_t s) {
  const int64_t N = g->n_aug;
  fill_i32(g->ng, -1, N, s, &g->prof);
  fill_i32(g->cand, -1, N, s, &g->prof);
  fates_reset(g, s);
}

// ng and root phases with a fixed number of rounds; nothing is read back.
static void enqueue_walks(pg_game *g, hipStream_t s) {
  const int32_t N = (int32_t)g->n_aug;
  Prof *pf = &g->prof;
  int32_t *ng = g->ng, *cand = g->cand;
  const WalkBudget wb = walk_budget(g);
  // the counters, and the parent sort's work buffer of a rank valuation
  clear_valuation(g->ctr, g->dense ? nullptr : g->rs1, N, s, pf);
  // own record 8, first successor record 8, result 4; state resets 5
  const int wblk = walk_block(g);
  PG_LAUNCH(pf, K_NG_WALK, 25.0 * N, k_ng_full, dim3(grid_for(N, wblk)),
            dim3(wblk), 0, s, N, g->sp, g->pri, ng, cand, g->ctr,
            wb.full, g->rs, (int32_t *)nullptr, g->wl_ng,
            g->wl_cap);
  // the rounds walk the listed vertices only: as many lists as the full
  // passes fill, each with up to kListBlocks blocks
  const int64_t fblocks = grid_for(N, wblk);
  const dim3 lgrid((unsigned)(
      fblocks <= kDistSlots
          ? fblocks
          : kDistSlots *
                std::min<int64_t>(kListBlocks,
                                  (fblocks + kDistSlots - 1) / kDistSlots)));
  for (int r = 1; r <= wb.rounds; ++r)
    PG_LAUNCH(pf, K_NG_ROUND, 0.0, k_ng_round_list, lgrid, dim3(kBlock), 0,
              s, N, g->sp, g->pri, ng, cand, g->ctr, (int)(r == wb.rounds),
              wb.walk, g->wl_ng, g->wl_cap);
  // own ng 4, parent's ng 4, sort key 4, rs 1 (+ rvpos 4 unless
  // relabeled); resets 12
  const int32_t *rvpos = kernel_rvpos(g);
  PG_LAUNCH(pf, K_ROOT_WALK, (rvpos ? 29.0 : 25.0) * N, k_root_full,
            dim3(grid_for(N, wblk)), dim3(wblk), 0, s, N, ng, g->rs,
            g->rcand, g->key, g->ctr, wb.full, g->fh, rvpos,
            g->sk0, (int32_t *)nullptr, g->wl_rt, g->wl_cap);
  for (int r = 1; r <= wb.rounds; ++r)
    PG_LAUNCH(pf, K_ROOT_ROUND, 0.0, k_root_round_list, lgrid,
              dim3(kBlock), 0, s, N, ng, g->rs, g->rcand, g->key, g->ctr,
              (int)(r == wb.rounds), wb.walk, rvpos, g->sk0, g->wl_rt,
              g->wl_cap);
  sum_dist(g->ctr, C_DIST_NF, C_NFIN, s, pf);
}

// Clears the distributed counter at C_DIST_MISC and C_MISC, runs `launch`
// (which counts its open vertices there) and reads the count back.
template <class F>
static pg_status counted(pg_game *g, hipStream_t s, F launch, int32_t *open) {
  Prof *pf = &g->prof;
  fill_i32(g->ctr + C_MISC, 0, 1, s, pf);
  fill_i32(g->ctr + C_DIST_MISC, 0, kDistSlots * kDistStride, s, pf);
  launch(g->ctr + C_DIST_MISC);
  sum_dist(g->ctr, C_DIST_MISC, C_MISC, s, pf);
  PG_TRY(read_ctr(g, s));
  *open = g->hctr[C_MISC];
  return PG_OK;
}

// ng and root phases looping on the host until every vertex is resolved.
static pg_status careful_walks(pg_game *g, hipStream_t s) {
  const int32_t N = (int32_t)g->n_aug;
  Prof *pf = &g->prof;
  const WalkBudget wb = walk_budget(g);
  int32_t *ng = g->ng, *cand = g->cand;
  fill_i32(ng, -1, N, s, pf);
  fill_i32(cand, -1, N, s, pf);
  clear_valuation(g->ctr, g->dense ? nullptr : g->rs1, N, s, pf);
  int32_t open = 0;
  const int wblk = walk_block(g);
  PG_TRY(counted(g, s, [&](int32_t *dist) {
    PG_LAUNCH(pf, K_NG_WALK, 25.0 * N, k_ng_full, dim3(grid_for(N, wblk)),
              dim3(wblk), 0, s, N, g->sp, g->pri, ng, cand, g->ctr,
              wb.full, g->rs, dist, (int32_t *)nullptr,
              (int64_t)0);
  }, &open));
  for (int r = 0; open > 0; ++r) {
    if (r >= kMaxRounds)
      return pg_fail(PG_EINTERNAL, "ng resolution did not converge");
    PG_TRY(counted(g, s, [&](int32_t *dist) {
      PG_LAUNCH(pf, K_NG_ROUND, 4.0 * N, k_ng_round, dim3(grid_for(N)),
                dim3(kBlock), 0, s, N, g->sp, g->pri, ng, cand, g->ctr, 0,
                wb.walk, dist);
    }, &open));
  }
  fill_i32(g->ctr + C_NFIN, 0, 1, s, pf);
  fill_i32(g->ctr + C_DIST_NF, 0, kDistSlots * kDistStride, s, pf);
  const int32_t *rvpos = kernel_rvpos(g);
  PG_TRY(counted(g, s, [&](int32_t *dist) {
    PG_LAUNCH(pf, K_ROOT_WALK, (rvpos ? 29.0 : 25.0) * N, k_root_full,
              dim3(grid_for(N, wblk)), dim3(wblk), 0, s, N, ng, g->rs,
              g->rcand, g->key, g->ctr, wb.full, g->fh, rvpos,
              g->sk0, dist, (int32_t *)nullptr, (int64_t)0);
  }, &open));
  for (int r = 0; open > 0; ++r) {
    if (r >= kMaxRounds)
      return pg_fail(PG_EINTERNAL, "root resolution did not converge");
    PG_TRY(counted(g, s, [&](int32_t *dist) {
      PG_LAUNCH(pf, K_ROOT_ROUND, 1.0 * N, k_root_round, dim3(grid_for(N)),
                dim3(kBlock), 0, s, N, ng, g->rs, g->rcand, g->key, g->ctr,
                0, wb.walk, rvpos, g->sk0, dist);
    }, &open));
  }
  sum_dist(g->ctr, C_DIST_NF, C_NFIN, s, pf);
  fill_i32(g->ctr + C_ABORT, 0, 1, s, pf);
  return PG_OK;
}

// sort, Euler list and the level-1 sublist sums; every kernel skips when
// C_ABORT is set.
static void enqueue_rank_list(pg_game *g, hipStream_t s) {
  const int32_t N = (int32_t)g->n_aug;
  Prof *pf = &g->prof;
  // the root walks wrote the keys in signed-priority order (the sort's
  // values are the positions in that order); sizes past the sort are only
  // known on the device: grids are sized for N
  const uint32_t *n_inner = nullptr;
  const int which = parent_sort(g->sk0, g->sv0, g->sk1, g->sv1, N,
                                (uint32_t)N, g->sort_bits, g->rs1, g->ctr, s,
                                pf, &n_inner);
  const uint32_t *skS = which ? g->sk1 : g->sk0;
  const uint32_t *svS = which ? g->sv1 : g->sv0;
  g->ps_k = skS;
  g->ps_ni = n_inner;
  // inner keys 4; fh at segment ends about 2 per inner child
  PG_LAUNCH_NI(pf, K_LINK_INFO, 0.0, 0.0, 6.0, k_link_info,
               dim3(grid_for(N)), dim3(kBlock), 0, s, N, skS, n_inner, g->fh,
               g->ctr);
  // keys and values 8 (+ perm 4 unless relabeled); fh 8; one element 8,
  // and per inner child about 8 more (leave elements)
  const int32_t *perm = kernel_perm(g);
  PG_LAUNCH_NI(pf, K_LINK_BUILD, 0.0, perm ? 28.0 : 24.0, 8.0, k_link_build,
               dim3(grid_for(N)), dim3(kBlock), 0, s, N, g->n_oddpri, skS, svS,
               n_inner, perm, g->fh, g->elem, g->ctr);
  const int s0 = g->tune.stride0;
  const int64_t Lmax = 2 * (int64_t)N + 2;
  const int64_t ns1 = level_size(Lmax, 1, s0);
  const int per1 = g->tune.per_thread;
  const int64_t thr1 = (ns1 + per1 - 1) / per1;
  // 8 B per list element and 8 B per splitter (2 F / s0 of them), a record
  // of 8 B per point.  The list has one element per leaf and two per inner
  // vertex: counted at one per finite vertex, its least length
  PG_LAUNCH_NF(pf, K_LR_SUM1, 16.5, k_lr_sum1, dim3(grid_for(thr1)),
            dim3(kBlock), 0, s, N, g->elem, per1, s0, g->lv[0].sum,
            g->lv[0].next, g->aux, g->ctr);
}

// The reduced lists ranked on the device (unless the level-1 bases come
// from the host), then the keys emitted from sorted positions.
static void enqueue_rank_emit(pg_game *g, hipStream_t s, bool device_reduced) {
  const int32_t N = (int32_t)g->n_aug;
  Prof *pf = &g->prof;
  const int nl = g->nlevels;
  const int s0 = g->tune.stride0;
  const int64_t Lmax = 2 * (int64_t)N + 2;
  for (int k = 1; device_reduced && k < nl; ++k) {
    const int64_t nsk = level_size(Lmax, k + 1, s0);
    // 8 B per element of the level-k list (about 2 nF / s0 / 8^(k-1))
    PG_LAUNCH_NF(pf, K_LR_SUMK,
                 16.0 * (double)level_size(Lmax, k, s0) / (double)Lmax,
                 k_lr_sumk, dim3(grid_for(nsk)), dim3(kBlock), 0, s,
                 g->lv[k - 1].next, g->lv[k - 1].sum, k, s0, g->lv[k].sum,
                 g->lv[k].next, g->ctr);
  }
  if (device_reduced)
    PG_LAUNCH(pf, K_LR_TOP, 12.0 * level_size(Lmax, nl, s0), k_lr_top,
              dim3(1), dim3(kTopThreads), 0, s, g->lv[nl - 1].next,
              g->lv[nl - 1].sum, nl, s0, g->lv[nl - 1].base, g->ctr);
  for (int k = nl - 1; device_reduced && k >= 1; --k) {
    const int64_t nsk = level_size(Lmax, k + 1, s0);
    PG_LAUNCH_NF(pf, K_LR_DISTK,
                 24.0 * (double)level_size(Lmax, k, s0) / (double)Lmax,
                 k_lr_distk, dim3(grid_for(nsk)), dim3(kBlock), 0, s,
                 g->lv[k - 1].next, g->lv[k - 1].sum, k, s0, g->lv[k].base,
                 g->lv[k - 1].base, g->ctr);
  }
  // per finite vertex: its key and element 12, the element's record 8, a
  // 4 B key written; leave elements of inner parents about 8 per inner child
  PG_LAUNCH_NI(pf, K_LR_EMIT1, 0.0, 24.0, 8.0, k_lr_emit1,
               dim3(grid_for(N + 1)), dim3(kBlock), 0, s, N, g->elem, g->aux,
               g->ps_k, g->ps_ni, g->lv[0].base, g->key, g->ctr);
}

// fresh: the switch counters are still zero from the valuation's own
// clearing (an iteration: walks, valuation, All_Odd in one sequence)
static void enqueue_switch(pg_game *g, bool odd, hipStream_t s, bool fresh) {
  const int32_t N = (int32_t)g->n_aug;
  Prof *pf = &g->prof;
  if (!fresh) fill_i32(g->ctr + C_DIST_SW, 0, kDistSlots * kDistStride, s, pf);
  // per vertex: id 4, two offsets 16, current choice 8 (read and write
  // counted once; its key is one of the row's) -> 28; per edge: target 4
  // and its key 4
  if (odd && g->tsw) {
    enqueue_tsw_odd(g, s);
  } else if (odd) {
    const int64_t cnt = g->n_odd;
    if (cnt > 0)
      PG_LAUNCH(pf, K_ODD_SWITCH, 28.0 * cnt + 8.0 * g->m_odd, k_odd_switch,
                dim3(grid_for(cnt)), dim3(kBlock), 0, s, N, cnt, g->odd_ids,
                g->off, g->tgt, g->key, g->pri, g->sp, g->ctr);
  } else {
    const int64_t cnt = N - g->n_odd;
    if (cnt > 0)
      PG_LAUNCH(pf, K_EVEN_SWITCH, 28.0 * cnt + 8.0 * (g->m_aug - g->m_odd),
                k_even_switch, dim3(grid_for(cnt)), dim3(kBlock), 0, s, N, cnt,
                g->even_ids, g->off, g->tgt, g->key, g->pri, g->sp, g->ctr);
  }
  // the host sums the switch count's slots when it reads the counters
}

// The valuation after the walks: rank keys (distinct priorities) or count
// vectors (pg_count.hip).
static void enqueue_values(pg_game *g, hipStream_t s) {
  if (g->dense) {
    enqueue_count(g, s);
  } else {
    enqueue_rank_list(g, s);
    enqueue_rank_emit(g, s, true);
  }
}

// The split of the paper's GPU-LR (PG_HOST_REDUCED_LIST, rank valuations):
// the device builds the list and sums the level-1 sublists, the host ranks
// the reduced list (one walk from the head) and the device emits the keys.
static pg_status host_reduced_rank(pg_game *g, hipStream_t s) {
  enqueue_rank_list(g, s);
  PG_TRY(read_ctr(g, s));
  if (g->hctr[C_ABORT] || g->hctr[C_ERR]) return PG_OK;  // the caller looks
  const int64_t nF = g->hctr[C_NFIN];
  const int64_t ns = level_size(2 * nF + 2, 1, g->tune.stride0);
  const int64_t cap = level_size(2 * g->n_aug + 2, 1, kStrideMin);
  if (!g->h_rl) {
    void *p = nullptr;
    PG_TRY(host_alloc(&p, sizeof(int32_t) * 3 * (size_t)cap));
    g->h_rl = (int32_t *)p;
  }
  int32_t *hn = g->h_rl, *hs = g->h_rl + cap, *hb = g->h_rl + 2 * cap;
  PG_HIP(hipMemcpyAsync(hn, g->lv[0].next, sizeof(int32_t) * ns,
                        hipMemcpyDeviceToHost, s));
  PG_HIP(hipMemcpyAsync(hs, g->lv[0].sum, sizeof(int32_t) * ns,
                        hipMemcpyDeviceToHost, s));
  PG_HIP(hipStreamSynchronize(s));
  int64_t acc = 0, steps = 0;
  for (int64_t j = 0; j >= 0; j = hn[j]) {
    if (++steps > ns || j >= ns)
      return pg_fail(PG_EINTERNAL, "reduced list walk exceeded its bound");
    hb[j] = (int32_t)acc;
    acc += hs[j];
  }
  if (acc != nF + 1)
    return pg_fail(PG_EINTERNAL, "list ranking lost elements");
  PG_HIP(hipMemcpyAsync(g->lv[0].base, hb, sizeof(int32_t) * ns,
                        hipMemcpyHostToDevice, s));
  enqueue_rank_emit(g, s, false);
  return PG_OK;
}

static pg_status values(pg_game *g, hipStream_t s) {
  if (g->host_rl && !g->dense) return host_reduced_rank(g, s);
  enqueue_values(g, s);
  return PG_OK;
}

static void enqueue_any_switch(pg_game *g, bool odd, hipStream_t s,
                               bool fresh) {
  if (g->dense) enqueue_count_switch(g, odd, s, fresh);
  else enqueue_switch(g, odd, s, fresh);
}

static pg_status check_ctr(pg_game *g) {
  const int e = g->hctr[C_ERR];
  if (e & ERR_INADMISSIBLE)
    return pg_fail(PG_EINADMISSIBLE,
                   "the play graph has a cycle whose largest priority is odd");
  if (e & ERR_LISTWALK)
    return pg_fail(PG_EINTERNAL, "list ranking walk exceeded its bound");
  if (e & ERR_RANKCOUNT)
    return pg_fail(PG_EINTERNAL, "list ranking lost elements");
  if (e & ERR_SORT)
    return pg_fail(PG_EINTERNAL, "radix sort look-back timed out");
  return PG_OK;
}

// One valuation (and, with odd_switch, the All_Odd step after it) with one
// host synchronisation on the common path.
// Captures one best-response iteration (fixed sizes and buffers: every size
// a kernel needs is read on the device) on a private stream, as a graph.
static pg_status capture_iteration(pg_game *g, hipGraphExec_t *ex) {
  if (!g->cap_stream)
    PG_HIP(hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking));
  hipStream_t cs = g->cap_stream;
  PG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  enqueue_walks(g, cs);
  enqueue_values(g, cs);
  enqueue_any_switch(g, true, cs, true);
  hipGraph_t gr = nullptr;
  hipError_t e = hipStreamEndCapture(cs, &gr);
  if (e == hipSuccess) e = hipGraphInstantiate(ex, gr, nullptr, nullptr, 0);
  if (gr) (void)hipGraphDestroy(gr);
  if (e != hipSuccess) {
    *ex = nullptr;
    return pg_fail(PG_EDEVICE, std::string("graph capture: ") +
                                   hipGetErrorString(e));
  }
  return PG_OK;
}

static pg_status run_valuation(pg_game *g, hipStream_t s, bool odd_switch,
                               int32_t *count, int64_t *n_finite) {
  g->nlevels = g->dense ? count_levels(g->n_aug, g->dw)
                        : plan_levels(g->n_aug, g->tune.stride0);
  if (g->timed && !g->ev_a) {
    PG_HIP(hipEventCreate(&g->ev_a));
    PG_HIP(hipEventCreate(&g->ev_b));
  }
  if (g->timed) PG_HIP(hipEventRecord(g->ev_a, s));
  bool replayed = false;
  if (odd_switch && g->use_graph && !g->careful && !g->prof.on &&
      !g->host_rl) {
    hipGraphExec_t &ex = g->iter_exec;
    if (!ex && capture_iteration(g, &ex) != PG_OK) {
      g->use_graph = false;  // capture refused: stay eager from now on
      (void)hipGetLastError();
    }
    if (ex) {
      PG_HIP(hipGraphLaunch(ex, s));
      replayed = true;
    }
  }
  if (!replayed) {
    if (g->careful) PG_TRY(careful_walks(g, s));
    else enqueue_walks(g, s);
    PG_TRY(values(g, s));
    if (odd_switch) {
      enqueue_any_switch(g, true, s, true);
    }
  }
  if (g->timed) PG_HIP(hipEventRecord(g->ev_b, s));
  pg_status st = read_ctr(g, s);
  if (st != PG_OK) return st;
  if (g->hctr[C_ABORT]) {
    // a walk outlasted the fixed rounds: finish on the host-driven path and
    // redo everything after the walks (the gated kernels did nothing)
    st = careful_walks(g, s);
    if (st != PG_OK) return st;
    st = values(g, s);
    if (st != PG_OK) return st;
    if (odd_switch) {
      enqueue_any_switch(g, true, s, true);
    }
    if (g->timed) PG_HIP(hipEventRecord(g->ev_b, s));
    st = read_ctr(g, s);
    if (st != PG_OK) return st;
  }
  if (!g->timed ||
      hipEventElapsedTime(&g->last_ms, g->ev_a, g->ev_b) != hipSuccess)
    g->last_ms = 0.0f;
  st = check_ctr(g);
  if (st != PG_OK) return st;
  if (count) *count = g->hctr[C_SWITCH];
  if (n_finite) *n_finite = (int64_t)g->hctr[C_NFIN] + 1;
  return PG_OK;
}

void enqueue_valuation(pg_game *g, hipStream_t s) {
  g->nlevels = g->dense ? count_levels(g->n_aug, g->dw)
                        : plan_levels(g->n_aug, g->tune.stride0);
  enqueue_walks(g, s);
  enqueue_values(g, s);
}

pg_status redo_valuation(pg_game *g, hipStream_t s) {
  PG_TRY(careful_walks(g, s));
  return values(g, s);
}

pg_status valuation_status(pg_game *g) { return check_ctr(g); }

pg_status valuation_device(pg_game *g, hipStream_t s, int64_t *n_finite_out) {
  return run_valuation(g, s, false, nullptr, n_finite_out);
}

pg_status iteration_device(pg_game *g, hipStream_t s, int32_t *count,
                           int64_t *n_finite) {
  return run_valuation(g, s, true, count, n_finite);
}

void mark_top(pg_game *g, hipStream_t s) {
  const int32_t N = (int32_t)g->n_aug;
  if (!g->mark_top || N == 0) return;
  PG_LAUNCH(&g->prof, K_OTHER, 9.0 * N, k_mark_top, dim3(grid_for(N)),
            dim3(kBlock), 0, s, N, g->rs, g->sp);
}

pg_status switch_device(pg_game *g, bool odd, hipStream_t s, int32_t *count) {
  fill_i32(g->ctr + C_ABORT, 0, 1, s, &g->prof);
  enqueue_any_switch(g, odd, s, false);
  pg_status st = read_ctr(g, s);
  if (st != PG_OK) return st;
  *count = g->hctr[C_SWITCH];
  return PG_OK;
}

}  // namespace pgk
