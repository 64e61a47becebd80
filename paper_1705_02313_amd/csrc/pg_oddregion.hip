// Admissibility without dummy vertices (PG_ODD_REGION).
//
// Section 3 ("The algorithm") starts strategy improvement from sigma_init,
// which sends every Even vertex to the sink; that strategy is admissible
// unless Odd can close a cycle with an odd largest priority through its own
// vertices only.  Instead of inserting dummy Even vertices, this removes the
// part of the game that Odd wins on its own and solves the rest unchanged:
//
//   X  the vertices from which Odd avoids every Even vertex forever (the
//      load's fixpoint rounds, inx)
//   R  the vertices of X from which Odd, moving inside X, reaches a cycle
//      whose largest priority is odd: strongly connected components of X
//      are peeled by colouring rounds -- every vertex takes the largest
//      (priority, id) that reaches it inside the live part of X (forward
//      max-propagation), a colour's root with the vertices of its colour
//      that reach the root is the root's component; a component with an
//      edge and an odd root goes to R's seed, a root of an even-rooted or
//      edgeless component is dropped (the rest of its component is coloured
//      again in the next round); then everything in X that reaches the seed
//      inside X
//   A  Odd's attractor of R in the whole game
//
// Odd wins A; G minus A is a trap for Odd in which every cycle of Odd
// vertices has an even largest priority, so sigma_init is admissible there
// and the solve runs on it with no preprocessing.
#include <algorithm>
#include <vector>

#include "pg_common.h"

namespace pgk {

namespace {

// raises *flag when pred holds in a lane of the wave: one atomic per wave
// at most, and none once the flag reads raised (a million waves' atomics on
// one address would serialise)
__device__ __forceinline__ void raise_flag(int32_t *flag, bool pred) {
  if (__ballot(pred) && (threadIdx.x & (kWave - 1)) == 0 &&
      __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
    atomicOr(flag, 1);
}

__device__ __forceinline__ uint64_t color_key(int32_t pri, int32_t v) {
  return ((uint64_t)(uint32_t)pri << 32) | (uint32_t)v;
}

// Lists of vertices are kept in increasing id order (neighbouring entries
// then share lines of every per-vertex array): a pass writes one keep flag
// per entry, an exclusive scan gives each kept entry its place, and
// k_or_scatter moves it there.

// keep flags for the vertices with a[v] (mode 0), a[v] && !b[v] (mode 1) or
// !a[v] (mode 2)
__global__ void k_or_select(int64_t n, const uint8_t *a, const uint8_t *b,
                            int mode, uint32_t *flag) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n)
    flag[v] = (mode == 0 ? a[v] != 0 : mode == 1 ? (a[v] && !b[v]) : !a[v])
                  ? 1u : 0u;
}

// keep flags for the entries of lst not yet decided (done[v] == 0)
__global__ void k_or_undecided(const int32_t *lst, int32_t cnt,
                               const uint8_t *done, uint32_t *flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) flag[i] = done[lst[i]] ? 0u : 1u;
}

// out[pos[i]] = the i-th entry (lst[i], or i itself when lst is null) for
// the entries kept; *total = the number kept
__global__ void k_or_scatter(const int32_t *lst, int64_t cnt,
                             const uint32_t *flag, const uint32_t *pos,
                             int32_t *out, int32_t *total) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  if (flag[i]) out[pos[i]] = lst ? lst[i] : (int32_t)i;
  if (i == cnt - 1) *total = (int32_t)(pos[i] + flag[i]);
}

// The colouring rounds work on the list of live vertices of X (lst, cnt).
__global__ void k_or_color_init(const int32_t *lst, int32_t cnt,
                                const int32_t *pri, unsigned long long *col,
                                uint8_t *reach, uint8_t *nontriv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const int32_t v = lst[i];
  col[v] = color_key(pri[v], v);
  reach[v] = 0;
  nontriv[v] = 0;
}

// col[w] = max over live v -> w of col[v]: one relaxation sweep.  A thread
// that raises a successor's colour goes on pushing from the first one it
// raised, up to kChase steps, so a colour runs down a chain of live
// vertices within one sweep instead of one link per sweep.
constexpr int kChase = 64;

__global__ void k_or_color_sweep(const int32_t *lst, int32_t cnt,
                                 const int64_t *off, const int32_t *tgt,
                                 const uint8_t *alive,
                                 unsigned long long *col, int32_t *changed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ch = false;
  if (i < cnt) {
    int32_t u = lst[i];
    unsigned long long c = col[u];
    for (int step = 0; step < kChase; ++step) {
      int32_t nx = -1;
      unsigned long long cn = 0;
      for (int64_t e = off[u]; e < off[u + 1]; ++e) {
        const int32_t w = tgt[e];
        if (alive[w] && col[w] < c) {
          const unsigned long long old = atomicMax(&col[w], c);
          if (old < c) {
            ch = true;
            if (nx < 0) {
              nx = w;
              cn = c;
            }
          }
        }
      }
      if (nx < 0) break;
      u = nx;
      c = cn;
    }
  }
  raise_flag(changed, ch);
}

// a colour's root reaches itself
__global__ void k_or_reach_init(const int32_t *lst, int32_t cnt,
                                const unsigned long long *col,
                                uint8_t *reach) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const int32_t v = lst[i];
  if ((int32_t)(uint32_t)col[v] == v) reach[v] = 1;
}

// v reaches its colour's root inside its colour when a successor of the
// same colour does: one sweep
__global__ void k_or_reach_sweep(const int32_t *lst, int32_t cnt,
                                 const int64_t *off, const int32_t *tgt,
                                 const uint8_t *alive,
                                 const unsigned long long *col, uint8_t *reach,
                                 int32_t *changed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ch = false;
  if (i < cnt) {
    const int32_t v = lst[i];
    if (!reach[v]) {
      const unsigned long long c = col[v];
      for (int64_t e = off[v]; e < off[v + 1]; ++e) {
        const int32_t w = tgt[e];
        if (alive[w] && col[w] == c && reach[w]) {
          reach[v] = 1;
          ch = true;
          break;
        }
      }
    }
  }
  raise_flag(changed, ch);
}

// a root's component has an edge when another vertex is in it or the root
// has a loop
__global__ void k_or_nontrivial(const int32_t *lst, int32_t cnt,
                                const int64_t *off, const int32_t *tgt,
                                const unsigned long long *col,
                                const uint8_t *reach, uint8_t *nontriv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const int32_t v = lst[i];
  if (!reach[v]) return;
  const int32_t r = (int32_t)(uint32_t)col[v];
  if (r != v) {
    nontriv[r] = 1;
    return;
  }
  for (int64_t e = off[v]; e < off[v + 1]; ++e)
    if (tgt[e] == v) {
      nontriv[v] = 1;
      return;
    }
}

// components with an odd root join the seed; roots of the others leave;
// the vertices still live form the next round's list
__global__ void k_or_peel(const int32_t *lst, int32_t cnt, uint8_t *alive,
                          const unsigned long long *col, const uint8_t *reach,
                          const uint8_t *nontriv, uint8_t *seed,
                          uint32_t *flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) {
    const int32_t v = lst[i];
    bool live = true;
    if (reach[v]) {
      const unsigned long long c = col[v];
      const int32_t r = (int32_t)(uint32_t)c;
      const bool odd = (c >> 32) & 1ull;
      if (nontriv[r] && odd) {
        seed[v] = 1;
        alive[v] = 0;
        live = false;
      } else if (r == v) {
        alive[v] = 0;
        live = false;
      }
    }
    flag[i] = live ? 1u : 0u;
  }
}

// R: v in X with a successor in R (inside X); lst holds X minus R
__global__ void k_or_back(const int32_t *lst, int32_t cnt, const int64_t *off,
                          const int32_t *tgt, const uint8_t *inx, uint8_t *R,
                          int32_t *changed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ch = false;
  if (i < cnt) {
    const int32_t v = lst[i];
    if (!R[v]) {
      for (int64_t e = off[v]; e < off[v + 1]; ++e) {
        const int32_t w = tgt[e];
        if (inx[w] && R[w]) {
          R[v] = 1;
          ch = true;
          break;
        }
      }
    }
  }
  raise_flag(changed, ch);
}

// Odd's attractor: an Odd vertex with a successor in A, an Even vertex with
// every successor in A; lst holds vertices outside A
__global__ void k_or_attr(const int32_t *lst, int32_t cnt, const int64_t *off,
                          const int32_t *tgt, const uint8_t *owner,
                          uint8_t *A, int32_t *changed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ch = false;
  if (i < cnt) {
    const int32_t v = lst[i];
    if (!A[v]) {
      const bool odd = owner[v] == 1;
      bool any = false, all = true;
      for (int64_t e = off[v]; e < off[v + 1]; ++e) {
        const bool in = A[tgt[e]];
        any |= in;
        all &= in;
        if (odd ? any : !all) break;
      }
      if (odd ? any : all) {
        A[v] = 1;
        ch = true;
      }
    }
  }
  raise_flag(changed, ch);
}

__global__ void k_or_keep(const uint8_t *A, uint32_t *keep, int64_t n) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) keep[v] = A[v] ? 0u : 1u;
}

// edges of a kept vertex that stay (their targets kept)
__global__ void k_or_rowlen(const int64_t *off, const int32_t *tgt,
                            const uint8_t *A, const uint32_t *newid,
                            int64_t *len, int64_t n) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || A[v]) return;
  int64_t c = 0;
  for (int64_t e = off[v]; e < off[v + 1]; ++e) c += A[tgt[e]] ? 0 : 1;
  len[newid[v]] = c;
}

__global__ void k_or_fill(const int64_t *off, const int32_t *tgt,
                          const uint8_t *owner, const int32_t *pri,
                          const uint8_t *A, const uint32_t *newid,
                          const int64_t *off2, int32_t *tgt2, uint8_t *owner2,
                          int32_t *pri2, int32_t *orig, int64_t n) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || A[v]) return;
  const uint32_t u = newid[v];
  int64_t o = off2[u];
  for (int64_t e = off[v]; e < off[v + 1]; ++e) {
    const int32_t w = tgt[e];
    if (!A[w]) tgt2[o++] = (int32_t)newid[w];
  }
  owner2[u] = owner[v];
  pri2[u] = pri[v];
  orig[u] = (int32_t)v;
}

// the removed vertices' map entries
__global__ void k_or_newmap(const uint8_t *A, const uint32_t *newid,
                            int32_t *newmap, int64_t n) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) newmap[v] = A[v] ? -1 : (int32_t)newid[v];
}

// Runs `sweep` over the list (*lst, cnt entries) in groups of four, one
// synchronisation each, until a group changes nothing or the list is empty.
// With `done`, the entries decided (done[v] != 0) leave the list after each
// group (compacted into *spare, then the two swap).  Fails after `bound`
// groups.
struct ListBufs {
  int32_t *a, *b;      // the list and its spare
  uint32_t *flag, *pos;
  int32_t *dcnt;
  void *stmp;          // scan scratch
};

// keeps the flagged entries of l->a (cnt of them; all ids 0..cnt-1 when
// `ids`) in order in l->b, swaps the two and queues the new count into
// *host (valid after the next synchronisation)
void list_keep(ListBufs *l, int64_t cnt, bool ids, hipStream_t s,
               int32_t *host) {
  scan_excl_u32(l->flag, l->pos, cnt, l->stmp, s);
  hipLaunchKernelGGL(k_or_scatter, dim3(grid_for(cnt)), dim3(kBlock), 0, s,
                     ids ? nullptr : l->a, cnt, l->flag, l->pos, l->b,
                     l->dcnt);
  (void)hipMemcpyAsync(host, l->dcnt, sizeof(int32_t), hipMemcpyDeviceToHost,
                       s);
  std::swap(l->a, l->b);
}

template <class F>
pg_status fixpoint_list(pg_game *g, hipStream_t s, int64_t bound,
                        ListBufs *l, int32_t *cnt, const uint8_t *done,
                        F sweep) {
  for (int64_t round = 0; *cnt > 0; ++round) {
    if (round > bound)
      return pg_fail(PG_EINTERNAL, "odd-region fixpoint did not converge");
    fill_i32(g->ctr + C_MISC, 0, 1, s);
    for (int k = 0; k < 4; ++k) sweep(l->a, *cnt, g->ctr + C_MISC);
    int32_t h[2] = {0, *cnt};
    if (done) {
      hipLaunchKernelGGL(k_or_undecided, dim3(grid_for(*cnt)), dim3(kBlock),
                         0, s, l->a, *cnt, done, l->flag);
      list_keep(l, *cnt, false, s, &h[1]);
    }
    PG_HIP(hipMemcpyAsync(&h[0], g->ctr + C_MISC, sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    *cnt = h[1];
    if (h[0] == 0) break;
  }
  return PG_OK;
}

}  // namespace

pg_status odd_region_reduce(pg_game *g, hipStream_t s, int64_t n, int64_t m,
                            const int64_t *off, const int32_t *tgt,
                            const uint8_t *owner, const int32_t *pri,
                            const uint8_t *inx) {
  const unsigned gn = grid_for(n);
  struct Tmp {
    hipStream_t s;
    std::vector<void *> p;
    ~Tmp() {
      if (!p.empty()) (void)hipStreamSynchronize(s);
      for (void *x : p) dev_free(x);
    }
  } tmp{s, {}};
  uint8_t *alive = nullptr, *reach = nullptr, *nontriv = nullptr,
          *seed = nullptr;
  unsigned long long *col = nullptr;
  PG_TRY(dev_alloc(&alive, n));
  tmp.p.push_back(alive);
  PG_TRY(dev_alloc(&reach, n));
  tmp.p.push_back(reach);
  PG_TRY(dev_alloc(&nontriv, n));
  tmp.p.push_back(nontriv);
  PG_TRY(dev_alloc(&seed, n));
  tmp.p.push_back(seed);
  PG_TRY(dev_alloc(&col, n));
  tmp.p.push_back(col);
  ListBufs L{};
  PG_TRY(dev_alloc(&L.a, n));
  tmp.p.push_back(L.a);
  PG_TRY(dev_alloc(&L.b, n));
  tmp.p.push_back(L.b);
  PG_TRY(dev_alloc(&L.flag, n));
  tmp.p.push_back(L.flag);
  PG_TRY(dev_alloc(&L.pos, n));
  tmp.p.push_back(L.pos);
  PG_TRY(dev_alloc(&L.dcnt, 1));
  tmp.p.push_back(L.dcnt);
  {
    const size_t need = scan_excl_u32(nullptr, nullptr, n, nullptr, s);
    PG_TRY(dev_alloc((uint8_t **)&L.stmp, (int64_t)need + 16));
    tmp.p.push_back(L.stmp);
  }
  // the list of the vertices selected from all n (see k_or_select)
  auto select = [&](const uint8_t *a, const uint8_t *b, int mode,
                    int32_t *cnt) -> pg_status {
    hipLaunchKernelGGL(k_or_select, dim3(gn), dim3(kBlock), 0, s, n, a, b,
                       mode, L.flag);
    list_keep(&L, n, true, s, cnt);
    PG_HIP(hipStreamSynchronize(s));
    return PG_OK;
  };
  PG_HIP(hipMemcpyAsync(alive, inx, n, hipMemcpyDeviceToDevice, s));
  fill_u8(seed, 0, n, s);
  const int64_t bound = n + 64;
  // peeling rounds over the live vertices of X: every round drops at least
  // every colour's root
  int32_t cnt = 0;
  PG_TRY(select(inx, nullptr, 0, &cnt));
  for (int64_t round = 0; cnt > 0; ++round) {
    if (round > n + 1)
      return pg_fail(PG_EINTERNAL, "odd-region peeling did not converge");
    const unsigned gc = grid_for(cnt);
    hipLaunchKernelGGL(k_or_color_init, dim3(gc), dim3(kBlock), 0, s, L.a,
                       cnt, pri, col, reach, nontriv);
    PG_TRY(fixpoint_list(g, s, bound, &L, &cnt, nullptr,
                         [&](const int32_t *l, int32_t c, int32_t *ch) {
      hipLaunchKernelGGL(k_or_color_sweep, dim3(grid_for(c)), dim3(kBlock), 0,
                         s, l, c, off, tgt, alive, col, ch);
    }));
    hipLaunchKernelGGL(k_or_reach_init, dim3(gc), dim3(kBlock), 0, s, L.a,
                       cnt, col, reach);
    PG_TRY(fixpoint_list(g, s, bound, &L, &cnt, nullptr,
                         [&](const int32_t *l, int32_t c, int32_t *ch) {
      hipLaunchKernelGGL(k_or_reach_sweep, dim3(grid_for(c)), dim3(kBlock), 0,
                         s, l, c, off, tgt, alive, col, reach, ch);
    }));
    hipLaunchKernelGGL(k_or_nontrivial, dim3(gc), dim3(kBlock), 0, s, L.a,
                       cnt, off, tgt, col, reach, nontriv);
    hipLaunchKernelGGL(k_or_peel, dim3(gc), dim3(kBlock), 0, s, L.a, cnt,
                       alive, col, reach, nontriv, seed, L.flag);
    int32_t next = 0;
    list_keep(&L, cnt, false, s, &next);
    PG_HIP(hipStreamSynchronize(s));
    cnt = next;
  }
  // R = what reaches the seed inside X (over X minus R); A = Odd's attractor
  // of R (over the vertices outside A), both in place
  PG_TRY(select(inx, seed, 1, &cnt));
  PG_TRY(fixpoint_list(g, s, bound, &L, &cnt, seed,
                       [&](const int32_t *l, int32_t c, int32_t *ch) {
    hipLaunchKernelGGL(k_or_back, dim3(grid_for(c)), dim3(kBlock), 0, s, l, c,
                       off, tgt, inx, seed, ch);
  }));
  PG_TRY(select(seed, nullptr, 2, &cnt));
  PG_TRY(fixpoint_list(g, s, bound, &L, &cnt, seed,
                       [&](const int32_t *l, int32_t c, int32_t *ch) {
    hipLaunchKernelGGL(k_or_attr, dim3(grid_for(c)), dim3(kBlock), 0, s, l, c,
                       off, tgt, owner, seed, ch);
  }));
  uint8_t *A = seed;
  // the game on the vertices kept, rows in their order
  uint32_t *keep = nullptr, *newid = nullptr;
  int64_t *len = nullptr;
  void *stmp = nullptr;
  PG_TRY(dev_alloc(&keep, n));
  tmp.p.push_back(keep);
  PG_TRY(dev_alloc(&newid, n));
  tmp.p.push_back(newid);
  hipLaunchKernelGGL(k_or_keep, dim3(gn), dim3(kBlock), 0, s, A, keep, n);
  const size_t need = std::max(scan_excl_u32(nullptr, nullptr, n, nullptr, s),
                               scan_excl_i64(nullptr, nullptr, n + 1, nullptr,
                                             s));
  PG_TRY(dev_alloc((uint8_t **)&stmp, (int64_t)need + 16));
  tmp.p.push_back(stmp);
  scan_excl_u32(keep, newid, n, stmp, s);
  uint32_t last[2] = {0, 0};
  PG_HIP(hipMemcpyAsync(&last[0], newid + (n - 1), 4, hipMemcpyDeviceToHost,
                        s));
  PG_HIP(hipMemcpyAsync(&last[1], keep + (n - 1), 4, hipMemcpyDeviceToHost,
                        s));
  PG_HIP(hipStreamSynchronize(s));
  const int64_t n2 = (int64_t)last[0] + last[1];
  g->or_removed = n - n2;
  PG_TRY(dev_alloc(&g->or_new, n));
  hipLaunchKernelGGL(k_or_newmap, dim3(gn), dim3(kBlock), 0, s, A, newid,
                     g->or_new, n);
  if (n2 == 0) {   // Odd wins everything on its own: an empty game
    PG_TRY(dev_alloc(&g->off, 1));
    fill_i32((int32_t *)g->off, 0, 2, s);
    g->n_aug = 0;
    g->m_aug = 0;
    return PG_OK;
  }
  PG_TRY(dev_alloc(&len, n2 + 1));
  tmp.p.push_back(len);
  fill_i32((int32_t *)len, 0, 2 * (n2 + 1), s);
  hipLaunchKernelGGL(k_or_rowlen, dim3(gn), dim3(kBlock), 0, s, off, tgt, A,
                     newid, len, n);
  PG_TRY(dev_alloc(&g->off, n2 + 1));
  scan_excl_i64(len, g->off, n2 + 1, stmp, s);
  int64_t m2 = 0;
  PG_HIP(hipMemcpyAsync(&m2, g->off + n2, 8, hipMemcpyDeviceToHost, s));
  PG_HIP(hipStreamSynchronize(s));
  PG_TRY(dev_alloc(&g->tgt, m2));
  PG_TRY(dev_alloc(&g->owner, n2));
  PG_TRY(dev_alloc(&g->pri, n2));
  PG_TRY(dev_alloc(&g->or_orig, n2));
  hipLaunchKernelGGL(k_or_fill, dim3(gn), dim3(kBlock), 0, s, off, tgt, owner,
                     pri, A, newid, g->off, g->tgt, g->owner, g->pri,
                     g->or_orig, n);
  g->n_aug = n2;
  g->m_aug = m2;
  (void)m;
  return PG_OK;
}

namespace {

// a caller's choice (original ids) in the reduced game's ids; a vertex of A
// or an id out of range becomes INT32_MAX, which the import reports
__device__ __forceinline__ int32_t to_reduced(int32_t x, const int32_t *newmap,
                                              int64_t n) {
  if (x == PG_SINK) return PG_SINK;
  if (x < 0 || x >= n) return 2147483647;
  const int32_t u = newmap[x];
  return u < 0 ? 2147483647 : u;
}

__global__ void k_or_strats_in(const int32_t *orig, const int32_t *newmap,
                               const int32_t *sigma, const int32_t *tau,
                               int32_t *s2, int32_t *t2, int64_t n2,
                               int64_t n) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n2) return;
  const int32_t v = orig[u];
  if (sigma) s2[u] = to_reduced(sigma[v], newmap, n);
  if (tau) t2[u] = to_reduced(tau[v], newmap, n);
}

__global__ void k_or_strats_out(const int32_t *orig, const int32_t *newmap,
                                const int32_t *s2, const int32_t *t2,
                                int32_t *sigma, int32_t *tau, int64_t n) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t u = newmap[v];
  if (sigma) {
    const int32_t x = u < 0 ? PG_SINK : s2[u];
    sigma[v] = x == PG_SINK ? PG_SINK : orig[x];
  }
  if (tau) {
    const int32_t x = u < 0 ? PG_SINK : t2[u];
    tau[v] = x == PG_SINK ? PG_SINK : orig[x];
  }
}

__global__ void k_or_winner_out(const int32_t *newmap, const uint8_t *w2,
                                uint8_t *winner, int64_t n) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t u = newmap[v];
  winner[v] = u < 0 ? 1 : w2[u];
}

}  // namespace

pg_status odd_region_strats_in(pg_game *g, const int32_t *sigma,
                               const int32_t *tau, bool dev, hipStream_t s,
                               int32_t *s2, int32_t *t2) {
  const int64_t n = g->n, n2 = g->n_aug;
  struct Tmp {
    int32_t *a = nullptr, *b = nullptr;
    ~Tmp() {
      dev_free(a);
      dev_free(b);
    }
  } tmp;
  const int32_t *ds = sigma, *dt = tau;
  if (!dev) {
    if (sigma) {
      PG_TRY(dev_alloc(&tmp.a, n));
      PG_TRY(copy_in(tmp.a, sigma, sizeof(int32_t) * n, false, s));
      ds = tmp.a;
    }
    if (tau) {
      PG_TRY(dev_alloc(&tmp.b, n));
      PG_TRY(copy_in(tmp.b, tau, sizeof(int32_t) * n, false, s));
      dt = tmp.b;
    }
  }
  if (n2 > 0)
    hipLaunchKernelGGL(k_or_strats_in, dim3(grid_for(n2)), dim3(kBlock), 0, s,
                       g->or_orig, g->or_new, ds, dt, s2, t2, n2, n);
  // the staging copies go back to the pool only after the kernel ran
  PG_HIP(hipStreamSynchronize(s));
  return PG_OK;
}

pg_status odd_region_strats_out(pg_game *g, const int32_t *s2,
                                const int32_t *t2, int32_t *sigma,
                                int32_t *tau, bool dev, hipStream_t s) {
  const int64_t n = g->n;
  struct Tmp {
    int32_t *a = nullptr, *b = nullptr;
    ~Tmp() {
      dev_free(a);
      dev_free(b);
    }
  } tmp;
  int32_t *ds = sigma, *dt = tau;
  if (!dev) {
    if (sigma) PG_TRY(dev_alloc(&tmp.a, n));
    if (tau) PG_TRY(dev_alloc(&tmp.b, n));
    ds = sigma ? tmp.a : nullptr;
    dt = tau ? tmp.b : nullptr;
  }
  hipLaunchKernelGGL(k_or_strats_out, dim3(grid_for(n)), dim3(kBlock), 0, s,
                     g->or_orig, g->or_new, s2, t2, ds, dt, n);
  if (!dev) {
    if (sigma) PG_TRY(copy_out(sigma, ds, sizeof(int32_t) * n, false, s));
    if (tau) PG_TRY(copy_out(tau, dt, sizeof(int32_t) * n, false, s));
  }
  PG_HIP(hipStreamSynchronize(s));
  return PG_OK;
}

pg_status odd_region_winner_out(pg_game *g, const uint8_t *w2,
                                uint8_t *winner, bool dev, hipStream_t s) {
  const int64_t n = g->n;
  struct Tmp {
    uint8_t *a = nullptr;
    ~Tmp() { dev_free(a); }
  } tmp;
  uint8_t *dw = winner;
  if (!dev) {
    PG_TRY(dev_alloc(&tmp.a, n));
    dw = tmp.a;
  }
  hipLaunchKernelGGL(k_or_winner_out, dim3(grid_for(n)), dim3(kBlock), 0, s,
                     g->or_new, w2, dw, n);
  if (!dev) PG_TRY(copy_out(winner, dw, n, false, s));
  PG_HIP(hipStreamSynchronize(s));
  return PG_OK;
}

}  // namespace pgk
