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

__device__ __forceinline__ uint64_t color_key(int32_t pri, int32_t v) {
  return ((uint64_t)(uint32_t)pri << 32) | (uint32_t)v;
}

__global__ void k_or_color_init(const uint8_t *alive, const int32_t *pri,
                                unsigned long long *col, int64_t n) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) col[v] = alive[v] ? color_key(pri[v], (int32_t)v) : 0ull;
}

// col[w] = max over live v -> w of col[v]: one relaxation sweep
__global__ void k_or_color_sweep(const int64_t *off, const int32_t *tgt,
                                 const uint8_t *alive,
                                 unsigned long long *col, int64_t n,
                                 int32_t *changed) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ch = false;
  if (v < n && alive[v]) {
    const unsigned long long c = col[v];
    for (int64_t e = off[v]; e < off[v + 1]; ++e) {
      const int32_t w = tgt[e];
      if (alive[w] && col[w] < c) {
        atomicMax(&col[w], c);
        ch = true;
      }
    }
  }
  if (__ballot(ch) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(changed, 1);
}

// a colour's root reaches itself; reset of the root flags
__global__ void k_or_reach_init(const uint8_t *alive,
                                const unsigned long long *col, uint8_t *reach,
                                uint8_t *nontriv, int64_t n) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  reach[v] = alive[v] && (int64_t)(uint32_t)col[v] == v;
  nontriv[v] = 0;
}

// v reaches its colour's root inside its colour when a successor of the
// same colour does: one sweep
__global__ void k_or_reach_sweep(const int64_t *off, const int32_t *tgt,
                                 const uint8_t *alive,
                                 const unsigned long long *col, uint8_t *reach,
                                 int64_t n, int32_t *changed) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ch = false;
  if (v < n && alive[v] && !reach[v]) {
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
  if (__ballot(ch) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(changed, 1);
}

// a root's component has an edge when another vertex is in it or the root
// has a loop
__global__ void k_or_nontrivial(const int64_t *off, const int32_t *tgt,
                                const uint8_t *alive,
                                const unsigned long long *col,
                                const uint8_t *reach, uint8_t *nontriv,
                                int64_t n) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || !alive[v] || !reach[v]) return;
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

// components with an odd root join the seed; roots of the others leave
__global__ void k_or_peel(uint8_t *alive, const unsigned long long *col,
                          const uint8_t *reach, const uint8_t *nontriv,
                          uint8_t *seed, int64_t n, int32_t *left) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool live = false;
  if (v < n && alive[v]) {
    live = true;
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
  }
  if (__ballot(live) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(left, 1);
}

// R: v in X with a successor in R (inside X)
__global__ void k_or_back(const int64_t *off, const int32_t *tgt,
                          const uint8_t *inx, uint8_t *R, int64_t n,
                          int32_t *changed) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ch = false;
  if (v < n && inx[v] && !R[v]) {
    for (int64_t e = off[v]; e < off[v + 1]; ++e) {
      const int32_t w = tgt[e];
      if (inx[w] && R[w]) {
        R[v] = 1;
        ch = true;
        break;
      }
    }
  }
  if (__ballot(ch) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(changed, 1);
}

// Odd's attractor: an Odd vertex with a successor in A, an Even vertex with
// every successor in A
__global__ void k_or_attr(const int64_t *off, const int32_t *tgt,
                          const uint8_t *owner, uint8_t *A, int64_t n,
                          int32_t *changed) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ch = false;
  if (v < n && !A[v]) {
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
  if (__ballot(ch) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(changed, 1);
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

// Repeats `sweep` (groups of four, one synchronisation each) until a group
// changes nothing; fails after `bound` groups.
template <class F>
pg_status fixpoint(pg_game *g, hipStream_t s, int64_t bound, F sweep) {
  for (int64_t round = 0;; ++round) {
    if (round > bound)
      return pg_fail(PG_EINTERNAL, "odd-region fixpoint did not converge");
    fill_i32(g->ctr + C_MISC, 0, 1, s);
    for (int k = 0; k < 4; ++k) sweep(g->ctr + C_MISC);
    PG_TRY(sync_ctr(g, s));
    if (g->hctr[C_MISC] == 0) return PG_OK;
  }
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
  PG_HIP(hipMemcpyAsync(alive, inx, n, hipMemcpyDeviceToDevice, s));
  fill_u8(seed, 0, n, s);
  const int64_t bound = n + 64;
  // peeling rounds: every round drops at least every colour's root
  for (int64_t round = 0;; ++round) {
    if (round > n + 1)
      return pg_fail(PG_EINTERNAL, "odd-region peeling did not converge");
    hipLaunchKernelGGL(k_or_color_init, dim3(gn), dim3(kBlock), 0, s, alive,
                       pri, col, n);
    PG_TRY(fixpoint(g, s, bound, [&](int32_t *ch) {
      hipLaunchKernelGGL(k_or_color_sweep, dim3(gn), dim3(kBlock), 0, s, off,
                         tgt, alive, col, n, ch);
    }));
    hipLaunchKernelGGL(k_or_reach_init, dim3(gn), dim3(kBlock), 0, s, alive,
                       col, reach, nontriv, n);
    PG_TRY(fixpoint(g, s, bound, [&](int32_t *ch) {
      hipLaunchKernelGGL(k_or_reach_sweep, dim3(gn), dim3(kBlock), 0, s, off,
                         tgt, alive, col, reach, n, ch);
    }));
    hipLaunchKernelGGL(k_or_nontrivial, dim3(gn), dim3(kBlock), 0, s, off,
                       tgt, alive, col, reach, nontriv, n);
    fill_i32(g->ctr + C_MISC, 0, 1, s);
    hipLaunchKernelGGL(k_or_peel, dim3(gn), dim3(kBlock), 0, s, alive, col,
                       reach, nontriv, seed, n, g->ctr + C_MISC);
    PG_TRY(sync_ctr(g, s));
    if (g->hctr[C_MISC] == 0) break;
  }
  // R = what reaches the seed inside X; A = Odd's attractor of R (in place)
  PG_TRY(fixpoint(g, s, bound, [&](int32_t *ch) {
    hipLaunchKernelGGL(k_or_back, dim3(gn), dim3(kBlock), 0, s, off, tgt, inx,
                       seed, n, ch);
  }));
  PG_TRY(fixpoint(g, s, bound, [&](int32_t *ch) {
    hipLaunchKernelGGL(k_or_attr, dim3(gn), dim3(kBlock), 0, s, off, tgt,
                       owner, seed, n, ch);
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
  if (n2 == 0) {   // Odd wins everything on its own
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
