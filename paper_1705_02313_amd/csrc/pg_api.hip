// The C ABI (include/pg.h): game loading and validation, the admissibility
// preprocessing, strategy import/export and the loops of Algorithm 1.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <string>
#include <vector>

#include "pg_common.h"

static thread_local std::string g_last_error;

pg_status pg_fail(pg_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

namespace pgk {

// ---------------------------------------------------------------------------
// validation (section 2: every vertex owned by one player, has an outgoing
// edge and a priority; distinct priorities are required by the rank keys)
// ---------------------------------------------------------------------------
__global__ void k_off32_to_64(const int32_t *in, int64_t *out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
}

__global__ void k_check_offsets(const int64_t *off, int64_t n, int64_t m,
                                int32_t *ctr) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int64_t a = off[v], b = off[v + 1];
  bool bad = (b <= a) || (b > m) || (a < 0);
  if (v == 0 && a != 0) bad = true;
  if (v == n - 1 && b != m) bad = true;
  if (bad) atomicOr(&ctr[C_ERR], ERR_OFFSETS);
}

__global__ void k_check_targets(const int32_t *tgt, int64_t m, int64_t n,
                                int32_t *ctr) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const int32_t t = tgt[e];
  if (t < 0 || (int64_t)t >= n) atomicOr(&ctr[C_ERR], ERR_INVAL);
}

__global__ void k_dup_check(const uint32_t *sk, int64_t n, int32_t *flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > 0 && i < n && sk[i] == sk[i - 1]) *flag = 1;
}

__global__ void k_max_i32(const int32_t *a, int64_t n, int32_t *out) {
  int32_t mx = -1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    mx = a[i] > mx ? a[i] : mx;
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const int32_t y = __shfl_down(mx, o, kWave);
    mx = y > mx ? y : mx;
  }
  if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(out, mx);
}

// One bit per priority value: a bit found set already is a repeat.
__global__ void k_dup_bits(const int32_t *pri, int64_t n, uint32_t *bits,
                           int32_t *flag) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint32_t p = (uint32_t)pri[v];
  const uint32_t b = 1u << (p & 31u);
  if (atomicOr(&bits[p >> 5], b) & b) *flag = 1;
}

__global__ void k_check_vertices(const uint8_t *owner, const int32_t *pri,
                                 int64_t n, int32_t *ctr) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  if (owner[v] > 1 || pri[v] < 0) atomicOr(&ctr[C_ERR], ERR_INVAL);
}

// ---------------------------------------------------------------------------
// preprocessing (section 3, "The algorithm")
// ---------------------------------------------------------------------------
// X: the largest set of Odd vertices each with a successor in X, found by
// removing Odd vertices without a successor in X until nothing changes.
// Updates are made in place; any interleaving of them converges to the same
// largest fixpoint.
__device__ __forceinline__ int32_t ld_flag(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_x_init(const uint8_t *owner, uint8_t *inx, int64_t n) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) inx[v] = owner[v] == 1;
}

// One round of the greatest fixpoint X (rounds update inx in place).  X
// only shrinks, so a member's row is scanned from the entry that last
// showed a successor in X (wit[v], relative to the row; 0 at first): the
// entries before it have left X for good.  Over all rounds each row is read
// about once.
__global__ void k_x_round(const int64_t *__restrict__ off,
                          const int32_t *__restrict__ tgt, uint8_t *inx,
                          uint32_t *wit, int64_t n, int32_t *ctr) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool drop = false;
  if (v < n && __hip_atomic_load(&inx[v], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT)) {
    const int64_t e0 = off[v], end = off[v + 1];
    const uint32_t w0 = wit[v];
    int64_t e = e0 + w0;
    bool any = false;
    for (; e < end; ++e)
      if (__hip_atomic_load(&inx[tgt[e]], __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT)) {
        any = true;
        break;
      }
    if (!any) {
      __hip_atomic_store(&inx[v], (uint8_t)0, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      drop = true;
    } else if (e - e0 != (int64_t)w0) {
      // a witness beyond 32 bits of row offset is not kept (rescan)
      wit[v] = (e - e0 <= 0xffffffffLL) ? (uint32_t)(e - e0) : 0u;
    }
  }
  // a change flag: most waves find it already set and only read it
  if (__ballot(drop) && (threadIdx.x & (kWave - 1)) == 0 &&
      ld_flag(&ctr[C_MISC]) == 0)
    atomicOr(&ctr[C_MISC], 1);
}

// X': members of X with a predecessor in X
__global__ void k_xp_mark(const int64_t *__restrict__ off,
                          const int32_t *__restrict__ tgt,
                          const uint8_t *__restrict__ inx, uint32_t *xp,
                          int64_t n) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || !inx[v]) return;
  for (int64_t e = off[v], end = off[v + 1]; e < end; ++e) {
    const int32_t w = tgt[e];
    if (inx[w]) xp[w] = 1u;
  }
}

// The modified game: rows of original vertices keep their length, edges
// between members of X go through the dummy of their target; the dummy of the
// i-th member w of X' is vertex n + i, Even, priority i, row [w].  Original
// priorities rise by K (|X'| rounded up to even).
__global__ void k_aug_build(int64_t n, int64_t m, int64_t K, int dense,
                            const int64_t *__restrict__ off,
                            const int32_t *__restrict__ tgt,
                            const uint8_t *__restrict__ owner,
                            const int32_t *__restrict__ pri,
                            const uint8_t *__restrict__ inx,
                            const uint32_t *__restrict__ xp,
                            const uint32_t *__restrict__ did, int64_t *off2,
                            int32_t *tgt2, uint8_t *owner2, int32_t *pri2,
                            int32_t *ctr) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  off2[v] = off[v];
  if (v == n - 1) off2[n] = off[n];
  const bool vx = inx[v] != 0;
  for (int64_t e = off[v], end = off[v + 1]; e < end; ++e) {
    const int32_t w = tgt[e];
    tgt2[e] = (vx && inx[w]) ? (int32_t)(n + did[w]) : w;
  }
  owner2[v] = owner[v];
  const int64_t p = (int64_t)pri[v] + K;
  if (p > 2147483647LL) atomicOr(&ctr[C_ERR], ERR_INVAL);
  pri2[v] = (int32_t)p;
  if (xp[v]) {
    const int64_t i = did[v];
    owner2[n + i] = 0;
    pri2[n + i] = dense ? 0 : (int32_t)i;
    tgt2[m + i] = (int32_t)v;
    off2[n + i + 1] = m + i + 1;
  }
}

// signed-priority order: odd priorities descending, then even ascending
__global__ void k_rv_keys(const int32_t *pri, uint32_t *sk, uint32_t *sv,
                          int64_t n) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint32_t p = (uint32_t)pri[v];
  sk[v] = (p & 1u) ? (0x7fffffffu - p) : (0x80000000u + p);
  sv[v] = (uint32_t)v;
}

__global__ void k_rv_finish(const uint32_t *skS, const uint32_t *svS,
                            int32_t *perm, int32_t *rvpos, int64_t n,
                            int check_dup, int32_t *ctr) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool odd = false;
  if (i < n) {
    perm[i] = (int32_t)svS[i];
    rvpos[svS[i]] = (int32_t)i;
    odd = skS[i] < 0x80000000u;
    if (check_dup && i > 0 && skS[i] == skS[i - 1])
      atomicOr(&ctr[C_ERR], ERR_DUPPRI);
  }
  count_block(&ctr[C_DIST_MISC], odd);
}

// Relabelling: vertex i of the new game is vertex from[i] of the old one,
// and a target t of the old game becomes to[t].  Rows keep their edge order
// (so the first entry of a row stays the first).  k_relabel_vertices writes
// the new row lengths into off2 (scanned afterwards; off2[n] = 0 before the
// scan), the owners and the priorities; k_relabel_rows copies the rows.
// With from = perm, to = rvpos a game goes into signed order; with from =
// rvpos, to = perm it comes back.
__global__ void k_relabel_vertices(const int64_t *off, const uint8_t *owner,
                                   const int32_t *pri, const int32_t *from,
                                   int64_t *off2, uint8_t *owner2,
                                   int32_t *pri2, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  if (i == n) {
    off2[n] = 0;
    return;
  }
  const int32_t v = from[i];
  off2[i] = off[v + 1] - off[v];
  owner2[i] = owner[v];
  pri2[i] = pri[v];
}

__global__ void k_relabel_rows(const int64_t *off, const int32_t *tgt,
                               const int32_t *from, const int32_t *to,
                               const int64_t *off2, int32_t *tgt2, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t v = from[i];
  const int64_t e0 = off[v], len = off[v + 1] - e0, o = off2[i];
  for (int64_t k = 0; k < len; ++k) tgt2[o + k] = to[tgt[e0 + k]];
}

// Odd vertices and Even vertices as two increasing lists (for the switch
// kernels), from the exclusive scan `oscan` of the Odd flags.
__global__ void k_split_players(const uint8_t *owner, const uint32_t *oscan,
                                int32_t *odd_ids, int32_t *even_ids,
                                int64_t n) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  if (owner[v] == 1) odd_ids[oscan[v]] = (int32_t)v;
  else even_ids[v - oscan[v]] = (int32_t)v;
}

__global__ void k_odd_flags(const uint8_t *owner, uint32_t *f, int64_t n) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) f[v] = owner[v] == 1;
}

// ---------------------------------------------------------------------------
// strategies <-> play graph
// ---------------------------------------------------------------------------
// sp[v] = {successor, priority of the successor}; the sink's is INT32_MAX
__global__ void k_sp_init(const int64_t *off, const int32_t *tgt,
                          const uint8_t *owner, const int32_t *pri, int2 *sp,
                          int32_t N) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v == 0) sp[N] = make_int2(N, 2147483647);
  if (v >= N) return;
  const int32_t s = owner[v] ? tgt[off[v]] : N;
  sp[v] = make_int2(s, s == N ? 2147483647 : pri[s]);
}



// The strategy arrays at the C ABI use the caller's vertex ids; for a
// relabeled game perm/rvpos translate them (both null otherwise).  A null
// sigma (tau) leaves the Even (Odd) entries of sp as they are.
__global__ void k_sp_import(const uint8_t *owner, const int32_t *pri,
                            const int32_t *sigma, const int32_t *tau,
                            const int32_t *perm, const int32_t *rvpos,
                            int2 *sp, int32_t N, int32_t *ctr) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int32_t v = perm ? perm[i] : (int32_t)i;
  const bool even = owner[i] == 0;
  const int32_t *strat = even ? sigma : tau;
  if (!strat) return;  // that player keeps its current choices
  int32_t s = strat[v];
  if (even && s == PG_SINK) {
    s = N;
  } else if (s < 0 || s >= N) {
    atomicOr(&ctr[C_ERR], ERR_INVAL);
    s = N;
  } else if (rvpos) {
    s = rvpos[s];
  }
  sp[i] = make_int2(s, s == N ? 2147483647 : pri[s]);
}

// With `report` (the outputs of a solve), an Odd choice of a dummy d_w
// (caller id >= n_orig) is given as w, the only entry of the dummy's row:
// the dummy stands in the middle of the original edge to w (section 3).
__global__ void k_sp_export(const uint8_t *owner, const int2 *sp,
                            const int32_t *perm, const int32_t *rvpos,
                            const int64_t *off, const int32_t *tgt,
                            int64_t n_orig, int report, int32_t *sigma,
                            int32_t *tau, int32_t N) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const int32_t i = rvpos ? rvpos[v] : (int32_t)v;
  const int32_t si = sp[i].x;
  int32_t s = (perm && si != N) ? perm[si] : si;
  const bool even = owner[i] == 0;
  if (report && !even && s != N && s >= n_orig) {
    const int32_t w = tgt[off[si]];
    s = perm ? perm[w] : w;
  }
  if (sigma) sigma[v] = even ? (s == N ? PG_SINK : s) : PG_SINK;
  if (tau) tau[v] = even ? PG_SINK : s;
}

__global__ void k_initial(const int64_t *off, const int32_t *tgt,
                          const uint8_t *owner, const int32_t *perm,
                          const int32_t *rvpos, int32_t *sigma, int32_t *tau,
                          int32_t N) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const int32_t i = rvpos ? rvpos[v] : (int32_t)v;
  if (sigma) sigma[v] = PG_SINK;
  if (tau) {
    const int32_t t = owner[i] ? tgt[off[i]] : PG_SINK;
    tau[v] = (perm && t != PG_SINK) ? perm[t] : t;
  }
}

// Rank keys in the caller's ids: key2[v] = key[rvpos[v]]; the sink's key
// (index N) stays where it is.
__global__ void k_key_export(const int32_t *key, const int32_t *rvpos,
                             int32_t *key2, int32_t N) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v > N) return;
  key2[v] = key[v == N ? N : rvpos[v]];
}

// Polynomial hash of the keys in the caller's ids (the order k_key_export
// writes): h = sum over v of ((uint32)key'[v] + 1) * M^(N - v) mod 2^64,
// which is the value of h = h * M + key'[v] + 1 folded from v = 0 to N.
// Each thread raises M by square-and-multiply; one atomic per block.
constexpr unsigned long long kHashMul = 1099511628211ull;
__global__ void k_key_hash(const int32_t *key, const int32_t *rvpos,
                           int32_t N, unsigned long long *out) {
  __shared__ unsigned long long part[kBlock / kWave];
  unsigned long long acc = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= N;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t k = key[(v == N || !rvpos) ? v : rvpos[v]];
    unsigned long long e = (unsigned long long)(N - v), pw = 1ull,
                       b = kHashMul;
    while (e) {
      if (e & 1ull) pw *= b;
      b *= b;
      e >>= 1;
    }
    acc += ((unsigned long long)(uint32_t)k + 1ull) * pw;
  }
  for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_down(acc, o, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < kBlock / kWave; ++w) t += part[w];
    atomicAdd(out, t);
  }
}

// Edges of the Odd rows (for the switch kernels' byte counts): a grid-stride
// sum with one atomic per block.
__global__ void k_count_odd_edges(const int64_t *off, const uint8_t *owner,
                                  int64_t n, unsigned long long *out) {
  __shared__ unsigned long long part[kBlock / kWave];
  unsigned long long e = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    if (owner[v] == 1) e += (unsigned long long)(off[v + 1] - off[v]);
  for (int o = kWave / 2; o > 0; o >>= 1) e += __shfl_down(e, o, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < kBlock / kWave; ++w) t += part[w];
    atomicAdd(out, t);
  }
}

// SI-Reset: every Odd vertex back to the first entry of its row.
__global__ void k_sp_reset_odd(const int64_t *off, const int32_t *tgt,
                               const uint8_t *owner, const int32_t *pri,
                               int2 *sp, int32_t N) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N || owner[v] != 1) return;
  const int32_t u = tgt[off[v]];
  sp[v] = make_int2(u, pri[u]);
}

// Theorem 1: Even wins exactly where the final valuation is top (the walks
// of the last valuation marked those vertices with rs = 2).
__global__ void k_winner(const uint8_t *rs, const int32_t *rvpos,
                         uint8_t *winner, int64_t n) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) winner[v] = rs[rvpos ? rvpos[v] : v] == 2 ? 0 : 1;
}

}  // namespace pgk

using namespace pgk;

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
namespace pgk {

struct DevGuard {
  int prev = -1;
  explicit DevGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DevGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev)
      (void)hipSetDevice(prev);
  }
};



// Copies count elements to or from the caller's buffer, which is on the
// device when `device` is true.
pg_status copy_in(void *dst, const void *src, size_t bytes, bool device,
                  hipStream_t s) {
  if (bytes == 0) return PG_OK;
  PG_HIP(hipMemcpyAsync(dst, src, bytes,
                        device ? hipMemcpyDeviceToDevice
                               : hipMemcpyHostToDevice,
                        s));
  return PG_OK;
}

pg_status copy_out(void *dst, const void *src, size_t bytes, bool device,
                   hipStream_t s) {
  if (bytes == 0) return PG_OK;
  PG_HIP(hipMemcpyAsync(dst, src, bytes,
                        device ? hipMemcpyDeviceToDevice
                               : hipMemcpyDeviceToHost,
                        s));
  return PG_OK;
}

thread_local DevPool *tl_pool = nullptr;

pg_status DevPool::alloc(void **p, size_t bytes, bool host) {
  std::lock_guard<std::mutex> lock(mu);
  if (bump_dev) {
    size_t &used = host ? bump_hused : bump_used;
    const size_t cap = host ? bump_hcap : bump_cap;
    const size_t at = (used + 255) & ~size_t(255);
    if (at > cap || bytes > cap - at) {
      *p = nullptr;
      return pg_fail(PG_ENOMEM,
                     std::string("the game does not fit the ") +
                         (host ? "host" : "device") +
                         " scratch of pg_solve_noalloc (" +
                         std::to_string(cap) + " bytes)");
    }
    *p = (host ? bump_host : bump_dev) + at;
    used = at + bytes;
    return PG_OK;
  }
  const size_t b = bucket(bytes);
  auto &fl = host ? host_free[b] : dev_free[b];
  if (fl.empty()) {
    const bool slab = b <= kSlabBlockMax;
    const size_t total = slab ? b * kSlabBlocks : b;
    void *base = nullptr;
    hipError_t e = host ? hipHostMalloc(&base, total, hipHostMallocDefault)
                        : hipMalloc(&base, total);
    if (e != hipSuccess) {
      *p = nullptr;
      return pg_fail(PG_ENOMEM, std::string("pool allocation failed: ") +
                                    hipGetErrorString(e));
    }
    auto &sizes = host ? host_size : dev_size;
    if (slab) {
      Slab sl;
      sl.base = base;
      sl.block = b;
      sl.host = host;
      slabs.push_back(sl);
      // blocks handed out from the end of the free list: keep the slab's
      // first block last so that it is taken first
      for (size_t k = kSlabBlocks; k-- > 0;) {
        void *q = (char *)base + k * b;
        sizes[q] = b;
        slab_of[q] = slabs.size() - 1;
        fl.push_back(q);
      }
    } else {
      sizes[base] = b;
      fl.push_back(base);
    }
  }
  *p = fl.back();
  fl.pop_back();
  auto it = slab_of.find(*p);
  if (it != slab_of.end()) ++slabs[it->second].in_use;
  return PG_OK;
}

bool DevPool::release(void *p) {
  std::lock_guard<std::mutex> lock(mu);
  if (bump_dev) {
    const uint8_t *q = (const uint8_t *)p;
    return (q >= bump_dev && q < bump_dev + bump_cap) ||
           (q >= bump_host && q < bump_host + bump_hcap);
  }
  auto it = dev_size.find(p);
  bool host = false;
  if (it == dev_size.end()) {
    it = host_size.find(p);
    if (it == host_size.end()) return false;
    host = true;
  }
  (host ? host_free : dev_free)[it->second].push_back(p);
  auto si = slab_of.find(p);
  if (si != slab_of.end()) --slabs[si->second].in_use;
  return true;
}

void DevPool::trim() {
  std::lock_guard<std::mutex> lock(mu);
  // slabs none of whose blocks is in use leave with all their blocks
  std::vector<bool> gone(slabs.size(), false);
  for (size_t i = 0; i < slabs.size(); ++i)
    gone[i] = slabs[i].base && slabs[i].in_use == 0;
  for (int h = 0; h < 2; ++h) {
    auto &lists = h ? host_free : dev_free;
    auto &sizes = h ? host_size : dev_size;
    for (auto &kv : lists) {
      std::vector<void *> keep;
      for (void *q : kv.second) {
        auto si = slab_of.find(q);
        if (si == slab_of.end()) {
          // a block of its own, not in use
          if (h) (void)hipHostFree(q);
          else (void)hipFree(q);
          sizes.erase(q);
        } else if (gone[si->second]) {
          sizes.erase(q);
          slab_of.erase(si);
        } else {
          keep.push_back(q);
        }
      }
      kv.second.swap(keep);
    }
  }
  for (size_t i = 0; i < slabs.size(); ++i)
    if (gone[i]) {
      if (slabs[i].host) (void)hipHostFree(slabs[i].base);
      else (void)hipFree(slabs[i].base);
      slabs[i].base = nullptr;   // the index stays: other blocks name theirs
    }
}

// One cache per device, kept until the process ends.  Single games allocate
// from it and pg_free returns their memory to it; a block goes back only
// after the work that used it has finished (every return follows a
// synchronisation), so a load on another thread's stream may reuse it.
static std::mutex g_cache_mu;
static std::map<int, DevPool *> g_caches;

DevPool *game_cache(int device) {
  std::lock_guard<std::mutex> lock(g_cache_mu);
  DevPool *&c = g_caches[device];
  if (!c) c = new DevPool();
  return c;
}

static void trim_caches() {
  std::lock_guard<std::mutex> lock(g_cache_mu);
  int prev = -1;
  (void)hipGetDevice(&prev);
  for (auto &kv : g_caches) {
    (void)hipSetDevice(kv.first);
    kv.second->trim();
  }
  if (prev >= 0) (void)hipSetDevice(prev);
}

void DevPool::clear() {
  std::lock_guard<std::mutex> lock(mu);
  for (auto &kv : dev_size)
    if (!slab_of.count(kv.first)) (void)hipFree(kv.first);
  for (auto &kv : host_size)
    if (!slab_of.count(kv.first)) (void)hipHostFree(kv.first);
  for (Slab &sl : slabs)
    if (sl.base) {
      if (sl.host) (void)hipHostFree(sl.base);
      else (void)hipFree(sl.base);
    }
  dev_size.clear();
  host_size.clear();
  dev_free.clear();
  host_free.clear();
  slabs.clear();
  slab_of.clear();
}

void dev_free(void *p) {
  if (!p) return;
  if (tl_pool && tl_pool->release(p)) return;
  (void)hipFree(p);
}

void host_free(void *p) {
  if (!p) return;
  if (tl_pool && tl_pool->release(p)) return;
  (void)hipHostFree(p);
}

pg_status host_alloc(void **p, size_t bytes) {
  if (tl_pool) return tl_pool->alloc(p, bytes, true);
  PG_HIP(hipHostMalloc(p, bytes, hipHostMallocDefault));
  return PG_OK;
}

pg_status sync_ctr(pg_game *g, hipStream_t s) {
  PG_HIP(hipMemcpyAsync(g->hctr, g->ctr, sizeof(int32_t) * C_COUNT,
                        hipMemcpyDeviceToHost, s));
  PG_HIP(hipStreamSynchronize(s));
  fold_switches(g->hctr);
  if (g->prof.on) g->prof.flush();
  return PG_OK;
}

void free_game(pg_game *g) {
  if (!g) return;
  void *ptrs[] = {g->off,      g->tgt,      g->owner,    g->pri,
                  g->perm,     g->rvpos,    g->odd_ids,  g->even_ids,
                  g->sp,       g->key,      g->ng,       g->cand,
                  g->rcand,    g->wl0,      g->wl_ng,    g->wl_rt,
                  g->wl1,      g->rs,       g->sk0,      g->sv0,
                  g->sk1,      g->sv1,      g->tile_cnt, g->scan_tmp,
                  g->kids,     g->fh,       g->pos,      g->elem,
                  g->aux,      g->or_new,   g->or_orig,
                  g->ctr,      g->u64tmp,   g->cvals,    g->pidx,
                  g->cnt,      g->elem4,    g->rs1,      g->cnt2,
                  g->tsw_t,    g->tsw_slot, g->tsw_g,    g->tsw_tz,
                  g->tsw_sz,   g->tsw_bs,   g->tsw_r};
  for (void *p : ptrs) dev_free(p);
  for (int k = 0; k < pgk::kMaxLevels; ++k) {
    dev_free(g->lv[k].sum);
    dev_free(g->lv[k].next);
    dev_free(g->lv[k].base);
    dev_free(g->vsum[k]);
    dev_free(g->vbase[k]);
  }
  host_free(g->hctr);
  host_free(g->h_rl);
  if (g->iter_exec) (void)hipGraphExecDestroy(g->iter_exec);
  if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
  if (g->ev_a) (void)hipEventDestroy(g->ev_a);
  if (g->ev_b) (void)hipEventDestroy(g->ev_b);
  g->prof.release();
  delete g;
}

// Allocates the per-solve state for games of up to `cap` vertices (the
// modified game's own size for a single game, the arena size for a batch).
pg_status alloc_state(pg_game *g, int64_t cap) {
  const int64_t N = cap;
  PG_TRY(dev_alloc(&g->odd_ids, N));
  PG_TRY(dev_alloc(&g->even_ids, N));
  PG_TRY(dev_alloc(&g->u64tmp, 2));
  PG_TRY(dev_alloc(&g->perm, N));
  PG_TRY(dev_alloc(&g->rvpos, N));
  PG_TRY(dev_alloc(&g->sp, N + 1));
  PG_TRY(dev_alloc(&g->key, N + 1));
  PG_TRY(dev_alloc(&g->ng, N));
  PG_TRY(dev_alloc(&g->cand, N));
  PG_TRY(dev_alloc(&g->rcand, N));
  g->wl_cap = (N + kDistSlots - 1) / kDistSlots + 2 * kBlock;
  PG_TRY(dev_alloc(&g->wl_ng, kDistSlots * g->wl_cap));
  PG_TRY(dev_alloc(&g->wl_rt, kDistSlots * g->wl_cap));
  PG_TRY(dev_alloc(&g->wl0, N));
  PG_TRY(dev_alloc(&g->wl1, N));
  PG_TRY(dev_alloc(&g->rs, N + 1));
  PG_TRY(dev_alloc(&g->sk0, N));
  PG_TRY(dev_alloc(&g->sv0, N));
  PG_TRY(dev_alloc(&g->sk1, N));
  PG_TRY(dev_alloc(&g->sv1, N));
  g->tiles = radix_tiles(N);
  PG_TRY(dev_alloc(&g->tile_cnt, 256 * g->tiles));
  PG_TRY(dev_alloc(&g->rs1, onesweep_words(N)));
  g->scan_tmp_bytes = radix_scan_tmp_bytes(N);
  size_t s2 = scan_excl_u32(nullptr, nullptr, N, nullptr, 0);
  if (s2 > g->scan_tmp_bytes) g->scan_tmp_bytes = s2;
  PG_TRY(dev_alloc((uint8_t **)&g->scan_tmp, (int64_t)g->scan_tmp_bytes + 16));
  PG_TRY(dev_alloc(&g->kids, N));
  PG_TRY(dev_alloc(&g->fh, N + 1));
  PG_TRY(dev_alloc(&g->pos, N + 1));
  fill_i32(g->pos, 0, N + 1, 0);
  PG_TRY(dev_alloc(&g->elem, 2 * N + 2));
  PG_TRY(dev_alloc(&g->aux, 2 * N + 2));
  // sublist levels for the longest possible Euler list (down to one
  // splitter, which every plan stops before)
  for (int k = 0; k < kMaxLevels; ++k) {
    const int64_t ns = level_size(2 * N + 2, k + 1, kStrideMin);
    PG_TRY(dev_alloc(&g->lv[k].sum, ns));
    PG_TRY(dev_alloc(&g->lv[k].next, ns));
    PG_TRY(dev_alloc(&g->lv[k].base, ns));
    if (ns <= 1) break;
  }
  return PG_OK;
}

pg_status check_err(pg_game *g, const char *what) {
  const int e = g->hctr[C_ERR];
  if (e & ERR_INVAL) return pg_fail(PG_EINVAL, std::string(what));
  if (e & ERR_DUPPRI)
    return pg_fail(PG_EINVAL, "priorities must be pairwise distinct");
  if (e & ERR_INADMISSIBLE)
    return pg_fail(PG_EINADMISSIBLE,
                   "the play graph has a cycle whose largest priority is odd");
  if (e & (ERR_LISTWALK | ERR_RANKCOUNT))
    return pg_fail(PG_EINTERNAL, "list ranking failed a consistency check");
  if (e & ERR_SORT)
    return pg_fail(PG_EINTERNAL, "radix sort look-back timed out");
  return PG_OK;
}

// Validates a game and builds its modified game in g->off, g->tgt,
// g->owner, g->pri (section 3 preprocessing unless PG_NO_PREPROCESS).  For
// rank valuations the dummies get the distinct priorities 0, 1, ... and the
// original ones are raised by |X'| rounded up to even; for count valuations
// (dense) every dummy gets priority 0 and the original ones are raised by 2
// when there is a dummy, so that few distinct priorities stay few.
pg_status load_modified(int64_t n, int64_t m, const void *offsets,
                        const int32_t *targets, const uint8_t *owner,
                        const int32_t *priority, uint32_t flags, hipStream_t s,
                        pg_game *g, LoadMode mode) {
  const bool dev = flags & PG_PTR_DEVICE;
  g->n = n;
  g->m = m;
  PG_TRY(host_alloc((void **)&g->hctr, sizeof(int32_t) * C_COUNT));
  PG_TRY(dev_alloc(&g->ctr, C_TOTAL));
  fill_i32(g->ctr, 0, C_TOTAL, s);

  // input copies.  The temporaries go back to the shared per-device cache
  // only after the stream has drained: the kernels queued last (the
  // modified game's build, or the copies) still read them, and a load on
  // another thread may take a returned block at once.
  int64_t *off_in = nullptr;
  int32_t *tgt_in = nullptr, *pri_in = nullptr;
  uint8_t *own_in = nullptr;
  struct Tmp {
    hipStream_t s;
    std::vector<void *> p;
    ~Tmp() {
      if (!p.empty()) (void)hipStreamSynchronize(s);
      for (void *x : p) dev_free(x);
    }
  } tmp{s, {}};
  PG_TRY(dev_alloc(&off_in, n + 1));
  tmp.p.push_back(off_in);
  PG_TRY(dev_alloc(&tgt_in, m));
  tmp.p.push_back(tgt_in);
  PG_TRY(dev_alloc(&own_in, n));
  tmp.p.push_back(own_in);
  PG_TRY(dev_alloc(&pri_in, n));
  tmp.p.push_back(pri_in);
  if (flags & PG_OFFSETS_I32) {
    int32_t *o32 = nullptr;
    PG_TRY(dev_alloc(&o32, n + 1));
    tmp.p.push_back(o32);
    PG_TRY(copy_in(o32, offsets, sizeof(int32_t) * (n + 1), dev, s));
    hipLaunchKernelGGL(k_off32_to_64, dim3(grid_for(n + 1)), dim3(kBlock), 0,
                       s, o32, off_in, n + 1);
  } else {
    PG_TRY(copy_in(off_in, offsets, sizeof(int64_t) * (n + 1), dev, s));
  }
  PG_TRY(copy_in(tgt_in, targets, sizeof(int32_t) * m, dev, s));
  PG_TRY(copy_in(own_in, owner, n, dev, s));
  PG_TRY(copy_in(pri_in, priority, sizeof(int32_t) * n, dev, s));

  // the three checks are independent: one synchronisation
  hipLaunchKernelGGL(k_check_offsets, dim3(grid_for(n)), dim3(kBlock), 0, s,
                     off_in, n, m, g->ctr);
  hipLaunchKernelGGL(k_check_targets, dim3(grid_for(m)), dim3(kBlock), 0, s,
                     tgt_in, m, n, g->ctr);
  hipLaunchKernelGGL(k_check_vertices, dim3(grid_for(n)), dim3(kBlock), 0, s,
                     own_in, pri_in, n, g->ctr);
  PG_TRY(sync_ctr(g, s));
  if (g->hctr[C_ERR] & ERR_OFFSETS)
    return pg_fail(PG_EINVAL,
                   "offsets must start at 0, end at m and give every vertex "
                   "a non-empty row");
  if (g->hctr[C_ERR])
    return pg_fail(PG_EINVAL,
                   "targets must lie in [0, n), owners in {0, 1} and "
                   "priorities be >= 0");

  g->dense = mode == kLoadCount;
  if (mode == kLoadAuto) {
    // repeated input priorities select count valuations.  Fewer values
    // than vertices repeat by pigeonhole; otherwise one bit per priority
    // value when the largest is below 32 n (each word then serves a few
    // scattered vertices), else a sort of the priorities and a look at
    // neighbours
    fill_i32(g->ctr + C_MISC, -1, 1, s);
    hipLaunchKernelGGL(k_max_i32, dim3(512), dim3(kBlock), 0, s, pri_in, n,
                       g->ctr + C_MISC);
    PG_TRY(sync_ctr(g, s));
    const int64_t maxpri = g->hctr[C_MISC];
    fill_i32(g->ctr + C_MISC, 0, 1, s);
    if (maxpri + 1 < n) {
      g->dense = true;
    } else if (maxpri < 32 * n) {
      uint32_t *bits = nullptr;
      const int64_t words = maxpri / 32 + 1;
      PG_TRY(dev_alloc(&bits, words));
      tmp.p.push_back(bits);
      fill_i32((int32_t *)bits, 0, words, s);
      hipLaunchKernelGGL(k_dup_bits, dim3(grid_for(n)), dim3(kBlock), 0, s,
                         pri_in, n, bits, g->ctr + C_MISC);
      PG_TRY(sync_ctr(g, s));
      g->dense = g->hctr[C_MISC] != 0;
    } else {
      uint32_t *k0 = nullptr, *v0 = nullptr, *k1 = nullptr, *v1 = nullptr;
      uint32_t *tc = nullptr;
      uint8_t *st = nullptr;
      PG_TRY(dev_alloc(&k0, n));
      tmp.p.push_back(k0);
      PG_TRY(dev_alloc(&v0, n));
      tmp.p.push_back(v0);
      PG_TRY(dev_alloc(&k1, n));
      tmp.p.push_back(k1);
      PG_TRY(dev_alloc(&v1, n));
      tmp.p.push_back(v1);
      PG_TRY(dev_alloc(&tc, 256 * radix_tiles(n)));
      tmp.p.push_back(tc);
      PG_TRY(dev_alloc(&st, (int64_t)radix_scan_tmp_bytes(n) + 16));
      tmp.p.push_back(st);
      PG_HIP(hipMemcpyAsync(k0, pri_in, sizeof(int32_t) * n,
                            hipMemcpyDeviceToDevice, s));
      const int w = radix_sort(k0, v0, k1, v1, n, 32, tc, st, s, nullptr,
                               nullptr, true);
      hipLaunchKernelGGL(k_dup_check, dim3(grid_for(n)), dim3(kBlock), 0, s,
                         w ? k1 : k0, n, g->ctr + C_MISC);
      PG_TRY(sync_ctr(g, s));
      g->dense = g->hctr[C_MISC] != 0;
    }
  }
  const bool dense = g->dense;

  int64_t nxp = 0;
  uint8_t *inx = nullptr;
  uint32_t *xp = nullptr, *did = nullptr;
  if (!(flags & PG_NO_PREPROCESS)) {
    PG_TRY(dev_alloc(&inx, n));
    tmp.p.push_back(inx);
    PG_TRY(dev_alloc(&xp, n));
    tmp.p.push_back(xp);
    PG_TRY(dev_alloc(&did, n));
    tmp.p.push_back(did);
    hipLaunchKernelGGL(k_x_init, dim3(grid_for(n)), dim3(kBlock), 0, s, own_in,
                       inx, n);
    // xp holds the rounds' row witnesses until X is known
    fill_i32((int32_t *)xp, 0, n, s);
    for (int64_t round = 0;; round += 4) {
      if (round > 4 * n + 64)
        return pg_fail(PG_EINTERNAL, "preprocessing did not converge");
      fill_i32(g->ctr + C_MISC, 0, 1, s);
      for (int k = 0; k < 4; ++k)
        hipLaunchKernelGGL(k_x_round, dim3(grid_for(n)), dim3(kBlock), 0, s,
                           off_in, tgt_in, inx, xp, n, g->ctr);
      PG_TRY(sync_ctr(g, s));
      if (g->hctr[C_MISC] == 0) break;
    }
    if (flags & PG_ODD_REGION) {
      // no dummies: the game without Odd's own winning region instead
      g->odd_region = true;
      return odd_region_reduce(g, s, n, m, off_in, tgt_in, own_in, pri_in,
                               inx);
    }
    fill_i32((int32_t *)xp, 0, n, s);
    hipLaunchKernelGGL(k_xp_mark, dim3(grid_for(n)), dim3(kBlock), 0, s,
                       off_in, tgt_in, inx, xp, n);
    size_t need = scan_excl_u32(nullptr, nullptr, n, nullptr, s);
    void *stmp = nullptr;
    PG_TRY(dev_alloc((uint8_t **)&stmp, (int64_t)need + 16));
    tmp.p.push_back(stmp);
    scan_excl_u32(xp, did, n, stmp, s);
    uint32_t last[2] = {0, 0};
    PG_HIP(hipMemcpyAsync(&last[0], did + (n - 1), 4, hipMemcpyDeviceToHost,
                          s));
    PG_HIP(hipMemcpyAsync(&last[1], xp + (n - 1), 4, hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    nxp = (int64_t)last[0] + last[1];
  }
  g->n_aug = n + nxp;
  g->m_aug = m + nxp;
  if (g->n_aug > kMaxVertices)
    return pg_fail(PG_EINVAL, "too many vertices after preprocessing");

  PG_TRY(dev_alloc(&g->off, g->n_aug + 1));
  PG_TRY(dev_alloc(&g->tgt, g->m_aug));
  PG_TRY(dev_alloc(&g->owner, g->n_aug));
  PG_TRY(dev_alloc(&g->pri, g->n_aug));
  if (flags & PG_NO_PREPROCESS) {
    PG_HIP(hipMemcpyAsync(g->off, off_in, sizeof(int64_t) * (n + 1),
                          hipMemcpyDeviceToDevice, s));
    PG_HIP(hipMemcpyAsync(g->tgt, tgt_in, sizeof(int32_t) * m,
                          hipMemcpyDeviceToDevice, s));
    PG_HIP(hipMemcpyAsync(g->owner, own_in, n, hipMemcpyDeviceToDevice, s));
    PG_HIP(hipMemcpyAsync(g->pri, pri_in, sizeof(int32_t) * n,
                          hipMemcpyDeviceToDevice, s));
  } else {
    const int64_t K = dense ? (nxp > 0 ? 2 : 0) : nxp + (nxp & 1);
    hipLaunchKernelGGL(k_aug_build, dim3(grid_for(n)), dim3(kBlock), 0, s, n,
                       m, K, (int)dense, off_in, tgt_in, own_in, pri_in, inx,
                       xp, did, g->off, g->tgt, g->owner, g->pri, g->ctr);
  }
  // a priority above INT32_MAX (ERR_INVAL) is reported at the caller's
  // next synchronisation: the wrapped values only make later keys wrong
  return PG_OK;
}

// Rebuilds a game of N vertices and M edges with vertex i taken from vertex
// from[i] and targets mapped by `to` (see k_relabel_vertices).  The new
// arrays are allocated; the old ones are left to the caller.
pg_status relabel_game(const int64_t *off, const int32_t *tgt,
                       const uint8_t *owner, const int32_t *pri,
                       const int32_t *from, const int32_t *to,
                       int64_t N, int64_t M, int64_t **off2,
                       int32_t **tgt2, uint8_t **owner2,
                       int32_t **pri2, hipStream_t s, bool drain) {
  PG_TRY(dev_alloc(off2, N + 1));
  PG_TRY(dev_alloc(tgt2, M));
  PG_TRY(dev_alloc(owner2, N));
  PG_TRY(dev_alloc(pri2, N));
  struct Tmp {
    uint8_t *p = nullptr;
    ~Tmp() { dev_free(p); }
  } stmp;
  const size_t need = scan_excl_i64(nullptr, nullptr, N + 1, nullptr, s);
  PG_TRY(dev_alloc(&stmp.p, (int64_t)need + 16));
  hipLaunchKernelGGL(k_relabel_vertices, dim3(grid_for(N + 1)), dim3(kBlock),
                     0, s, off, owner, pri, from, *off2, *owner2, *pri2, N);
  scan_excl_i64(*off2, *off2, N + 1, stmp.p, s);
  hipLaunchKernelGGL(k_relabel_rows, dim3(grid_for(N)), dim3(kBlock), 0, s,
                     off, tgt, from, to, *off2, *tgt2, N);
  if (drain) PG_HIP(hipStreamSynchronize(s));
  return PG_OK;
}

// The signed-priority order (and the distinctness check), the initial play
// graph and the two players' vertex lists of the modified game in g->off,
// g->tgt, g->owner, g->pri (state allocated by alloc_state).  A game with
// distinct priorities (rank valuations) is then stored in signed order
// (pg_game::relabeled).
pg_status finalize_state(pg_game *g, hipStream_t s, bool init_sp,
                         bool distinct) {
  const int64_t N = g->n_aug;
  int bits = 1;
  while ((int64_t(1) << bits) <= N + 1) ++bits;
  g->sort_bits = bits;
  // every counter but the error bits, which may hold the preprocessing's
  // priority overflow
  fill_i32(g->ctr + 1, 0, C_TOTAL - 1, s);
  hipLaunchKernelGGL(k_rv_keys, dim3(grid_for(N)), dim3(kBlock), 0, s, g->pri,
                     g->sk0, g->sv0, N);
  int which = radix_sort(g->sk0, g->sv0, g->sk1, g->sv1, N, 32, g->tile_cnt,
                         g->scan_tmp, s);
  hipLaunchKernelGGL(k_rv_finish, dim3(grid_for(N)), dim3(kBlock), 0, s,
                     which ? g->sk1 : g->sk0, which ? g->sv1 : g->sv0, g->perm,
                     g->rvpos, N, (int)distinct, g->ctr);
  sum_dist(g->ctr, C_DIST_MISC, C_MISC, s);
  PG_TRY(sync_ctr(g, s));
  PG_TRY(check_err(g, "a priority exceeds INT32_MAX after preprocessing"));
  if (distinct) {
    int64_t *off2 = nullptr;
    int32_t *tgt2 = nullptr, *pri2 = nullptr;
    uint8_t *owner2 = nullptr;
    pg_status st = relabel_game(g->off, g->tgt, g->owner, g->pri, g->perm,
                                g->rvpos, N, g->m_aug, &off2, &tgt2, &owner2,
                                &pri2, s);
    if (st != PG_OK) {
      (void)hipStreamSynchronize(s);
      dev_free(off2);
      dev_free(tgt2);
      dev_free(owner2);
      dev_free(pri2);
      return st;
    }
    dev_free(g->off);
    dev_free(g->tgt);
    dev_free(g->owner);
    dev_free(g->pri);
    g->off = off2;
    g->tgt = tgt2;
    g->owner = owner2;
    g->pri = pri2;
    g->relabeled = true;
  }
  if (init_sp)
    hipLaunchKernelGGL(k_sp_init, dim3(grid_for(N)), dim3(kBlock), 0, s,
                       g->off, g->tgt, g->owner, g->pri, g->sp, (int32_t)N);
  g->n_oddpri = g->hctr[C_MISC];
  // the two players' vertex lists and the Odd rows' edge count
  uint32_t *flags = g->sk0, *oscan = g->sk1;
  hipLaunchKernelGGL(k_odd_flags, dim3(grid_for(N)), dim3(kBlock), 0, s,
                     g->owner, flags, N);
  scan_excl_u32(flags, oscan, N, g->scan_tmp, s);
  uint32_t last[2] = {0, 0};
  PG_HIP(hipMemcpyAsync(&last[0], oscan + (N - 1), 4, hipMemcpyDeviceToHost,
                        s));
  PG_HIP(hipMemcpyAsync(&last[1], flags + (N - 1), 4, hipMemcpyDeviceToHost,
                        s));
  fill_i32((int32_t *)g->u64tmp, 0, 2, s);
  hipLaunchKernelGGL(k_count_odd_edges, dim3(1024), dim3(kBlock), 0, s,
                     g->off, g->owner, N, g->u64tmp);
  unsigned long long me = 0;
  PG_HIP(hipMemcpyAsync(&me, g->u64tmp, sizeof(me), hipMemcpyDeviceToHost, s));
  hipLaunchKernelGGL(k_split_players, dim3(grid_for(N)), dim3(kBlock), 0, s,
                     g->owner, oscan, g->odd_ids, g->even_ids, N);
  PG_HIP(hipStreamSynchronize(s));
  g->n_odd = (int64_t)last[0] + last[1];
  g->m_odd = (int64_t)me;
  return PG_OK;
}

// The maps between the caller's vertex ids and a relabeled game's (null for
// a game stored in the caller's order).
static const int32_t *io_perm(const pg_game *g) {
  return g->relabeled ? g->perm : nullptr;
}
static const int32_t *io_rvpos(const pg_game *g) {
  return g->relabeled ? g->rvpos : nullptr;
}

// Stages caller strategy arrays (host or device) into the play graph.
pg_status import_strats(pg_game *g, const int32_t *sigma, const int32_t *tau,
                        bool dev, hipStream_t s) {
  const int64_t N = g->n_aug;
  const int32_t *ds = sigma, *dt = tau;
  if (!dev) {
    // a null array leaves that player's choices as they are
    if (sigma) PG_TRY(copy_in(g->wl0, sigma, sizeof(int32_t) * N, false, s));
    if (tau) PG_TRY(copy_in(g->wl1, tau, sizeof(int32_t) * N, false, s));
    ds = sigma ? g->wl0 : nullptr;
    dt = tau ? g->wl1 : nullptr;
  }
  fill_i32(g->ctr, 0, C_COUNT, s);
  hipLaunchKernelGGL(k_sp_import, dim3(grid_for(N)), dim3(kBlock), 0, s,
                     g->owner, g->pri, ds, dt, io_perm(g), io_rvpos(g), g->sp,
                     (int32_t)N, g->ctr);
  PG_TRY(sync_ctr(g, s));
  if (g->hctr[C_ERR] & ERR_INVAL)
    return pg_fail(PG_EINVAL,
                   "a strategy entry is out of range (Even: a vertex id or "
                   "PG_SINK, Odd: a vertex id)");
  return PG_OK;
}

pg_status export_strats(pg_game *g, int32_t *sigma, int32_t *tau, bool dev,
                        hipStream_t s, bool report) {
  const int64_t N = g->n_aug;
  if (!sigma && !tau) return PG_OK;
  int32_t *ds = dev ? sigma : (sigma ? g->wl0 : nullptr);
  int32_t *dt = dev ? tau : (tau ? g->wl1 : nullptr);
  hipLaunchKernelGGL(k_sp_export, dim3(grid_for(N)), dim3(kBlock), 0, s,
                     g->owner, g->sp, io_perm(g), io_rvpos(g), g->off, g->tgt,
                     g->n, (int)report, ds, dt, (int32_t)N);
  if (!dev) {
    if (sigma) PG_TRY(copy_out(sigma, g->wl0, sizeof(int32_t) * N, false, s));
    if (tau) PG_TRY(copy_out(tau, g->wl1, sizeof(int32_t) * N, false, s));
  }
  PG_HIP(hipStreamSynchronize(s));
  return PG_OK;
}

// Rank keys in the caller's ids.  Host output of a relabeled game is staged
// in g->elem, which every valuation rebuilds before reading it.
pg_status export_keys(pg_game *g, int32_t *key, bool dev, hipStream_t s) {
  const int64_t N = g->n_aug;
  if (!g->relabeled)
    return copy_out(key, g->key, sizeof(int32_t) * (N + 1), dev, s);
  int32_t *dk = dev ? key : (int32_t *)g->elem;
  hipLaunchKernelGGL(k_key_export, dim3(grid_for(N + 1)), dim3(kBlock), 0, s,
                     g->key, g->rvpos, dk, (int32_t)N);
  if (!dev) PG_TRY(copy_out(key, dk, sizeof(int32_t) * (N + 1), false, s));
  return PG_OK;
}

}  // namespace pgk

namespace {

// The per-valuation trace of pg_solve (pg_solve_opts.trace_*): counts and
// times go straight to the host arrays; key hashes are summed on the device
// into dhash and copied out once at the end.
struct Trace {
  const pg_solve_opts *o = nullptr;
  int64_t n = 0;
  unsigned long long *dhash = nullptr;
  void record(pg_game *g, hipStream_t s, int32_t switches, int64_t nf) {
    if (!o || n >= o->trace_cap) return;
    if (o->trace_finite) o->trace_finite[n] = nf;
    if (o->trace_switches) o->trace_switches[n] = switches;
    if (o->trace_ms) o->trace_ms[n] = g->last_ms;
    if (dhash && !g->dense) {
      // the next iteration overwrites the keys: it is ordered after this
      // kernel on the same stream
      const int32_t N = (int32_t)g->n_aug;
      hipLaunchKernelGGL(k_key_hash, dim3(grid_for(N + 1) < 2048u
                                              ? grid_for(N + 1) : 2048u),
                         dim3(kBlock), 0, s, g->key,
                         g->relabeled ? g->rvpos : nullptr, N, dhash + n);
    }
    ++n;
  }
};

// The inner loop of Algorithm 1 on the play graph in g->sp.
pg_status inner_loop(pg_game *g, int32_t max_inner, hipStream_t s,
                     int64_t *n_val, int64_t *n_sw, Trace *tr = nullptr,
                     double *iter_ms = nullptr) {
  int32_t inner = 0;
  for (;;) {
    if (max_inner > 0 && inner >= max_inner)
      return pg_fail(PG_EITERLIMIT, "best response: valuation cap reached");
    int32_t c = 0;
    int64_t nf = 0;
    PG_TRY(iteration_device(g, s, &c, &nf));
    if (iter_ms) *iter_ms += g->last_ms;
    if (tr) tr->record(g, s, c, nf);
    ++inner;
    ++*n_val;
    *n_sw += c;
    if (c == 0) return PG_OK;
  }
}

}  // namespace

// ===========================================================================
// the C ABI
// ===========================================================================
namespace {

pg_status check_load_args(int64_t n, int64_t m, const void *offsets,
                          const int32_t *targets, const uint8_t *owner,
                          const int32_t *priority, uint32_t flags) {
  if (n < 1 || m < n) return pg_fail(PG_EINVAL, "need n >= 1 and m >= n");
  if (n > kMaxVertices || m > 0x7fffffffLL * 4)
    return pg_fail(PG_EINVAL, "game too large");
  if (!offsets || !targets || !owner || !priority)
    return pg_fail(PG_EINVAL, "a game array is NULL");
  if ((flags & PG_OFFSETS_I32) && m > 0x7fffffffLL)
    return pg_fail(PG_EINVAL, "int32 offsets cannot address m edges");
  if ((flags & PG_SWITCH_ROWS) && (flags & PG_SWITCH_BUCKETS))
    return pg_fail(PG_EINVAL,
                   "PG_SWITCH_ROWS and PG_SWITCH_BUCKETS exclude each other");
  if ((flags & PG_ODD_REGION) && (flags & PG_NO_PREPROCESS))
    return pg_fail(PG_EINVAL,
                   "PG_ODD_REGION and PG_NO_PREPROCESS exclude each other");
  return PG_OK;
}

// pg_load_csr's work on g (g->device set), allocating from the current pool.
pg_status load_game(int64_t n, int64_t m, const void *offsets,
                    const int32_t *targets, const uint8_t *owner,
                    const int32_t *priority, uint32_t flags, hipStream_t s,
                    pg_game *g) {
  // count valuations when asked for or when the priorities repeat
  pg_status st =
      load_modified(n, m, offsets, targets, owner, priority, flags, s, g,
                    (flags & PG_COUNT_VALUATION) ? kLoadCount : kLoadAuto);
  // Odd's own region may be the whole game: nothing left to solve
  if (st == PG_OK && g->odd_region && g->n_aug == 0) return PG_OK;
  if (st == PG_OK) st = alloc_state(g, g->n_aug);
  if (st == PG_OK) st = finalize_state(g, s, true, !g->dense);
  if (st == PG_OK && g->dense) st = count_setup(g, s);
  // All_Odd over the bucketed layout: rank valuations, large Odd rows or
  // PG_SWITCH_BUCKETS, unless PG_SWITCH_ROWS
  if (st == PG_OK && !g->dense && !(flags & PG_SWITCH_ROWS) &&
      ((flags & PG_SWITCH_BUCKETS) || g->m_odd >= kTswMinEdges) &&
      tsw_fits(g->device, g->n_odd, g->m_odd)) {
    st = tsw_build(g, s);
    // without room for the layout the row form serves (same results)
    if (st == PG_ENOMEM && !(flags & PG_SWITCH_BUCKETS)) {
      (void)hipStreamSynchronize(s);
      tsw_release(g);
      g_last_error.clear();
      st = PG_OK;
    }
  }
  g->careful = flags & PG_CAREFUL_WALKS;
  g->use_graph = !(flags & PG_NO_GRAPH);
  g->host_rl = (flags & PG_HOST_REDUCED_LIST) && !g->dense;
  if (st == PG_OK && !g->dense) apply_tuning(g, tuning_for(g->n_aug));
  g->mark_top = true;
  return st;
}

pg_status solve_game(pg_game *g, const pg_solve_opts *opts, uint8_t *winner,
                     int32_t *sigma, int32_t *tau, pg_stats *stats,
                     hipStream_t s);

}  // namespace

namespace {

// pg_solve on a PG_ODD_REGION game that Odd's own region covers: Odd wins
// every vertex and no strategy is left (PG_SINK everywhere)
pg_status solve_all_removed(pg_game *g, uint8_t *winner, int32_t *sigma,
                            int32_t *tau, pg_stats *stats, bool dev,
                            hipStream_t s) {
  const int64_t n = g->n;
  if (dev) {
    fill_u8(winner, 1, n, s);
    if (sigma) fill_i32(sigma, PG_SINK, n, s);
    if (tau) fill_i32(tau, PG_SINK, n, s);
    PG_HIP(hipStreamSynchronize(s));
  } else {
    std::fill(winner, winner + n, uint8_t(1));
    if (sigma) std::fill(sigma, sigma + n, int32_t(PG_SINK));
    if (tau) std::fill(tau, tau + n, int32_t(PG_SINK));
  }
  if (stats) {
    *stats = pg_stats{};
    stats->n = g->n;
    stats->m = g->m;
  }
  return PG_OK;
}

// pg_solve's work on a loaded game, allocating from the current pool.
pg_status solve_game(pg_game *g, const pg_solve_opts *opts, uint8_t *winner,
                     int32_t *sigma, int32_t *tau, pg_stats *stats,
                     hipStream_t s) {
  pg_solve_opts o{};
  if (opts) o = *opts;
  const bool dev = o.flags & PG_PTR_DEVICE;
  if (o.best_response < PG_BR_SI || o.best_response > PG_BR_BELLMAN_FORD)
    return pg_fail(PG_EINVAL, "unknown best-response selector");
  if (o.best_response == PG_BR_BELLMAN_FORD && !g->dense)
    return pg_fail(PG_EINVAL, "Bellman-Ford best responses need a game with "
                              "count valuations");
  if (o.trace_cap < 0) return pg_fail(PG_EINVAL, "trace_cap < 0");
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t N = g->n_aug;
  if (g->odd_region && N == 0) return solve_all_removed(g, winner, sigma, tau,
                                                        stats, dev, s);
  // the reduced game's strategies and winners (PG_ODD_REGION): its own ids
  struct OrBuf {
    int32_t *s2 = nullptr, *t2 = nullptr;
    uint8_t *w2 = nullptr;
    ~OrBuf() {
      dev_free(s2);
      dev_free(t2);
      dev_free(w2);
    }
  } ob;
  if (g->odd_region) {
    PG_TRY(dev_alloc(&ob.s2, N));
    PG_TRY(dev_alloc(&ob.t2, N));
    PG_TRY(dev_alloc(&ob.w2, N));
  }
  // sigma and tau out: directly, or through the reduced game's ids
  auto strats_out = [&](bool report) -> pg_status {
    if (!g->odd_region) return export_strats(g, sigma, tau, dev, s, report);
    if (!sigma && !tau) return PG_OK;
    PG_TRY(export_strats(g, sigma ? ob.s2 : nullptr, tau ? ob.t2 : nullptr,
                         true, s, false));
    return odd_region_strats_out(g, ob.s2, ob.t2, sigma, tau, dev, s);
  };
  hipLaunchKernelGGL(k_sp_init, dim3(grid_for(N)), dim3(kBlock), 0, s, g->off,
                     g->tgt, g->owner, g->pri, g->sp, (int32_t)N);
  // warm start: the given strategies replace the initial ones
  if ((o.init_sigma || o.init_tau) && g->odd_region) {
    PG_TRY(odd_region_strats_in(g, o.init_sigma, o.init_tau, dev, s, ob.s2,
                                ob.t2));
    PG_TRY(import_strats(g, o.init_sigma ? ob.s2 : nullptr,
                         o.init_tau ? ob.t2 : nullptr, true, s));
  } else if (o.init_sigma || o.init_tau) {
    PG_TRY(import_strats(g, o.init_sigma, o.init_tau, dev, s));
  }
  valuation_reset(g, s);
  Trace tr;
  tr.o = &o;
  struct HashBuf {
    unsigned long long *p = nullptr;
    ~HashBuf() { dev_free(p); }
  } hb;
  if (o.trace_key_hash && o.trace_cap > 0) {
    PG_TRY(dev_alloc(&hb.p, o.trace_cap));
    fill_i32((int32_t *)hb.p, 0, 2 * (int64_t)o.trace_cap, s);
    tr.dhash = hb.p;
  }
  int64_t n_major = 0, n_val = 0, n_odd = 0, n_even = 0;
  double iter_ms = 0.0;
  pg_status st = PG_OK;
  for (;;) {
    if (o.max_major > 0 && n_major >= o.max_major) {
      st = pg_fail(PG_EITERLIMIT, "solve: outer iteration cap reached");
      break;
    }
    ++n_major;
    if (o.best_response == PG_BR_SI_RESET)
      hipLaunchKernelGGL(k_sp_reset_odd, dim3(grid_for(N)), dim3(kBlock), 0, s,
                         g->off, g->tgt, g->owner, g->pri, g->sp, (int32_t)N);
    if (o.best_response == PG_BR_BELLMAN_FORD) {
      int64_t rounds = 0;
      st = bf_best_response(g, s, &rounds);
      n_val += rounds;
    } else {
      st = inner_loop(g, o.max_inner, s, &n_val, &n_odd, &tr, &iter_ms);
      // a best response: its top vertices stay top from here on
      if (st == PG_OK) mark_top(g, s);
    }
    if (st != PG_OK) break;
    int32_t c = 0;
    st = switch_device(g, false, s, &c);
    if (st != PG_OK) break;
    n_even += c;
    if (c == 0) break;
    // a new inner loop: Even's switches may make finite vertices top
    fates_reset(g, s);
  }
  if (tr.dhash && tr.n > 0) {
    // the trace is the caller's even when the run stopped early
    const std::string err = pg_last_error();
    PG_HIP(hipMemcpyAsync(o.trace_key_hash, tr.dhash,
                          sizeof(uint64_t) * (size_t)tr.n,
                          hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    if (st != PG_OK) pg_fail(st, err);
  }
  if (o.trace_key_hash && g->dense)
    for (int64_t i = 0; i < tr.n; ++i) o.trace_key_hash[i] = 0;
  if (stats) {
    stats->n = g->n;
    stats->m = g->m;
    stats->n_aug = g->n_aug;
    stats->m_aug = g->m_aug;
    stats->n_major = n_major;
    stats->n_valuations = n_val;
    stats->n_odd_switches = n_odd;
    stats->n_even_switches = n_even;
    stats->iteration_ms = iter_ms;
    stats->n_traced = tr.n;
  }
  const bool report = !(o.flags & PG_KEEP_DUMMIES);
  if (st == PG_EITERLIMIT) {
    // a checkpoint: the strategies reached, from which a warm start resumes
    const std::string err = pg_last_error();
    PG_TRY(strats_out(report));
    return pg_fail(st, err);
  }
  if (st != PG_OK) return st;
  if (g->odd_region) {
    hipLaunchKernelGGL(k_winner, dim3(grid_for(N)), dim3(kBlock), 0, s, g->rs,
                       io_rvpos(g), ob.w2, N);
    PG_TRY(odd_region_winner_out(g, ob.w2, winner, dev, s));
  } else {
    uint8_t *dw = winner;
    if (!dev) dw = (uint8_t *)g->wl0;
    hipLaunchKernelGGL(k_winner, dim3(grid_for(g->n)), dim3(kBlock), 0, s,
                       g->rs, io_rvpos(g), dw, g->n);
    if (!dev) PG_TRY(copy_out(winner, dw, g->n, false, s));
    PG_HIP(hipStreamSynchronize(s));
  }
  PG_TRY(strats_out(report));
  const auto t1 = std::chrono::steady_clock::now();
  if (stats) stats->seconds = std::chrono::duration<double>(t1 - t0).count();
  return PG_OK;
}

}  // namespace

// ---- the allocation-free entry point ---------------------------------------
// pg_solve_noalloc carves every device buffer of a load and a solve from this
// array (bump allocation, nothing handed back until the call ends) and the
// counter mirror from a small static host buffer.  In host code the array's
// name is not its device address: hipGetSymbolAddress gives that, once per
// device (each device holds its own copy), and only that address is used.
constexpr size_t kScratchBytes = size_t(PG_NOALLOC_SCRATCH_MIB) << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];
constexpr int kScratchDevices = 64;
constexpr size_t kScratchHostBytes = 16384;   // the counter mirror
static std::mutex g_scratch_mu;
static uint8_t *g_scratch_dev[kScratchDevices];
alignas(256) static uint8_t g_scratch_host[kScratchDevices][kScratchHostBytes];

namespace {
pg_status scratch_address(int device, uint8_t **out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return pg_fail(PG_EDEVICE, std::string("scratch address: ") +
                                     hipGetErrorString(e));
    g_scratch_dev[device] = (uint8_t *)ptr;
  }
  *out = g_scratch_dev[device];
  return PG_OK;
}
}  // namespace

namespace {
// per-vertex arrays of the calls below are in the stored game's ids, which
// for PG_ODD_REGION are not the caller's
pg_status solve_only(const pg_game *g) {
  if (g->odd_region)
    return pg_fail(PG_EINVAL, "a game loaded with PG_ODD_REGION supports "
                              "pg_solve (not the per-vertex calls)");
  return PG_OK;
}
}  // namespace

extern "C" {

const char *pg_last_error(void) { return g_last_error.c_str(); }

pg_status pg_load_csr(int64_t n, int64_t m, const void *offsets,
                      const int32_t *targets, const uint8_t *owner,
                      const int32_t *priority, uint32_t flags,
                      void *hip_stream, pg_game **out_game) {
  g_last_error.clear();
  if (!out_game) return pg_fail(PG_EINVAL, "out_game is NULL");
  *out_game = nullptr;
  PG_TRY(check_load_args(n, m, offsets, targets, owner, priority, flags));
  pg_game *g = new (std::nothrow) pg_game();
  if (!g) return pg_fail(PG_ENOMEM, "host allocation failed");
  if (hipGetDevice(&g->device) != hipSuccess) {
    delete g;
    return pg_fail(PG_EDEVICE, "no HIP device");
  }
  hipStream_t s = (hipStream_t)hip_stream;
  PoolScope cache(game_cache(g->device));
  const pg_status st = load_game(n, m, offsets, targets, owner, priority,
                                 flags, s, g);
  if (st != PG_OK) {
    (void)hipStreamSynchronize(s);
    free_game(g);
    return st;
  }
  *out_game = g;
  return PG_OK;
}

pg_status pg_count_info(const pg_game *g, int32_t *d, int32_t *values) {
  if (!g || !d) return pg_fail(PG_EINVAL, "NULL argument");
  *d = g->dense ? g->d : 0;
  if (values && g->dense)
    for (int j = 0; j < g->d; ++j) values[j] = g->values[j];
  return PG_OK;
}

pg_status pg_game_info(const pg_game *g, int64_t *n, int64_t *m,
                       int64_t *n_aug, int64_t *m_aug) {
  if (!g) return pg_fail(PG_EINVAL, "game is NULL");
  if (n) *n = g->n;
  if (m) *m = g->m;
  if (n_aug) *n_aug = g->n_aug;
  if (m_aug) *m_aug = g->m_aug;
  return PG_OK;
}

pg_status pg_export_game(const pg_game *gc, int64_t *offsets, int32_t *targets,
                         uint8_t *owner, int32_t *priority, uint32_t flags,
                         void *hip_stream) {
  if (!gc) return pg_fail(PG_EINVAL, "game is NULL");
  pg_game *g = const_cast<pg_game *>(gc);
  DevGuard guard(g->device);
  PoolScope cache(game_cache(g->device));
  hipStream_t s = (hipStream_t)hip_stream;
  const bool dev = flags & PG_PTR_DEVICE;
  // a relabeled game goes back to the caller's vertex ids first
  struct Tmp {
    int64_t *off = nullptr;
    int32_t *tgt = nullptr, *pri = nullptr;
    uint8_t *owner = nullptr;
    ~Tmp() {
      dev_free(off);
      dev_free(tgt);
      dev_free(owner);
      dev_free(pri);
    }
  } ext;
  const int64_t *off = g->off;
  const int32_t *tgt = g->tgt, *pri = g->pri;
  const uint8_t *own = g->owner;
  if (g->relabeled) {
    pg_status st = relabel_game(g->off, g->tgt, g->owner, g->pri, g->rvpos,
                                g->perm, g->n_aug, g->m_aug, &ext.off,
                                &ext.tgt, &ext.owner, &ext.pri, s);
    if (st != PG_OK) {
      (void)hipStreamSynchronize(s);
      return st;
    }
    off = ext.off;
    tgt = ext.tgt;
    own = ext.owner;
    pri = ext.pri;
  }
  pg_status st = PG_OK;
  if (st == PG_OK && offsets)
    st = copy_out(offsets, off, sizeof(int64_t) * (g->n_aug + 1), dev, s);
  if (st == PG_OK && targets)
    st = copy_out(targets, tgt, sizeof(int32_t) * g->m_aug, dev, s);
  if (st == PG_OK && owner) st = copy_out(owner, own, g->n_aug, dev, s);
  if (st == PG_OK && priority)
    st = copy_out(priority, pri, sizeof(int32_t) * g->n_aug, dev, s);
  // the temporaries are freed only after the copies ran
  PG_HIP(hipStreamSynchronize(s));
  return st;
}

pg_status pg_initial_strategies(pg_game *g, int32_t *sigma, int32_t *tau,
                                uint32_t flags, void *hip_stream) {
  if (!g) return pg_fail(PG_EINVAL, "game is NULL");
  PG_TRY(solve_only(g));
  DevGuard guard(g->device);
  hipStream_t s = (hipStream_t)hip_stream;
  const bool dev = flags & PG_PTR_DEVICE;
  const int64_t N = g->n_aug;
  int32_t *ds = dev ? sigma : (sigma ? g->wl0 : nullptr);
  int32_t *dt = dev ? tau : (tau ? g->wl1 : nullptr);
  hipLaunchKernelGGL(k_initial, dim3(grid_for(N)), dim3(kBlock), 0, s, g->off,
                     g->tgt, g->owner, io_perm(g), io_rvpos(g), ds, dt,
                     (int32_t)N);
  if (!dev) {
    if (sigma) PG_TRY(copy_out(sigma, g->wl0, sizeof(int32_t) * N, false, s));
    if (tau) PG_TRY(copy_out(tau, g->wl1, sizeof(int32_t) * N, false, s));
  }
  PG_HIP(hipStreamSynchronize(s));
  return PG_OK;
}

pg_status pg_valuation(pg_game *g, const int32_t *sigma, const int32_t *tau,
                       int32_t *key, int64_t *n_finite, uint32_t flags,
                       void *hip_stream) {
  if (!g) return pg_fail(PG_EINVAL, "game is NULL");
  PG_TRY(solve_only(g));
  if (!sigma || !tau || !key) return pg_fail(PG_EINVAL, "NULL argument");
  if (g->dense)
    return pg_fail(PG_EINVAL, "a count-valuation game has no rank keys: use "
                              "pg_valuation_counts");
  DevGuard guard(g->device);
  PoolScope cache(game_cache(g->device));
  hipStream_t s = (hipStream_t)hip_stream;
  const bool dev = flags & PG_PTR_DEVICE;
  PG_TRY(import_strats(g, sigma, tau, dev, s));
  valuation_reset(g, s);
  PG_TRY(valuation_device(g, s, n_finite));
  PG_TRY(export_keys(g, key, dev, s));
  PG_TRY(sync_ctr(g, s));
  PG_TRY(check_err(g, "invalid strategy"));
  return PG_OK;
}

pg_status pg_valuation_counts(pg_game *g, const int32_t *sigma,
                              const int32_t *tau, int32_t *counts,
                              uint8_t *top, int64_t *n_finite, uint32_t flags,
                              void *hip_stream) {
  if (!g) return pg_fail(PG_EINVAL, "game is NULL");
  PG_TRY(solve_only(g));
  if (!sigma || !tau || !counts) return pg_fail(PG_EINVAL, "NULL argument");
  if (!g->dense)
    return pg_fail(PG_EINVAL, "not a count-valuation game: use pg_valuation");
  DevGuard guard(g->device);
  PoolScope cache(game_cache(g->device));
  hipStream_t s = (hipStream_t)hip_stream;
  const bool dev = flags & PG_PTR_DEVICE;
  PG_TRY(import_strats(g, sigma, tau, dev, s));
  valuation_reset(g, s);
  PG_TRY(valuation_device(g, s, n_finite));
  PG_TRY(export_counts(g, counts, top, dev, s));
  return PG_OK;
}

pg_status pg_best_response(pg_game *g, const int32_t *sigma, int32_t *tau,
                           int32_t *key, int32_t *n_valuations,
                           int32_t max_inner, uint32_t flags,
                           void *hip_stream) {
  if (!g) return pg_fail(PG_EINVAL, "game is NULL");
  PG_TRY(solve_only(g));
  if (!sigma || !tau) return pg_fail(PG_EINVAL, "NULL argument");
  if (key && g->dense)
    return pg_fail(PG_EINVAL, "a count-valuation game has no rank keys: "
                              "pass key = NULL");
  DevGuard guard(g->device);
  PoolScope cache(game_cache(g->device));
  hipStream_t s = (hipStream_t)hip_stream;
  const bool dev = flags & PG_PTR_DEVICE;
  PG_TRY(import_strats(g, sigma, tau, dev, s));
  valuation_reset(g, s);
  int64_t nv = 0, nsw = 0;
  pg_status st = inner_loop(g, max_inner, s, &nv, &nsw);
  if (n_valuations) *n_valuations = (int32_t)nv;
  if (st != PG_OK) return st;
  PG_TRY(export_strats(g, nullptr, tau, dev, s, false));
  if (key) PG_TRY(export_keys(g, key, dev, s));
  PG_HIP(hipStreamSynchronize(s));
  return PG_OK;
}

pg_status pg_solve(pg_game *g, const pg_solve_opts *opts, uint8_t *winner,
                   int32_t *sigma, int32_t *tau, pg_stats *stats,
                   void *hip_stream) {
  if (!g) return pg_fail(PG_EINVAL, "game is NULL");
  if (!winner) return pg_fail(PG_EINVAL, "winner is NULL");
  DevGuard guard(g->device);
  PoolScope cache(game_cache(g->device));
  return solve_game(g, opts, winner, sigma, tau, stats,
                    (hipStream_t)hip_stream);
}

pg_status pg_solve_noalloc(int64_t n, int64_t m, const void *offsets,
                           const int32_t *targets, const uint8_t *owner,
                           const int32_t *priority, uint32_t flags,
                           const pg_solve_opts *opts, uint8_t *winner,
                           int32_t *sigma, int32_t *tau, pg_stats *stats,
                           void *hip_stream) {
  g_last_error.clear();
  PG_TRY(check_load_args(n, m, offsets, targets, owner, priority, flags));
  if (!winner) return pg_fail(PG_EINVAL, "winner is NULL");
  if (n > PG_NOALLOC_MAX_VERTICES || m > PG_NOALLOC_MAX_EDGES)
    return pg_fail(PG_EINVAL,
                   "pg_solve_noalloc takes at most " +
                       std::to_string(PG_NOALLOC_MAX_VERTICES) +
                       " vertices and " + std::to_string(PG_NOALLOC_MAX_EDGES) +
                       " edges; load larger games with pg_load_csr");
  if (flags & (PG_SWITCH_BUCKETS | PG_HOST_REDUCED_LIST))
    return pg_fail(PG_EINVAL, "pg_solve_noalloc takes neither "
                              "PG_SWITCH_BUCKETS nor PG_HOST_REDUCED_LIST");
  if (opts && (opts->trace_key_hash || opts->trace_finite ||
               opts->trace_switches || opts->trace_ms))
    return pg_fail(PG_EINVAL, "pg_solve_noalloc keeps no trace");
  int device = -1;
  if (hipGetDevice(&device) != hipSuccess || device < 0)
    return pg_fail(PG_EDEVICE, "no HIP device");
  if (device >= kScratchDevices)
    return pg_fail(PG_EDEVICE, "device index beyond the scratch table");
  uint8_t *dev_scratch = nullptr;
  PG_TRY(scratch_address(device, &dev_scratch));
  hipStream_t s = (hipStream_t)hip_stream;
  DevPool bump;
  bump.bump_dev = dev_scratch;
  bump.bump_cap = kScratchBytes;
  bump.bump_host = g_scratch_host[device];
  bump.bump_hcap = kScratchHostBytes;
  PoolScope scope(&bump);
  // the game lives on this call's stack; every buffer it points to is in
  // the scratch; no events, no graphs, rows for All_Odd
  pg_game g;
  g.device = device;
  g.timed = false;
  pg_status st = load_game(n, m, offsets, targets, owner, priority,
                           flags | PG_NO_GRAPH | PG_SWITCH_ROWS, s, &g);
  if (st == PG_OK) st = solve_game(&g, opts, winner, sigma, tau, stats, s);
  // the scratch is free again once the stream has drained
  (void)hipStreamSynchronize(s);
  return st;
}

pg_status pg_profile_enable(pg_game *g, int32_t on) {
  if (!g) return pg_fail(PG_EINVAL, "game is NULL");
  g->prof.on = on != 0;
  g->prof.reset();
  return PG_OK;
}

int32_t pg_profile_kinds(void) { return (int32_t)K_COUNT; }

pg_status pg_profile_read(const pg_game *g, int32_t kind, const char **name,
                          double *ms, int64_t *calls, double *bytes) {
  if (!g) return pg_fail(PG_EINVAL, "game is NULL");
  if (kind < 0 || kind >= K_COUNT) return pg_fail(PG_EINVAL, "bad kind");
  if (name) *name = kKernelNames[kind];
  if (ms) *ms = g->prof.ms[kind];
  if (calls) *calls = g->prof.calls[kind];
  if (bytes) *bytes = g->prof.bytes[kind];
  return PG_OK;
}

pg_status pg_free(pg_game *g) {
  if (!g) return PG_OK;
  DevGuard guard(g->device);
  PoolScope cache(game_cache(g->device));
  (void)hipDeviceSynchronize();
  free_game(g);
  return PG_OK;
}

pg_status pg_release_cache(void) {
  trim_caches();
  return PG_OK;
}

}  // extern "C"
