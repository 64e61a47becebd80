// All_Odd over a bucketed edge layout (rank valuations, single games).
//
// All_Odd (section 4) gives every Odd vertex the first successor of least
// key when that key is strictly below the current choice's.  Read row by
// row, every edge costs one random key gather: a whole memory line for four
// bytes, and the step runs at the chip's rate of random line transactions.
// The game's edges never change during a solve, so the load lays the Odd
// rows' edges out once for a two-kernel step whose memory traffic is
// coalesced:
//
//   stage   the edges in increasing target order, cut into chunks of
//           kTswChunk: a block gathers its chunk's keys (nearly sequential
//           reads, since the targets increase), drops each into the edge's
//           slot in LDS, and writes the slots out in order.  Slots are
//           grouped by bucket (kTswBucket consecutive Odd vertices), so each
//           bucket receives one contiguous run per chunk;
//   min     one block per bucket takes the least (key, target) pair of each
//           of its vertices with LDS atomics, finds the current choice's
//           key among the same entries, and applies the rule.
//
// Finite keys are pairwise distinct, so the least (key, target) pair names
// the row's first entry of least key; when the least key is top no switch
// happens, whichever top entry it names.  The layout is three stable radix
// sorts at load: the edges by target; those by bucket, which gives each
// edge's place in bucket order; the places by chunk, which gives each edge's
// slot in its chunk.
#include "pg_common.h"

namespace pgk {

// Sizes: a 16384-edge chunk (64 KiB of LDS, two stage blocks per CU) and
// 4096-vertex buckets, each taken by a 1024-thread min block.  Larger
// buckets give longer runs per chunk in the stage's writes; on the
// 10M-vertex random game stage + min went 91 + 72 -> 82 + 63 us per step
// against 32768-edge chunks and 2048-vertex buckets of 256 threads (1M
// vertices: 16 + 21 -> 12 + 15 us).  8192- and 6144-vertex buckets, or 512
// threads per min block, were slower.
constexpr int kTswChunk = 16384;   // edges per stage block
constexpr int kTswBucket = 4096;   // Odd vertices per min block

// ---- layout (load time) ----------------------------------------------------

// row lengths of the Odd vertices, in list order
__global__ void k_tsw_len(const int32_t *ids, const int64_t *off,
                          uint32_t *len, int64_t no) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o < no) {
    const int32_t v = ids[o];
    len[o] = (uint32_t)(off[v + 1] - off[v]);
  }
}

// one (target, list position) pair per edge of an Odd row
__global__ void k_tsw_expand(const int32_t *ids, const int64_t *off,
                             const int32_t *tgt, const uint32_t *start,
                             uint32_t *kt, uint32_t *vo, int64_t no) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= no) return;
  const int32_t v = ids[o];
  uint32_t p = start[o];
  for (int64_t e = off[v]; e < off[v + 1]; ++e, ++p) {
    kt[p] = (uint32_t)tgt[e];
    vo[p] = (uint32_t)o;
  }
}

// in target order: keep the targets and list positions; sort key the bucket
__global__ void k_tsw_keep(uint32_t *kt, const uint32_t *vo, int32_t *tx,
                           int32_t *ox, int64_t m) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const uint32_t o = vo[j];
  tx[j] = (int32_t)kt[j];
  ox[j] = (int32_t)o;
  kt[j] = o / kTswBucket;
}

// z[p] = the edge (target-order index) at bucket-order place p, zb[p] its
// bucket: each place's target, vertex within the bucket and the bucket
// starts; sort key the edge's chunk (the places stay in bucket order within
// a chunk)
__global__ void k_tsw_places(const uint32_t *z, const uint32_t *zb,
                             const int32_t *tx, const int32_t *ox,
                             int32_t *tz, uint16_t *sz, int32_t *bs,
                             uint32_t *kc, int64_t m, int64_t nb) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m) return;
  const uint32_t j = z[p];
  tz[p] = tx[j];
  sz[p] = (uint16_t)((uint32_t)ox[j] % kTswBucket);
  kc[p] = j / kTswChunk;
  const uint32_t b = zb[p];
  if (p == 0 || zb[p - 1] != b) bs[b] = (int32_t)p;
  if (p == m - 1) bs[nb] = (int32_t)m;
}

// w[q] = the place of the edge in chunk-sorted position q: slot q % chunk
// of its chunk
__global__ void k_tsw_slots(const uint32_t *w, const uint32_t *z,
                            uint16_t *slot, int32_t *gpos, int64_t m) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const uint32_t p = w[q];
  gpos[q] = (int32_t)p;
  slot[z[p]] = (uint16_t)(q % kTswChunk);
}

// ---- the step (every valuation) --------------------------------------------

constexpr int kTswStageBlock = 1024;
constexpr int kTswMinBlock = 1024;
constexpr int kTswUnroll = 8;

__global__ __launch_bounds__(kTswStageBlock) void k_tsw_stage(
    int64_t m, const int32_t *__restrict__ tx, const uint16_t *__restrict__ slot,
    const int32_t *__restrict__ gpos, const int32_t *__restrict__ key,
    int32_t *__restrict__ r, const int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  __shared__ int32_t st[kTswChunk];
  const int64_t c0 = (int64_t)blockIdx.x * kTswChunk;
  const int len = (int)min((int64_t)kTswChunk, m - c0);
  constexpr int kIt = kTswChunk / kTswStageBlock;
  for (int k = 0; k < kIt; k += kTswUnroll) {
    int32_t t[kTswUnroll], kv[kTswUnroll];
    int sl[kTswUnroll];
#pragma unroll
    for (int u = 0; u < kTswUnroll; ++u) {
      const int i = (k + u) * kTswStageBlock + threadIdx.x;
      t[u] = i < len ? tx[c0 + i] : -1;
      sl[u] = i < len ? slot[c0 + i] : 0;
    }
#pragma unroll
    for (int u = 0; u < kTswUnroll; ++u) kv[u] = t[u] >= 0 ? key[t[u]] : 0;
#pragma unroll
    for (int u = 0; u < kTswUnroll; ++u)
      if (t[u] >= 0) st[sl[u]] = kv[u];
  }
  __syncthreads();
  for (int k = 0; k < kIt; k += kTswUnroll) {
    int32_t g[kTswUnroll];
#pragma unroll
    for (int u = 0; u < kTswUnroll; ++u) {
      const int i = (k + u) * kTswStageBlock + threadIdx.x;
      g[u] = i < len ? gpos[c0 + i] : -1;
    }
#pragma unroll
    for (int u = 0; u < kTswUnroll; ++u) {
      const int i = (k + u) * kTswStageBlock + threadIdx.x;
      if (g[u] >= 0) r[g[u]] = st[i];
    }
  }
}

__global__ __launch_bounds__(kTswMinBlock) void k_tsw_min(
    int64_t no, const int32_t *__restrict__ ids, const int32_t *__restrict__ bs,
    const int32_t *__restrict__ r, const int32_t *__restrict__ tz,
    const uint16_t *__restrict__ sz, const int32_t *__restrict__ key,
    const int32_t *__restrict__ pri, int2 *sp, int32_t *ctr) {
  if (ctr[C_ABORT]) return;
  __shared__ unsigned long long best[kTswBucket];
  __shared__ int32_t curt[kTswBucket], curk[kTswBucket];
  const int64_t o0 = (int64_t)blockIdx.x * kTswBucket;
  const int ns = (int)min((int64_t)kTswBucket, no - o0);
  for (int i = threadIdx.x; i < ns; i += kTswMinBlock) {
    best[i] = ~0ull;
    curt[i] = sp[ids[o0 + i]].x;
    curk[i] = -1;   // keys are >= 0: not met yet
  }
  __syncthreads();
  const int32_t p0 = bs[blockIdx.x], p1 = bs[blockIdx.x + 1];
  for (int32_t p = p0 + threadIdx.x; p < p1; p += kTswMinBlock * 4) {
    int32_t k[4], t[4];
    int s[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t q = p + u * kTswMinBlock;
      t[u] = q < p1 ? tz[q] : -1;
      k[u] = q < p1 ? r[q] : 0;
      s[u] = q < p1 ? sz[q] : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (t[u] < 0) continue;
      atomicMin(&best[s[u]], ((unsigned long long)(uint32_t)k[u] << 32) |
                                 (uint32_t)t[u]);
      // every entry naming the current choice carries the same key
      if (t[u] == curt[s[u]]) curk[s[u]] = k[u];
    }
  }
  __syncthreads();
  int sw = 0;
  for (int i = threadIdx.x; i < ns; i += kTswMinBlock) {
    const unsigned long long x = best[i];
    const int32_t kb = (int32_t)(x >> 32), bt = (int32_t)(uint32_t)x;
    int32_t kc = curk[i];
    if (kc < 0) kc = key[curt[i]];   // a current choice outside the row
    if (kb < kc) {
      sp[ids[o0 + i]] = make_int2(bt, pri[bt]);
      ++sw;
    }
  }
  add_block(&ctr[C_DIST_SW], sw);
}

// ---- host side -------------------------------------------------------------

static int bits_for(int64_t max_value) {
  int b = 1;
  while (b < 32 && (int64_t(1) << b) <= max_value) ++b;
  return b;
}

// places, slots and bucket starts are int32; the stage kernel's chunk
// needs its LDS in one block
bool tsw_fits(int device, int64_t n_odd, int64_t m_odd) {
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                            device) != hipSuccess ||
      lds < (int)sizeof(int32_t) * kTswChunk)
    return false;
  return n_odd > 0 && m_odd > 0 && m_odd < (int64_t(1) << 31) - kTswChunk;
}

pg_status tsw_build(pg_game *g, hipStream_t s) {
  const int64_t no = g->n_odd, m = g->m_odd;
  if (!tsw_fits(g->device, no, m))
    return pg_fail(PG_EINVAL, "no bucketed layout");
  const int64_t nb = (no + kTswBucket - 1) / kTswBucket;
  const int64_t nc = (m + kTswChunk - 1) / kTswChunk;
  PG_TRY(dev_alloc(&g->tsw_t, m));
  PG_TRY(dev_alloc(&g->tsw_slot, m));
  PG_TRY(dev_alloc(&g->tsw_g, m));
  PG_TRY(dev_alloc(&g->tsw_tz, m));
  PG_TRY(dev_alloc(&g->tsw_sz, m));
  PG_TRY(dev_alloc(&g->tsw_r, m));
  PG_TRY(dev_alloc(&g->tsw_bs, nb + 1));
  g->tsw_nb = nb;
  g->tsw_nc = nc;
  // temporaries: four sort buffers, a fifth key buffer, the scans' and
  // sorts' scratch
  uint32_t *a[5] = {};
  uint32_t *tiles = nullptr;
  void *tmp = nullptr;
  struct Free {
    uint32_t **a;
    uint32_t **tiles;
    void **tmp;
    hipStream_t s;
    ~Free() {
      (void)hipStreamSynchronize(s);
      for (int i = 0; i < 5; ++i) dev_free(a[i]);
      dev_free(*tiles);
      dev_free(*tmp);
    }
  } release{a, &tiles, &tmp, s};
  for (int i = 0; i < 5; ++i) PG_TRY(dev_alloc(&a[i], m < no + 1 ? no + 1 : m));
  PG_TRY(dev_alloc(&tiles, 256 * radix_tiles(m)));
  size_t tb = radix_scan_tmp_bytes(m);
  const size_t tb2 = scan_excl_u32(nullptr, nullptr, no + 1, nullptr, s);
  if (tb2 > tb) tb = tb2;
  PG_TRY(dev_alloc((uint8_t **)&tmp, (int64_t)tb));
  // the Odd rows' edges as (target, list position)
  hipLaunchKernelGGL(k_tsw_len, dim3(grid_for(no)), dim3(kBlock), 0, s,
                     g->odd_ids, g->off, a[4], no);
  fill_i32((int32_t *)a[4] + no, 0, 1, s);
  scan_excl_u32(a[4], a[4], no + 1, tmp, s);
  hipLaunchKernelGGL(k_tsw_expand, dim3(grid_for(no)), dim3(kBlock), 0, s,
                     g->odd_ids, g->off, g->tgt, a[4], a[0], a[1], no);
  // by target; targets and list positions in that order go to tsw_t and
  // tsw_r (free until the first step)
  int w = radix_sort(a[0], a[1], a[2], a[3], m, bits_for(g->n_aug), tiles,
                     tmp, s);
  uint32_t *k0 = a[2 * w], *v0 = a[2 * w + 1];
  uint32_t *k1 = a[2 - 2 * w], *v1 = a[3 - 2 * w];
  hipLaunchKernelGGL(k_tsw_keep, dim3(grid_for(m)), dim3(kBlock), 0, s, k0,
                     v0, g->tsw_t, g->tsw_r, m);
  // by bucket (stable: target order within a bucket) -> places
  w = radix_sort(k0, v0, k1, v1, m, bits_for(nb - 1), tiles, tmp, s, nullptr,
                 nullptr, true);
  uint32_t *zk = w ? k1 : k0, *zv = w ? v1 : v0;
  uint32_t *fk = w ? k0 : k1, *fv = w ? v0 : v1;   // the free pair
  hipLaunchKernelGGL(k_tsw_places, dim3(grid_for(m)), dim3(kBlock), 0, s, zv,
                     zk, g->tsw_t, g->tsw_r, g->tsw_tz, g->tsw_sz, g->tsw_bs,
                     a[4], m, nb);
  // places by chunk (stable: bucket order within a chunk) -> slots
  w = radix_sort(a[4], zk, fk, fv, m, bits_for(nc - 1), tiles, tmp, s,
                 nullptr, nullptr, true);
  hipLaunchKernelGGL(k_tsw_slots, dim3(grid_for(m)), dim3(kBlock), 0, s,
                     w ? fv : zk, zv, g->tsw_slot, g->tsw_g, m);
  PG_HIP(hipGetLastError());
  g->tsw = true;
  return PG_OK;
}

void tsw_release(pg_game *g) {
  void *ptrs[] = {g->tsw_t, g->tsw_slot, g->tsw_g, g->tsw_tz,
                  g->tsw_sz, g->tsw_bs,   g->tsw_r};
  for (void *p : ptrs) dev_free(p);
  g->tsw_t = g->tsw_g = g->tsw_tz = g->tsw_bs = g->tsw_r = nullptr;
  g->tsw_slot = g->tsw_sz = nullptr;
  g->tsw = false;
  g->tsw_nb = g->tsw_nc = 0;
}

void enqueue_tsw_odd(pg_game *g, hipStream_t s) {
  Prof *pf = &g->prof;
  const int64_t m = g->m_odd, no = g->n_odd;
  // a target and its key per edge
  PG_LAUNCH(pf, K_ODD_STAGE, 8.0 * m, k_tsw_stage, dim3((unsigned)g->tsw_nc),
            dim3(kTswStageBlock), 0, s, m, g->tsw_t, g->tsw_slot, g->tsw_g,
            g->key, g->tsw_r, g->ctr);
  // per vertex: id 4, two row offsets 16, current choice 8 (the row form's
  // figure: the step's algorithmic bytes do not depend on the layout)
  PG_LAUNCH(pf, K_ODD_SWITCH, 28.0 * no, k_tsw_min, dim3((unsigned)g->tsw_nb),
            dim3(kTswMinBlock), 0, s, no, g->odd_ids, g->tsw_bs, g->tsw_r,
            g->tsw_tz, g->tsw_sz, g->key, g->pri, g->sp, g->ctr);
}

}  // namespace pgk
