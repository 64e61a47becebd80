// Data-parallel primitives: fills, device-wide exclusive scans and a stable
// LSD radix sort.  Written for wave64: wave-level scans use lane shuffles and
// the radix sort ranks digits inside a wave with ballots (a match of the
// eight digit bits), so no LDS atomics decide an order.
#include "pg_common.h"

namespace pgk {

const char *const kKernelNames[K_COUNT] = {
    "fill",       "ng_walk",   "ng_round",   "root_walk",  "root_round",
    "sort_split", "sort_hist", "scan",       "sort_pass",  "link_info",
    "link_build", "lr_sum1",   "lr_sumk",    "lr_top",     "lr_distk",
    "lr_emit1",   "odd_switch", "even_switch", "odd_stage", "other"};

hipEvent_t Prof::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

void Prof::flush() {
  for (Pend &p : pend) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
      ms[p.kid] += t;
      calls[p.kid] += 1;
      bytes[p.kid] += p.bytes + p.per_nf * nf + p.per_ni * ni;
    }
    pool.push_back(p.a);
    pool.push_back(p.b);
  }
  pend.clear();
}

void Prof::reset() {
  for (int k = 0; k < K_COUNT; ++k) {
    ms[k] = 0.0;
    calls[k] = 0;
    bytes[k] = 0.0;
  }
}

void Prof::release() {
  for (Pend &p : pend) {
    pool.push_back(p.a);
    pool.push_back(p.b);
  }
  pend.clear();
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  pool.clear();
}

// ---------------------------------------------------------------------------
// fills (kernels rather than hipMemsetAsync, so the calls can live in a
// captured graph)
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

// zeroes three ranges in one launch (the counters and the parent sort's
// work buffer)
__global__ void k_zero3(int32_t *a, int64_t na, int32_t *b, int64_t nb,
                        int32_t *c, int64_t nc) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < na + nb + nc; i += stride) {
    if (i < na) a[i] = 0;
    else if (i < na + nb) b[i - na] = 0;
    else c[i - na - nb] = 0;
  }
}

__global__ void k_fill_u8(uint8_t *p, uint8_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

static unsigned capped_grid(int64_t n) {
  unsigned g = grid_for(n);
  return g > 65536u ? 65536u : g;
}

void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s, Prof *prof) {
  if (n <= 0) return;
  PG_LAUNCH(prof, K_FILL, 4.0 * n, k_fill_i32, dim3(capped_grid(n)),
            dim3(kBlock), 0, s, p, v, n);
}

void fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s, Prof *prof) {
  if (n <= 0) return;
  PG_LAUNCH(prof, K_FILL, 1.0 * n, k_fill_u8, dim3(capped_grid(n)),
            dim3(kBlock), 0, s, p, v, n);
}

__global__ void k_sum_dist(int32_t *ctr, int dist, int dst) {
  int32_t v = ctr[dist + threadIdx.x * kDistStride];
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
  if (threadIdx.x == 0) ctr[dst] += v;
}

void sum_dist(int32_t *ctr, int dist, int dst, hipStream_t s, Prof *prof) {
  static_assert(kDistSlots == kWave, "one lane per slot");
  PG_LAUNCH(prof, K_OTHER, 0.0, k_sum_dist, dim3(1), dim3(kDistSlots), 0, s,
            ctr, dist, dst);
}

// ---------------------------------------------------------------------------
// exclusive scan: reduce tiles, scan the tile sums (recursively), then scan
// each tile with its offset
// ---------------------------------------------------------------------------
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;  // 2048

template <typename T>
__device__ T wave_incl_scan(T x) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    T y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  return x;
}

// Exclusive scan of one value per thread across the block; returns the
// thread's exclusive prefix and writes the block total to *total.
template <typename T>
__device__ T block_excl_scan(T x, T *total) {
  __shared__ T wsum[kBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  T inc = wave_incl_scan(x);
  if (lane == kWave - 1) wsum[w] = inc;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < kBlock / kWave; ++i) {
    T s = wsum[i];
    if (i < w) before += s;
    all += s;
  }
  __syncthreads();
  *total = all;
  return before + inc - x;
}

template <typename T>
__global__ void k_scan_reduce(const T *in, T *part, int64_t n,
                              const int32_t *gate) {
  if (gate && *gate) return;
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  T acc = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = base + (int64_t)j * kBlock + threadIdx.x;
    if (i < n) acc += in[i];
  }
  T tot;
  block_excl_scan(acc, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

template <typename T>
__global__ void k_scan_down(const T *in, T *out, const T *part, int64_t n,
                            const int32_t *gate) {
  if (gate && *gate) return;
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  // blocked arrangement: thread t owns items [base + t*8, base + t*8 + 8)
  T v[kScanItems];
  T acc = 0;
  const int64_t my = base + (int64_t)threadIdx.x * kScanItems;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = my + j;
    v[j] = (i < n) ? in[i] : (T)0;
    acc += v[j];
  }
  T tot;
  T run = block_excl_scan(acc, &tot) + (part ? part[blockIdx.x] : (T)0);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = my + j;
    if (i < n) out[i] = run;
    run += v[j];
  }
}

template <typename T>
static size_t scan_tmp_need(int64_t n) {
  size_t bytes = 0;
  while (n > kScanTile) {
    int64_t t = (n + kScanTile - 1) / kScanTile;
    bytes += (size_t)t * sizeof(T);
    n = t;
  }
  return bytes;
}

template <typename T>
static void scan_rec(const T *in, T *out, int64_t n, T *tmp, hipStream_t s,
                     Prof *prof, const int32_t *gate) {
  if (n <= 0) return;
  if (n <= kScanTile) {
    PG_LAUNCH(prof, K_SCAN, 2.0 * sizeof(T) * n, k_scan_down<T>, dim3(1),
              dim3(kBlock), 0, s, in, out, (const T *)nullptr, n, gate);
    return;
  }
  int64_t t = (n + kScanTile - 1) / kScanTile;
  PG_LAUNCH(prof, K_SCAN, 1.0 * sizeof(T) * n, k_scan_reduce<T>,
            dim3((unsigned)t), dim3(kBlock), 0, s, in, tmp, n, gate);
  scan_rec<T>(tmp, tmp, t, tmp + t, s, prof, gate);
  PG_LAUNCH(prof, K_SCAN, 2.0 * sizeof(T) * n, k_scan_down<T>,
            dim3((unsigned)t), dim3(kBlock), 0, s, in, out, (const T *)tmp, n,
            gate);
}

size_t scan_excl_i64(const int64_t *in, int64_t *out, int64_t n, void *tmp,
                     hipStream_t s) {
  if (!tmp) return scan_tmp_need<int64_t>(n);
  scan_rec<int64_t>(in, out, n, (int64_t *)tmp, s, nullptr, nullptr);
  return 0;
}

size_t scan_excl_u32(const uint32_t *in, uint32_t *out, int64_t n, void *tmp,
                     hipStream_t s, Prof *prof, const int32_t *gate) {
  if (!tmp) return scan_tmp_need<uint32_t>(n);
  scan_rec<uint32_t>(in, out, n, (uint32_t *)tmp, s, prof, gate);
  return 0;
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, 8-bit digits
// ---------------------------------------------------------------------------
constexpr int kRsItems = 16;
constexpr int kRsTile = kBlock * kRsItems;  // 4096 keys per tile
constexpr int kRsWaves = kBlock / kWave;    // 4

int64_t radix_tiles(int64_t n) { return (n + kRsTile - 1) / kRsTile; }

size_t radix_scan_tmp_bytes(int64_t n) {
  return scan_tmp_need<uint32_t>(256 * radix_tiles(n));
}

__global__ __launch_bounds__(kBlock) void k_rs_upsweep(const uint32_t *keys,
                                                       int64_t n, int shift,
                                                       uint32_t *tile_cnt,
                                                       int64_t tiles,
                                                       const int32_t *gate) {
  if (gate && *gate) return;
  __shared__ uint32_t hist[256];
  hist[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll 4
  for (int r = 0; r < kRsItems; ++r) {
    int64_t i = base + (int64_t)r * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&hist[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  tile_cnt[(int64_t)threadIdx.x * tiles + blockIdx.x] = hist[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_rs_downsweep(
    const uint32_t *kin, const uint32_t *__restrict__ vin, uint32_t *kout,
    uint32_t *vout,
    int64_t n, int shift, const uint32_t *tile_off, int64_t tiles,
    const int32_t *gate) {
  if (gate && *gate) return;
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[kRsWaves][256];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int w = tid / kWave;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  run[tid] = tile_off[(int64_t)tid * tiles + blockIdx.x];
#pragma unroll
  for (int j = 0; j < kRsWaves; ++j) wcnt[j][tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int r = 0; r < kRsItems; ++r) {
    const int64_t i = base + (int64_t)r * kBlock + tid;
    const bool valid = i < n;
    uint32_t k = valid ? kin[i] : 0u;
    // without an input value array the value is the input position
    uint32_t v = valid ? (vin ? vin[i] : (uint32_t)i) : 0u;
    const uint32_t d = (k >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t before = (uint32_t)__popcll(peers & lt);
    if (valid && before == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t p = run[d] + before;
      for (int j = 0; j < w; ++j) p += wcnt[j][d];
      kout[p] = k;
      vout[p] = v;
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int j = 0; j < kRsWaves; ++j) {
      add += wcnt[j][tid];
      wcnt[j][tid] = 0;
    }
    run[tid] += add;
    __syncthreads();
  }
}

int radix_sort(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1,
               int64_t n, int bits, uint32_t *tile_cnt, void *scan_tmp,
               hipStream_t s, Prof *prof, const int32_t *gate,
               bool index_values) {
  if (n <= 0 || bits <= 0) return 0;
  const int64_t tiles = radix_tiles(n);
  int cur = 0;
  for (int shift = 0; shift < bits; shift += 8) {
    uint32_t *ki = cur ? k1 : k0;
    // with index_values the first pass takes each key's input position as
    // its value instead of reading v0
    const uint32_t *vi =
        cur ? v1 : ((index_values && shift == 0) ? nullptr : v0);
    uint32_t *ko = cur ? k0 : k1, *vo = cur ? v0 : v1;
    // algorithmic bytes: keys read (4 B) and 1 KiB of counts per tile;
    // then keys and values read and written (16 B)
    PG_LAUNCH(prof, K_SORT_HIST, 4.0 * n + 1024.0 * tiles, k_rs_upsweep,
              dim3((unsigned)tiles), dim3(kBlock), 0, s, ki, n, shift,
              tile_cnt, tiles, gate);
    scan_excl_u32(tile_cnt, tile_cnt, 256 * tiles, scan_tmp, s, prof, gate);
    PG_LAUNCH(prof, K_SORT_PASS, 16.0 * n + 1024.0 * tiles, k_rs_downsweep,
              dim3((unsigned)tiles), dim3(kBlock), 0, s, ki, vi, ko, vo, n,
              shift, tile_cnt, tiles, gate);
    cur ^= 1;
  }
  return cur;
}

// ---------------------------------------------------------------------------
// one-sweep stable LSD radix sort, 8-bit digits (the parent sort of a
// valuation): a split pass sets the sink's children aside (they are already
// in order), compacts the other finite vertices and counts their digits of
// every pass; then each pass is one kernel in which a tile
// (taken in launch order from a counter) ranks its keys in LDS, learns
// its global offset per digit by decoupled look-back over the tiles before
// it, and writes each digit's run out contiguously.  A tile waits only on
// tiles that took their number earlier and never wait on later ones, so the
// look-back always ends; a bounded spin turns a broken protocol into an
// error instead of a hang.
// ---------------------------------------------------------------------------
// Tile shapes.  kBlock threads with ITEMS keys each, 4096-key tiles below
// kLargeTileFrom keys and 8192-key tiles from there on, lay out the status
// words.  The split and the digit
// passes take 1024-thread blocks with tiles at least as large (so never
// more tiles than there are status words for): a pass holds its keys and
// values in LDS, 16384 keys (128 KiB) on a large sort, one block per CU at
// 16 waves, where 8192-key tiles of 256 threads left 2 waves per SIMD
// (205 VGPRs) with nothing to cover the look-back and the LDS ranking; the
// split keeps nothing in LDS and takes 32768 keys.  On the 10M-vertex game
// per valuation: digit pass 48 -> 41 us, split 63 -> 48 us; on the
// 1M-vertex game 18.6 -> 16.6 and 20.4 -> 15.9 us (4096- and 8192-key
// tiles there).  Fewer, larger tiles shorten the look-back chains of a
// large sort, smaller ones keep a small sort's grid wide.
constexpr int k1sItemsSmall = 16, k1sItemsLarge = 32;
constexpr int64_t kLargeTileFrom = 4194304;
constexpr int kPassBlockSmall = 1024, kPassItemsSmall = 4;
constexpr int kPassBlockLarge = 1024, kPassItemsLarge = 16;
constexpr int kSplitBlockSmall = 1024, kSplitItemsSmall = 8;
constexpr int kSplitBlockLarge = 1024, kSplitItemsLarge = 32;
static_assert(kSplitBlockSmall * kSplitItemsSmall >= kBlock * k1sItemsSmall &&
                  kSplitBlockLarge * kSplitItemsLarge >=
                      kBlock * k1sItemsLarge,
              "the split has at most as many tiles as its status words");
static_assert(kPassBlockSmall * kPassItemsSmall >= kBlock * k1sItemsSmall &&
                  kPassBlockLarge * kPassItemsLarge >= kBlock * k1sItemsLarge,
              "a digit pass has at most as many tiles as its status words");
inline int sort_items(int64_t n) {
  return n >= kLargeTileFrom ? k1sItemsLarge : k1sItemsSmall;
}
constexpr uint32_t kStAgg = 1u << 30;        // tile count published
constexpr uint32_t kStPre = 1u << 31;        // inclusive prefix published
constexpr uint32_t kStVal = (1u << 30) - 1;
constexpr int kSpinMax = 1 << 22;
constexpr int k1sMaxPasses = 4;
constexpr int k1sCopies = 64;   // histogram copies (blocks spread over them)

int64_t onesweep_tiles(int64_t n, int items) {
  const int64_t t = (int64_t)kBlock * items;
  return (n + t - 1) / t;
}

// work buffer: [counters 8 | histograms 64 copies x 4 x 256 | bases 4 x 256
//               | status 4 x tiles x 256 | split status 2 x tiles]
// counters: 0-3 tile numbers of the digit passes, 4 of the split pass,
// 5 the prefix length (finite vertices whose parent is not the sink)
constexpr int k1sCounters = 8;
constexpr int64_t k1sHistWords = (int64_t)k1sCopies * k1sMaxPasses * 256;

int64_t onesweep_words(int64_t n) {
  const int64_t tiles = onesweep_tiles(n, k1sItemsSmall);   // the most
  return k1sCounters + k1sHistWords + k1sMaxPasses * 256 +
         k1sMaxPasses * tiles * 256 + 2 * tiles;
}

// lanes of the wave (among `valid` ones) whose 8-bit digit equals mine
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bb = __ballot(bit);
    peers &= bit ? bb : ~bb;
  }
  return peers;
}

// digit bases of every pass: exclusive scans of the histograms, summed
// over their copies; thread group p (256 threads) takes pass p, so that the
// passes' copies are read and scanned together
constexpr int kBaseThreads = k1sMaxPasses * 256;
__global__ __launch_bounds__(kBaseThreads) void k_1s_base(
    const uint32_t *glob, int passes, uint32_t *base, const int32_t *gate) {
  if (gate && *gate) return;
  __shared__ uint32_t wsum[kBaseThreads / kWave];
  const int p = threadIdx.x / 256, d = threadIdx.x & 255;
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  uint32_t c = 0;
  if (p < passes) {
#pragma unroll 16
    for (int j = 0; j < k1sCopies; ++j)
      c += glob[(int64_t)j * (k1sMaxPasses * 256) + p * 256 + d];
  }
  const uint32_t inc = wave_incl_scan(c);
  if (lane == kWave - 1) wsum[w] = inc;
  __syncthreads();
  uint32_t before = 0;
  for (int i = p * (256 / kWave); i < w; ++i) before += wsum[i];
  if (p < passes) base[p * 256 + d] = before + inc - c;
}

__device__ __forceinline__ uint32_t ld_status(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_status(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive scan of one value per thread over a block of BS threads.
template <typename T, int BS>
__device__ T block_excl_scan_bs(T x, T *total) {
  __shared__ T wsum[BS / kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  T inc = wave_incl_scan(x);
  if (lane == kWave - 1) wsum[w] = inc;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < BS / kWave; ++i) {
    T s = wsum[i];
    if (i < w) before += s;
    all += s;
  }
  __syncthreads();
  *total = all;
  return before + inc - x;
}

// BS threads take a tile of BS * ITEMS keys.  Wave w of a tile owns the
// w-th of BS / 64 equal stretches of the tile's keys, 64 at a time in order,
// so wave order then round order then lane order is input order: ranks come
// out stable without barriers inside the loop.  The first 256 threads then
// take one digit each.
template <int BS, int ITEMS>
__global__ __launch_bounds__(BS) void k_1s_pass(
    const uint32_t *kin, const uint32_t *__restrict__ vin, uint32_t *kout,
    uint32_t *vout, const uint32_t *n_dev, int shift,
    const uint32_t *__restrict__ dbase, uint32_t *status, uint32_t *tile_ctr,
    int32_t *err, const int32_t *gate) {
  constexpr int kT = BS * ITEMS;   // keys per tile
  constexpr int kW = BS / kWave;   // waves per tile
  static_assert(BS >= 256 && BS % 256 == 0, "one thread per digit");
  if (gate && *gate) return;
  const int64_t n = *n_dev;
  // the grid is sized for the most keys: blocks past the tiles needed leave
  // before taking a tile number, so the ones that stay take exactly the
  // numbers of the tiles there are
  if ((int64_t)blockIdx.x * kT >= n) return;
  __shared__ uint32_t s_tile;
  __shared__ uint32_t lk[kT];
  __shared__ uint32_t lv[kT];
  __shared__ uint32_t wc[kW][256];   // per wave: digit counts, then the
                                     // wave's first slot per digit
  __shared__ uint32_t start[256], goff[256];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int w = tid / kWave;
  const bool dig = tid < 256;        // thread tid owns digit tid
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  if (tid == 0) s_tile = atomicAdd(tile_ctr, 1u);
  for (int j = lane; j < 256; j += kWave) wc[w][j] = 0;
  __syncthreads();
  const uint32_t tile = s_tile;
  const int64_t base = (int64_t)tile * kT;
  const int64_t rem = n - base;
  const int tn = rem < kT ? (int)rem : kT;   // keys of this tile
  uint32_t k[ITEMS], v[ITEMS], rk[ITEMS];
  // every load in flight before the first ballot waits on one
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int j = w * (kT / kW) + r * kWave + lane;
    const bool valid = j < tn;
    k[r] = valid ? kin[base + j] : 0u;
    v[r] = valid ? vin[base + j] : 0u;
  }
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int j = w * (kT / kW) + r * kWave + lane;
    const bool valid = j < tn;
    const uint32_t d = (k[r] >> shift) & 255u;
    const uint64_t peers = digit_peers(d, valid);
    const uint32_t before = (uint32_t)__popcll(peers & lt);
    const uint32_t cur = wc[w][d];
    rk[r] = cur + before;
    if (valid && before == 0) wc[w][d] = cur + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  uint32_t c[kW], cnt = 0;
  if (dig) {
#pragma unroll
    for (int j = 0; j < kW; ++j) {
      c[j] = wc[j][tid];
      cnt += c[j];
    }
    // publish this tile's count at once (its prefix, for the first tile)
    st_status(&status[(int64_t)tile * 256 + tid],
              (tile == 0 ? kStPre : kStAgg) | cnt);
  }
  uint32_t tot;
  const uint32_t st0 = block_excl_scan_bs<uint32_t, BS>(cnt, &tot);
  if (dig) {
    start[tid] = st0;
    uint32_t o = st0;
#pragma unroll
    for (int j = 0; j < kW; ++j) {
      wc[j][tid] = o;
      o += c[j];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int j = w * (kT / kW) + r * kWave + lane;
    if (j < tn) {
      const uint32_t slot = wc[w][(k[r] >> shift) & 255u] + rk[r];
      lk[slot] = k[r];
      lv[slot] = v[r];
    }
  }
  // decoupled look-back for digit tid
  if (dig) {
    uint32_t excl = 0;
    if (tile > 0) {
      int64_t t = (int64_t)tile - 1;
      int spins = 0;
      for (;;) {
        const uint32_t sv = ld_status(&status[t * 256 + tid]);
        if (!(sv & (kStAgg | kStPre))) {
          if (++spins > kSpinMax) {
            atomicOr(err, ERR_SORT);
            break;
          }
          continue;
        }
        excl += sv & kStVal;
        if ((sv & kStPre) || t == 0) break;
        --t;
      }
      st_status(&status[(int64_t)tile * 256 + tid], kStPre | (excl + cnt));
    }
    goff[tid] = dbase[tid] + excl;
  }
  __syncthreads();
  // each digit's run goes out contiguously
#pragma unroll 4
  for (int r = 0; r < ITEMS; ++r) {
    const int sl = r * BS + tid;
    if (sl < tn) {
      const uint32_t key = lk[sl];
      const uint32_t d = (key >> shift) & 255u;
      const uint32_t pos = goff[d] + (uint32_t)sl - start[d];
      kout[pos] = key;
      vout[pos] = lv[sl];
    }
  }
}

// Split pass of the parent sort: key < npar (the vertex has an inner
// parent) goes to kout/vout in input order with its index as value; key ==
// npar (a child of the sink) only needs its index, written to cout at
// nF - 1 - (its rank among the sink's children), so that the prefix length
// need not be known; larger keys (top vertices) are dropped.  Tiles find
// their offsets for the two classes by decoupled look-back (two status
// words per tile); the last tile publishes the prefix length and checks that
// the two classes add up to the finite count.  The split also builds the
// digit histograms of every pass over the keys it keeps: each wave adds its
// inner keys' digits to its own LDS counters with atomics (lanes of a wave
// that hit one counter are serialised by the LDS, which costs less than
// finding the groups of equal digits with ballots, eight per digit: 47 ->
// 13 us per valuation on the 10M-vertex random game, then in a kernel of
// its own that read the kept keys again; folded in here they add 9 us to
// the split against that kernel's 15 us).
template <int BS, int ITEMS>
__global__ __launch_bounds__(BS) void k_ps_split(
    const uint32_t *kin, int64_t n, uint32_t npar, uint32_t *kout,
    uint32_t *vout, uint32_t *cout, uint32_t *status, uint32_t *tile_ctr,
    uint32_t *n_inner, int passes, uint32_t *glob, int32_t *ctr) {
  constexpr int kT = BS * ITEMS;   // keys per tile
  constexpr int kW = BS / kWave;   // waves per tile
  if (ctr[C_ABORT]) return;
  __shared__ uint32_t s_tile;
  __shared__ uint32_t wcnt[2][kW];
  __shared__ uint32_t s_excl[2], s_total[2];
  __shared__ uint32_t h[kW][k1sMaxPasses][256];   // per wave: digit counts
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int w = tid / kWave;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  if (tid == 0) s_tile = atomicAdd(tile_ctr, 1u);
  for (int q = lane; q < k1sMaxPasses * 256; q += kWave)
    h[w][q / 256][q & 255] = 0;
  __syncthreads();
  const uint32_t tile = s_tile;
  const int64_t base = (int64_t)tile * kT + w * (kT / kW);
  uint32_t k[ITEMS], r0[ITEMS], r1[ITEMS];
  uint32_t c0 = 0, c1 = 0;
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int64_t i = base + r * kWave + lane;
    k[r] = i < n ? kin[i] : 0xffffffffu;
  }
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const uint64_t b0 = __ballot(k[r] < npar);
    const uint64_t b1 = __ballot(k[r] == npar);
    r0[r] = c0 + (uint32_t)__popcll(b0 & lt);
    r1[r] = c1 + (uint32_t)__popcll(b1 & lt);
    c0 += (uint32_t)__popcll(b0);
    c1 += (uint32_t)__popcll(b1);
  }
  // the digit histogram of every pass over the inner keys
  for (int p = 0; p < passes; ++p) {
#pragma unroll
    for (int r = 0; r < ITEMS; ++r)
      if (k[r] < npar) atomicAdd(&h[w][p][(k[r] >> (8 * p)) & 255u], 1u);
  }
  if (lane == 0) {
    wcnt[0][w] = c0;
    wcnt[1][w] = c1;
  }
  __syncthreads();
  {
    // blocks add into one of k1sCopies copies: one counter hit by every
    // block serialises on its address
    uint32_t *copy =
        glob + (int64_t)(blockIdx.x % k1sCopies) * (k1sMaxPasses * 256);
    for (int q = tid; q < passes * 256; q += BS) {
      uint32_t t = 0;
#pragma unroll
      for (int j = 0; j < kW; ++j) t += h[j][q / 256][q & 255];
      if (t) atomicAdd(&copy[q], t);
    }
  }
  if (tid < 2) {
    uint32_t cnt = 0;
    for (int j = 0; j < kW; ++j) cnt += wcnt[tid][j];
    st_status(&status[(int64_t)tile * 2 + tid],
              (tile == 0 ? kStPre : kStAgg) | cnt);
    uint32_t excl = 0;
    if (tile > 0) {
      int64_t t = (int64_t)tile - 1;
      int spins = 0;
      for (;;) {
        const uint32_t sv = ld_status(&status[t * 2 + tid]);
        if (!(sv & (kStAgg | kStPre))) {
          if (++spins > kSpinMax) {
            atomicOr(&ctr[C_ERR], ERR_SORT);
            break;
          }
          continue;
        }
        excl += sv & kStVal;
        if ((sv & kStPre) || t == 0) break;
        --t;
      }
      st_status(&status[(int64_t)tile * 2 + tid], kStPre | (excl + cnt));
    }
    s_excl[tid] = excl;
    s_total[tid] = excl + cnt;
  }
  __syncthreads();
  const int64_t nf = ctr[C_NFIN];
  if (tid == 0 && (int64_t)(tile + 1) * kT >= n) {
    *n_inner = s_total[0];
    ctr[C_NINNER] = (int32_t)s_total[0];
    if ((int64_t)s_total[0] + s_total[1] != nf)
      atomicOr(&ctr[C_ERR], ERR_RANKCOUNT);
  }
  uint32_t o0 = s_excl[0], o1 = s_excl[1];
  for (int j = 0; j < w; ++j) {
    o0 += wcnt[0][j];
    o1 += wcnt[1][j];
  }
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int64_t i = base + r * kWave + lane;
    if (k[r] < npar) {
      const uint32_t q = o0 + r0[r];
      kout[q] = k[r];
      vout[q] = (uint32_t)i;
    } else if (k[r] == npar) {
      const int64_t q = (int64_t)o1 + r1[r];
      if (q < nf) cout[nf - 1 - q] = (uint32_t)i;   // else flagged above
    }
  }
}

void clear_valuation(int32_t *ctr, uint32_t *work, int64_t n, hipStream_t s,
                     Prof *prof) {
  if (!work) {
    fill_i32(ctr, 0, C_TOTAL, s, prof);
    return;
  }
  // [counters | histograms] and [status | split status] (the bases are
  // written before they are read)
  const int64_t tiles = onesweep_tiles(n, sort_items(n));
  const int64_t na = k1sCounters + k1sHistWords;
  const int64_t nb = (int64_t)k1sMaxPasses * tiles * 256 + 2 * tiles;
  uint32_t *status = work + na + k1sMaxPasses * 256;
  PG_LAUNCH(prof, K_FILL, 4.0 * (C_TOTAL + na + nb), k_zero3,
            dim3(capped_grid(C_TOTAL + na + nb)), dim3(kBlock), 0, s, ctr,
            (int64_t)C_TOTAL, (int32_t *)work, na, (int32_t *)status, nb);
}

int parent_sort(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1,
                int64_t n, uint32_t npar, int bits, uint32_t *work,
                int32_t *ctr, hipStream_t s, Prof *prof,
                const uint32_t **n_inner) {
  const int passes = (bits + 7) / 8;
  const int items = sort_items(n);
  const int64_t tiles = onesweep_tiles(n, items);
  uint32_t *wctr = work, *glob = work + k1sCounters;
  uint32_t *base = glob + k1sHistWords;
  uint32_t *status = base + k1sMaxPasses * 256;
  uint32_t *sstat = status + (int64_t)k1sMaxPasses * tiles * 256;
  uint32_t *ni = wctr + 5;
  const int32_t *gate = ctr + C_ABORT;
  *n_inner = ni;
  // the tile counters, histograms and status words are zero
  // (clear_valuation, at the start of the valuation)
  // the digit passes alternate between the pairs and end in pair 0 after
  // an odd number of passes: the sink's children go straight to that pair
  const int fin = (passes & 1) ? 0 : 1;
  {
    // the split takes its own tiles too (no more of them than `tiles`, for
    // which its status words are laid out)
    const bool large = items == k1sItemsLarge;
    const int sbs = large ? kSplitBlockLarge : kSplitBlockSmall;
    const int sitems = large ? kSplitItemsLarge : kSplitItemsSmall;
    const int64_t stiles =
        (n + (int64_t)sbs * sitems - 1) / ((int64_t)sbs * sitems);
    // keys read (4 B each); 8 B per inner child, 4 B per child of the sink
    PG_LAUNCH_NI(prof, K_SORT_SPLIT, 4.0 * n, 4.0, 4.0,
                 (large ? k_ps_split<kSplitBlockLarge, kSplitItemsLarge>
                        : k_ps_split<kSplitBlockSmall, kSplitItemsSmall>),
                 dim3((unsigned)stiles), dim3(sbs), 0, s, k0, n, npar, k1,
                 v1, fin ? v1 : v0, sstat, wctr + 4, ni, passes, glob, ctr);
  }
  PG_LAUNCH(prof, K_SCAN, 0.0, k_1s_base, dim3(1), dim3(kBaseThreads), 0, s,
            glob, passes, base, gate);
  // the digit passes take their own tiles (no more of them than `tiles`,
  // for which the status words of a pass are laid out)
  const bool large = items == k1sItemsLarge;
  const int pbs = large ? kPassBlockLarge : kPassBlockSmall;
  const int pitems = large ? kPassItemsLarge : kPassItemsSmall;
  const int64_t ptiles =
      (n + (int64_t)pbs * pitems - 1) / ((int64_t)pbs * pitems);
  int cur = 1;
  for (int p = 0; p < passes; ++p) {
    uint32_t *ki = cur ? k1 : k0, *vi = cur ? v1 : v0;
    uint32_t *ko = cur ? k0 : k1, *vo = cur ? v0 : v1;
    // keys and values read and written (16 B), 1 KiB of status per tile
    PG_LAUNCH_NI(prof, K_SORT_PASS, 0.0, 0.0, 16.0 + 1024.0 / (pbs * pitems),
                 (large ? k_1s_pass<kPassBlockLarge, kPassItemsLarge>
                        : k_1s_pass<kPassBlockSmall, kPassItemsSmall>),
                 dim3((unsigned)ptiles), dim3(pbs), 0, s, ki, vi, ko, vo,
                 ni, 8 * p, base + p * 256, status + (int64_t)p * tiles * 256,
                 wctr + p, ctr + C_ERR, gate);
    cur ^= 1;
  }
  return cur;
}

}  // namespace pgk
