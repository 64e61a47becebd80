// Internal definitions shared by the library's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/pg.h"

namespace pgk {

constexpr int kBlock = 256;            // threads per block for flat kernels
// sp[v].y (the priority of v's successor) of a vertex known to stay top for
// the rest of a solve: its play, and every play through it, is infinite
constexpr int32_t kTopMark = INT32_MIN;
constexpr int kWave = 64;              // CDNA wavefront width
constexpr int kMaxVertices = (1 << 30) - 2;

// Counters and flags kept in one small device array so that a single
// device-to-host copy returns all of them.
enum Counter : int {
  C_ERR = 0,          // error bits (ERR_*)
  C_NFIN = 1,         // finite vertices excluding the sink
  C_SWITCH = 2,       // switches made by the last switch kernel
  C_ABORT = 3,        // nonzero: bounded rounds left work; later kernels skip
  C_MISC = 4,         // scratch counter (preprocessing changes, odd count,
                      // open vertices of host-driven walk rounds)
  C_NINNER = 5,       // finite vertices whose parent is not the sink
  // Hot counts are spread over kDistSlots slots kDistStride ints apart (one
  // atomic per block into slot blockIdx % kDistSlots) and summed afterwards:
  // a single address hit by every block serialises.  The switch slots are
  // summed by the host (fold_switches), the others by a small kernel (a
  // last-block-done sum inside the producing kernel would need a release
  // fence per block, which writes back the L2 each time: 10x slower).
  C_DIST_SW = 32,
  C_COUNT = 32 + 1024,   // the part copied back to the host
  C_DIST_NF = C_COUNT,
  C_DIST_MISC = C_COUNT + 1024,
  // lengths of the open-walk lists (one list per slot, see append_block)
  C_DIST_WLNG = C_COUNT + 2048,
  C_DIST_WLRT = C_COUNT + 3072,
  C_TOTAL = C_COUNT + 4096
};
constexpr int kDistSlots = 64;
constexpr int kDistStride = 16;

// After a copy of the first C_COUNT counters to the host: the switch count
// is the sum of its slots.
inline void fold_switches(int32_t *hctr) {
  int32_t s = 0;
  for (int k = 0; k < kDistSlots; ++k) s += hctr[C_DIST_SW + k * kDistStride];
  hctr[C_SWITCH] = s;
}

enum ErrBit : int {
  ERR_INADMISSIBLE = 1,  // a cycle whose largest priority is odd
  ERR_LISTWALK = 2,      // a list walk exceeded its bound (broken list)
  ERR_INVAL = 4,         // input validation failed
  ERR_DUPPRI = 8,        // repeated priority
  ERR_RANKCOUNT = 16,    // list ranking did not emit every finite vertex
  ERR_SORT = 32,         // a radix-sort look-back gave up waiting
  ERR_OFFSETS = 64,      // input validation: bad CSR offsets
};

// Kernel kinds for the optional event profiler (pg_profile_* in pg.h).
enum KId : int {
  K_FILL = 0, K_NG_WALK, K_NG_ROUND, K_ROOT_WALK, K_ROOT_ROUND,
  K_SORT_SPLIT, K_SORT_HIST, K_SCAN, K_SORT_PASS, K_LINK_INFO, K_LINK_BUILD,
  K_LR_SUM1, K_LR_SUMK, K_LR_TOP, K_LR_DISTK, K_LR_EMIT1, K_ODD_SWITCH,
  K_EVEN_SWITCH, K_ODD_STAGE, K_OTHER, K_COUNT
};
extern const char *const kKernelNames[K_COUNT];

// Records a pair of HIP events around each profiled launch on the launch's
// stream; elapsed times are collected after the stream has been synchronised.
struct Prof {
  bool on = false;
  double ms[K_COUNT] = {};
  int64_t calls[K_COUNT] = {};
  double bytes[K_COUNT] = {};
  struct Pend {
    int kid;
    double bytes;     // fixed part
    double per_nf;    // plus this many bytes per finite vertex
    double per_ni;    // and per finite vertex whose parent is not the sink
    hipEvent_t a, b;
  };
  double nf = 0.0;    // counts of the valuation being flushed
  double ni = 0.0;
  std::vector<hipEvent_t> pool;
  std::vector<Pend> pend;
  hipEvent_t get();
  void flush();     // call only after the stream has been synchronised
  void reset();
  void release();
};

struct ProfScope {
  Prof *p;
  hipStream_t s;
  Prof::Pend e{};
  ProfScope(Prof *prof, int kid, double bytes, hipStream_t st,
            double per_nf = 0.0, double per_ni = 0.0)
      : p(prof && prof->on ? prof : nullptr), s(st) {
    if (!p) return;
    e.kid = kid;
    e.bytes = bytes;
    e.per_nf = per_nf;
    e.per_ni = per_ni;
    e.a = p->get();
    e.b = p->get();
    (void)hipEventRecord(e.a, s);
  }
  ~ProfScope() {
    if (!p) return;
    (void)hipEventRecord(e.b, s);
    p->pend.push_back(e);
  }
};

// Launch with profiling: `bytes` are the kernel's algorithmic bytes.
#define PG_LAUNCH(prof, kid, bytes, kern, grid, block, smem, stream, ...) \
  do {                                                                    \
    ::pgk::ProfScope ps_((prof), (kid), (double)(bytes), (stream));       \
    hipLaunchKernelGGL(kern, grid, block, smem, stream, __VA_ARGS__);     \
  } while (0)

// Same, for kernels whose bytes are `per_nf` per finite vertex (the count
// is read back with the valuation's counters).
#define PG_LAUNCH_NF(prof, kid, per_nf, kern, grid, block, smem, stream, ...) \
  do {                                                                        \
    ::pgk::ProfScope ps_((prof), (kid), 0.0, (stream), (double)(per_nf));    \
    hipLaunchKernelGGL(kern, grid, block, smem, stream, __VA_ARGS__);         \
  } while (0)

// Same, with `per_nf` bytes per finite vertex and `per_ni` per finite vertex
// whose parent is not the sink (both read back with the counters).
#define PG_LAUNCH_NI(prof, kid, bytes, per_nf, per_ni, kern, grid, block,   \
                     smem, stream, ...)                                    \
  do {                                                                     \
    ::pgk::ProfScope ps_((prof), (kid), (double)(bytes), (stream),         \
                         (double)(per_nf), (double)(per_ni));              \
    hipLaunchKernelGGL(kern, grid, block, smem, stream, __VA_ARGS__);      \
  } while (0)

// Levels of the recursive sublist list ranking a game holds arrays for: with
// a level-0 stride of at least kStrideMin and kStrideUp = 4 above it, an
// Euler list of 2^32 elements is down to one splitter by level 15.
constexpr int kMaxLevels = 16;

// Per-level arrays of the recursive sublist list ranking.
struct RankLevel {
  int64_t size = 0;      // elements of this level
  int stride = 0;        // splitter stride (elements e with e % stride == 0)
  int64_t nsplit = 0;    // splitters = elements of the next level
  int32_t *sum = nullptr;   // per splitter: weight of its sublist
  int32_t *next = nullptr;  // per splitter: index of the next splitter or -1
  int32_t *base = nullptr;  // per splitter: exclusive rank of its sublist
};

}  // namespace pgk

struct pg_game {
  int device = 0;
  int64_t n = 0, m = 0;          // original game
  int64_t n_aug = 0, m_aug = 0;  // modified game (sink not counted)
  int32_t n_oddpri = 0;          // vertices with an odd priority
  int64_t n_odd = 0, m_odd = 0;  // Odd vertices and the edges of their rows
  int sort_bits = 0;             // bits of a parent id key (ids 0..n_aug+1)
  bool careful = false;          // PG_CAREFUL_WALKS: host-driven walk rounds
  // a solve marks, after each best response, the vertices whose valuation
  // is top (kTopMark); single games (a batch marks in its own step)
  bool mark_top = false;
  // PG_HOST_REDUCED_LIST: the host ranks the level-1 reduced list (pinned
  // next, sum and base arrays in h_rl)
  bool host_rl = false;
  int32_t *h_rl = nullptr;
  // one best-response iteration (walks, valuation, All_Odd) captured as a
  // HIP graph and replayed (unless PG_NO_GRAPH)
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t iter_exec = nullptr;
  // All_Odd over the bucketed edge layout (pg_switch.hip): the Odd rows'
  // edges in target order (tsw_t) with each edge's slot in its chunk
  // (tsw_slot) and that slot's place in bucket order (tsw_g); per place the
  // target (tsw_tz) and the vertex within its bucket (tsw_sz); bucket starts
  // (tsw_bs, tsw_nb + 1); keys in bucket order each step (tsw_r)
  bool tsw = false;
  int64_t tsw_nb = 0, tsw_nc = 0;
  int32_t *tsw_t = nullptr, *tsw_g = nullptr, *tsw_tz = nullptr;
  int32_t *tsw_bs = nullptr, *tsw_r = nullptr;
  uint16_t *tsw_slot = nullptr, *tsw_sz = nullptr;

  // modified game, device resident
  int64_t *off = nullptr;   // [n_aug+1]
  int32_t *tgt = nullptr;   // [m_aug]
  uint8_t *owner = nullptr; // [n_aug]
  int32_t *pri = nullptr;   // [n_aug]
  // Signed-priority order: perm[i] is the i-th vertex in that order, rvpos
  // (below) its inverse.  A rank-valuation game is stored in that order
  // (relabeled): internal vertex i is the caller's vertex perm[i], with its
  // row in the caller's edge order, so the valuation kernels use neither map
  // and the two only translate vertex ids at the C ABI.
  int32_t *perm = nullptr;  // [n_aug]
  bool relabeled = false;
  // PG_ODD_REGION: the stored game is the original one minus Odd's own
  // winning region A (pg_oddregion.hip); or_new[v] is vertex v's id in it
  // (-1 for A), or_orig[u] the original id of its vertex u
  bool odd_region = false;
  int64_t or_removed = 0;     // |A|
  int32_t *or_new = nullptr;  // [n]
  int32_t *or_orig = nullptr; // [n_aug]

  // play graph and valuation state
  // [n_aug+1] {successor (the sink is n_aug), priority of that successor}
  int2 *sp = nullptr;
  int32_t *key = nullptr;   // [n_aug+1] valuation keys; n_aug is the sink
  int32_t *ng = nullptr;    // [n_aug] nearest greater vertex (-1: open)
  int32_t *cand = nullptr;  // [n_aug] walk candidates of open vertices
  int32_t *rcand = nullptr; // [n_aug]   root-walk candidates
  // vertices whose ng (wl_ng) or fate (wl_rt) the full pass left open, in
  // kDistSlots lists of wl_cap entries (see append_block)
  int32_t *wl_ng = nullptr, *wl_rt = nullptr;
  int64_t wl_cap = 0;
  int32_t *wl0 = nullptr;   // [n_aug]   staging of host strategies
  int32_t *wl1 = nullptr;   // [n_aug]
  uint8_t *rs = nullptr;    // [n_aug+1] 0 unknown, 1 finite, 2 top

  // sorting
  uint32_t *sk0 = nullptr, *sv0 = nullptr, *sk1 = nullptr, *sv1 = nullptr;
  uint32_t *tile_cnt = nullptr;  // [256 * tiles]
  uint32_t *rs1 = nullptr;       // [onesweep_words(n_aug)] one-sweep sort
  int64_t tiles = 0;
  void *scan_tmp = nullptr;      // device-wide scan partials
  size_t scan_tmp_bytes = 0;

  // Euler list of the nearest-greater-ancestor tree
  int32_t *kids = nullptr;   // [n_aug]   count valuations: compacted vertices
  // [n_aug+1] rank valuations: {0, 0} for a leaf, else the sorted positions
  // of the first and the last child, + 1 each (count valuations: the list
  // starts, as int32)
  uint2 *fh = nullptr;
  // where the last parent sort left its sorted keys, and the device word
  // holding its count of inner positions
  const uint32_t *ps_k = nullptr, *ps_ni = nullptr;
  int32_t *pos = nullptr;    // [n_aug+1] sorted position of each finite vertex
  int32_t *rvpos = nullptr;  // [n_aug] position of each vertex in perm
  int32_t *odd_ids = nullptr;   // [n_odd]  Odd vertices, increasing
  int32_t *even_ids = nullptr;  // [n_aug - n_odd] Even vertices, increasing
  // [2*n_aug+2] {next element or -1, node | weight bits}
  int2 *elem = nullptr;
  // [2*n_aug+2] per element carrying a point: {level-1 sublist, weight
  // before the element in that sublist}, by sorted position: element 2i+2
  // at i, 2i+3 at n_aug + i, element 1 at 2 n_aug
  int2 *aux = nullptr;

  pgk::RankLevel lv[pgk::kMaxLevels];
  int nlevels = 0;

  // count valuations (repeated priorities; see pg_count.hip)
  bool dense = false;
  int32_t d = 0;              // distinct priorities in use
  int32_t dw = 0;             // ints per count row: d rounded up to 4/8/16/32
  uint32_t odd_cols = 0;      // bit j: the j-th smallest priority is odd
  int32_t values[32] = {};    // the distinct priorities, increasing
  int32_t *cvals = nullptr;   // [32] the same on the device
  uint8_t *pidx = nullptr;    // [n_aug] column of each vertex's priority
  int32_t *cnt = nullptr;     // [(n_aug+1) * dw] counts; row n_aug: the sink
  int32_t *cnt2 = nullptr;    // the same size: Bellman-Ford's second buffer
  int4 *elem4 = nullptr;      // [2*n_aug+2] {next, vertex | up bit, column}
  int32_t *vsum[pgk::kMaxLevels] = {};   // per level: dw ints per splitter
  int32_t *vbase[pgk::kMaxLevels] = {};

  unsigned long long *u64tmp = nullptr;  // [2] scratch for 64-bit sums
  int32_t *ctr = nullptr;    // [C_TOTAL] device counters
  int32_t *hctr = nullptr;   // pinned host mirror

  pgk::Prof prof;
  // launch and walk parameters of the rank valuation (pg_tuning)
  pg_tuning tune{32, 1, 16, 64, 3, 256};
  // false: no HIP events are created or recorded (pg_solve_noalloc)
  bool timed = true;
  // HIP events around each best-response iteration on the call's stream
  // (created at first use); the last iteration's device time
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
  float last_ms = 0.0f;
};

// The signed-order maps the valuation kernels take: none for a relabeled
// game, whose vertex ids already are positions in that order.
inline const int32_t *kernel_rvpos(const pg_game *g) {
  return g->relabeled ? nullptr : g->rvpos;
}
inline const int32_t *kernel_perm(const pg_game *g) {
  return g->relabeled ? nullptr : g->perm;
}

// ---- error reporting (pg_api.hip) -----------------------------------------
pg_status pg_fail(pg_status st, const std::string &msg);

#define PG_HIP(call)                                                        \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess)                                                   \
      return pg_fail(e_ == hipErrorOutOfMemory ? PG_ENOMEM : PG_EDEVICE,    \
                     std::string(#call) + ": " + hipGetErrorString(e_));   \
  } while (0)

#define PG_TRY(expr)                   \
  do {                                 \
    pg_status st_ = (expr);            \
    if (st_ != PG_OK) return st_;      \
  } while (0)

// ---- primitives (pg_prims.hip) --------------------------------------------
namespace pgk {

// Adds the number of threads of the block with `pred` to the distributed
// counter starting at `dist` (see C_DIST_*).  Every thread of the block must
// call it.
__device__ __forceinline__ void count_block(int32_t *dist, bool pred) {
  __shared__ int32_t blk;
  if (threadIdx.x == 0) blk = 0;
  __syncthreads();
  const uint64_t b = __ballot(pred);
  if ((threadIdx.x & (kWave - 1)) == 0 && b) atomicAdd(&blk, (int)__popcll(b));
  __syncthreads();
  if (threadIdx.x == 0 && blk)
    atomicAdd(&dist[(blockIdx.x % kDistSlots) * kDistStride], blk);
}

// Adds n (per thread) to the distributed counter at `dist`.  Every thread of
// the block must call it.
__device__ __forceinline__ void add_block(int32_t *dist, int32_t n) {
  __shared__ int32_t blk;
  if (threadIdx.x == 0) blk = 0;
  __syncthreads();
  if (n) atomicAdd(&blk, n);
  __syncthreads();
  if (threadIdx.x == 0 && blk)
    atomicAdd(&dist[(blockIdx.x % kDistSlots) * kDistStride], blk);
}

// Appends v (where pred holds) to the list of slot blockIdx % kDistSlots,
// whose length counts at cnt[slot * kDistStride]: one LDS atomic per wave
// and one device atomic per block, spread over the slots' counters.  A slot
// receives at most ceil(blocks / kDistSlots) blocks' vertices, so cap =
// ceil(n / kDistSlots) + 2 * kBlock entries per slot suffice for blocks of
// up to kBlock threads.  Every thread of the block must call it.
__device__ __forceinline__ void append_block(int32_t *cnt, int32_t *list,
                                             int64_t cap, bool pred,
                                             int32_t v) {
  __shared__ int32_t s_n, s_base;
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  const uint64_t b = __ballot(pred);
  const int lane = threadIdx.x & (kWave - 1);
  int32_t off = 0;
  if (b) {
    int32_t wbase = 0;
    if (lane == 0) wbase = atomicAdd(&s_n, (int32_t)__popcll(b));
    wbase = __shfl(wbase, 0);
    off = wbase + (int32_t)__popcll(b & ((1ull << lane) - 1ull));
  }
  __syncthreads();
  const int slot = blockIdx.x % kDistSlots;
  if (threadIdx.x == 0 && s_n)
    s_base = atomicAdd(&cnt[slot * kDistStride], s_n);
  __syncthreads();
  if (pred) list[(int64_t)slot * cap + s_base + off] = v;
}

__device__ __forceinline__ int ld_relaxed(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_relaxed(int32_t *p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Splitter strides of the sublist ranking: the Euler list (level 0) is walked
// by many threads at once and is bound by its loads; the reduced lists are
// short, and a level's time is its longest sublist walk (sublist lengths are
// about geometric, so the longest is near stride x ln(sublists)): there a
// small stride wins.  The level-0 stride s0 is a power of two: rank
// valuations take pg_tuning::stride0, count valuations count_stride.  Above
// level 0, stride 4 against 8 (more levels, each shorter): per iteration
// 1M-vertex game 0.321 -> 0.317 ms, 10M 1.598 -> 1.590 ms, 10M with 4
// priorities 3.20 -> 3.17 ms; 16 was slower on all three.
constexpr int kStrideUp = 4;       // level k -> k + 1 for k >= 1
constexpr int kStrideMin = 8;      // least level-0 stride (sizes the levels)

// size of level k of the sublist ranking for an Euler list of L elements
// whose level-0 stride is s0
__device__ __host__ __forceinline__ int64_t level_size(int64_t L, int k,
                                                       int s0) {
  if (k >= 1) L = (L + s0 - 1) / s0;
  for (int j = 1; j < k; ++j) L = (L + kStrideUp - 1) / kStrideUp;
  return L;
}

// ctr[dst] += sum of the distributed counter at ctr + dist (one block).
void sum_dist(int32_t *ctr, int dist, int dst, hipStream_t s,
              Prof *prof = nullptr);

inline unsigned grid_for(int64_t n, int block = kBlock) {
  int64_t g = (n + block - 1) / block;
  return (unsigned)(g < 1 ? 1 : g);
}

void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s,
              Prof *prof = nullptr);
void fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s,
             Prof *prof = nullptr);

// Exclusive prefix sum of int64 values (in and out may alias).  Returns the
// number of temporary bytes needed when tmp == nullptr.
size_t scan_excl_i64(const int64_t *in, int64_t *out, int64_t n, void *tmp,
                     hipStream_t s);
size_t scan_excl_u32(const uint32_t *in, uint32_t *out, int64_t n, void *tmp,
                     hipStream_t s, Prof *prof = nullptr,
                     const int32_t *gate = nullptr);

// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of the
// key.  Ping-pongs between (k0, v0) and (k1, v1); returns 0 if the result is
// in (k0, v0), 1 if in (k1, v1).  tile_cnt must hold 256 * radix_tiles(n).
int64_t radix_tiles(int64_t n);
// `gate` (nullable) points at a device word; when it is nonzero the sort's
// kernels return at once.
int radix_sort(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1,
               int64_t n, int bits, uint32_t *tile_cnt, void *scan_tmp,
               hipStream_t s, Prof *prof = nullptr,
               const int32_t *gate = nullptr, bool index_values = false);
size_t radix_scan_tmp_bytes(int64_t n);

// The parent sort of a valuation (one kernel per 8-bit pass, decoupled
// look-back).  k0[i] is the parent of the vertex at signed-order position i:
// npar for the sink, above npar for a top vertex.  Finite vertices come out
// grouped by parent, stably: position i < n_inner (*n_inner on the device,
// also in ctr[C_NINNER]) holds parent skS[i] and position svS[i]; a position
// n_inner <= i < nF = ctr[C_NFIN] holds a child of the sink, at
// svS[n_inner + nF - 1 - i].  Returns which pair holds skS/svS (1: k1/v1).
// `work` holds onesweep_words(n) words, cleared by clear_valuation since
// the last sort; a look-back that waits too long sets ERR_SORT, a finite
// count that disagrees with the keys ERR_RANKCOUNT.
int64_t onesweep_words(int64_t n);
int parent_sort(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1,
                int64_t n, uint32_t npar, int bits, uint32_t *work,
                int32_t *ctr, hipStream_t s, Prof *prof,
                const uint32_t **n_inner);
// Clears the counters (C_TOTAL words) and, unless `work` is null, the parts
// of the parent sort's work buffer for n keys that the sort needs cleared,
// in one launch.
void clear_valuation(int32_t *ctr, uint32_t *work, int64_t n, hipStream_t s,
                     Prof *prof);

}  // namespace pgk

// ---- valuation and switching (pg_val.hip) ---------------------------------
namespace pgk {
// The table entry for a rank game of n_aug vertices (pg_tune.hip).
pg_tuning tuning_for(int64_t n_aug);
bool tuning_valid(const pg_tuning &t);
// Applies t to g (rank valuations); drops captured iteration graphs.
void apply_tuning(pg_game *g, const pg_tuning &t);
// Clears the walk state; call once before a sequence of valuations.
void valuation_reset(pg_game *g, hipStream_t s);
// One valuation of the play graph held in g->sp; writes g->key.
pg_status valuation_device(pg_game *g, hipStream_t s, int64_t *n_finite_out);
// The walks and the valuation of g->sp with no host synchronisation (for
// graph capture); the counters are not read back.
void enqueue_valuation(pg_game *g, hipStream_t s);
// After a valuation whose bounded walks left vertices open (C_ABORT read
// back into g->hctr): the host-driven walks and the valuation again.
pg_status redo_valuation(pg_game *g, hipStream_t s);
// The error bits of the counters read back in g->hctr, as a status.
pg_status valuation_status(pg_game *g);
// One All_Odd (odd = true) or All_Even step on g->sp from g->key.
pg_status switch_device(pg_game *g, bool odd, hipStream_t s, int32_t *count);
// marks the vertices whose valuation (the best response's) is top, for
// later walks to stop at (g->mark_top games; see k_mark_top)
void mark_top(pg_game *g, hipStream_t s);
// forgets every vertex's fate: at the start of a solve and after each Even
// switch step (a valuation keeps the finite fates of the previous one of
// the same inner loop; valuation_reset includes this)
void fates_reset(pg_game *g, hipStream_t s);
// One best-response iteration (valuation, then All_Odd) with a single
// host synchronisation; returns the number of Odd switches and (nullable)
// the finite vertices, the sink included.  g->last_ms receives the
// iteration's device time between two HIP events on s.
pg_status iteration_device(pg_game *g, hipStream_t s, int32_t *count,
                           int64_t *n_finite = nullptr);
}  // namespace pgk

// ---- count valuations (pg_count.hip) ---------------------------------------
namespace pgk {
constexpr int kCountMax = 32;   // most distinct priorities of a count game
// After finalize_state: the distinct priorities, each vertex's column and
// the count buffers.  PG_EINVAL when more than kCountMax priorities are used.
pg_status count_setup(pg_game *g, hipStream_t s);
// walking levels of the vector list ranking for games of n_aug vertices
int count_levels(int64_t n_aug, int dw);
// level-0 stride of a count valuation's list ranking (8 or 16)
int count_stride(int64_t n_aug);
// Euler list and vector list ranking after the walks; gated by C_ABORT.
void enqueue_count(pg_game *g, hipStream_t s);
// All_Odd (odd) or All_Even on count valuations; counts into C_DIST_SW.
// fresh: the switch counters are still zero from this valuation's clearing
void enqueue_count_switch(pg_game *g, bool odd, hipStream_t s, bool fresh);
// All_Odd over a bucketed edge layout (pg_switch.hip; rank valuations).
// tsw_fits: the layout's indices fit its 32-bit fields and the device
// gives a block the stage kernel's LDS.
bool tsw_fits(int device, int64_t n_odd, int64_t m_odd);
pg_status tsw_build(pg_game *g, hipStream_t s);
// frees the layout (after the stream has drained); the row form serves
void tsw_release(pg_game *g);
void enqueue_tsw_odd(pg_game *g, hipStream_t s);
// Odd-row edges from which a single game takes the bucketed layout by
// default (smaller games read rows directly)
constexpr int64_t kTswMinEdges = int64_t(1) << 20;
// Bellman-Ford best response against the sigma in g->sp: labels into
// g->cnt, tau into g->sp, finite/top into g->rs; *rounds = Jacobi rounds.
pg_status bf_best_response(pg_game *g, hipStream_t s, int64_t *rounds);
// counts[(n_aug+1) * d] row-major (top rows zero) and top[n_aug]
pg_status export_counts(pg_game *g, int32_t *counts, uint8_t *top, bool dev,
                        hipStream_t s);
}  // namespace pgk

// ---- device memory ---------------------------------------------------------
namespace pgk {
// Size-bucketed memory for the many small games of a batch: blocks (device,
// and pinned host for the counter mirrors) go back to free lists by
// power-of-two size instead of to hipFree, which waits for the device, and
// come back from them instead of from hipMalloc.  Everything is released by
// clear() when the batch is freed.
// Blocks of up to kSlabBlockMax bytes are carved from slabs of
// kSlabBlocks blocks (one runtime allocation instead of one per block: a
// game allocates a dozen small buffers, and a first pass over many games
// otherwise pays a hipMalloc or hipHostMalloc for each); a slab goes back to
// the runtime once none of its blocks is in use.
struct DevPool {
  static constexpr size_t kSlabBlockMax = size_t(1) << 20;
  static constexpr size_t kSlabBlocks = 32;
  struct Slab {
    void *base = nullptr;
    size_t block = 0;
    bool host = false;
    int64_t in_use = 0;
  };
  std::mutex mu;           // calls on different games may overlap
  std::map<size_t, std::vector<void *>> dev_free, host_free;
  std::unordered_map<void *, size_t> dev_size, host_size;
  std::vector<Slab> slabs;
  std::unordered_map<void *, size_t> slab_of;   // block -> index in slabs
  // Bump mode (pg_solve_noalloc): blocks are carved in turn from the device
  // range [bump_dev, bump_dev + bump_cap) and the host range [bump_host,
  // bump_host + bump_hcap); nothing goes back block by block and nothing is
  // asked of the HIP runtime.
  uint8_t *bump_dev = nullptr, *bump_host = nullptr;
  size_t bump_cap = 0, bump_used = 0, bump_hcap = 0, bump_hused = 0;
  static size_t bucket(size_t bytes) {
    size_t b = 256;
    while (b < bytes) b <<= 1;
    return b;
  }
  pg_status alloc(void **p, size_t bytes, bool host);
  bool release(void *p);   // false: not a block of this pool
  void clear();            // every block, in use or not
  void trim();             // the blocks not in use
};
// The cache of the calling thread's current device that single games
// allocate from and return their memory to (see pg_release_cache).
DevPool *game_cache(int device);
// allocations of the calling thread go to this pool while it is set
extern thread_local DevPool *tl_pool;
struct PoolScope {
  DevPool *prev;
  explicit PoolScope(DevPool *p) : prev(tl_pool) { tl_pool = p; }
  ~PoolScope() { tl_pool = prev; }
};
void dev_free(void *p);            // to the current pool, else hipFree
void host_free(void *p);           // to the current pool, else hipHostFree
pg_status host_alloc(void **p, size_t bytes);
}  // namespace pgk

// ---- loading helpers shared by single games and batches (pg_api.hip) ------
namespace pgk {
__global__ void k_rv_keys(const int32_t *pri, uint32_t *sk, uint32_t *sv,
                          int64_t n);
// the admissibility preprocessing's kernels (pg_api.hip): X starts as the Odd
// vertices; a round removes members without a successor in X (wit: each
// row's last witness; ctr[C_MISC] set on a change); xp marks the members of
// X with a predecessor in X
__global__ void k_x_init(const uint8_t *owner, uint8_t *inx, int64_t n);
__global__ void k_x_round(const int64_t *off, const int32_t *tgt, uint8_t *inx,
                          uint32_t *wit, int64_t n, int32_t *ctr);
__global__ void k_xp_mark(const int64_t *off, const int32_t *tgt,
                          const uint8_t *inx, uint32_t *xp, int64_t n);
// perm/rvpos from the sorted signed keys; odd-priority count into
// C_DIST_MISC; ERR_DUPPRI on a repeat when check_dup
__global__ void k_rv_finish(const uint32_t *skS, const uint32_t *svS,
                            int32_t *perm, int32_t *rvpos, int64_t n,
                            int check_dup, int32_t *ctr);
__global__ void k_odd_flags(const uint8_t *owner, uint32_t *f, int64_t n);
__global__ void k_split_players(const uint8_t *owner, const uint32_t *oscan,
                                int32_t *odd_ids, int32_t *even_ids,
                                int64_t n);
__global__ void k_count_odd_edges(const int64_t *off, const uint8_t *owner,
                                  int64_t n, unsigned long long *out);
template <typename T>
pg_status dev_alloc(T **p, int64_t count) {
  size_t bytes = sizeof(T) * (size_t)(count > 0 ? count : 1);
  if (tl_pool) return tl_pool->alloc((void **)p, bytes, false);
  hipError_t e = hipMalloc((void **)p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return pg_fail(PG_ENOMEM, "hipMalloc of " + std::to_string(bytes) +
                                  " bytes failed: " + hipGetErrorString(e));
  }
  return PG_OK;
}
pg_status copy_in(void *dst, const void *src, size_t bytes, bool device,
                  hipStream_t s);
pg_status copy_out(void *dst, const void *src, size_t bytes, bool device,
                   hipStream_t s);
pg_status sync_ctr(pg_game *g, hipStream_t s);
void free_game(pg_game *g);
pg_status alloc_state(pg_game *g, int64_t cap);
pg_status check_err(pg_game *g, const char *what);
// flag when two neighbours of a sorted key array are equal
__global__ void k_dup_check(const uint32_t *sk, int64_t n, int32_t *flag);
// *out = max(*out, max of a[0..n)); *out must start at or below it
__global__ void k_max_i32(const int32_t *a, int64_t n, int32_t *out);
// kLoadAuto: count valuations when the input priorities repeat (sets
// g->dense); kLoadRank / kLoadCount: that representation.
enum LoadMode { kLoadRank = 0, kLoadCount = 1, kLoadAuto = 2 };
pg_status load_modified(int64_t n, int64_t m, const void *offsets,
                        const int32_t *targets, const uint8_t *owner,
                        const int32_t *priority, uint32_t flags, hipStream_t s,
                        pg_game *g, LoadMode mode);
// PG_ODD_REGION (pg_oddregion.hip): from X (inx, the vertices from which
// Odd avoids Even forever) and the validated input copies, builds the game
// without Odd's own winning region in g->off, g->tgt, g->owner, g->pri and
// the id maps g->or_new, g->or_orig; g->n_aug may be 0
pg_status odd_region_reduce(pg_game *g, hipStream_t s, int64_t n, int64_t m,
                            const int64_t *off, const int32_t *tgt,
                            const uint8_t *owner, const int32_t *pri,
                            const uint8_t *inx);
// strategies in original ids (n entries, host or device) to the reduced
// game's ids (device, n_aug entries; an entry naming a removed vertex or out
// of range becomes INT32_MAX, which import_strats rejects); and back (a
// removed vertex gets PG_SINK in both)
pg_status odd_region_strats_in(pg_game *g, const int32_t *sigma,
                               const int32_t *tau, bool dev, hipStream_t s,
                               int32_t *s2, int32_t *t2);
pg_status odd_region_strats_out(pg_game *g, const int32_t *s2,
                                const int32_t *t2, int32_t *sigma,
                                int32_t *tau, bool dev, hipStream_t s);
// winners of the reduced game (device) to the original ids (removed: Odd)
pg_status odd_region_winner_out(pg_game *g, const uint8_t *w2,
                                uint8_t *winner, bool dev, hipStream_t s);
// distinct: reject repeated priorities (rank valuations)
pg_status finalize_state(pg_game *g, hipStream_t s, bool init_sp,
                         bool distinct = true);
// A game of N vertices and M edges rebuilt with vertex i taken from vertex
// from[i] and every target t mapped to to[t]; rows keep their edge order.
// The new arrays are allocated (the old ones are the caller's).  With
// `drain` it returns after the stream has drained; without, its scratch goes
// back to the current pool at once, which is safe only when that pool is
// reused in the order of this stream (a batch's submissions).
pg_status relabel_game(const int64_t *off, const int32_t *tgt,
                       const uint8_t *owner, const int32_t *pri,
                       const int32_t *from, const int32_t *to, int64_t N,
                       int64_t M, int64_t **off2, int32_t **tgt2,
                       uint8_t **owner2, int32_t **pri2, hipStream_t s,
                       bool drain = true);
}  // namespace pgk
