// Launch and walk parameters of the rank valuation per size class.
//
// The entries below were measured on one MI355X by
// paper_1705_02313_amd/tune.py (which rewrites this table): for each size
// class a random game of that size is solved under candidate parameters,
// one parameter at a time from the previous best, and the set with the
// least device time per best-response iteration is kept.  Every candidate
// must give the same valuations, strategies and counts (the parameters
// change only how the work is split and scheduled).
#include "pg_common.h"

namespace pgk {

namespace {
struct TuneEntry {
  int64_t min_n_aug;
  pg_tuning t;   // stride0, per_thread, walk_full, walk_round, walk_rounds,
                 // walk_block
};

// BEGIN TABLE (tune.py)
const TuneEntry kTuneTable[] = {
    {0, {8, 1, 16, 128, 2, 64}},
    {4096, {8, 1, 16, 128, 2, 256}},
    {32768, {8, 1, 8, 128, 2, 256}},
    {262144, {8, 1, 12, 128, 2, 128}},
    {1048576, {16, 1, 8, 128, 2, 256}},
    {4194304, {8, 4, 12, 32, 2, 256}},
    {8388608, {16, 8, 24, 128, 2, 64}},
};
// END TABLE
constexpr int kTuneEntries = (int)(sizeof(kTuneTable) / sizeof(kTuneTable[0]));

bool pow2_in(int32_t v, int32_t lo, int32_t hi) {
  return v >= lo && v <= hi && (v & (v - 1)) == 0;
}
}  // namespace

bool tuning_valid(const pg_tuning &t) {
  return pow2_in(t.stride0, kStrideMin, 64) && pow2_in(t.per_thread, 1, 8) &&
         t.walk_full >= 2 && t.walk_full <= 64 && t.walk_round >= 8 &&
         t.walk_round <= 256 && t.walk_rounds >= 1 && t.walk_rounds <= 8 &&
         pow2_in(t.walk_block, 64, kBlock);
}

pg_tuning tuning_for(int64_t n_aug) {
  int k = 0;
  while (k + 1 < kTuneEntries && n_aug >= kTuneTable[k + 1].min_n_aug) ++k;
  return kTuneTable[k].t;
}

void apply_tuning(pg_game *g, const pg_tuning &t) {
  g->tune = t;
  // captured iterations carry the old launch shapes: capture again
  if (g->iter_exec) {
    (void)hipGraphExecDestroy(g->iter_exec);
    g->iter_exec = nullptr;
  }
}

}  // namespace pgk

extern "C" {

pg_status pg_get_tuning(const pg_game *g, pg_tuning *t) {
  if (!g || !t) return pg_fail(PG_EINVAL, "NULL argument");
  *t = g->tune;
  return PG_OK;
}

pg_status pg_set_tuning(pg_game *g, const pg_tuning *t) {
  if (!g || !t) return pg_fail(PG_EINVAL, "NULL argument");
  if (g->dense)
    return pg_fail(PG_EINVAL, "tuning applies to rank valuations");
  if (g->n_aug == 0)
    return pg_fail(PG_EINVAL, "no vertex is left to solve in this game");
  if (!pgk::tuning_valid(*t))
    return pg_fail(PG_EINVAL, "a tuning value is outside its range");
  // a graph may still run on the game's stream: drain it before the
  // captured graphs go
  (void)hipDeviceSynchronize();
  pgk::apply_tuning(g, *t);
  return PG_OK;
}

int32_t pg_tuning_table(pg_tuning *entries, int64_t *min_n_aug,
                        int32_t capacity) {
  for (int i = 0; i < pgk::kTuneEntries && i < capacity; ++i) {
    if (entries) entries[i] = pgk::kTuneTable[i].t;
    if (min_n_aug) min_n_aug[i] = pgk::kTuneTable[i].min_n_aug;
  }
  return pgk::kTuneEntries;
}

}  // extern "C"
