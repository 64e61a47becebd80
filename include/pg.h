/*
 * pg.h -- C ABI of the MI355X parity-game strategy-improvement library.
 *
 * The library solves parity games by greedy all-switches strategy
 * improvement with one-player strategy improvement for best responses
 * (Fearnley, "Efficient Parallel Strategy Improvement for Parity Games",
 * Algorithm 1 in section 4).  Every step of that loop -- preprocessing,
 * valuation (cycle marking, nearest-greater-ancestor tree, Euler-tour list
 * construction, list ranking) and the switching rules -- runs in HIP kernels
 * on the GPU the caller's stream belongs to.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every call returns a pg_status.  Nothing throws or aborts across the
 *    ABI.  On failure pg_last_error() returns a description; it is per
 *    thread and stays valid until that thread's next call.
 *  - Vertex ids are int32.  A game may have at most 2^30 - 2 vertices after
 *    preprocessing; offsets are int64 (or int32 with PG_OFFSETS_I32).
 *  - Buffers belong to the caller.  Without PG_PTR_DEVICE in `flags` they are
 *    host pointers; with it they are device pointers on the current device
 *    (for example torch tensors' data_ptr()).  Calls that write outputs
 *    return after the outputs are written (the stream is synchronised).
 *  - `hip_stream` is a hipStream_t (NULL = the default stream).  The game's
 *    device memory is allocated by pg_load_csr and released by pg_free.
 *  - Calls on one game must not overlap; different games are independent.
 *
 * Game model (section 2, "Parity games"): vertices 0..n-1, each owned by Even
 * (0) or Odd (1), each with a priority and at least one outgoing edge.  With
 * pairwise distinct priorities the library represents a valuation by its
 * rank (rank valuations); when priorities repeat it keeps the paper's count
 * vectors (count valuations, at most 32 distinct priorities; see
 * pg_load_csr).
 *
 * The modified game (section 3, "A modified game" and "The algorithm"): a
 * sink s gets an implicit edge from every Even vertex; preprocessing then
 * appends dummy Even vertices d_w (ids n, n+1, ...) so that Odd cannot close
 * a cycle of Odd vertices against the initial strategy.  n_aug and m_aug
 * count the modified game without the sink.  Strategies and keys below are
 * indexed in the modified game; PG_SINK names the sink as a successor.
 */
#ifndef PG_H
#define PG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pg_game pg_game;

typedef enum pg_status {
    PG_OK = 0,
    PG_EINVAL = 1,          /* invalid argument or game                      */
    PG_ENOMEM = 2,          /* device or host allocation failed              */
    PG_EDEVICE = 3,         /* a HIP runtime call failed                     */
    PG_EITERLIMIT = 4,      /* an iteration cap was reached                  */
    PG_EINADMISSIBLE = 5,   /* a cycle with odd largest priority was found   */
    PG_EINTERNAL = 6        /* an internal consistency check failed          */
} pg_status;

/* Successor id meaning "the sink" in an Even entry of sigma. */
#define PG_SINK (-1)
/* Valuation key of a vertex whose play is infinite (the valuation top). */
#define PG_KEY_TOP 2147483647

enum {
    PG_PTR_DEVICE = 1u,     /* buffer arguments are device pointers          */
    PG_NO_PREPROCESS = 2u,  /* pg_load_csr: do not insert dummy vertices     */
    PG_OFFSETS_I32 = 4u,    /* pg_load_csr: offsets are int32, not int64     */
    PG_CAREFUL_WALKS = 8u,  /* pg_load_csr: host-driven walk rounds (below)  */
    PG_COUNT_VALUATION = 16u,/* pg_load_csr: count valuations (below)        */
    PG_NO_GRAPH = 32u,      /* pg_load_csr: launch every kernel one by one   */
    PG_HOST_REDUCED_LIST = 64u,/* pg_load_csr: rank the reduced list on the
                                  host (the paper's GPU-LR split; below)     */
    PG_SWITCH_ROWS = 128u,  /* pg_load_csr: All_Odd reads rows (below)       */
    PG_SWITCH_BUCKETS = 256u,/* pg_load_csr: All_Odd by buckets (below)      */
    PG_KEEP_DUMMIES = 512u, /* pg_solve: tau in the modified game's ids      */
    PG_ODD_REGION = 1024u   /* pg_load_csr: admissibility without dummies
                               (below)                                       */
};

/*
 * pg_load_csr -- validate a game and copy it to the device.
 *
 *   n, m      vertex and edge counts (n >= 1, m >= n)
 *   offsets   n+1 entries: row v is targets[offsets[v] .. offsets[v+1]);
 *             offsets[0] = 0, offsets[n] = m, every row non-empty (the paper
 *             assumes no terminal vertices, section 2)
 *   targets   m int32 successor ids in [0, n); self-loops and repeated
 *             edges are allowed
 *   owner     n bytes: 0 = Even, 1 = Odd
 *   priority  n int32 priorities, >= 0 (they may repeat; see below)
 *   flags     PG_PTR_DEVICE, PG_NO_PREPROCESS, PG_OFFSETS_I32,
 *             PG_CAREFUL_WALKS, PG_COUNT_VALUATION, PG_NO_GRAPH,
 *             PG_HOST_REDUCED_LIST, PG_SWITCH_ROWS, PG_SWITCH_BUCKETS,
 *             PG_ODD_REGION
 *
 * Two representations of valuations (section 3, "Valuations").  With
 * pairwise distinct priorities a finite valuation is the set of priorities
 * on a path and the library ranks the vertices by it (rank valuations,
 * pg_valuation).  When priorities repeat -- the paper's own setting, with a
 * handful of priorities -- or PG_COUNT_VALUATION is given, the library keeps
 * the paper's count vectors (one count per priority in use) and ranks the
 * Euler tour of the play graph's tree with vector addition (section 5,
 * "Formal reduction to list ranking"); at most 32 distinct priorities after
 * preprocessing (pg_count_info, pg_valuation_counts).
 *
 * Unless PG_NO_PREPROCESS is given, the admissibility preprocessing of
 * section 3 ("The algorithm") runs on the device: X is the largest set of
 * Odd vertices that each have a successor in X; for every w in X with a
 * predecessor in X a dummy Even vertex d_w is appended (in increasing w),
 * with the single row [w]; every edge (u, w) with u, w in X is redirected to
 * d_w in place.  With rank valuations the dummies get priorities 0, 1, ...
 * (the index of w) and the original priorities are raised by that count
 * rounded up to even; with count valuations every dummy gets priority 0 and
 * the original priorities are raised by 2 when there is a dummy.  Both keep
 * the order and parity of the original priorities below which the dummies
 * lie, so every winner is kept.
 *
 * PG_ODD_REGION replaces the dummies (section 3 offers them as one simple
 * preprocessing, not the only one): from X the load computes R, the vertices of X
 * from which Odd, moving inside X, reaches a cycle whose largest priority
 * is odd (strongly connected components of X peeled on the device by
 * colouring rounds), and A, Odd's attractor of R.  Odd wins A on its own;
 * the stored game is the original one without A (rows lose their edges
 * into A; ids renumbered in increasing original id), in which every
 * all-Odd cycle has an even largest priority, so the initial strategy is
 * admissible there and no dummy is needed.  n_aug, m_aug (pg_game_info,
 * pg_stats) are that game's sizes (n_aug may be 0: Odd wins everything) and
 * pg_export_game returns it.  Such a game takes pg_solve (and pg_stats,
 * pg_count_info, pg_*_tuning, profiling) only: pg_valuation,
 * pg_valuation_counts, pg_best_response and pg_initial_strategies give
 * PG_EINVAL, and so does a batch.  With PG_NO_PREPROCESS: PG_EINVAL.  The
 * colouring needs one round per level of the components' condensation
 * (each round removes every colour's root), so a game whose X holds long
 * chains of components loads slowly; the dummies stay the default.
 *
 * Every valuation first walks the play graph with a fixed number of device
 * rounds and falls back by itself to rounds driven from the host (each one
 * followed by a read-back of the count of open walks) when those leave work.
 * PG_CAREFUL_WALKS makes every valuation of this game take the host-driven
 * rounds directly: slower, same results; it exists to test that path.
 *
 * A best-response iteration (walks, valuation, All_Odd) of pg_solve and
 * pg_best_response is captured once per game as a HIP graph (on a stream of
 * the library's own) and replayed on the caller's stream; the event
 * profiler and the host-driven fallback launch kernels one by one.
 * PG_NO_GRAPH launches every kernel one by one: same results.
 *
 * PG_HOST_REDUCED_LIST (rank valuations; ignored for count valuations) is
 * the split of the paper's GPU-LR implementation (section 6): the device
 * builds the Euler list and sums its sublists, the host ranks the reduced
 * list (one walk from the head over a copy of it) and the device emits the
 * keys.  Same results; each valuation then waits for the host and no graph
 * is captured.  It exists to measure that split against the device-only
 * ranking.
 *
 * All_Odd (section 4) of a rank-valuation game with at least 2^20 edges in
 * Odd rows runs over a bucketed copy of those edges made at load (about
 * 24 bytes per edge): one kernel gathers the keys in target order and
 * regroups them by blocks of Odd vertices, a second takes each vertex's
 * least entry in LDS.  Same results as reading each row's keys, with
 * coalesced instead of random memory traffic.  PG_SWITCH_BUCKETS takes the
 * bucketed form at any size, PG_SWITCH_ROWS never (both: PG_EINVAL); count
 * valuations always read rows.  When the layout does not fit in device
 * memory the load keeps the row form, unless PG_SWITCH_BUCKETS asked for it
 * (then PG_ENOMEM); so does a device that cannot give one block 128 KiB of
 * LDS (with either flag setting).
 *
 * The inputs may be freed when the call returns.  Errors: PG_EINVAL for a
 * malformed game (bad offsets, a terminal vertex, a target out of range, an
 * owner not in {0,1}, a negative priority, a shifted priority above
 * INT32_MAX, too many vertices, more than 32 distinct priorities with count
 * valuations, both PG_SWITCH_ flags), PG_ENOMEM, PG_EDEVICE.
 */
pg_status pg_load_csr(int64_t n, int64_t m, const void *offsets,
                      const int32_t *targets, const uint8_t *owner,
                      const int32_t *priority, uint32_t flags,
                      void *hip_stream, pg_game **out_game);

/*
 * pg_count_info -- *d = the number of distinct priorities of the modified
 * game when it uses count valuations, else 0; values (nullable, room for 32)
 * receives them in increasing order: column j of a count row counts
 * values[j].
 */
pg_status pg_count_info(const pg_game *game, int32_t *d, int32_t *values);

/* Sizes of the original and the modified game (any pointer may be NULL). */
pg_status pg_game_info(const pg_game *game, int64_t *n, int64_t *m,
                       int64_t *n_aug, int64_t *m_aug);

/*
 * pg_export_game -- copy the modified game out (for inspection and tests).
 *   offsets  n_aug+1 int64;  targets  m_aug int32;  owner  n_aug bytes;
 *   priority n_aug int32.   Any pointer may be NULL.
 */
pg_status pg_export_game(const pg_game *game, int64_t *offsets,
                         int32_t *targets, uint8_t *owner, int32_t *priority,
                         uint32_t flags, void *hip_stream);

/*
 * pg_initial_strategies -- the strategies Algorithm 1 starts from:
 * sigma_init(v) = PG_SINK for every Even vertex (section 3, "The
 * algorithm"), and for every Odd vertex the first entry of its row (the
 * "arbitrary" initial Odd strategy of Algorithm 1).  sigma and tau have
 * n_aug entries; entries of the other player are PG_SINK.
 */
pg_status pg_initial_strategies(pg_game *game, int32_t *sigma, int32_t *tau,
                                uint32_t flags, void *hip_stream);

/*
 * pg_valuation -- one valuation Val^{sigma,tau} (section 3, "Valuations";
 * computed as in section 5).
 *
 *   sigma   n_aug entries; for Even vertices a successor id or PG_SINK
 *   tau     n_aug entries; for Odd vertices a successor id
 *           (entries of the other player are ignored; every chosen successor
 *           must be an edge of the modified game -- this is not checked)
 *   key     n_aug+1 outputs: for a vertex whose play reaches the sink, the
 *           rank of its valuation among all such vertices and the sink
 *           (0 = smallest in the paper's order); PG_KEY_TOP for an infinite
 *           play.  key[n_aug] is the sink's own rank.
 *   n_finite (nullable) number of finite entries of key (the sink included)
 *
 * Returns PG_EINADMISSIBLE if the play graph has a cycle whose largest
 * priority is odd (sigma is not admissible, section 3); key is then
 * unspecified.  PG_EINVAL for a game with count valuations.
 */
pg_status pg_valuation(pg_game *game, const int32_t *sigma,
                       const int32_t *tau, int32_t *key, int64_t *n_finite,
                       uint32_t flags, void *hip_stream);

/*
 * pg_valuation_counts -- one valuation of a count-valuation game as the
 * paper defines it (section 3, "Valuations"), computed by list ranking the
 * Euler tour of the tree of finite vertices with vector addition (section 5,
 * "Formal reduction to list ranking"; the list is built with the atomic
 * exchange of "Constructing the list ranking instance in parallel").
 *
 *   sigma, tau  as in pg_valuation
 *   counts      (n_aug+1) * d int32, row-major: row v holds, for each
 *               column j, how many vertices of priority values[j]
 *               (pg_count_info) the play from v visits before the sink; row
 *               n_aug is the sink's (zero); rows of top vertices are zero
 *   top         (nullable) n_aug bytes: 1 where the play is infinite (top)
 *   n_finite    (nullable) vertices with a finite play, the sink included
 *
 * PG_EINVAL for a game with rank valuations; PG_EINADMISSIBLE as in
 * pg_valuation.
 */
pg_status pg_valuation_counts(pg_game *game, const int32_t *sigma,
                              const int32_t *tau, int32_t *counts,
                              uint8_t *top, int64_t *n_finite, uint32_t flags,
                              void *hip_stream);

/*
 * pg_best_response -- the inner loop of Algorithm 1: one-player strategy
 * improvement for Odd against a fixed admissible sigma (section 4).  Starting
 * from tau, it repeats valuation and All_Odd -- every Odd vertex whose row
 * has a successor of strictly smaller key moves to the first such successor
 * of least key -- until no Odd vertex switches.
 *
 *   sigma         n_aug entries (as in pg_valuation), admissible
 *   tau           n_aug entries; in: the start strategy; out: br(sigma)
 *   key           n_aug+1 outputs (nullable): Val^{sigma, br(sigma)} as
 *                 ranks; must be NULL for a count-valuation game (whose
 *                 valuations compare count rows by Maxdiff instead of keys)
 *   n_valuations  (nullable) number of valuations computed
 *   max_inner     cap on valuations (0 = none); PG_EITERLIMIT when reached
 */
pg_status pg_best_response(pg_game *game, const int32_t *sigma, int32_t *tau,
                           int32_t *key, int32_t *n_valuations,
                           int32_t max_inner, uint32_t flags,
                           void *hip_stream);

/*
 * Best responses of pg_solve (section 4; section 6 compares the three):
 *   PG_BR_SI             one-player strategy improvement, each best response
 *                        starting from the previous one (Algorithm 1)
 *   PG_BR_SI_RESET       the same, each best response starting again from
 *                        the initial Odd strategy (first entry of each row)
 *   PG_BR_BELLMAN_FORD   shortest paths to the sink under the valuation
 *                        order by Jacobi rounds of Bellman-Ford (count
 *                        valuations only); tau(v) is then the first row
 *                        position of least valuation.  n_valuations counts
 *                        its rounds.
 * All three give the same valuations, hence the same outer iterations,
 * final sigma and winners; tau can differ where successors tie.
 */
enum {
    PG_BR_SI = 0,
    PG_BR_SI_RESET = 1,
    PG_BR_BELLMAN_FORD = 2
};

typedef struct pg_solve_opts {
    int32_t max_major;      /* cap on outer iterations (0 = none)            */
    int32_t max_inner;      /* cap on valuations per best response (0=none)  */
    uint32_t flags;         /* PG_PTR_DEVICE for init_sigma, init_tau and the
                               output buffers; PG_KEEP_DUMMIES (below)       */
    int32_t best_response;  /* PG_BR_* (0 = PG_BR_SI)                        */
    /* Warm start (nullable; n_aug entries each, in the modified game's ids
     * as pg_valuation takes them): the run starts from these strategies
     * instead of sigma_init and the first entry of every row.  init_sigma
     * must be admissible (section 3).  A run stopped by a cap hands back
     * its current strategies (pg_solve, PG_EITERLIMIT); started from them
     * with PG_KEEP_DUMMIES it continues exactly where it stopped.          */
    const int32_t *init_sigma;
    const int32_t *init_tau;
    /* Per-valuation trace (host arrays, each nullable, trace_cap entries;
     * entry i belongs to the i-th valuation of the run; beyond trace_cap
     * nothing is written; stats->n_traced says how many were):
     *   trace_key_hash   h = h * 1099511628211 + (uint32_t)key[v] + 1 over
     *                    the keys of pg_valuation's output, v = 0..n_aug
     *                    (the sink last), starting from h = 0, modulo 2^64
     *                    (rank valuations; 0 for count valuations; computed
     *                    on the device, one extra kernel per valuation)
     *   trace_finite     vertices with a finite play, the sink included
     *   trace_switches   Odd vertices switched by the All_Odd step that
     *                    follows the valuation (0 ends a best response)
     *   trace_ms         device time of the best-response iteration (the
     *                    valuation and its All_Odd step) between two HIP
     *                    events on the call's stream                      */
    int32_t trace_cap;
    int32_t reserved;
    uint64_t *trace_key_hash;
    int64_t *trace_finite;
    int64_t *trace_switches;
    float *trace_ms;
} pg_solve_opts;

typedef struct pg_stats {
    int64_t n, m, n_aug, m_aug;
    int64_t n_major;        /* outer iterations, the final one included      */
    int64_t n_valuations;   /* valuations over the whole solve               */
    int64_t n_odd_switches; /* vertices switched by All_Odd, summed          */
    int64_t n_even_switches;/* vertices switched by All_Even, summed         */
    double seconds;         /* wall time of the solve on the host clock      */
    double iteration_ms;    /* device time of the best-response iterations,
                               summed (HIP events on the call's stream
                               around each; 0 for Bellman-Ford and batches) */
    int64_t n_traced;       /* entries written to the trace arrays           */
} pg_stats;

/*
 * pg_solve -- Algorithm 1 from the initial strategies (or opts->init_sigma,
 * opts->init_tau) to the end.  The outer
 * loop switches Even by greedy all-switches (section 3, "Switching rules"):
 * among the sink (option 0) and the row, the first option of greatest
 * valuation replaces sigma(v) if its valuation is strictly greater.  It
 * stops when no Even vertex switches; by Theorem 1 the vertices whose
 * valuation is then top are exactly Even's winning set.
 *
 *   opts     nullable (no caps; host outputs; PG_BR_SI).  PG_EINVAL for
 *            PG_BR_BELLMAN_FORD on a game with rank valuations or a
 *            negative trace_cap.  The trace covers the iterations of one-
 *            player strategy improvement (Bellman-Ford rounds are not
 *            traced).
 *   winner   n outputs (original vertices): 0 = W_Even, 1 = W_Odd
 *   sigma    n_aug outputs (nullable): the final sigma* (PG_SINK for the
 *            sink); vertices Even wins never map to the sink
 *   tau      n_aug outputs (nullable): the final tau* = br(sigma*), with
 *            an Odd choice of a dummy d_w given as w (the dummy only stands
 *            in the middle of the original edge to w), so the Odd choices of
 *            the n original vertices are edges of the original game; with
 *            PG_KEEP_DUMMIES in opts->flags the dummy itself (the form
 *            pg_best_response and init_tau use)
 *   stats    nullable
 *
 * For a game loaded with PG_ODD_REGION, winner, sigma and tau (and
 * init_sigma, init_tau) have n entries in the original ids: a vertex of
 * Odd's own region A has winner 1 and PG_SINK in sigma and tau, the others
 * the results of the game without A, whose strategies never lead into A.
 * A start strategy that chooses a vertex of A: PG_EINVAL.
 *
 * When a cap stops the run (PG_EITERLIMIT: max_major outer iterations
 * done, or max_inner valuations in one best response), winner is not
 * written, but sigma and tau (when given) receive the strategies reached:
 * a checkpoint.  A later pg_solve with them as init_sigma and init_tau
 * (PG_KEEP_DUMMIES form) takes exactly the remaining iterations of the
 * uninterrupted run.
 */
pg_status pg_solve(pg_game *game, const pg_solve_opts *opts, uint8_t *winner,
                   int32_t *sigma, int32_t *tau, pg_stats *stats,
                   void *hip_stream);

/*
 * Kernel profiling.  When enabled, every kernel the library launches for this
 * game is bracketed by two HIP events on the call's stream, and after each
 * synchronisation the elapsed times are added up per kernel kind together
 * with the kernel's algorithmic bytes (the bytes the step must move, as
 * computed from its sizes; not measured traffic).
 *
 * pg_profile_enable: on != 0 enables and clears the counters; 0 disables.
 * pg_profile_kinds:  number of kernel kinds.
 * pg_profile_read:   totals for one kind: name (static string), summed
 *                    milliseconds, launches, summed algorithmic bytes.
 */
pg_status pg_profile_enable(pg_game *game, int32_t on);
int32_t pg_profile_kinds(void);
pg_status pg_profile_read(const pg_game *game, int32_t kind, const char **name,
                          double *ms, int64_t *calls, double *bytes);

/*
 * Batched and continuously served solving.  A batch is an arena on the
 * device that holds many games at once; one pg_batch_step advances every game
 * in it by one best-response iteration of Algorithm 1 (a valuation, All_Odd,
 * and All_Even for the games whose All_Odd switched nothing), all games in
 * the same kernel launches.  Each game follows its own copy of Algorithm 1,
 * so its strategies, winners and counts are those pg_solve gives it alone.
 *
 * pg_batch_create  an arena for up to max_vertices / max_edges of modified
 *                  games (the HBM footprint budget) and max_games games.
 * pg_batch_submit  (may be called from another thread than the other
 *                  pg_batch_* calls: it works on a stream of the batch's
 *                  own and takes the batch's lock only to queue the game)
 *                  validates and preprocesses one game (arguments as
 *                  pg_load_csr) and queues it; returns a ticket.  PG_ENOMEM
 *                  if the game alone exceeds the arena; PG_EINVAL for
 *                  repeated priorities (batches take games with rank
 *                  valuations only: the arena ranks all its games together,
 *                  and for PG_ODD_REGION).
 *                  Queued games join the arena, first come first served, at
 *                  a step where they fit beside the games already in it.  A
 *                  game's memory comes from a pool that the batch keeps
 *                  until pg_batch_free.
 * pg_batch_submit_many  submits count games at once (arrays of their
 *                  arguments; flags shared): the same checks, preprocessing
 *                  and queueing as count pg_batch_submit calls in order, but
 *                  done together over the games' disjoint union, a few dozen
 *                  kernels and a handful of synchronisations for the whole
 *                  call instead of for each game.  status[i] is game i's
 *                  outcome (as pg_batch_submit would return it) and
 *                  tickets[i] its ticket (-1 if refused; pg_last_error
 *                  holds the message of a refused game).  The call returns
 *                  PG_OK when every game got its status, else the error
 *                  that stopped it (games not queued then carry it too).
 *                  Games larger than 2^29 - 1 vertices: PG_EINVAL.
 * pg_batch_step    lays the arena out again when finished games hold a
 *                  quarter of it, or to admit queued games that fit: once
 *                  they add up to an eighth of the arena's vertices, once
 *                  one has waited 8 steps, or when no game is running; then
 *                  advances every live game once.  Outputs (nullable):
 *                  games running, games queued, games finished by this
 *                  step.
 * pg_batch_poll    done = 1 once the game has finished; then writes its
 *                  winner (n), sigma and tau (n_aug, as pg_solve) and
 *                  stats, and releases the ticket.  With winner, sigma and
 *                  tau all NULL it only reports done and stats and keeps the
 *                  ticket (a query, to size the outputs).  flags:
 *                  PG_PTR_DEVICE for device output buffers.
 * pg_batch_poll_many  the same for count tickets at once (arrays of
 *                  output pointers, each array and each entry nullable):
 *                  one wait for all the copies.  PG_EINVAL for an unknown
 *                  ticket, before anything is written.
 * pg_batch_finished  tickets of finished games not yet polled (up to
 *                  capacity of them; *count = how many there are).
 * pg_batch_info    games running and queued, current arena size.
 * pg_batch_free    releases everything, including unpolled games.
 *
 * Calls on one batch must not overlap.
 */
typedef struct pg_batch pg_batch;
pg_status pg_batch_create(int64_t max_vertices, int64_t max_edges,
                          int32_t max_games, void *hip_stream,
                          pg_batch **out);
pg_status pg_batch_submit(pg_batch *batch, int64_t n, int64_t m,
                          const void *offsets, const int32_t *targets,
                          const uint8_t *owner, const int32_t *priority,
                          uint32_t flags, int64_t *ticket);
pg_status pg_batch_submit_many(pg_batch *batch, int32_t count,
                               const int64_t *n, const int64_t *m,
                               const void *const *offsets,
                               const int32_t *const *targets,
                               const uint8_t *const *owner,
                               const int32_t *const *priority, uint32_t flags,
                               int64_t *tickets, pg_status *status);
pg_status pg_batch_step(pg_batch *batch, int32_t *n_live, int32_t *n_queued,
                        int32_t *n_finished);
pg_status pg_batch_poll(pg_batch *batch, int64_t ticket, int32_t *done,
                        uint8_t *winner, int32_t *sigma, int32_t *tau,
                        pg_stats *stats, uint32_t flags);
pg_status pg_batch_poll_many(pg_batch *batch, int32_t count,
                             const int64_t *tickets, int32_t *done,
                             uint8_t *const *winner, int32_t *const *sigma,
                             int32_t *const *tau, pg_stats *stats,
                             uint32_t flags);
pg_status pg_batch_finished(const pg_batch *batch, int64_t *tickets,
                            int32_t capacity, int32_t *count);
pg_status pg_batch_info(const pg_batch *batch, int32_t *n_live,
                        int32_t *n_queued, int64_t *arena_vertices,
                        int64_t *arena_edges);
pg_status pg_batch_free(pg_batch *batch);

/*
 * pg_solve_noalloc -- pg_load_csr, pg_solve and the release of the game in
 * one call that allocates nothing: for callers that cannot allocate device
 * memory (tight serving loops that must not call hipMalloc or hipFree,
 * harnesses that forbid allocation).  Same arguments, results and errors
 * as pg_load_csr followed by pg_solve, with these limits:
 *
 *   size     n <= PG_NOALLOC_MAX_VERTICES, m <= PG_NOALLOC_MAX_EDGES, else
 *            PG_EINVAL (load larger games with pg_load_csr).  A game
 *            within them fits the scratch below; PG_ENOMEM if not.
 *   scratch  every device buffer of the load and the solve is carved from
 *            one static device array of PG_NOALLOC_SCRATCH_MIB MiB (held by
 *            each GPU the library runs on until the process ends), the
 *            counter mirror from a static host buffer; the game descriptor
 *            lives on the call's stack.  No hipMalloc, hipFree, pinned host
 *            allocation, HIP event or graph.
 *   sharing  all calls on one GPU share that GPU's scratch, which keeps the
 *            last call's contents (everything a call reads it writes
 *            first): calls that overlap on one GPU, from two threads or on
 *            two streams, race.  Calls on different GPUs do not.
 *   forms    All_Odd reads rows (PG_SWITCH_ROWS); PG_SWITCH_BUCKETS and
 *            PG_HOST_REDUCED_LIST are refused (PG_EINVAL), and so is a
 *            per-valuation trace in opts.  Iterations are not timed
 *            (stats->iteration_ms = 0).
 *
 * sigma and tau (nullable) need room for n_aug entries, which the caller
 * does not know before the load: n_aug <= 2 n (one dummy at most per
 * original vertex), and stats->n_aug (when stats is given) says how many
 * were written; with PG_ODD_REGION n entries, as pg_solve.  The call returns after the stream has drained; outputs are
 * written then.
 */
#define PG_NOALLOC_MAX_VERTICES 65536
#define PG_NOALLOC_MAX_EDGES 1048576
#define PG_NOALLOC_SCRATCH_MIB 128
pg_status pg_solve_noalloc(int64_t n, int64_t m, const void *offsets,
                           const int32_t *targets, const uint8_t *owner,
                           const int32_t *priority, uint32_t flags,
                           const pg_solve_opts *opts, uint8_t *winner,
                           int32_t *sigma, int32_t *tau, pg_stats *stats,
                           void *hip_stream);

/*
 * Tuning of the rank valuation (games with distinct priorities): launch and
 * walk parameters that change the speed of a valuation, never its result.
 * pg_load_csr (and each batch arena) takes them from a table measured on
 * MI355X per size class of n_aug (pg_tuning_table);
 * paper_1705_02313_amd/tune.py measures the table again.
 *
 *   stride0      list ranking (section 5, "List ranking"): every stride0-th
 *                element of the Euler list is a splitter; 8, 16, 32 or 64
 *   per_thread   level-1 sublists walked by one thread: 1, 2, 4 or 8
 *   walk_full    plain play steps of the full ng pass and ng-chain steps
 *                of the full root pass: 2..64
 *   walk_round   shortcut steps of one later round: 8..256
 *   walk_rounds  rounds enqueued before the host looks: 1..8 (a vertex
 *                still open after them is finished on the host-driven path)
 *   walk_block   threads per block of the full ng and root passes: 64, 128
 *                or 256
 *
 * pg_set_tuning: PG_EINVAL for a value outside these sets or a game with
 * count valuations; the new values serve the next valuation (a captured
 * iteration graph is captured again).
 * pg_tuning_table: copies up to `capacity` entries (nullable arrays) and
 * returns the table's length; entry i serves games with n_aug >= min_n_aug[i]
 * below the next entry's bound.
 */
typedef struct pg_tuning {
    int32_t stride0;
    int32_t per_thread;
    int32_t walk_full;
    int32_t walk_round;
    int32_t walk_rounds;
    int32_t walk_block;
} pg_tuning;

pg_status pg_get_tuning(const pg_game *game, pg_tuning *tuning);
pg_status pg_set_tuning(pg_game *game, const pg_tuning *tuning);
int32_t pg_tuning_table(pg_tuning *entries, int64_t *min_n_aug,
                        int32_t capacity);

/* Release the game.  NULL is accepted.  Its device and pinned host memory
 * goes to a per-device cache that later pg_load_csr calls on that device
 * take their memory from (blocks are returned only after the device has
 * finished with them), so loading many games does not pay hipMalloc and
 * hipFree for each. */
pg_status pg_free(pg_game *game);

/* Hand the cached memory of freed games back to the HIP runtime (every
 * device).  Memory of games still loaded is not touched.  Small blocks are
 * carved from shared slabs of 32; a slab goes back once none of its blocks
 * belongs to a loaded game (its free blocks stay cached until then). */
pg_status pg_release_cache(void);

/* Description of the calling thread's last error ("" if none). */
const char *pg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PG_H */
