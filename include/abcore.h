/*
 * abcore.h -- C ABI of libabcore, (alpha,beta)-core computation and
 * on-the-fly edge queries on bipartite graphs, for AMD Instinct MI355X
 * (gfx950).  Method: Feng et al., "Efficient (alpha,beta)-core Computation
 * and On-the-fly Query at Billion Scale with GPUs".
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Vertices use unified ids (Sec. IV-A): upper vertex u is id u in
 *    [0, n_upper); lower vertex v is id n_upper + v.  Edge endpoints in the
 *    API are given per layer: u in [0, n_upper), v in [0, n_lower).
 *  - Membership bitmasks are arrays of ceil(n/32) uint32 words in DEVICE
 *    memory owned by the caller; bit (x % 32) of word x / 32 (least
 *    significant bit first) is 1 iff vertex x belongs to the result.  Padding
 *    bits past n are written as 0.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it; calls documented as synchronous also wait for it.
 *  - Every entry point returns an abcore_status and never throws.  On any
 *    error no state changes: a rejected update is not applied.  The message
 *    of the last error of the calling thread is abcore_last_error().
 *  - A handle is not thread-safe: calls on one handle must be serialised by
 *    the caller.  Handles own all of their device memory.
 *  - All arithmetic is integer; results are exact and independent of thread
 *    scheduling (the (alpha,beta)-core is unique, Definition 1).
 */
#ifndef ABCORE_H
#define ABCORE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct abcore_graph_s *abcore_graph;

typedef enum {
  ABCORE_OK = 0,
  ABCORE_EINVAL = 1,  /* bad argument: null pointer, id out of range, alpha or beta 0 */
  ABCORE_ENOMEM = 2,  /* device or host allocation failed */
  ABCORE_EDEVICE = 3, /* a HIP call failed */
  ABCORE_ENOENT = 4,  /* deletion of an edge that is not present */
  ABCORE_EEXIST = 5,  /* insertion of an edge that is already present */
  ABCORE_EBUSY = 6,   /* no admission slot free, or the handle is serving */
  ABCORE_EAGAIN = 7,  /* abcore_poll: the request has not finished yet */
  ABCORE_ETIMEDOUT = 8 /* abcore_poll: past its deadline, query dropped */
} abcore_status;

/* Algorithms of Sec. IV. */
enum { ABCORE_GCC = 0, ABCORE_GCC_PLUS = 1 };

/* Counters of one computation (filled when a stats pointer is passed; that
 * forces a synchronisation of the stream). */
typedef struct {
  int64_t removed;        /* vertices outside the result (|V| - |core|) */
  int64_t rounds;         /* peel rounds (frontier generations) */
  int64_t entries_read;   /* adjacency entries read by the peel */
  int64_t initial;        /* vertices in the first frontier (scan phase) */
  int64_t uncertain;      /* GCC+: vertices with delta_l <= core < delta_q */
  int64_t launches;       /* kernels launched for the peel phase */
  int64_t pulled;         /* 1 if the first round ran in pull form */
  int64_t rank_order;     /* 1 if the query ran on the degree-rank relabelling
                             of an unchanged graph (survivors of the scan are
                             the vertices of degree >= threshold, Sec. IV-A) */
} abcore_stats;

/* One edge update for the on-the-fly query (Problem 2, Sec. III). */
typedef struct {
  int32_t u;  /* upper index in [0, n_upper) */
  int32_t v;  /* lower index in [0, n_lower) */
  int32_t op; /* +1 insertion, -1 deletion */
} abcore_edge_update;

/* Message describing the last error on this thread ("" if none). */
const char *abcore_last_error(void);

/* Graph construction (Sec. III: CSR storage; Sec. IV-A: unified ids).
 * d_eu, d_ev: DEVICE arrays of m int32 endpoints (u in [0,n_upper), v in
 * [0,n_lower)), read during the call and not retained.  Duplicate pairs are
 * removed (the edge set E is a set).  Builds one CSR over unified ids holding
 * both adjacencies, rows sorted ascending.  Requires n_upper, n_lower >= 0,
 * n_upper + n_lower < 2^31 and m < 2^31.  Synchronous.
 * out: receives the handle.  out_m_distinct (nullable): distinct edge count.
 * Errors: EINVAL (null pointer, negative size, id out of range), ENOMEM,
 * EDEVICE. */
abcore_status abcore_build_csr(int32_t n_upper, int32_t n_lower, const int32_t *d_eu,
                               const int32_t *d_ev, int64_t m, void *stream,
                               abcore_graph *out, int64_t *out_m_distinct);

/* What a handle's build cost and what it holds (the paper reports GPU
 * memory per dataset, Sec. VI Fig. 4; Table II separates preprocessing from
 * query time).  Times are wall-clock milliseconds of abcore_build_csr's
 * phases, each ended by a synchronisation: the CSR (dedupe, both
 * adjacencies), the row pieces, and the degree-rank copy -- an optional
 * index the build adds for queries on an unchanged graph (0 when the build
 * skipped it); Algorithm 1 itself needs none of it.  Bytes: the graph (CSR
 * offsets and columns, degrees, row pieces), the degree-rank copy, and the
 * frontier sub-queues of the handle's working set. */
typedef struct {
  double build_ms;      /* whole abcore_build_csr */
  double csr_ms;        /* dedupe and the unified CSR */
  double pieces_ms;     /* row pieces of rows longer than 64 entries */
  double ranks_ms;      /* degree-rank copy and its tables */
  int64_t graph_bytes;  /* off, cols, deg0, row pieces */
  int64_t ranks_bytes;  /* degree-rank copy: ranks, relabelled CSR, pieces, degree slots */
  int64_t queue_bytes;  /* frontier sub-queues of the handle's working set */
  /* last core decomposition's h-index phase (zeros if it did not run):
   * switch level k0, vertices of the k0-core, the adjacency slots it used
   * (its vertices' degrees in the graph), half sweeps (one layer each) */
  int64_t core_top[4];
  double core_levels_ms;  /* levels peeled before the switch (wall clock) */
  double core_top_ms;     /* the h-index phase (wall clock) */
} abcore_report;

abcore_status abcore_graph_report(abcore_graph g, abcore_report *out);

/* Device memory the library holds, summed over all handles and devices:
 * current bytes and the peak since the last reset (reset_peak != 0 sets the
 * peak to the current value after reading).  Host bookkeeping only. */
abcore_status abcore_device_memory(int64_t *current, int64_t *peak, int32_t reset_peak);

/* Process-wide cap on the device bytes the library holds (every handle and
 * device together; 0 = none, the default).  An allocation that would exceed
 * it fails as out of memory: the entry point that needed it returns
 * ABCORE_ENOMEM and changes nothing (a build creates no handle; a computation
 * leaves the handle as it was), except abcore_serve_start, which admits with
 * fewer device working sets when at least one fits (see there).  Lowering
 * the budget frees nothing.  Errors: EINVAL (negative). */
abcore_status abcore_set_memory_budget(int64_t bytes);

/* Releases every resource of the handle.  NULL is accepted. */
abcore_status abcore_destroy(abcore_graph g);

/* Debug builds only (libabcore_debug.so, compiled with ABC_DEBUG_ENQUEUE):
 * every vertex id appended to the frontier queues is counted per vertex, so
 * that a test can check the crossing rule of Algorithm 1's peel -- a vertex
 * is queued when its degree crosses its threshold, once -- and the scan's
 * frontier.  The counts accumulate over computations on the handle.
 * d_counts (DEVICE int32[n], nullable) receives them; reset != 0 zeroes them
 * afterwards.  Synchronous on `stream`.  Errors: EINVAL (null handle, or a
 * release build, which keeps no counts), EBUSY (serving), EDEVICE. */
abcore_status abcore_debug_enqueue_counts(abcore_graph g, int32_t *d_counts, int32_t reset,
                                          void *stream);

/* Sizes: n_upper, n_lower and the current number of distinct edges. */
abcore_status abcore_graph_info(abcore_graph g, int32_t *n_upper, int32_t *n_lower,
                                int64_t *m);

/* Copies the current CSR to DEVICE buffers: d_off (n+1 int64) and d_cols
 * (2m int32), rows sorted ascending, edges inserted after the build included
 * and deleted ones left out.  Either pointer may be NULL to only query
 * *out_entries (= 2m).  Synchronous. */
abcore_status abcore_export_csr(abcore_graph g, int64_t *d_off, int32_t *d_cols,
                                int64_t *out_entries, void *stream);

/* Problem 1 of Sec. III: the vertex set of the (alpha,beta)-core
 * (Definition 1).  algo = ABCORE_GCC runs the scan and peel phases of
 * Algorithm 1 (Sec. IV-A); ABCORE_GCC_PLUS runs Algorithm 2 (Sec. IV-B):
 * core-number classification by Lemma 1, then the peel restricted to the
 * vertices with min(alpha,beta) <= core < max(alpha,beta), whose degrees
 * count only neighbours with core >= min(alpha,beta).  GCC+ computes and
 * caches the core numbers on first use (abcore_core_numbers).
 * alpha, beta >= 1 (EINVAL otherwise).  d_bitmask: DEVICE, ceil(n/32)
 * words, every word written.  stats: nullable.  Asynchronous on `stream`
 * unless stats is requested. */
abcore_status abcore_compute(abcore_graph g, uint32_t alpha, uint32_t beta, int32_t algo,
                             uint32_t *d_bitmask, abcore_stats *stats, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the GCC
 * computation of abcore_compute(g, alpha, beta, ABCORE_GCC, d_bitmask, NULL,
 * stream), bit for bit, with no allocation and no free of any kind.  Its
 * per-query working set (working degrees, frontier sub-queues, peel state,
 * partial sums, survivor bitmap) lives in a static device array of 64 MiB
 * that the library holds on every device it runs on until the process ends;
 * the handle's graph arrays are read only.  It fits graphs whose working set,
 * 4 * (2n + pieces) + 4.125 n bytes plus about 600 KB (pieces: one per 64
 * adjacency entries of each row longer than 64), is at most 64 MiB -- about
 * 5,000,000 vertices at the degree skew of a power-law graph; larger graphs
 * return ABCORE_EINVAL and change nothing.  Every call on a device
 * shares that device's array and starts by filling it afresh (queue slots
 * empty, state zero), with kernels only (no memset node), on `stream`:
 * calls that overlap on one device, on any handles or streams, race, and
 * the caller must serialise them.  Asynchronous on `stream`.  Errors: EINVAL
 * (null handle or bitmask, alpha or beta 0, graph too large), EBUSY
 * (serving), EDEVICE. */
abcore_status abcore_compute_static(abcore_graph g, uint32_t alpha, uint32_t beta,
                                    uint32_t *d_bitmask, void *stream);

/* Batch of q queries (thresholds h_alpha[i], h_beta[i], HOST arrays of q
 * values >= 1) computed in one call.  Result i is written to d_bitmasks +
 * i * ceil(n/32) (DEVICE, q * ceil(n/32) words, every word written) and equals
 * abcore_compute(g, h_alpha[i], h_beta[i], ...) bit for bit.
 * Method: the cores are nested -- the (a,b)-core lies inside the
 * (a',b')-core whenever a' <= a and b' <= b, the property behind Lemma 1's
 * proof (Sec. IV-B).  Each query starts from the final degrees and
 * survivors of a query it dominates and peels only the difference
 * (Algorithm 1's scan and peel on that state); equal queries share one
 * computation.  The plan is abcore_batch_plan's.  The working degrees need
 * `states` buffers of n int32, allocated on first use and kept by the handle
 * (ENOMEM if they do not fit).  In the default peel mode the whole batch is
 * captured into one HIP graph, cached for the same thresholds, output pointer
 * and graph version, and replayed.  Synchronous.
 * Errors: EINVAL (null pointer, q < 0, a threshold 0), ENOMEM, EDEVICE. */
abcore_status abcore_compute_batch(abcore_graph g, const uint32_t *h_alpha,
                                   const uint32_t *h_beta, int32_t q, uint32_t *d_bitmasks,
                                   void *stream);

/* The plan abcore_compute_batch follows, on the host only (no device call).
 * h_parent[i] (nullable, HOST q int32): the query whose final state query i
 * starts from (it is dominated: alpha and beta both <=), or -1 to start from
 * the graph; equal queries name the first of them.  h_order (nullable, HOST
 * q int32): execution order, parents first.  out_states (nullable): number
 * of n-int32 degree buffers the plan needs.  Errors: EINVAL. */
abcore_status abcore_batch_plan(const uint32_t *h_alpha, const uint32_t *h_beta, int32_t q,
                                int32_t *h_parent, int32_t *h_order, int32_t *out_states);

/* Core numbers (Definition 2): core(x) = largest delta with x in the
 * (delta,delta)-core, 0 for isolated vertices.  Computed once per graph
 * version and cached for GCC+.  d_core: DEVICE n int32, or NULL to only fill
 * the cache.  max_core (nullable): largest core number (delta of Table I).
 * The handle keeps the buffers of the decomposition's deep part (the k0-core's
 * rows, about 4 GB at 10^9 edges) for the next decomposition, until it is
 * destroyed; they count in abcore_device_memory.  Under a memory budget
 * that leaves no room for them the levels finish the decomposition alone.
 * Synchronous. */
abcore_status abcore_core_numbers(abcore_graph g, int32_t *d_core, int32_t *max_core,
                                  void *stream);

/* Connected-component labels (GFQ preprocessing, Sec. V): label = smallest
 * unified id in the component.  Maintained under updates by abcore_query.
 * d_comp: DEVICE n int32 or NULL (only compute the labels).  Synchronous. */
abcore_status abcore_components(abcore_graph g, int32_t *d_comp, void *stream);

/* Problem 2 of Sec. III / GFQ (Sec. V).  Applies the update permanently,
 * updates the component labels (union on insertion, re-labelling of the old
 * component on deletion), peels only the component(s) holding u and v, and
 * answers whether both endpoints belong to the (alpha,beta)-core of the
 * updated graph (for an insertion this is membership of the edge, the core
 * being an induced subgraph).  h_answer: HOST int32, 1 or 0.
 * h_endpoint_bits (nullable, HOST): bit0 = u in core, bit1 = v in core.
 * Errors: EINVAL (ids, op, alpha/beta 0), EEXIST (insertion of a present
 * edge), ENOENT (deletion of an absent edge); the graph is unchanged on
 * error.  Synchronous. */
abcore_status abcore_query(abcore_graph g, abcore_edge_update upd, uint32_t alpha,
                           uint32_t beta, int32_t *h_answer, uint32_t *h_endpoint_bits,
                           void *stream);

/* Query parameters of Sec. VI-B.  *out_delta (nullable): delta of Table I,
 * the largest value with a non-empty (delta,delta)-core (the largest core
 * number, Definition 2; core numbers are computed and cached if needed).
 * h_offset[i] (HOST, q entries): alpha_offset(h_alpha[i]), the largest beta
 * with a non-empty (h_alpha[i], beta)-core, 0 when even the (h_alpha[i],
 * 1)-core is empty.  The cores are nested in beta, so a binary search of
 * GCC+ queries finds it exactly (non-empty at beta = delta when alpha <=
 * delta, empty above the largest lower degree).  h_alpha: HOST, q values >= 1.
 * Errors: EINVAL, EBUSY, ENOMEM, EDEVICE.  Synchronous. */
abcore_status abcore_alpha_offsets(abcore_graph g, const uint32_t *h_alpha, int32_t q,
                                   uint32_t *h_offset, int32_t *out_delta, void *stream);

/* The default query of Sec. VI-B: alpha = 0.4 delta and beta = 0.6
 * alpha_offset(alpha), each rounded down and at least 1.  Synchronous. */
abcore_status abcore_default_query(abcore_graph g, uint32_t *alpha, uint32_t *beta,
                                   void *stream);

/* Remark of Sec. V: GFQ returning the vertex set instead of one bit.  Does
 * what abcore_query does (the update, the component maintenance, the peel
 * scoped to the component(s) of u and v, the answer in *h_answer and
 * *h_endpoint_bits) and writes to d_bitmask (DEVICE, ceil(n/32) words, every
 * word written) the vertices that peel leaves: the (alpha,beta)-core members
 * in the component(s) of u and v in the updated graph; with connected != 0
 * only the members connected to u or v through members (the connected part
 * of the core that holds them; empty when neither is a member).
 * out_count (nullable, HOST): the set's size.  Errors as abcore_query, and
 * EINVAL for a null bitmask.  Synchronous. */
abcore_status abcore_query_set(abcore_graph g, abcore_edge_update upd, uint32_t alpha,
                               uint32_t beta, int32_t connected, int32_t *h_answer,
                               uint32_t *h_endpoint_bits, uint32_t *d_bitmask,
                               int64_t *out_count, void *stream);

/* Remark of Sec. V: localized community search in the static setting.
 * Algorithm 1 runs on the connected component of vertex q (a unified id)
 * only, as GFQ scopes its peel; d_bitmask (DEVICE, ceil(n/32) words, every
 * word written) receives the (alpha,beta)-core members of that component,
 * or with connected != 0 only the members connected to q through members:
 * the connected part of the (alpha,beta)-core containing q, empty when q is
 * not in the core.  For a query edge (u, v), take q = u: if the edge is in
 * the core, v is in the same connected part (the core is an induced
 * subgraph).  The graph is not changed.  out_count (nullable, HOST): the
 * set's size.  Errors: EINVAL (null pointer, q out of range, alpha or beta
 * 0), EBUSY (serving), ENOMEM, EDEVICE.  Synchronous. */
abcore_status abcore_community(abcore_graph g, int32_t q, uint32_t alpha, uint32_t beta,
                               int32_t connected, uint32_t *d_bitmask, int64_t *out_count,
                               void *stream);

/* ---- Serving: a stream of on-the-fly queries (Problem 2, Sec. V) -------
 * Requests are the calls abcore_query would get, in submission order; each
 * result equals what abcore_query returns when the requests are applied one
 * at a time in ticket order (answer, endpoint bits, or the EEXIST/ENOENT
 * rejection of an update that does not apply to the graph as the earlier
 * requests left it).  A worker thread of the library takes the admitted
 * requests in windows: it applies a window's updates in order (each at its
 * own graph version: deletions keep their version, insertions take new
 * edge slots), then peels each valid query's component(s) (GFQ's scoped
 * Algorithm 1) on its own device working set, all working sets running
 * concurrently on separate streams.  A new window starts as soon as working
 * sets free up, while earlier queries still run.  Component labels only
 * merge while serving (a stale label's component is a superset of the
 * current ones, which keeps the scoped peel exact).  While a handle serves,
 * every other entry point except abcore_graph_info and abcore_kernel_timing
 * returns EBUSY. */

/* Starts the engine (abcore_submit starts it with defaults if needed).
 * max_inflight: admitted-but-unfinished requests allowed (0 = 1024);
 * device_slots: concurrent device working sets, n + 16 * (2n + pieces)
 * int32 each (0 = 2, at most 256: on graphs of hundreds of millions of
 * edges a single query already saturates the device's random-access
 * throughput, and two working sets measured best); window: most updates
 * per window (0 = 64, at most 64).  Computes the component labels if needed.  Synchronous.
 * Under a memory budget (abcore_set_memory_budget) it creates as many working
 * sets as fit, at least one (ENOMEM if none does; abcore_serve_counters
 * reports how many): windows then take fewer requests and the rest wait,
 * admitted, until abcore_submit's EBUSY at max_inflight.
 * Errors: EINVAL, ENOMEM, EDEVICE. */
abcore_status abcore_serve_start(abcore_graph g, int64_t max_inflight, int32_t device_slots,
                                 int32_t window);

/* Admits one request: the update (u, v, op) and the (alpha,beta) membership
 * question on the updated graph.  *ticket receives its number (consecutive
 * from 0 per handle).  EBUSY when max_inflight requests are admitted and
 * unfinished (retry later); EINVAL for ids out of range, op not +1/-1 or a
 * threshold 0 (the request is not admitted); EDEVICE once the engine failed.
 * Thread-safe with abcore_poll. */
abcore_status abcore_submit(abcore_graph g, abcore_edge_update upd, uint32_t alpha,
                            uint32_t beta, uint64_t *ticket);

/* Result of a ticket.  ABCORE_OK: *answer (1 if both endpoints are in the
 * core of the graph after that update), *endpoint_bits (bit0 u, bit1 v) and
 * *t_done_ns (steady-clock nanoseconds, CLOCK_MONOTONIC, when the engine saw
 * it finish) are written (each pointer nullable) and the result is released.
 * EEXIST / ENOENT: the update was rejected (graph unchanged by it).
 * EAGAIN: not finished yet, or already taken.  EINVAL: a ticket never
 * issued.  ETIMEDOUT: the deadline (ABCORE_OPT_SERVE_DEADLINE_US) passed
 * before the request's query started: its update was applied as usual, the
 * query was dropped and nothing else is written.  EDEVICE: the engine
 * failed.  Thread-safe with abcore_submit. */
abcore_status abcore_poll(abcore_graph g, uint64_t ticket, int32_t *answer,
                          uint32_t *endpoint_bits, uint64_t *t_done_ns);

/* Counters of the serving engine (HOST int64[count], count <= 8): windows
 * run, requests answered, requests rejected, requests decided without a
 * peel by stale core-number pruning, core-number snapshots taken, their
 * total wall time in microseconds, requests past their deadline, and device
 * working sets in use.  Valid while serving and after abcore_serve_stop. */
abcore_status abcore_serve_counters(abcore_graph g, int64_t *out, int32_t count);

/* Waits for every admitted request to finish, stops the worker and frees the
 * working sets (unpolled results stay available).  counters (nullable, HOST
 * int64[3]): windows run, requests answered, requests rejected. */
abcore_status abcore_serve_stop(abcore_graph g, int64_t *counters);

/* Tuning knobs (non-negative values; 0 restores the default).
 *   ABCORE_OPT_PEEL_MODE : 1 = one kernel per peel round, host-checked in
 *                          batches; 2 = all rounds in one cooperative launch
 *                          with a grid barrier between rounds; 3 (default) =
 *                          asynchronous worklist: one launch, no rounds,
 *                          waves take queued vertices as soon as they are
 *                          appended (stats.rounds is then -1).  Modes 2 and 3
 *                          fall back to 1 when the device reports no
 *                          co-residency of the grid.  For core numbers,
 *                          mode 3 peels level by level (a scan and an
 *                          asynchronous peel per level) and modes 1 and 2
 *                          run rounds.
 *   ABCORE_OPT_GRID      : workgroups per peel launch.
 *   ABCORE_OPT_ROUNDS_PER_SYNC : round kernels enqueued between checks.
 *   ABCORE_OPT_TIMING    : 1 = record a HIP event pair on the caller's stream
 *                          around every launch (or batch of launches) of the
 *                          GCC kernels; read with abcore_kernel_timing.
 *   ABCORE_OPT_PULL      : first GCC round in pull form: 0 = decided on the
 *                          device from the scan frontier, 1 = never, 2 = always.
 *   ABCORE_OPT_CLAIM     : queue slots a wave of the asynchronous peel takes
 *                          at a time, 1..64 (0 = 32).
 *   ABCORE_OPT_RANK_ORDER: 1 (default) = a GCC query whose first round is
 *                          pulled runs on the degree-rank relabelling of the
 *                          graph while it is unchanged since the build (the
 *                          scan's survivors are then known in advance, Sec.
 *                          IV-A), and other first pull rounds count on it;
 *                          2 = index-free: every query runs in vertex order
 *                          on the CSR alone, as Algorithm 1 does.
 *   ABCORE_OPT_AUTOTUNE  : 0 or 1 (default) = take mappings from the tuning
 *                          cache and tune batches on first use (below);
 *                          2 = off.  Setting ABCORE_OPT_GRID or
 *                          ABCORE_OPT_CLAIM to a non-zero value fixes the
 *                          mapping (no cache lookups).
 *   ABCORE_OPT_SERVE_PRUNE: stale core-number pruning of served requests
 *                          (set before abcore_serve_start).  0 (default) =
 *                          off; 1 = on, with the snapshot of the core numbers
 *                          taken at serve start; k >= 2 = on, with a new
 *                          snapshot after every k applied updates.  An edge
 *                          update changes only the core numbers equal to
 *                          min(core(u), core(v)), each by one (the k-core
 *                          maintenance property; beyond the paper), so the
 *                          engine keeps an interval per snapshot value that
 *                          holds the current core numbers of its vertices.
 *                          A request whose two endpoints Lemma 1 decides on
 *                          those intervals (lower end >= max(alpha,beta): in;
 *                          upper end < min(alpha,beta): out) is answered
 *                          without a peel.  Results stay exact.
 *   ABCORE_OPT_KCORE_SWITCH: core numbers (default peel mode): levels are
 *                          peeled one by one until at most `value` vertices
 *                          are live (0 = 1048576; checked between batches of
 *                          levels); the rest -- the k0-core, whose core
 *                          numbers in G are its own -- is finished by the
 *                          h-index fixpoint (iterate est(x) <- h-index of the
 *                          neighbours' est, from the degrees, until nothing
 *                          changes).  1 = levels only.  Results are
 *                          identical either way.
 *   ABCORE_OPT_SPIN_LIMIT: failure injection for tests: polls a waiting wave
 *                          of the asynchronous peel makes before it declares
 *                          a hang and aborts (0 = the default, 2^21, i.e.
 *                          seconds; small values make peels abort at once).
 *   ABCORE_OPT_SERVE_DEADLINE_US: per-request deadline of the serving
 *                          engine, from admission (set before
 *                          abcore_serve_start; 0 = none, the default): a
 *                          request whose query would start later is answered
 *                          ABCORE_ETIMEDOUT by abcore_poll; its update is
 *                          applied all the same, so the stream stays ordered.
 *   ABCORE_OPT_APPEND_SUBQUEUE: test of the frontier queue's shared capacity
 *                          (the 16 sub-queues together hold the bound of
 *                          2n + pieces + 256 appends per computation, each a
 *                          16th plus 4,096 slots; an append that does not fit
 *                          one goes to the next): 0 (default) = each
 *                          workgroup appends to its own sub-queue first;
 *                          j in 1..16 = every append tries sub-queue j-1
 *                          first, so that it fills and the rest overflow.
 *                          Results are identical either way.
 *
 * Aborts.  Every device-side wait is bounded.  A computation whose wait
 * exceeds its bound leaves an invalid result; a call that requested stats
 * (or that synchronises internally) returns ABCORE_EDEVICE at once.  An
 * asynchronous call cannot know yet: its peel sets a pinned host word when it
 * ends, and the first later computing call on the handle that finds the word
 * set (abcore_compute, _compute_batch, _core_numbers, _query, _autotune,
 * _serve_start) returns ABCORE_EDEVICE without computing, after resetting the
 * handle's workspace, so that the calls after it are exact again.  Results of
 * calls enqueued between the aborted one and that report may be invalid too.
 */
enum {
  ABCORE_OPT_PEEL_MODE = 1,
  ABCORE_OPT_GRID = 2,
  ABCORE_OPT_ROUNDS_PER_SYNC = 3,
  ABCORE_OPT_TIMING = 4,
  ABCORE_OPT_PULL = 5,
  ABCORE_OPT_CLAIM = 6,
  ABCORE_OPT_RANK_ORDER = 7,
  ABCORE_OPT_SPIN_LIMIT = 8,
  ABCORE_OPT_AUTOTUNE = 9,
  ABCORE_OPT_SERVE_PRUNE = 10,
  ABCORE_OPT_KCORE_SWITCH = 11,
  ABCORE_OPT_APPEND_SUBQUEUE = 12,
  ABCORE_OPT_SERVE_DEADLINE_US = 13
};
abcore_status abcore_set_option(abcore_graph g, int32_t option, int64_t value);

/* Autotuner of the peel's work mapping for this graph: times the query
 * (alpha, beta) with algorithm algo (3 runs after a warm run, median) for
 * every pair of asynchronous-peel grid size (1/2, 3/4, 1, 3/2, 2, 3
 * workgroups of 8 waves per compute unit, within the co-resident capacity)
 * and claim size (64, 32, 16 queue slots per wave), then sets ABCORE_OPT_GRID
 * and ABCORE_OPT_CLAIM to the fastest.  out_grid, out_claim, out_ms
 * (nullable): the choice and its time in milliseconds.  Results of every
 * computation stay exact whatever the choice.  Synchronous.
 * Errors: EINVAL, ENOMEM, EDEVICE, EBUSY (serving). */
abcore_status abcore_autotune(abcore_graph g, uint32_t alpha, uint32_t beta, int32_t algo,
                              int32_t *out_grid, int32_t *out_claim, double *out_ms,
                              void *stream);

/* Tuning cache.  abcore_autotune stores its choice under the device's
 * architecture name, compute-unit count, graph shape (floor log2 of the
 * vertex count and of the 2m adjacency entries) and kind 0 (single
 * queries); later handles of that shape take it on their first
 * abcore_compute unless the caller set the grid or claim.  A batch
 * (abcore_compute_batch, kind 1) looks its mapping up there and, the first
 * time a shape is seen, tunes it on the batch's median query (by alpha +
 * beta) and stores it; it applies to that call only.  ABCORE_OPT_AUTOTUNE:
 * 0 or 1 = on (default), 2 = off.  abcore_tuned reads the entry for the
 * handle's shape (*found = 0 if none).  abcore_tune_cache: mode 0 loads
 * (merges) the text file at path, 1 saves the cache there, 2 clears it
 * (path unused); one entry per line: arch cu nlog elog kind grid claim ms. */
abcore_status abcore_tuned(abcore_graph g, int32_t kind, int32_t *out_grid, int32_t *out_claim,
                           double *out_ms, int32_t *found);
abcore_status abcore_tune_cache(const char *path, int32_t mode);

/* Kernel kinds timed while ABCORE_OPT_TIMING is on: the push peel
 * (Algorithm 1, peel phase), the pull-form first round, the scan phase, the
 * bitmask pack and the pull round's completion (split rows below threshold
 * queued, round range advanced). */
enum {
  ABCORE_KERNEL_PEEL = 0,
  ABCORE_KERNEL_PULL = 1,
  ABCORE_KERNEL_SCAN = 2,
  ABCORE_KERNEL_PACK = 3,
  ABCORE_KERNEL_FIXUP = 4
};

/* GPU time of one kernel kind recorded while ABCORE_OPT_TIMING is on:
 * *ms = summed elapsed time of its event pairs (recorded on the stream the
 * kernel is launched on), *launches = launches they bracket.  Waits for the
 * recorded events.  reset != 0 clears the records of that kind.
 * EINVAL for an unknown kind. */
abcore_status abcore_kernel_timing(abcore_graph g, int32_t kernel, double *ms,
                                   int64_t *launches, int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* ABCORE_H */
