// Internal declarations of libabcore (device layout, launch helpers).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "abcore.h"

namespace abc {

constexpr int kWave = 64;
constexpr int kBlock = 256;             // flat kernels (scan, classify, pack)
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kPeelBlock = 512;         // peel kernels: 8 waves per workgroup
constexpr int kPeelWaves = kPeelBlock / kWave;
constexpr int kPullBlock = 1024;        // pull round: one workgroup per CU
constexpr int kPullWaves = kPullBlock / kWave;
// Per-wave frontier buffer in LDS (the warp-local queue of Algorithm 1,
// sized for a 64-lane wavefront); flushed per workgroup at round ends.
constexpr int kLocalQueue = 256;
constexpr int kPullLocalQueue = 128;
// Row piece length (entries) for load balancing over skewed degrees.
constexpr int kPiece = 64;

// Spread append counters: workgroup b appends to sub-queue b % kSub (the
// next one with room when it is full), each with its own counter on its own
// 64-byte line.  Same-address device-scope atomics serialise (about 11 ns
// each on MI355X), so no counter may take more than a few dozen increments
// per launch.
constexpr int kSub = 16;
// Largest single append (a scan workgroup's chunk).
constexpr int kMaxAppend = 4096;
// A slot filled by an append that did not fit its sub-queue: consumers take
// it and count it as processed, and nothing else.
constexpr int32_t kSkipItem = INT32_MIN;
// Slots per sub-queue.  A computation appends at most 2n + pieces +
// kLocalQueue items (a vertex at most twice: GCC+'s uncertain list and
// frontier, or a split row's two queueings after a pull round; a piece
// once); the sub-queues share that bound, each with kMaxAppend of slack.
inline int64_t queue_capacity(int64_t n, int64_t npieces) {
  return (2 * n + npieces + kLocalQueue + kSub - 1) / kSub + kMaxAppend;
}
constexpr int kPad = 16;      // int32 words per 64-byte line
constexpr int kGroups = 16;   // grid-barrier / last-workgroup groups
constexpr int kMaxBlocks = 4096;
// Queue slots an asynchronous-peel wave claims at a time.  Fewer than 64
// spreads a small frontier over more waves (the batch's entries are still
// spread over all 64 lanes).
constexpr int kDefaultClaim = 32;

// GCC+ class encoding in the working degree array (Sec. IV-B, Lemma 1):
// certain members are never decremented, certain non-members never counted.
constexpr int32_t kDegIn = 0x7FFFFFFF;
constexpr int32_t kDegOut = -1;
// Polls of one waiting wave of the asynchronous peel before it declares a
// hang (each poll takes at least a few microseconds, so this is seconds: far
// beyond any legitimate wait of a peel).  ABCORE_OPT_SPIN_LIMIT lowers it.
constexpr uint32_t kAsyncSpinLimit = 1u << 21;
// Live vertices at or below which the core decomposition leaves the level
// peel for the h-index fixpoint (measured best at 2^20 on the 2e7-, 5e8- and
// 1e9-edge power-law graphs: 10, 78 and 131 ms, against 12, 96 and 152 ms
// at 2^18).
constexpr int64_t kKcoreSwitch = 1 << 20;
// Largest usable threshold: kDegIn must stay above every threshold.
constexpr int32_t kMaxThreshold = 0x7FFFFFFE;
// Degree of a removed split row once a consumer has claimed it (far below
// any degree a vertex reaches by decrements, since degrees stay below 2^30).
constexpr int32_t kClaimedDeg = -(1 << 30);

// Hierarchical arrival counters: workgroups arrive on their group's line,
// the last of each group on the top line.
struct Arrival {
  uint32_t group[kGroups][kPad];
  uint32_t top[kPad];
  uint32_t gen[kPad];  // grid barrier generation (persistent kernels)
};

// Peel bookkeeping shared by every multi-round computation (one instance in
// device memory per handle).  Each vertex enters the frontier queues at most
// once per computation (twice for GCC+: uncertain list, then frontier), so
// the queues are append-only and a round is the ranges [lo[j], hi[j]) of the
// kSub sub-queues.  Whoever completes a round (the last workgroup of a
// launch, or the last arrival of a grid barrier) advances the ranges to the
// items appended meanwhile.
struct PeelState {
  int32_t tail[kSub][kPad];  // append cursors
  int32_t head[kSub][kPad];  // asynchronous peel: next slot to claim
  int32_t consumed[kSub][kPad];  // asynchronous peel: slots processed
  int32_t started[kGroups][kPad];  // asynchronous peel: workgroups past their start phase
  int32_t fin[kGroups][kPad];  // asynchronous peel: termination detected (one copy per group)
  int32_t lo[kSub];
  int32_t hi[kSub];
  Arrival arr;
  int32_t rounds;       // non-empty rounds completed
  int32_t first;        // size of the initial frontier
  int32_t k;            // core decomposition: current level
  int32_t next_k;       // core decomposition: level of the next scan
  int32_t alive_cur;    // core decomposition: entries in the current alive list
  int32_t alive_sel;    // which alive list is current (0/1)
  int32_t kept;         // core decomposition: live vertices after the last scan
  int32_t compact;      // core decomposition: compact the alive list next
  int32_t done;         // computation finished
  int32_t max_core;     // largest level with removals
  int32_t status;       // device-side status for updates (0 ok)
  int32_t aux0, aux1;   // small results (uncertain count, labels, answer bits)
  int32_t pulled;       // first round ran in pull form
  int32_t abort_flag;   // a grid barrier exceeded its spin limit
  int32_t dead;         // core decomposition: alive-list entries found removed by a scan
  int32_t live;         // core decomposition: live entries of the alive list after a scan
  int32_t pad0;
  int64_t launches;     // launches that did work
  // arrival counters of the workspace reset only (never zeroed: that kernel
  // always completes, so they always return to zero)
  Arrival rst;
};

// Per-workgroup partial results, one slot line per workgroup (no atomics).
enum PartField : int {
  kPartEntries = 0,   // adjacency entries read
  kPartF0 = 1,        // initial-frontier vertices
  kPartF0Deg = 2,     // their degree sum
  kPartKept = 3,      // core decomposition: kept vertices of the last scan
  kPartMin = 4,       // core decomposition: smallest kept degree
  kPartF1 = 5,        // vertices a pull round found below their threshold
  kPartRest = 6,      // nested scan: entries of the rows that survive it
  kPartAliveU = 7,    // GCC scan: upper vertices that survive it
  kPartAliveL = 8,    // GCC scan: lower vertices that survive it
  kPartFields = 10
};

// Dynamic edge storage for updates after the build (Sec. V).  Deleted CSR
// entries are tombstoned in place as ~col (negative, order-preserving after
// decoding); inserted edges live in per-vertex singly linked lists of
// half-edges.  Half-edge 2j is the entry of pair j in the upper row, 2j+1 in
// the lower row; a deleted half-edge stores ~other.
struct Delta {
  int32_t *head = nullptr;   // n, -1 = empty list
  int32_t *next = nullptr;   // 2*cap
  int32_t *other = nullptr;  // 2*cap: neighbour id (negative = deleted)
  int64_t cap = 0;
  int64_t count = 0;         // pairs used
};

struct Server;  // serving engine (serve.hip)

// Execution plan of a batch of queries (make_batch_plan).
struct BatchPlan {
  std::vector<int32_t> order;   // execution order (query indices)
  std::vector<int32_t> parent;  // query whose final state seeds it, -1 = the graph
  std::vector<uint8_t> dup;     // 1: same thresholds as parent, bitmask copied
  std::vector<uint8_t> copy;    // 1: starts from a copy of the parent's state
  std::vector<int32_t> slot;    // state buffer (-1 for duplicates)
  // 1: runs from scratch as a root does (in its buffer) although it has a
  // parent, because that measured faster (see abcore_compute_batch)
  std::vector<uint8_t> scratch;
  int nslots = 0;
};
BatchPlan make_batch_plan(const int32_t *tu, const int32_t *tl, int32_t q);

// A captured batch of nested queries, replayed while the same batch is
// asked for again on an unchanged graph.
struct BatchCache {
  std::vector<int32_t> key;  // thresholds of the queries, then options
  uint32_t *bits = nullptr;  // output the graph writes
  int version = -1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int parity = 0;  // Graph::rs_parity when captured (the state it refers to)
};

struct Graph {
  int device = 0;
  char arch[64] = "";  // gcnArchName of the device (key of the tuning cache)
  int autotune = 1;    // ABCORE_OPT_AUTOTUNE: batches take a tuned mapping
  // ABCORE_OPT_SERVE_PRUNE: 0 off; 1 stale core-number pruning of served
  // requests from the snapshot taken at serve start; k >= 2 the same with a
  // new snapshot after every k applied updates
  int64_t serve_prune = 0;
  // ABCORE_OPT_KCORE_SWITCH: core numbers finish by the h-index fixpoint
  // once at most kcore_switch vertices are live (checked between batches of
  // levels)
  int64_t kcore_switch = kKcoreSwitch;
  bool kcore_top_used = false;  // the last core decomposition used it
  // its switch level, vertices, adjacency entries, sweeps and phase times
  int64_t top_stats[4] = {0, 0, 0, 0};
  double top_ms[2] = {0, 0};  // levels before the switch, the h-index phase
  bool tuned = false;  // grid and claim chosen (by a tuner or by the caller)
  int32_t nU = 0, nL = 0;
  int64_t n = 0;
  int64_t m = 0;      // current distinct edges
  int64_t m_csr = 0;  // pairs stored in the CSR at build
  int64_t *off = nullptr;   // n+1
  int32_t *cols = nullptr;  // 2*m_csr
  int32_t *deg0 = nullptr;  // current degree of every vertex
  int32_t *deg = nullptr;   // working degree (per computation)
  int32_t *queue = nullptr; // kSub sub-queues of qcap entries
  int64_t qcap = 0;
  uint32_t *alive_bits = nullptr;  // n bits: alive after the scan (pull round)
  uint32_t *row_bits = nullptr;    // n bits: rows a GCC+ pull round counts (uncertain)
  int32_t *list = nullptr;  // n: alive list 0 (core decomposition)
  int32_t *list2 = nullptr; // n: alive list 1
  int64_t *part = nullptr;  // kMaxBlocks * kPartFields
  PeelState *state = nullptr;
  PeelState *h_state = nullptr;  // pinned host mirror
  int64_t *h_part = nullptr;     // pinned host mirror of part
  int32_t *core = nullptr;  // cached core numbers
  uint32_t *kdead = nullptr;  // n bits: vertices the level peel has removed
  // the h-index phase's buffers (hipMalloc), kept for the next decomposition
  void *top_buf[20] = {};
  size_t top_cap[20] = {};
  bool core_valid = false;
  int32_t max_core = 0;
  // Rows longer than kPiece entries are split into pieces of kPiece entries
  // so that no wave batch walks a hub alone (fixed by the offsets, so built
  // once per handle).  Pieces are ordered by row; upper rows come first.
  int32_t *piece_row = nullptr;    // npieces
  int64_t *piece_start = nullptr;  // npieces: absolute position in cols
  int32_t *piece_first = nullptr;  // n: first piece of a split row, else -1
  // At the slot of a split row's first piece: the degree a nested scan left
  // in place for a pull round to replace (npieces).
  int32_t *split_written = nullptr;
  int32_t *heavy_rows = nullptr;   // nheavy: the split rows, ascending
  int64_t npieces = 0, npieces_upper = 0;
  int64_t nheavy = 0, nheavy_upper = 0;
  // Degree ranks (the build's degrees): rank[x] is x's position within its
  // layer in the order of decreasing degree (ties by id); rank_vtx maps the
  // global rank R (a layer's ranks follow its first unified id) back to the
  // vertex.  rcols holds the rows in rank order (row R at roff[R]), each as
  // its neighbours' global ranks, ascending: the rank rows are the graph
  // relabelled by rank, a layer's vertices keeping their id range.  A scan
  // leaves alive exactly the K
  // vertices of a layer with degree >= its threshold, i.e. ranks [0, K): the
  // surviving rows are a prefix of the rank order (the split rows first),
  // and a row's surviving neighbours are the prefix of its rank row below
  // the other layer's K.  A first pull round on an unchanged graph counts
  // them so.  (Null when the build could not afford them.)
  int32_t *rank = nullptr;      // n
  int32_t *rank_vtx = nullptr;  // n
  int64_t *roff = nullptr;      // n + 1
  int32_t *rcols = nullptr;     // 2*m_csr
  // The rank rows' pieces (as piece_row/start/first for the vertex rows), and
  // per layer, indexed by a threshold t <= its largest degree + 1, the
  // vertices of degree >= t (K) and their entries (host copies): a query on
  // an unchanged graph runs in rank order, its survivors known in advance.
  int32_t *rp_row = nullptr;    // npieces
  int64_t *rp_start = nullptr;  // npieces
  int32_t *rp_first = nullptr;  // n
  std::vector<int64_t> rk_cnt[2], rk_ent[2];
  // Working degrees of a query in rank order, at hashed slots: the hubs lead
  // each layer's ranks and would otherwise share cache lines and channels
  // under the peel's atomics (rdeg_mask + 1 entries, a power of two >= n).
  int32_t *rdeg = nullptr;
  uint32_t rdeg_mask = 0;
  bool rank_order = true;  // ABCORE_OPT_RANK_ORDER
  // Second workspace state and partial sums: queries in rank order alternate
  // between the two, each leaving the other one zeroed and the queue empty
  // (rs_ready).  Any other launch through make_args clears rs_ready.
  PeelState *state_alt = nullptr;
  int64_t *part_alt = nullptr;
  int32_t *rs_fail = nullptr;  // device word, see PeelArgs
  bool rs_ready = false;
  // Pinned host word set by a peel that ended by a spin-limit abort (see
  // PeelArgs::abort_host); the next computing call reports it and resets
  // the workspace.
  int32_t *h_abort = nullptr;
  uint32_t spin_limit = 0;  // ABCORE_OPT_SPIN_LIMIT (0 = kAsyncSpinLimit)
  int32_t append_sub = -1;  // ABCORE_OPT_APPEND_SUBQUEUE - 1
  int32_t *dbg_enqueue = nullptr;  // debug builds: int32[n] enqueue counts
  int64_t serve_deadline_us = 0;   // ABCORE_OPT_SERVE_DEADLINE_US (0: none)
  int rs_parity = 0;  // flips with every exchange of state and state_alt
  // Pull round work split: workgroup k of a cu_count grid walks the upper
  // rows [b[k], b[k+1]) and the lower rows [b[G+1+k], b[G+2+k]), ranges of
  // equal weight (entries of unsplit rows plus a per-row cost).
  int32_t *pull_bounds = nullptr;  // 2 * (pull_bounds_grid + 1)
  int pull_bounds_grid = 0;
  int64_t *aux = nullptr;   // small counters of the vertex-set searches (4)
  uint32_t *probe_bits = nullptr;  // ceil(n/32) words: results of offset probes
  int32_t *comp = nullptr;  // component labels
  bool comp_valid = false;
  int32_t *parent = nullptr; // union-find scratch
  Delta delta;
  int version = 0;
  // wall times of the build's phases: CSR, row pieces, degree-rank copy, all
  double build_ms[4] = {0, 0, 0, 0};
  // device facts and options
  int cu_count = 256;
  size_t lds_per_block = 65536;
  int peel_mode = 3;        // 1 = round kernels, 2 = rounds in one cooperative
                            // launch, 3 = asynchronous worklist
  int pull_mode = 0;        // 0 = auto, 1 = never, 2 = always
  int grid = 0;             // 0 = derived from the device
  int rounds_per_sync = 16;
  int claim = kDefaultClaim;  // slots a wave of the asynchronous peel claims
  int persistent_grid = 0;  // co-resident workgroups of the persistent kernels
  int kcore_grid = 0;
  int async_grid = 0;       // co-resident workgroups of the asynchronous peel
  // serving: versions of deletions (per base entry, per inserted pair) and
  // the count of applied served updates; the engine while it runs
  int32_t *del_ver = nullptr;
  int32_t *pair_del_ver = nullptr;
  int64_t pair_del_cap = 0;
  int32_t upd_version = 0;
  Server *server = nullptr;
  // batched queries: working-degree states (n int32 each) and the cache
  std::vector<int32_t *> slots;
  BatchCache batch;
  hipStream_t capture_stream = nullptr;
  // kernel timing (ABCORE_OPT_TIMING): event pairs per kernel kind
  bool timing = false;
  static constexpr int kKernelKinds = 5;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events[kKernelKinds];
  std::vector<hipEvent_t> event_pool;
  int64_t timed_launches[kKernelKinds] = {0, 0, 0, 0, 0};
};

// Serving: at most kWindowMax updates per window, hence at most kCorrMax
// degree corrections for one query's view.
constexpr int kWindowMax = 64;
constexpr int kCorrMax = 2 * kWindowMax;

// Outcome of one served update (update_window_kernel).
struct WindowRecord {
  int32_t status;       // 0, -ABCORE_EEXIST or -ABCORE_ENOENT
  int32_t version;      // version of the graph after it (valid updates)
  int32_t pairs_after;  // inserted pairs allocated after it
  int32_t label_u, label_v;  // component labels of the endpoints before the window
  int32_t pad[3];
};

// Peel flavours.
enum PeelKind : int { kGCC = 0, kGCCPlus = 1, kKCore = 2 };

// Parameters of a peel, passed by value to kernels.
struct PeelArgs {
  const int64_t *off;
  const int32_t *cols;
  int32_t *deg;
  int32_t *queue;
  int64_t qcap;
  PeelState *st;
  int64_t *part;
  const int32_t *ins_head;  // nullable
  const int32_t *ins_next;
  const int32_t *ins_other;
  int32_t *core;            // kKCore: output core numbers
  // kKCore (nullable): a bit per removed vertex, set when the peel takes it;
  // decrements of a vertex found removed are skipped (a bit still clear
  // only costs the decrement)
  uint32_t *kdead;
  const int32_t *piece_row;
  const int64_t *piece_start;
  const int32_t *piece_first;
  // Versioned view (served queries, whose updates are applied while older
  // queries still peel): a tombstoned entry at position p is still an edge of
  // this query iff del_ver[p] > ver; inserted pair j exists iff
  // j < pair_limit and it is live or pair_del_ver[j] > ver.  del_ver ==
  // nullptr: the current graph.
  const int32_t *del_ver;
  const int32_t *pair_del_ver;
  int32_t ver;
  int32_t pair_limit;
  int32_t claim;  // asynchronous peel: slots per claim, 1..64
  // asynchronous peel, fused work (all nullable): split rows of a pull round
  // to queue when below their threshold (start phase, before any workgroup
  // may end: start_expect workgroups must have started), and the membership
  // bitmask to write after termination
  const int32_t *fix_rows;
  const uint32_t *fix_bits;
  int64_t nfix;
  uint32_t *pack_bits;
  int32_t start_expect;
  // vertices alive after the scan (bit set; nullable): GCC skips decrements
  // of the scan frontier, which is out of the core whatever its degree
  const uint32_t *alive0;
  // the frontier a pushed first round queues, when not the scan's clear bits
  const uint32_t *f0_bits;
  // Rank order (klim_u >= 0): ids are global ranks, the scan's survivors are
  // the ranks below klim_u (upper) and nU + klim_l (lower), which replaces
  // alive0.  pack_vtx (global rank -> vertex, non-null in rank order): the
  // result bitmask already holds the scan's survivors and the peel clears
  // each vertex it removes (no pack after termination).
  int32_t klim_u, klim_l;
  const int32_t *pack_vtx;
  // Rank order: a rank's degree sits at slot (rank * kRankMul) & rs_mask of
  // a power-of-two array (0: the degree array is indexed by id).
  uint32_t rs_mask;
  // Rank order (nullable): the peel returns each queue slot to empty as it
  // takes the slot's item, and after termination zeroes this state and these
  // partial sums, the next query's workspace (its own stay readable for the
  // statistics).
  PeelState *rs_next_st;
  int64_t *rs_next_part;
  // Rank order: set when a peel ended without termination (a spin-limit
  // abort) and so left the queue as it was; later queries in rank order
  // then abort at once until a preparation clears it.
  int32_t *rs_fail;
  // Polls of a waiting wave before it declares a hang (kAsyncSpinLimit
  // unless lowered by ABCORE_OPT_SPIN_LIMIT).
  uint32_t spin_limit;
  // Host-visible word (pinned, coherent; nullable) the peel sets when it
  // ends by an abort, so the host learns of it without a synchronisation.
  int32_t *abort_host;
  // Sub-queue every append tries first (-1: the producer's own; a fixed one
  // makes appends overflow into the others, ABCORE_OPT_APPEND_SUBQUEUE).
  int32_t append_sub;
  // Debug builds: per-vertex counts of appends to the frontier queues.
  int32_t *dbg_enqueue;
  int64_t n;
  int32_t nU;
  int32_t thrU, thrL;
};

void set_error(const char *fmt, ...);
PeelArgs make_args(Graph &g, int32_t thrU, int32_t thrL);

// Every device allocation of the library goes through these, which keep
// the library-wide current and peak byte counts (abcore_device_memory) and
// apply the budget (abcore_set_memory_budget).  Memory a handle keeps comes
// from hipMalloc; temporaries of one call (sort keys, scan storage, the
// deep core's rows) are stream-ordered on the caller's stream
// (hipMallocAsync / hipFreeAsync), so freeing them waits for nothing.
hipError_t dev_malloc_bytes(void **p, size_t bytes);
template <class T>
hipError_t dev_malloc(T **p, size_t bytes) {
  return dev_malloc_bytes(reinterpret_cast<void **>(p), bytes);
}
hipError_t dev_free(void *p);
hipError_t dev_malloc_async_bytes(void **p, size_t bytes, hipStream_t s);
template <class T>
hipError_t dev_malloc_async(T **p, size_t bytes, hipStream_t s) {
  return dev_malloc_async_bytes(reinterpret_cast<void **>(p), bytes, s);
}
hipError_t dev_free_async(void *p, hipStream_t s);

// Launchers (defined in the .hip files).
// keep_abort: leave the abort flag as it is (several computations in one
// sequence report a spin-limit abort of any of them)
hipError_t launch_init_state(Graph &g, hipStream_t s, bool keep_abort = false);
// The same for another working set (queue of g.qcap per sub-queue, state,
// partial sums) than the handle's own.
hipError_t launch_init_workspace(Graph &g, int32_t *queue, PeelState *state, int64_t *part,
                                 hipStream_t s, bool keep_abort = false);
hipError_t launch_scan_gcc(Graph &g, int32_t thrU, int32_t thrL, bool want_bits,
                           hipStream_t s);
// bits (nullable): also writes the survivor bitmap, the partial sums and the
// surviving split rows' degrees (g.split_written) a pull round needs
// (rest_part in the pull then compares the frontier's degrees with the
// survivors' row entries, and written_snap replaces deg0 as what the
// split rows' pieces subtract).
// src (nullable): the parent's state, copied into g.deg as it is read (a
// child that does not continue in its parent's buffer).  fbits (nullable,
// with bits): the frontier goes to this bitmap instead of the queue, and the
// pull kernel queues it if it pushes the first round (launch_pull_round's
// f0bits).
hipError_t launch_scan_nested(Graph &g, int32_t pU, int32_t pL, int32_t thrU, int32_t thrL,
                              hipStream_t s, uint32_t *bits = nullptr,
                              const int32_t *src = nullptr, uint32_t *fbits = nullptr);
// queue_f0: the scan did not queue its frontier (launch_scan_reset_gcc);
// a pushed first round then queues it from the bitmap.
hipError_t launch_scan_reset_gcc(Graph &g, int32_t thrU, int32_t thrL, hipStream_t s,
                                  bool keep_abort = false);
// A GCC query in rank order (g.rcols and g.rp_* present, unchanged graph):
// part 0 is the pulled first round (and the survivor bitmap into pack_bits),
// part 1 the asynchronous peel (clearing the removed vertices' bits, then
// readying g.state_alt, g.part_alt and the queue); ku and kl are the layers'
// survivor counts.
hipError_t launch_rank_query(Graph &g, int32_t thrU, int32_t thrL, int64_t ku, int64_t kl,
                             uint32_t *pack_bits, hipStream_t s, int part);
// Returns the queue's used slots (cursors in g.state) to empty and zeroes
// g.state_alt and g.part_alt: the workspace a query in rank order expects.
hipError_t launch_rank_prep(Graph &g, hipStream_t s);
// GCC+: the classification, fused with the workspace reset, that prepares
// a pull round (rowbits = g.row_bits, force = true) as its initialisation.
hipError_t launch_classify_reset(Graph &g, int32_t thrU, int32_t thrL, int32_t dl, int32_t dq,
                                  hipStream_t s);
// rowbits: the rows to count (nullptr: the rows whose bit is set in the
// lookup bitmap); force: pull whatever the pull mode and the frontier.
// rest_part: the pull cost is the scan's kPartRest sums (nested scans).
// rank: count by the degree-rank copy (Graph::rcols; the GCC scan's
// survivors on an unchanged graph only), completing split rows at once.
// f0bits (nullable, with queue_f0): the frontier to queue when pushing is
// this bitmap's set bits instead of the lookup bitmap's clear bits.
hipError_t launch_pull_round(Graph &g, int32_t thrU, int32_t thrL, hipStream_t s,
                             bool advance = false, bool queue_f0 = false,
                             const uint32_t *rowbits = nullptr, bool force = false,
                             bool rest_part = false, bool rank = false,
                             const uint32_t *f0bits = nullptr);
// Asynchronous peel fused with the pull round's completion (fix_bits: the
// scan's survivors, or nullptr when no pull round ran) and the bitmask pack
// (pack_bits nullable).
// split_done: the pull round completed its split rows itself (rank form):
// no start phase, fix_bits serves as the decrement filter only.
hipError_t launch_peel_async_fused(Graph &g, PeelKind kind, int32_t thrU, int32_t thrL,
                                   const uint32_t *fix_bits, uint32_t *pack_bits,
                                   hipStream_t s, bool split_done = false);
hipError_t launch_pull_fixup(Graph &g, int32_t thrU, int32_t thrL, hipStream_t s);
hipError_t launch_scan_component_of(Graph &g, int32_t thrU, int32_t thrL, int32_t x,
                                    int32_t y, hipStream_t s);
hipError_t launch_scan_component_view(Graph &g, const PeelArgs &a, int32_t x, int32_t y,
                                      const int32_t *corr_x, const int32_t *corr_d, int ncorr,
                                      uint32_t *bits, hipStream_t s);
// Pull-form first round for any working set: bits are the scan's survivors;
// corr_x/corr_d (ncorr entries, nullable) the degree corrections the scan
// applied (served views).
// advance: the pull round's last workgroup starts the next round itself
// (the asynchronous peel then queues the split rows in its start phase, in
// place of the separate completion kernel).
hipError_t launch_pull_round_args(Graph &g, const PeelArgs &a, const uint32_t *bits,
                                  const int32_t *corr_x, const int32_t *corr_d, int ncorr,
                                  bool advance, hipStream_t s, bool queue_f0 = false,
                                  const uint32_t *rowbits = nullptr, bool force = false,
                                  bool rest_part = false, bool rank = false);
hipError_t launch_pull_fixup_args(Graph &g, const PeelArgs &a, const uint32_t *bits,
                                  hipStream_t s);
hipError_t launch_peel_async_args(Graph &g, PeelKind kind, const PeelArgs &a, int grid,
                                  hipStream_t s);
hipError_t launch_peel_rounds(Graph &g, PeelKind kind, int32_t thrU, int32_t thrL,
                              int rounds, hipStream_t s);
hipError_t launch_peel_persistent(Graph &g, PeelKind kind, int32_t thrU, int32_t thrL,
                                  hipStream_t s);
hipError_t launch_peel_async(Graph &g, PeelKind kind, int32_t thrU, int32_t thrL,
                             hipStream_t s);
hipError_t launch_pack(Graph &g, int32_t thrU, int32_t thrL, uint32_t *bits,
                       hipStream_t s);
hipError_t launch_pack_from_core(Graph &g, int32_t k, uint32_t *bits, hipStream_t s);
hipError_t launch_classify(Graph &g, int32_t dl, int32_t dq, hipStream_t s);
hipError_t launch_restricted_init(Graph &g, int32_t thrU, int32_t thrL, int32_t dl,
                                  hipStream_t s);
hipError_t launch_kcore_init(Graph &g, hipStream_t s);
hipError_t launch_kcore_persistent(Graph &g, hipStream_t s);
hipError_t launch_kcore_steps(Graph &g, int steps, hipStream_t s);
hipError_t launch_kcore_levels(Graph &g, int levels, hipStream_t s);
hipError_t launch_cc(Graph &g, int32_t only_label, hipStream_t s);
hipError_t query_persistent_grids(Graph &g);
abcore_status build_pieces(Graph &g, hipStream_t s);
// Degree ranks and the rank-sorted adjacency copy (Graph::rank, rcols); on
// an allocation failure it leaves them null and succeeds.
abcore_status build_ranks(Graph &g, hipStream_t s);
hipError_t launch_answer_view(const PeelArgs &a, int32_t x, int32_t y, hipStream_t s);
// After a peel scoped to the components of vx and vy: the survivors of that
// scope, or with `connected` those reachable from vx or vy through
// survivors, into d_bits (every word); *count (nullable) their number.
// Synchronous.  Needs g.list and g.list2 for `connected`.
abcore_status scoped_set(Graph &g, int32_t vx, int32_t vy, int32_t thrU, int32_t thrL,
                         bool connected, uint32_t *d_bits, int64_t *count, hipStream_t s);
// Largest deg0 over ids [lo, hi); set bits of a ceil(n/32)-word bitmask.
// Synchronous.
abcore_status max_degree(Graph &g, int64_t lo, int64_t hi, int32_t *out, hipStream_t s);
// Core numbers (Definition 2) of the current graph into g.core (cached per
// graph version).  Synchronous.
abcore_status compute_core_numbers(Graph &g, hipStream_t s);
// The core numbers of the live vertices of an alive list (cnt entries,
// those with core < 0) once every vertex of core < k0 has its value, by the
// h-index fixpoint; *finished false if it needed more than max_halves
// half sweeps.
abcore_status kcore_top(Graph &g, const int32_t *alive, int64_t cnt, int32_t k0,
                        int max_halves, bool *finished, int32_t *top_max, hipStream_t s);
abcore_status count_bits(Graph &g, const uint32_t *bits, int64_t *out, hipStream_t s);
hipError_t launch_update_window(Graph &g, const int32_t *d_upd, int w, WindowRecord *d_rec,
                                hipStream_t s);
hipError_t launch_relabel(Graph &g, int32_t from, int32_t to, hipStream_t s);
void set_error(const char *fmt, ...);

int peel_grid(const Graph &g);
int wide_grid(const Graph &g);
int async_peel_grid(const Graph &g);

}  // namespace abc
