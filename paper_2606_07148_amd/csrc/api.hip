// C-ABI entry points of libabcore (declared in include/abcore.h).
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <tuple>
#include <mutex>
#include <new>
#include <unordered_map>

#include "abcore_internal.h"

namespace abc {

static thread_local char g_error[512] = "";

// ------------------------------------------------- allocation accounting --
static std::mutex g_mem_mu;
static std::unordered_map<void *, size_t> g_mem_sizes;
static int64_t g_mem_current = 0, g_mem_peak = 0;
static int64_t g_mem_budget = 0;  // abcore_set_memory_budget (0: none)

// Every device allocation of the library.  Under a budget the bytes are
// reserved before hipMalloc, so that concurrent callers cannot overrun it;
// a request beyond it fails as out of memory.
hipError_t dev_malloc_bytes(void **p, size_t bytes) {
  {
    std::lock_guard<std::mutex> lock(g_mem_mu);
    if (g_mem_budget > 0 && g_mem_current + (int64_t)bytes > g_mem_budget) {
      *p = nullptr;
      return hipErrorOutOfMemory;
    }
    g_mem_current += (int64_t)bytes;
  }
  hipError_t e = hipMalloc(p, bytes);
  std::lock_guard<std::mutex> lock(g_mem_mu);
  if (e == hipSuccess && *p != nullptr) {
    g_mem_sizes[*p] = bytes;
    g_mem_peak = std::max(g_mem_peak, g_mem_current);
  } else {
    g_mem_current -= (int64_t)bytes;
  }
  return e;
}

hipError_t dev_malloc_async_bytes(void **p, size_t bytes, hipStream_t s) {
  {
    std::lock_guard<std::mutex> lock(g_mem_mu);
    if (g_mem_budget > 0 && g_mem_current + (int64_t)bytes > g_mem_budget) {
      *p = nullptr;
      return hipErrorOutOfMemory;
    }
    g_mem_current += (int64_t)bytes;
  }
  hipError_t e = hipMallocAsync(p, bytes, s);
  std::lock_guard<std::mutex> lock(g_mem_mu);
  if (e == hipSuccess && *p != nullptr) {
    g_mem_sizes[*p] = bytes;
    g_mem_peak = std::max(g_mem_peak, g_mem_current);
  } else {
    *p = nullptr;
    g_mem_current -= (int64_t)bytes;
  }
  return e;
}

static void forget(void *p) {
  std::lock_guard<std::mutex> lock(g_mem_mu);
  auto it = g_mem_sizes.find(p);
  if (it != g_mem_sizes.end()) {
    g_mem_current -= (int64_t)it->second;
    g_mem_sizes.erase(it);
  }
}

hipError_t dev_free(void *p) {
  if (p == nullptr) return hipSuccess;
  forget(p);
  return hipFree(p);
}

hipError_t dev_free_async(void *p, hipStream_t s) {
  if (p == nullptr) return hipSuccess;
  forget(p);
  return hipFreeAsync(p, s);
}

// ----------------------------------------------------------- tuning cache --
// Mappings chosen by abcore_autotune, per device architecture, compute-unit
// count, graph shape (log2 of the vertex count and of the adjacency entries)
// and workload kind (0 = single query, 1 = batch), shared by every handle
// of the process and savable to a text file.
struct TuneKey {
  std::string arch;
  int cu, nlog, elog, kind;
  bool operator<(const TuneKey &o) const {
    return std::tie(arch, cu, nlog, elog, kind) < std::tie(o.arch, o.cu, o.nlog, o.elog, o.kind);
  }
};
struct TuneVal {
  int grid, claim;
  double ms;
};
static std::mutex g_tune_mu;
static std::map<TuneKey, TuneVal> g_tune;

static int floor_log2(int64_t v) {
  int l = 0;
  while (v > 1) {
    v >>= 1;
    ++l;
  }
  return l;
}

static TuneKey tune_key(const Graph &g, int kind) {
  return TuneKey{g.arch, g.cu_count, floor_log2(std::max<int64_t>(g.n, 1)),
                 floor_log2(std::max<int64_t>(2 * g.m, 1)), kind};
}

static void tune_store(const Graph &g, int kind, int grid, int claim, double ms) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune[tune_key(g, kind)] = TuneVal{grid, claim, ms};
}

static bool tune_find(const Graph &g, int kind, TuneVal *out) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune.find(tune_key(g, kind));
  if (it == g_tune.end()) return false;
  *out = it->second;
  return true;
}

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_error, sizeof(g_error), fmt, ap);
  va_end(ap);
}

abcore_status build_csr_device(Graph &g, const int32_t *eu, const int32_t *ev, int64_t m,
                               hipStream_t s);
hipError_t launch_relabel(Graph &g, int32_t from, int32_t to, hipStream_t s);
hipError_t launch_update(Graph &g, int32_t u, int32_t v, int32_t op, int64_t slot,
                         hipStream_t s);
hipError_t launch_answer(Graph &g, int32_t x, int32_t y, int32_t thrU, int32_t thrL,
                         hipStream_t s);
hipError_t launch_export(Graph &g, int64_t *out_off, int32_t *out_cols, hipStream_t s);
hipError_t prepare_pull_kernel(Graph &g);
bool serving(const Graph &g);
abcore_status serve_start(Graph &g, int64_t max_inflight, int32_t slots, int32_t window);
abcore_status serve_stop(Graph &g);
void destroy_server(Graph &g);
abcore_status serve_submit(Graph &g, const abcore_edge_update &upd, int32_t thrU, int32_t thrL,
                           uint64_t *ticket);
abcore_status serve_poll(Graph &g, uint64_t ticket, int32_t *answer, uint32_t *bits,
                         uint64_t *t_done);
void serve_counters(const Graph &g, int64_t *out, int count);

// Storage for edges inserted after the build: the per-vertex list heads and
// room for at least min_cap pairs (doubling), with a deletion version per
// pair (0 for pairs present before serving, so their tombstones hold for
// every served version).  Synchronous; moves the pair arrays.
abcore_status grow_delta(Graph &g, int64_t min_cap, hipStream_t s) {
  Delta &d = g.delta;
  hipError_t e = hipSuccess;
  if (d.head == nullptr) {
    e = dev_malloc(&d.head, sizeof(int32_t) * std::max<int64_t>(g.n, 1));
    if (e == hipSuccess)
      e = hipMemsetAsync(d.head, 0xFF, sizeof(int32_t) * std::max<int64_t>(g.n, 1), s);
    if (e != hipSuccess) {
      if (d.head) (void)dev_free(d.head);
      d.head = nullptr;
      set_error("delta allocation failed: %s", hipGetErrorString(e));
      return ABCORE_ENOMEM;
    }
  }
  if (min_cap <= d.cap && min_cap <= g.pair_del_cap) return ABCORE_OK;
  int64_t ncap = std::max<int64_t>(1024, d.cap);
  while (ncap < min_cap) ncap *= 2;
  int32_t *nn = nullptr, *no = nullptr, *nv = nullptr;
  e = dev_malloc(&nn, sizeof(int32_t) * 2 * ncap);
  if (e == hipSuccess) e = dev_malloc(&no, sizeof(int32_t) * 2 * ncap);
  if (e == hipSuccess) e = dev_malloc(&nv, sizeof(int32_t) * ncap);
  if (e == hipSuccess) e = hipMemsetAsync(nv, 0, sizeof(int32_t) * ncap, s);
  if (e == hipSuccess && d.count > 0) {
    e = hipMemcpyAsync(nn, d.next, sizeof(int32_t) * 2 * d.count, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(no, d.other, sizeof(int32_t) * 2 * d.count, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && g.pair_del_ver)
      e = hipMemcpyAsync(nv, g.pair_del_ver, sizeof(int32_t) * d.count, hipMemcpyDeviceToDevice,
                         s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    for (void *p : {(void *)nn, (void *)no, (void *)nv})
      if (p) (void)dev_free(p);
    set_error("delta growth failed: %s", hipGetErrorString(e));
    return ABCORE_ENOMEM;
  }
  if (d.next) (void)dev_free(d.next);
  if (d.other) (void)dev_free(d.other);
  if (g.pair_del_ver) (void)dev_free(g.pair_del_ver);
  d.next = nn;
  d.other = no;
  g.pair_del_ver = nv;
  d.cap = ncap;
  g.pair_del_cap = ncap;
  return ABCORE_OK;
}

namespace {

#define CHK(x)                                                                     \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) {                                                        \
      set_error("%s: %s failed: %s", __func__, #x, hipGetErrorString(e_));         \
      return e_ == hipErrorOutOfMemory ? ABCORE_ENOMEM : ABCORE_EDEVICE;           \
    }                                                                              \
  } while (0)

#define TRY(x)                                 \
  do {                                         \
    abcore_status s_ = (x);                    \
    if (s_ != ABCORE_OK) return s_;            \
  } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline int32_t clamp_thr(uint32_t t) {
  return (int32_t)std::min<uint64_t>(t, (uint64_t)kMaxThreshold);
}

void free_graph(Graph *g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  destroy_server(*g);
  if (g->del_ver) (void)dev_free(g->del_ver);
  if (g->pair_del_ver) (void)dev_free(g->pair_del_ver);
  for (auto &ev : g->events)
    for (auto &pr : ev) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : g->event_pool) (void)hipEventDestroy(e);
  if (g->batch.exec) (void)hipGraphExecDestroy(g->batch.exec);
  if (g->batch.graph) (void)hipGraphDestroy(g->batch.graph);
  if (g->capture_stream) (void)hipStreamDestroy(g->capture_stream);
  for (int32_t *p : g->slots)
    if (p) (void)dev_free(p);
  void *bufs[] = {g->off,        g->cols,        g->deg0,        g->deg,
                  g->queue,      g->list,        g->list2,       g->state,
                  g->core,       g->comp,        g->parent,      g->delta.head,
                  g->delta.next, g->delta.other, g->alive_bits,  g->part,
                  g->piece_row,  g->piece_start, g->piece_first, g->heavy_rows,
                  g->pull_bounds, g->row_bits,    g->split_written, g->rank,
                  g->rcols,       g->rank_vtx,    g->roff,        g->rp_row,
                  g->rp_start,    g->rp_first,    g->rdeg,        g->state_alt,
                  g->part_alt,    g->rs_fail,     g->aux,         g->probe_bits,
                  g->dbg_enqueue, g->kdead};
  for (void *p : bufs)
    if (p) (void)dev_free(p);
  for (void *p : g->top_buf)
    if (p) (void)dev_free(p);
  if (g->h_abort) (void)hipHostFree(g->h_abort);
  if (g->h_state) (void)hipHostFree(g->h_state);
  if (g->h_part) (void)hipHostFree(g->h_part);
  delete g;
}

template <class T>
abcore_status ensure(T **p, int64_t count) {
  if (*p) return ABCORE_OK;
  hipError_t e = dev_malloc(p, sizeof(T) * std::max<int64_t>(count, 1));
  if (e != hipSuccess) {
    *p = nullptr;
    set_error("device allocation of %lld elements failed: %s", (long long)count,
              hipGetErrorString(e));
    return ABCORE_ENOMEM;
  }
  return ABCORE_OK;
}

hipError_t take_event(Graph &g, hipEvent_t *e) {
  if (!g.event_pool.empty()) {
    *e = g.event_pool.back();
    g.event_pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

// Records an event pair of kernel kind `kind` around `launch` when timing
// is on (kinds: ABCORE_KERNEL_PEEL, _PULL, _SCAN, _PACK, _FIXUP).
template <class F>
hipError_t timed(Graph &g, int kind, hipStream_t s, int64_t nlaunch, F launch) {
  if (!g.timing) return launch();
  hipEvent_t a, b;
  hipError_t e = take_event(g, &a);
  if (e != hipSuccess) return e;
  if ((e = take_event(g, &b)) != hipSuccess) return e;
  if ((e = hipEventRecord(a, s)) != hipSuccess) return e;
  if ((e = launch()) != hipSuccess) return e;
  if ((e = hipEventRecord(b, s)) != hipSuccess) return e;
  g.events[kind].emplace_back(a, b);
  g.timed_launches[kind] += nlaunch;
  return hipSuccess;
}

abcore_status read_state(Graph &g, hipStream_t s) {
  CHK(hipMemcpyAsync(g.h_state, g.state, sizeof(PeelState), hipMemcpyDeviceToHost, s));
  CHK(hipStreamSynchronize(s));
  if (g.h_state->abort_flag) {
    g.rs_ready = false;  // the next query in rank order prepares the workspace
    if (g.h_abort) __atomic_store_n(g.h_abort, 0, __ATOMIC_RELEASE);  // reported here
    set_error("a device-side wait exceeded its spin limit; the result is invalid");
    return ABCORE_EDEVICE;
  }
  return ABCORE_OK;
}

// Reports a spin-limit abort of an earlier asynchronous computation on the
// handle (its peel set the pinned word when it ended) and readies the
// workspace again: the next query in rank order runs its preparation, which
// returns the queue's used slots to empty and clears the failure word, and
// any other computation resets the workspace as it starts.
abcore_status check_abort(Graph &g) {
  if (g.h_abort == nullptr || __atomic_load_n(g.h_abort, __ATOMIC_ACQUIRE) == 0)
    return ABCORE_OK;
  __atomic_store_n(g.h_abort, 0, __ATOMIC_RELEASE);
  g.rs_ready = false;
  set_error("an earlier computation on this handle ended by a spin-limit abort; its result "
            "was invalid (the workspace is reset; later calls are exact)");
  return ABCORE_EDEVICE;
}

int64_t sum_part(Graph &g, int field, hipStream_t s, abcore_status *st) {
  hipError_t e = hipMemcpyAsync(g.h_part, g.part, sizeof(int64_t) * kMaxBlocks * kPartFields,
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    set_error("reading partial sums failed: %s", hipGetErrorString(e));
    *st = ABCORE_EDEVICE;
    return 0;
  }
  int64_t t = 0;
  for (int b = 0; b < kMaxBlocks; ++b) t += g.h_part[(int64_t)b * kPartFields + field];
  *st = ABCORE_OK;
  return t;
}

// Runs the peel rounds of the current frontier to completion.  Persistent
// mode: one cooperative launch, no host involvement.  Round mode: round
// kernels in growing batches (4, 8, 16, ...), checking convergence between
// batches; a launch after convergence returns immediately.
abcore_status run_peel(Graph &g, PeelKind kind, int32_t thrU, int32_t thrL, hipStream_t s,
                       int64_t *launches) {
  if (g.peel_mode == 3) {
    CHK(timed(g, ABCORE_KERNEL_PEEL, s, 1,
              [&] { return launch_peel_async(g, kind, thrU, thrL, s); }));
    *launches += 1;
    return ABCORE_OK;
  }
  if (g.peel_mode == 2) {
    CHK(timed(g, ABCORE_KERNEL_PEEL, s, 1,
              [&] { return launch_peel_persistent(g, kind, thrU, thrL, s); }));
    *launches += 1;
    return ABCORE_OK;
  }
  // every non-empty round removes at least one vertex
  const int64_t max_launches = g.n + 4 * (int64_t)std::max(4, g.rounds_per_sync) + 8;
  int batch = 4;
  for (int64_t done = 0; done < max_launches; done += batch) {
    CHK(timed(g, ABCORE_KERNEL_PEEL, s, batch,
              [&] { return launch_peel_rounds(g, kind, thrU, thrL, batch, s); }));
    *launches += batch;
    TRY(read_state(g, s));
    bool empty = true;
    for (int j = 0; j < kSub; ++j) empty &= g.h_state->lo[j] >= g.h_state->hi[j];
    if (empty) return ABCORE_OK;
    batch = std::min(batch * 2, std::max(4, g.rounds_per_sync));
  }
  set_error("peel did not converge");
  return ABCORE_EDEVICE;
}

// After a scan: the first round in pull form (when pull is set and the
// device decides so), the peel to completion and, when bits is given, the
// bitmask.  In the asynchronous mode the pull round's completion (split
// rows below their threshold) and the pack run inside the peel kernel.
// Survivor counts of a query in rank order: ku upper and kl lower vertices
// of degree >= their threshold, and the entries of the other vertices (what
// pushing them would cost).  False when the graph has changed since the
// build or has no rank relabelling.
bool rank_counts(const Graph &g, int32_t thrU, int32_t thrL, int64_t &ku, int64_t &kl,
                 int64_t &f0deg) {
  if (g.version != 0 || g.delta.count > 0 || g.rcols == nullptr || g.rp_first == nullptr ||
      g.rdeg == nullptr ||
      g.rk_cnt[0].empty() || g.rk_cnt[1].empty())
    return false;
  auto at = [](const std::vector<int64_t> &v, int32_t t) {
    return t >= 0 && (size_t)t < v.size() ? v[t] : 0;
  };
  ku = at(g.rk_cnt[0], thrU);
  kl = at(g.rk_cnt[1], thrL);
  f0deg = 2 * g.m_csr - at(g.rk_ent[0], thrU) - at(g.rk_ent[1], thrL);
  return true;
}

abcore_status pull_peel_pack(Graph &g, PeelKind kind, int32_t thrU, int32_t thrL, bool pull,
                             uint32_t *bits, hipStream_t s, int64_t *launches,
                             bool queue_f0 = false, const uint32_t *rowbits = nullptr,
                             bool force = false, bool rest_part = false, bool rank = false,
                             const uint32_t *f0bits = nullptr) {
  const bool fused = g.peel_mode == 3;
  rank = rank && fused && g.rcols != nullptr;
  if (pull) {
    CHK(timed(g, ABCORE_KERNEL_PULL, s, 1, [&] {
      return launch_pull_round(g, thrU, thrL, s, fused, queue_f0, rowbits, force, rest_part,
                               rank, f0bits);
    }));
    if (!fused)
      CHK(timed(g, ABCORE_KERNEL_FIXUP, s, 1,
                [&] { return launch_pull_fixup(g, thrU, thrL, s); }));
  }
  if (fused) {
    CHK(timed(g, ABCORE_KERNEL_PEEL, s, 1, [&] {
      return launch_peel_async_fused(g, kind, thrU, thrL,
                                     pull ? (rowbits ? rowbits : g.alive_bits) : nullptr, bits,
                                     s, rank && pull);
    }));
    *launches += 1;
    return ABCORE_OK;
  }
  TRY(run_peel(g, kind, thrU, thrL, s, launches));
  if (bits)
    CHK(timed(g, ABCORE_KERNEL_PACK, s, 1,
              [&] { return launch_pack(g, thrU, thrL, bits, s); }));
  return ABCORE_OK;
}

abcore_status compute_core(Graph &g, hipStream_t s) {
  if (g.core_valid) return ABCORE_OK;
  TRY(ensure(&g.core, g.n));
  TRY(ensure(&g.list, g.n));
  TRY(ensure(&g.list2, g.n));
  TRY(ensure(&g.kdead, (g.n + 31) / 32));
  CHK(launch_kcore_init(g, s));
  g.kcore_top_used = false;
  for (int64_t &v : g.top_stats) v = 0;
  const auto t_levels = std::chrono::steady_clock::now();
  if (g.peel_mode == 3) {
    // levels of a scan and an asynchronous peel, in growing batches between
    // checks; every level either removes a vertex or jumps to one that does
    const int64_t max_levels = 2 * g.n + 8;
    int batch = 8;
    int64_t done = 0;
    bool top_tried = false;
    for (; done < max_levels; done += batch) {
      CHK(launch_kcore_levels(g, batch, s));
      TRY(read_state(g, s));
      if (g.h_state->done) break;
      // the deep levels by the h-index fixpoint once the live part (the
      // next_k-core) is small: at most kcore_switch vertices
      // (the list may still hold removed entries: the live count decides)
      const int64_t alive = g.h_state->live;
      if (!top_tried && g.h_state->next_k >= 1 && alive <= g.kcore_switch) {
        top_tried = true;
        bool fin = false;
        int32_t tmax = 0;
        const int32_t *L = g.h_state->alive_sel ? g.list2 : g.list;
        const auto t_top = std::chrono::steady_clock::now();
        g.top_ms[0] = std::chrono::duration<double, std::milli>(t_top - t_levels).count();
        // the h-index phase needs temporaries of the deep core's size; when
        // they do not fit the memory budget the levels finish the job
        const abcore_status ts =
            kcore_top(g, L, g.h_state->alive_cur, g.h_state->next_k, 8192, &fin, &tmax, s);
        if (ts != ABCORE_OK && ts != ABCORE_ENOMEM) return ts;
        g.top_ms[1] = std::chrono::duration<double, std::milli>(
                          std::chrono::steady_clock::now() - t_top).count();
        if (fin) {
          g.max_core = std::max(g.h_state->max_core, tmax);
          g.core_valid = true;
          g.kcore_top_used = true;
          return ABCORE_OK;
        }
      }
      batch = std::min(batch * 2, 256);
    }
    if (done >= max_levels) {
      set_error("core decomposition did not converge");
      return ABCORE_EDEVICE;
    }
  } else if (g.peel_mode >= 2 && g.kcore_grid > 0) {
    CHK(launch_kcore_persistent(g, s));
    TRY(read_state(g, s));
    if (!g.h_state->done) {
      set_error("core decomposition did not finish");
      return ABCORE_EDEVICE;
    }
  } else {
    // each step removes a vertex, raises the level past a live degree, or
    // compacts the alive list after a scan
    const int64_t max_steps = 4 * g.n + 256;
    int batch = 8;
    int64_t done = 0;
    for (; done < max_steps; done += batch) {
      CHK(launch_kcore_steps(g, batch, s));
      TRY(read_state(g, s));
      if (g.h_state->done) break;
      batch = std::min(batch * 2, 64);
    }
    if (done >= max_steps) {
      set_error("core decomposition did not converge");
      return ABCORE_EDEVICE;
    }
  }
  g.max_core = g.h_state->max_core;
  g.core_valid = true;
  return ABCORE_OK;
}

}  // namespace

abcore_status compute_core_numbers(Graph &g, hipStream_t s) { return compute_core(g, s); }

namespace {

abcore_status compute_components(Graph &g, hipStream_t s) {
  if (g.comp_valid) return ABCORE_OK;
  TRY(ensure(&g.comp, g.n));
  TRY(ensure(&g.parent, g.n));
  if (g.n > 0) CHK(launch_cc(g, -1, s));
  CHK(hipStreamSynchronize(s));
  g.comp_valid = true;
  return ABCORE_OK;
}

abcore_status ensure_delta(Graph &g, hipStream_t s) {
  return grow_delta(g, g.delta.count + 1, s);
}

// ------------------------------------------------------------- batches --
// Runs the nested sequence of a batch plan on stream s (every launch is
// stream-ordered with no host read, so the sequence can be captured).
// Working degrees of query i live in slot plan.slot[i]; g.deg is restored on
// every exit.
// Runs the plan on stream s.  times (nullable, q entries): the device time
// of each query's launches in milliseconds (an event pair around each;
// synchronises at the end), for the calibration of the first call.
abcore_status run_batch(Graph &g, const BatchPlan &plan, const int32_t *tu, const int32_t *tl,
                        uint32_t *bits, hipStream_t s, std::vector<float> *times = nullptr) {
  struct Restore {
    Graph &g;
    int32_t *deg;
    ~Restore() { g.deg = deg; }
  } restore{g, g.deg};
  const int64_t words = (g.n + 31) / 32;
  const bool pull = g.pull_mode != 1;
  int64_t launches = 0;
  CHK(launch_init_state(g, s));  // clears the abort flag once for the batch
  std::vector<hipEvent_t> ev;
  struct FreeEvents {
    std::vector<hipEvent_t> &ev;
    ~FreeEvents() {
      for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
  } free_events{ev};
  if (times) {
    times->assign(plan.parent.size(), 0.0f);
    ev.resize(2 * plan.parent.size(), nullptr);
    for (hipEvent_t &e : ev) CHK(hipEventCreate(&e));
  }
  for (int32_t i : plan.order) {
    uint32_t *out = bits + (int64_t)i * words;
    const int32_t p0 = plan.parent[i];
    if (plan.dup[i]) {
      if (words > 0)
        CHK(hipMemcpyAsync(out, bits + (int64_t)p0 * words, sizeof(uint32_t) * words,
                           hipMemcpyDeviceToDevice, s));
      continue;
    }
    // a query measured faster from scratch starts as a root does
    const int32_t p = !plan.scratch.empty() && plan.scratch[i] ? -1 : p0;
    if (times) CHK(hipEventRecord(ev[2 * i], s));
    struct Stop {
      std::vector<hipEvent_t> &ev;
      int32_t i;
      hipStream_t s;
      bool on;
      ~Stop() {
        if (on) (void)hipEventRecord(ev[2 * i + 1], s);
      }
    } stop{ev, i, s, times != nullptr};
    g.deg = g.slots[plan.slot[i]];
    if (p < 0 && pull && g.peel_mode == 3) {
      // a root runs as a single query does: the fused scan and reset, then a
      // first round counted on the degree-rank copy when the graph has one
      CHK(launch_scan_reset_gcc(g, tu[i], tl[i], s, true));
      TRY(pull_peel_pack(g, kGCC, tu[i], tl[i], true, out, s, &launches, true, nullptr, false,
                         false, g.rank_order && g.version == 0));
    } else if (p < 0) {
      CHK(launch_init_state(g, s, true));
      CHK(launch_scan_gcc(g, tu[i], tl[i], pull, s));
      TRY(pull_peel_pack(g, kGCC, tu[i], tl[i], pull, out, s, &launches));
    } else {
      // a child that does not continue in its parent's buffer copies the
      // parent's state as its scan reads it; a pull round over the parent's
      // survivors when the frontier is heavy (decided on the device from
      // the scan's sums), else the pull kernel queues the frontier from the
      // scan's frontier bitmap (fused mode; otherwise the scan queues it)
      const int32_t *src = plan.copy[i] ? g.slots[plan.slot[p]] : nullptr;
      uint32_t *fbits = pull && g.peel_mode == 3 && g.pull_mode != 1 ? g.row_bits : nullptr;
      CHK(launch_init_state(g, s, true));
      CHK(launch_scan_nested(g, tu[p], tl[p], tu[i], tl[i], s, pull ? g.alive_bits : nullptr,
                             src, fbits));
      TRY(pull_peel_pack(g, kGCC, tu[i], tl[i], pull, out, s, &launches, fbits != nullptr,
                         nullptr, false, true, false, fbits));
    }
  }
  if (times) {
    CHK(hipStreamSynchronize(s));
    for (int32_t i : plan.order) {
      if (plan.dup[i]) continue;
      float ms = 0.0f;
      CHK(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
      (*times)[i] = ms;
    }
  }
  return ABCORE_OK;
}

// The first call of a batch (before its capture) measures, per query with a
// parent, the nested start against a start from scratch as a root does (on
// an unchanged graph: the scan, then the first round counted on the
// degree-rank copy).  Nesting peels only the difference between the two
// cores, through atomic decrements; from scratch, the survivors of the
// degree scan count their surviving neighbours by a search of their sorted
// rank rows.  When the parent's core is much larger than the child's, the
// second wins (measured 2 ms against 0.06 ms).  Both leave a valid state
// for the query's own children (every survivor's degree in its core), so the
// choice is per query.  Two eager passes of the batch, then the plan.
abcore_status calibrate_batch(Graph &g, BatchPlan &plan, const int32_t *tu, const int32_t *tl,
                              uint32_t *bits, hipStream_t s) {
  const int32_t q = (int32_t)plan.parent.size();
  plan.scratch.assign(q, 0);
  std::vector<float> nested, fresh;
  TRY(run_batch(g, plan, tu, tl, bits, s, &nested));
  TRY(read_state(g, s));
  plan.scratch.assign(q, 1);
  TRY(run_batch(g, plan, tu, tl, bits, s, &fresh));
  TRY(read_state(g, s));
  for (int32_t i = 0; i < q; ++i)
    plan.scratch[i] = plan.parent[i] >= 0 && !plan.dup[i] && fresh[i] < nested[i] ? 1 : 0;
  return ABCORE_OK;
}

// The measured choice applies where a query from scratch starts as a root
// does in the asynchronous mode: first round in pull form, degree-rank copy
// available and the graph unchanged since its build.
bool pull_mode_allows_calibration(const Graph &g) {
  return g.peel_mode == 3 && g.pull_mode != 1 && g.rank_order && g.version == 0 &&
         g.rcols != nullptr;
}

abcore_status ensure_slots(Graph &g, int n_slots) {
  while ((int)g.slots.size() < n_slots) {
    int32_t *p = nullptr;
    hipError_t e = dev_malloc(&p, sizeof(int32_t) * std::max<int64_t>(g.n, 1));
    if (e != hipSuccess) {
      set_error("batch: allocation of degree state %d failed: %s", (int)g.slots.size(),
                hipGetErrorString(e));
      return ABCORE_ENOMEM;
    }
    g.slots.push_back(p);
  }
  return ABCORE_OK;
}

void drop_batch_cache(Graph &g) {
  if (g.batch.exec) (void)hipGraphExecDestroy(g.batch.exec);
  if (g.batch.graph) (void)hipGraphDestroy(g.batch.graph);
  g.batch = BatchCache();
}

}  // namespace

// Plan of a batch of queries (host only).  Query i computes the core for
// thresholds (tu[i], tl[i]).  The (a,b)-core is contained in the (a',b')-core
// whenever a' <= a and b' <= b (the nesting that the proof of Lemma 1 uses),
// so a query can start from the final state of any query it dominates and
// peel only the difference.  Queries are taken in lexicographic order of
// (tu, tl), a topological order of dominance; each picks as parent the
// dominated earlier query with the largest tu + tl (the smallest core it
// can expect), among the last kPlanWindow distinct ones.  Equal queries copy
// the bitmask of the first.  The tree runs depth first, the child with the
// largest subtree last: that child continues in its parent's state buffer,
// the others start from a copy, and a buffer returns to the pool when the
// chain using it ends at a leaf.
BatchPlan make_batch_plan(const int32_t *tu, const int32_t *tl, int32_t q) {
  constexpr int kPlanWindow = 4096;
  BatchPlan plan;
  plan.parent.assign(q, -1);
  plan.dup.assign(q, 0);
  plan.copy.assign(q, 0);
  plan.slot.assign(q, -1);
  std::vector<int32_t> idx(q);
  for (int32_t i = 0; i < q; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) {
    return tu[a] != tu[b] ? tu[a] < tu[b] : tl[a] < tl[b];
  });
  std::vector<int32_t> reps;  // distinct queries in sorted order
  std::vector<std::vector<int32_t>> dups(q);
  for (int32_t k = 0; k < q; ++k) {
    const int32_t i = idx[k];
    if (!reps.empty() && tu[reps.back()] == tu[i] && tl[reps.back()] == tl[i]) {
      plan.parent[i] = reps.back();
      plan.dup[i] = 1;
      dups[reps.back()].push_back(i);
      continue;
    }
    int32_t best = -1;
    int64_t best_score = -1;
    const int lo = std::max(0, (int)reps.size() - kPlanWindow);
    for (int r = (int)reps.size() - 1; r >= lo; --r) {
      const int32_t j = reps[r];
      if (tu[j] <= tu[i] && tl[j] <= tl[i]) {
        const int64_t score = (int64_t)tu[j] + tl[j];
        if (score > best_score) {
          best_score = score;
          best = j;
        }
      }
    }
    plan.parent[i] = best;
    reps.push_back(i);
  }
  // children and subtree sizes (a parent precedes its children in reps)
  std::vector<std::vector<int32_t>> kids(q);
  std::vector<int64_t> size(q, 1);
  std::vector<int32_t> roots;
  for (int32_t i : reps) {
    if (plan.parent[i] >= 0)
      kids[plan.parent[i]].push_back(i);
    else
      roots.push_back(i);
  }
  for (auto it = reps.rbegin(); it != reps.rend(); ++it)
    if (plan.parent[*it] >= 0) size[plan.parent[*it]] += size[*it];
  for (int32_t i : reps)
    std::stable_sort(kids[i].begin(), kids[i].end(),
                     [&](int32_t a, int32_t b) { return size[a] < size[b]; });
  // depth-first order and buffer assignment
  std::vector<int32_t> free_slots;
  auto take = [&]() {
    if (!free_slots.empty()) {
      const int32_t s = free_slots.back();
      free_slots.pop_back();
      return s;
    }
    return (int32_t)plan.nslots++;
  };
  std::vector<int32_t> stack;
  for (auto it = roots.rbegin(); it != roots.rend(); ++it) stack.push_back(*it);
  while (!stack.empty()) {
    const int32_t i = stack.back();
    stack.pop_back();
    const int32_t p = plan.parent[i];
    if (p < 0) {
      plan.slot[i] = take();
    } else if (kids[p].back() == i) {
      plan.slot[i] = plan.slot[p];
    } else {
      plan.slot[i] = take();
      plan.copy[i] = 1;
    }
    plan.order.push_back(i);
    for (int32_t d : dups[i]) plan.order.push_back(d);
    if (kids[i].empty()) free_slots.push_back(plan.slot[i]);
    for (auto it = kids[i].rbegin(); it != kids[i].rend(); ++it) stack.push_back(*it);
  }
  return plan;
}

// --------------------------------------------- allocation-free variant --
// abcore_compute_static runs GCC's vertex-order path with its per-query
// working set -- working degrees, frontier sub-queues, peel state, partial
// sums, survivor bitmap -- in this file-scope device array instead of the
// handle's buffers, so the call allocates nothing.  Each device that loads
// the library holds its own copy for the life of the process.  In host code
// the name `scratch` only stands in for the symbol: its device address comes
// from hipGetSymbolAddress, once per device (scratch_base).
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static uint8_t *g_scratch_ptr[kMaxDevices] = {};

// This device's copy of `scratch` (the device must be current).
abcore_status scratch_base(int device, uint8_t **out) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("static scratch: device %d out of range", device);
    return ABCORE_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device] == nullptr) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      set_error("static scratch: hipGetSymbolAddress failed: %s", hipGetErrorString(e));
      return ABCORE_EDEVICE;
    }
    g_scratch_ptr[device] = static_cast<uint8_t *>(p);
  }
  *out = g_scratch_ptr[device];
  return ABCORE_OK;
}

// Byte offsets of the working set in the scratch array (256-byte aligned).
struct StaticLayout {
  size_t queue, deg, bits, state, part, total;
};

StaticLayout static_layout(const Graph &g) {
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  StaticLayout L;
  size_t at = 0;
  L.queue = at;
  at += up(sizeof(int32_t) * (size_t)kSub * (size_t)g.qcap);
  L.deg = at;
  at += up(sizeof(int32_t) * (size_t)std::max<int64_t>(g.n, 1));
  L.bits = at;
  at += up(sizeof(uint32_t) * (size_t)((g.n + 31) / 32 + 1));
  L.state = at;
  at += up(sizeof(PeelState));
  L.part = at;
  at += up(sizeof(int64_t) * (size_t)kMaxBlocks * kPartFields);
  L.total = at;
  return L;
}

// The working set as a fresh one: every queue slot empty, the survivor
// bitmap, the state (cursors, flags, arrival counters) and the partial sums
// zero.  A plain fill kernel, so that a caller may capture the call.
__global__ void static_fill_kernel(uint32_t *queue, int64_t nqueue, uint32_t *zero,
                                   int64_t nzero) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = tid; i < nqueue; i += stride) queue[i] = 0xFFFFFFFFu;  // kEmpty
  for (int64_t i = tid; i < nzero; i += stride) zero[i] = 0u;
}

}  // namespace abc

using namespace abc;

static abcore_status busy_error(const char *fn) {
  set_error("%s: the handle is serving (abcore_serve_stop first)", fn);
  return ABCORE_EBUSY;
}

extern "C" {

const char *abcore_last_error(void) { return g_error; }

abcore_status abcore_build_csr(int32_t n_upper, int32_t n_lower, const int32_t *d_eu,
                               const int32_t *d_ev, int64_t m, void *stream, abcore_graph *out,
                               int64_t *out_m_distinct) {
  if (!out) {
    set_error("abcore_build_csr: out is NULL");
    return ABCORE_EINVAL;
  }
  *out = nullptr;
  if (n_upper < 0 || n_lower < 0 || m < 0 || (int64_t)n_upper + n_lower >= 0x3FFFFFFFLL ||
      m >= 0x7FFFFFFFLL || (m > 0 && (!d_eu || !d_ev))) {
    set_error("abcore_build_csr: invalid sizes or null edge arrays");
    return ABCORE_EINVAL;
  }
  Graph *g = new (std::nothrow) Graph();
  if (!g) {
    set_error("abcore_build_csr: host allocation failed");
    return ABCORE_ENOMEM;
  }
  hipStream_t s = as_stream(stream);
  abcore_status st = ABCORE_OK;
  const auto t_build = std::chrono::steady_clock::now();
  do {
    if (hipGetDevice(&g->device) != hipSuccess) {
      set_error("abcore_build_csr: no HIP device");
      st = ABCORE_EDEVICE;
      break;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, g->device) == hipSuccess) {
      if (prop.multiProcessorCount > 0) g->cu_count = prop.multiProcessorCount;
      snprintf(g->arch, sizeof(g->arch), "%s", prop.gcnArchName);
      for (char *c = g->arch; *c; ++c)
        if (*c == ' ' || *c == '\t') *c = '_';
      if (prop.sharedMemPerBlock > 0) g->lds_per_block = prop.sharedMemPerBlock;
    }
    g->nU = n_upper;
    g->nL = n_lower;
    g->n = (int64_t)n_upper + n_lower;
    {
      // set-up of the allocation-free variant on this device (a failure is
      // reported again by abcore_compute_static, which retries)
      uint8_t *unused = nullptr;
      if (scratch_base(g->device, &unused) != ABCORE_OK) set_error("");
    }
    // each phase ends synchronised, so its wall time is its own
    auto now = [] { return std::chrono::steady_clock::now(); };
    auto ms_since = [&](std::chrono::steady_clock::time_point t) {
      return std::chrono::duration<double, std::milli>(now() - t).count();
    };
    auto t0 = now();
    st = build_csr_device(*g, d_eu, d_ev, m, s);
    if (st == ABCORE_OK && hipStreamSynchronize(s) != hipSuccess) st = ABCORE_EDEVICE;
    if (st != ABCORE_OK) break;
    g->build_ms[0] = ms_since(t0);
    t0 = now();
    st = build_pieces(*g, s);
    if (st == ABCORE_OK && hipStreamSynchronize(s) != hipSuccess) st = ABCORE_EDEVICE;
    if (st != ABCORE_OK) break;
    g->build_ms[1] = ms_since(t0);
    t0 = now();
    st = build_ranks(*g, s);
    if (st == ABCORE_OK && hipStreamSynchronize(s) != hipSuccess) st = ABCORE_EDEVICE;
    if (st != ABCORE_OK) break;
    g->build_ms[2] = ms_since(t0);
    g->qcap = queue_capacity(g->n, g->npieces);
    if ((st = ensure(&g->deg, g->n)) != ABCORE_OK) break;
    if ((st = ensure(&g->queue, (int64_t)kSub * g->qcap)) != ABCORE_OK) break;
    if (hipMemsetAsync(g->queue, 0xFF, sizeof(int32_t) * kSub * g->qcap, s) != hipSuccess) {
      set_error("abcore_build_csr: queue initialisation failed");
      st = ABCORE_EDEVICE;
      break;
    }
    if ((st = ensure(&g->alive_bits, (g->n + 31) / 32 + 1)) != ABCORE_OK) break;
    if ((st = ensure(&g->row_bits, (g->n + 31) / 32 + 1)) != ABCORE_OK) break;
    if ((st = ensure(&g->part, (int64_t)kMaxBlocks * kPartFields)) != ABCORE_OK) break;
    if ((st = ensure(&g->part_alt, (int64_t)kMaxBlocks * kPartFields)) != ABCORE_OK) break;
    hipError_t e = dev_malloc(&g->state, sizeof(PeelState));
    // the state is read (queue tails) by the first initialisation: zero it
    if (e == hipSuccess) e = hipMemsetAsync(g->state, 0, sizeof(PeelState), s);
    if (e == hipSuccess) e = dev_malloc(&g->state_alt, sizeof(PeelState));
    if (e == hipSuccess) e = hipMemsetAsync(g->state_alt, 0, sizeof(PeelState), s);
    if (e == hipSuccess) e = dev_malloc(&g->rs_fail, sizeof(int32_t));
    if (e == hipSuccess) e = hipMemsetAsync(g->rs_fail, 0, sizeof(int32_t), s);
    if (e == hipSuccess) e = hipHostMalloc(&g->h_state, sizeof(PeelState));
    if (e == hipSuccess)
      e = hipHostMalloc(&g->h_abort, sizeof(int32_t), hipHostMallocCoherent);
    if (e == hipSuccess) *g->h_abort = 0;
    if (e == hipSuccess)
      e = hipHostMalloc(&g->h_part, sizeof(int64_t) * kMaxBlocks * kPartFields);
    if (e != hipSuccess) {
      set_error("abcore_build_csr: state allocation failed: %s", hipGetErrorString(e));
      st = ABCORE_ENOMEM;
      break;
    }
    memset(g->h_state, 0, sizeof(PeelState));
#ifdef ABC_DEBUG_ENQUEUE
    if ((st = ensure(&g->dbg_enqueue, g->n)) != ABCORE_OK) break;
    if (hipMemsetAsync(g->dbg_enqueue, 0, sizeof(int32_t) * std::max<int64_t>(g->n, 1), s) !=
        hipSuccess) {
      set_error("abcore_build_csr: debug counter initialisation failed");
      st = ABCORE_EDEVICE;
      break;
    }
#endif
    if (query_persistent_grids(*g) != hipSuccess) {
      // no co-residency information: the cooperative kernels are not used
      g->persistent_grid = 0;
      g->kcore_grid = 0;
      g->async_grid = 0;
      g->peel_mode = 1;
    }
    (void)prepare_pull_kernel(*g);
    if (launch_init_state(*g, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
      set_error("abcore_build_csr: state initialisation failed");
      st = ABCORE_EDEVICE;
      break;
    }
  } while (0);
  if (st != ABCORE_OK) {
    free_graph(g);
    return st;
  }
  g->build_ms[3] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                             t_build).count();
  if (out_m_distinct) *out_m_distinct = g->m;
  *out = reinterpret_cast<abcore_graph>(g);
  return ABCORE_OK;
}

abcore_status abcore_graph_report(abcore_graph h, abcore_report *out) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (!g || !out) {
    set_error("abcore_graph_report: null handle or output");
    return ABCORE_EINVAL;
  }
  out->build_ms = g->build_ms[3];
  out->csr_ms = g->build_ms[0];
  out->pieces_ms = g->build_ms[1];
  out->ranks_ms = g->rcols != nullptr ? g->build_ms[2] : 0.0;
  const int64_t n = g->n, np = g->npieces;
  out->graph_bytes = 8 * (n + 1) + 4 * 2 * g->m_csr + 4 * n + (4 + 8 + 4) * np + 4 * n +
                     4 * g->nheavy;
  out->ranks_bytes = g->rcols == nullptr
                         ? 0
                         : 4 * n + 4 * n + 8 * (n + 1) + 4 * 2 * g->m_csr +
                               (g->rp_row != nullptr ? (4 + 8) * np + 4 * n : 0) +
                               (g->rdeg != nullptr ? 4 * ((int64_t)g->rdeg_mask + 1) : 0);
  out->queue_bytes = 4 * (int64_t)kSub * g->qcap;
  for (int i = 0; i < 4; ++i) out->core_top[i] = g->kcore_top_used ? g->top_stats[i] : 0;
  out->core_levels_ms = g->kcore_top_used ? g->top_ms[0] : 0.0;
  out->core_top_ms = g->kcore_top_used ? g->top_ms[1] : 0.0;
  return ABCORE_OK;
}

abcore_status abcore_set_memory_budget(int64_t bytes) {
  if (bytes < 0) {
    set_error("abcore_set_memory_budget: negative budget");
    return ABCORE_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_mem_mu);
  g_mem_budget = bytes;
  return ABCORE_OK;
}

abcore_status abcore_device_memory(int64_t *current, int64_t *peak, int32_t reset_peak) {
  std::lock_guard<std::mutex> lock(g_mem_mu);
  if (current) *current = g_mem_current;
  if (peak) *peak = g_mem_peak;
  if (reset_peak) g_mem_peak = g_mem_current;
  return ABCORE_OK;
}

abcore_status abcore_destroy(abcore_graph h) {
  free_graph(reinterpret_cast<Graph *>(h));
  return ABCORE_OK;
}

abcore_status abcore_debug_enqueue_counts(abcore_graph h, int32_t *d_counts, int32_t reset,
                                          void *stream) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (!g) {
    set_error("abcore_debug_enqueue_counts: null handle");
    return ABCORE_EINVAL;
  }
  if (serving(*g)) return busy_error(__func__);
  if (g->dbg_enqueue == nullptr) {
    set_error("abcore_debug_enqueue_counts: not a debug build (ABC_DEBUG_ENQUEUE)");
    return ABCORE_EINVAL;
  }
  (void)hipSetDevice(g->device);
  hipStream_t s = as_stream(stream);
  const size_t bytes = sizeof(int32_t) * (size_t)std::max<int64_t>(g->n, 1);
  if (d_counts != nullptr)
    CHK(hipMemcpyAsync(d_counts, g->dbg_enqueue, bytes, hipMemcpyDeviceToDevice, s));
  if (reset) CHK(hipMemsetAsync(g->dbg_enqueue, 0, bytes, s));
  CHK(hipStreamSynchronize(s));
  return ABCORE_OK;
}

abcore_status abcore_graph_info(abcore_graph h, int32_t *n_upper, int32_t *n_lower,
                                int64_t *m) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (!g) {
    set_error("abcore_graph_info: null handle");
    return ABCORE_EINVAL;
  }
  if (n_upper) *n_upper = g->nU;
  if (n_lower) *n_lower = g->nL;
  if (m) *m = g->m;
  return ABCORE_OK;
}

abcore_status abcore_export_csr(abcore_graph h, int64_t *d_off, int32_t *d_cols,
                                int64_t *out_entries, void *stream) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (g && serving(*g)) return busy_error(__func__);
  if (!g) {
    set_error("abcore_export_csr: null handle");
    return ABCORE_EINVAL;
  }
  if (out_entries) *out_entries = 2 * g->m;
  if (!d_off) return ABCORE_OK;
  CHK(hipSetDevice(g->device));
  CHK(launch_export(*g, d_off, d_cols, as_stream(stream)));
  return ABCORE_OK;
}

abcore_status abcore_set_option(abcore_graph h, int32_t option, int64_t value) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (g && serving(*g)) return busy_error(__func__);
  if (!g || value < 0) {
    set_error("abcore_set_option: null handle or negative value");
    return ABCORE_EINVAL;
  }
  switch (option) {
    case ABCORE_OPT_PEEL_MODE:
      if (value > 3 || (value >= 2 && g->persistent_grid <= 0)) {
        set_error("abcore_set_option: peel mode %lld not available", (long long)value);
        return ABCORE_EINVAL;
      }
      g->peel_mode = value != 0 ? (int)value : g->persistent_grid > 0 ? 3 : 1;
      return ABCORE_OK;
    case ABCORE_OPT_GRID:
      g->grid = (int)std::min<int64_t>(value, kMaxBlocks);
      g->tuned = value != 0;  // the caller's choice stands
      return ABCORE_OK;
    case ABCORE_OPT_KCORE_SWITCH:
      g->kcore_switch = value == 0 ? kKcoreSwitch : value;
      g->core_valid = false;
      return ABCORE_OK;
    case ABCORE_OPT_SERVE_PRUNE:
      g->serve_prune = value;
      return ABCORE_OK;
    case ABCORE_OPT_AUTOTUNE:
      if (value > 2) {
        set_error("abcore_set_option: autotune mode %lld unknown", (long long)value);
        return ABCORE_EINVAL;
      }
      g->autotune = value != 2;
      return ABCORE_OK;
    case ABCORE_OPT_ROUNDS_PER_SYNC:
      g->rounds_per_sync = value == 0 ? 16 : (int)std::min<int64_t>(value, 4096);
      return ABCORE_OK;
    case ABCORE_OPT_TIMING:
      g->timing = value != 0;
      return ABCORE_OK;
    case ABCORE_OPT_PULL:
      if (value > 2) {
        set_error("abcore_set_option: pull mode %lld unknown", (long long)value);
        return ABCORE_EINVAL;
      }
      g->pull_mode = (int)value;
      return ABCORE_OK;
    case ABCORE_OPT_RANK_ORDER:
      if (value > 2) {
        set_error("abcore_set_option: rank order mode %lld unknown", (long long)value);
        return ABCORE_EINVAL;
      }
      g->rank_order = value != 2;
      return ABCORE_OK;
    case ABCORE_OPT_SERVE_DEADLINE_US:
      g->serve_deadline_us = value;
      return ABCORE_OK;
    case ABCORE_OPT_APPEND_SUBQUEUE:
      if (value > kSub) {
        set_error("abcore_set_option: sub-queue %lld above %d", (long long)value, kSub);
        return ABCORE_EINVAL;
      }
      g->append_sub = (int32_t)value - 1;
      return ABCORE_OK;
    case ABCORE_OPT_SPIN_LIMIT:
      g->spin_limit = (uint32_t)std::min<int64_t>(value, (int64_t)kAsyncSpinLimit);
      return ABCORE_OK;
    case ABCORE_OPT_CLAIM:
      if (value > kWave) {
        set_error("abcore_set_option: claim %lld above %d", (long long)value, kWave);
        return ABCORE_EINVAL;
      }
      g->claim = value == 0 ? kDefaultClaim : (int)value;
      g->tuned = value != 0;
      return ABCORE_OK;
    default:
      set_error("abcore_set_option: unknown option %d", option);
      return ABCORE_EINVAL;
  }
}

abcore_status abcore_kernel_timing(abcore_graph h, int32_t kernel, double *ms,
                                   int64_t *launches, int32_t reset) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (!g || kernel < 0 || kernel >= Graph::kKernelKinds) {
    set_error("abcore_kernel_timing: null handle or unknown kernel kind");
    return ABCORE_EINVAL;
  }
  CHK(hipSetDevice(g->device));
  double total = 0.0;
  auto &ev = g->events[kernel];
  for (auto &pr : ev) {
    CHK(hipEventSynchronize(pr.second));
    float t = 0.f;
    CHK(hipEventElapsedTime(&t, pr.first, pr.second));
    total += t;
  }
  if (ms) *ms = total;
  if (launches) *launches = g->timed_launches[kernel];
  if (reset) {
    for (auto &pr : ev) {
      g->event_pool.push_back(pr.first);
      g->event_pool.push_back(pr.second);
    }
    ev.clear();
    g->timed_launches[kernel] = 0;
  }
  return ABCORE_OK;
}

abcore_status abcore_core_numbers(abcore_graph h, int32_t *d_core, int32_t *max_core,
                                  void *stream) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (g && serving(*g)) return busy_error(__func__);
  if (!g) {
    set_error("abcore_core_numbers: null handle");
    return ABCORE_EINVAL;
  }
  CHK(hipSetDevice(g->device));
  TRY(check_abort(*g));
  hipStream_t s = as_stream(stream);
  TRY(compute_core(*g, s));
  if (d_core && g->n > 0)
    CHK(hipMemcpyAsync(d_core, g->core, sizeof(int32_t) * g->n, hipMemcpyDeviceToDevice, s));
  CHK(hipStreamSynchronize(s));
  if (max_core) *max_core = g->max_core;
  return ABCORE_OK;
}

abcore_status abcore_components(abcore_graph h, int32_t *d_comp, void *stream) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (g && serving(*g)) return busy_error(__func__);
  if (!g) {
    set_error("abcore_components: null handle");
    return ABCORE_EINVAL;
  }
  CHK(hipSetDevice(g->device));
  hipStream_t s = as_stream(stream);
  TRY(compute_components(*g, s));
  if (d_comp && g->n > 0)
    CHK(hipMemcpyAsync(d_comp, g->comp, sizeof(int32_t) * g->n, hipMemcpyDeviceToDevice, s));
  CHK(hipStreamSynchronize(s));
  return ABCORE_OK;
}

abcore_status abcore_compute(abcore_graph h, uint32_t alpha, uint32_t beta, int32_t algo,
                             uint32_t *d_bitmask, abcore_stats *stats, void *stream) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (g && serving(*g)) return busy_error(__func__);
  if (!g || (!d_bitmask && g->n > 0)) {
    set_error("abcore_compute: null handle or bitmask");
    return ABCORE_EINVAL;
  }
  if (alpha < 1 || beta < 1) {
    set_error("abcore_compute: alpha and beta must be >= 1");
    return ABCORE_EINVAL;
  }
  if (algo != ABCORE_GCC && algo != ABCORE_GCC_PLUS) {
    set_error("abcore_compute: unknown algorithm %d", algo);
    return ABCORE_EINVAL;
  }
  CHK(hipSetDevice(g->device));
  TRY(check_abort(*g));
  hipStream_t s = as_stream(stream);
  if (g->autotune && !g->tuned) {
    // a mapping tuned for single queries on this architecture and shape
    TuneVal v{};
    if (tune_find(*g, 0, &v)) {
      g->grid = v.grid;
      g->claim = v.claim;
    }
  }
  const int32_t thrU = clamp_thr(alpha), thrL = clamp_thr(beta);
  int64_t launches = 0;
  bool plus_pull = false;  // GCC+ initialised by a pull round
  bool rank_order = false;
  int64_t ku = 0, kl = 0, f0deg = 0;
  if (algo == ABCORE_GCC) {
    const bool pull = g->pull_mode != 1;
    // On an unchanged graph the scan's survivors are known in advance (the
    // ranks below K of each layer) and so are the frontier's entries: a
    // pulled first round then runs in rank order, without a scan.
    rank_order = pull && g->peel_mode == 3 && g->rank_order &&
                 rank_counts(*g, thrU, thrL, ku, kl, f0deg) &&
                 (g->pull_mode == 2 || (f0deg > 0 && f0deg * 2 >= ku + kl));
    if (rank_order) {
      // No scan launch: the pull round writes the survivor bitmap into the
      // result (the peel clears the vertices it removes).  The workspace
      // alternates between two states; the previous query in rank order left
      // this one zeroed and the queue empty, else one launch prepares them.
      if (!g->rs_ready)
        CHK(timed(*g, ABCORE_KERNEL_SCAN, s, 1, [&] { return launch_rank_prep(*g, s); }));
      std::swap(g->state, g->state_alt);
      std::swap(g->part, g->part_alt);
      g->rs_parity ^= 1;
      CHK(timed(*g, ABCORE_KERNEL_PULL, s, 1, [&] {
        return launch_rank_query(*g, thrU, thrL, ku, kl, d_bitmask, s, 0);
      }));
      CHK(timed(*g, ABCORE_KERNEL_PEEL, s, 1, [&] {
        return launch_rank_query(*g, thrU, thrL, ku, kl, d_bitmask, s, 1);
      }));
      g->rs_ready = true;
      launches += 1;
    } else if (pull && g->peel_mode == 3) {
      // scan and workspace reset in one launch; the frontier is queued only
      // if the first round is pushed (by the pull kernel, from the bitmap)
      CHK(timed(*g, ABCORE_KERNEL_SCAN, s, 1,
                [&] { return launch_scan_reset_gcc(*g, thrU, thrL, s); }));
      // an unchanged graph counts the first round on its degree-rank copy
      TRY(pull_peel_pack(*g, kGCC, thrU, thrL, true, d_bitmask, s, &launches, true, nullptr,
                         false, false, g->rank_order && g->version == 0));
    } else {
      CHK(launch_init_state(*g, s));
      CHK(timed(*g, ABCORE_KERNEL_SCAN, s, 1,
                [&] { return launch_scan_gcc(*g, thrU, thrL, pull, s); }));
      TRY(pull_peel_pack(*g, kGCC, thrU, thrL, pull, d_bitmask, s, &launches));
    }
  } else {
    TRY(compute_core(*g, s));
    const int32_t dl = std::min(thrU, thrL), dq = std::max(thrU, thrL);
    plus_pull = dl != dq && g->peel_mode == 3 && g->pull_mode != 1;
    if (!plus_pull) CHK(launch_init_state(*g, s));
    if (dl == dq) {
      CHK(launch_pack_from_core(*g, dl, d_bitmask, s));
    } else if (plus_pull) {
      // the uncertain rows' degrees inside G[{core >= delta_l}] by a pull
      // round over LDS-staged bitmaps, then the asynchronous peel
      CHK(timed(*g, ABCORE_KERNEL_SCAN, s, 1,
                [&] { return launch_classify_reset(*g, thrU, thrL, dl, dq, s); }));
      TRY(pull_peel_pack(*g, kGCCPlus, thrU, thrL, true, d_bitmask, s, &launches, false,
                         g->row_bits, true));
    } else {
      CHK(launch_classify(*g, dl, dq, s));
      CHK(launch_restricted_init(*g, thrU, thrL, dl, s));
      TRY(pull_peel_pack(*g, kGCCPlus, thrU, thrL, false, d_bitmask, s, &launches));
    }
  }
  if (stats) {
    TRY(read_state(*g, s));
    abcore_status st = ABCORE_OK;
    const int64_t entries = sum_part(*g, kPartEntries, s, &st);
    if (st != ABCORE_OK) return st;
    const PeelState &p = *g->h_state;
    // queue items count pieces of split rows, so removals are counted from
    // the result: every vertex outside the core
    const int64_t nwords = (g->n + 31) / 32;
    std::vector<uint32_t> words((size_t)std::max<int64_t>(nwords, 1));
    if (nwords > 0) {
      CHK(hipMemcpyAsync(words.data(), d_bitmask, sizeof(uint32_t) * nwords,
                         hipMemcpyDeviceToHost, s));
      CHK(hipStreamSynchronize(s));
    }
    int64_t members = 0;
    for (int64_t i = 0; i < nwords; ++i) members += __builtin_popcount(words[i]);
    const bool plus = algo == ABCORE_GCC_PLUS;
    stats->removed = g->n - members;
    // the asynchronous peel has no rounds
    stats->rounds = (g->peel_mode == 3 && !(algo == ABCORE_GCC_PLUS && thrU == thrL)) ? -1
                                                                                     : p.rounds;
    stats->entries_read = entries;
    // GCC: the scan frontier (its per-workgroup counts; it need not be
    // queued).  GCC+: the uncertain vertices below their threshold after the
    // initialisation, and the uncertain count.
    if (rank_order)
      stats->initial = g->n - ku - kl;
    else if (!plus)
      stats->initial = sum_part(*g, kPartF0, s, &st);
    else if (plus_pull)
      stats->initial = sum_part(*g, kPartF1, s, &st);
    else
      stats->initial = p.first;
    if (st != ABCORE_OK) return st;
    stats->uncertain = !plus ? 0 : (plus_pull ? sum_part(*g, kPartF0, s, &st) : p.aux0);
    if (st != ABCORE_OK) return st;
    stats->launches = launches;
    stats->pulled = p.pulled;
    stats->rank_order = rank_order ? 1 : 0;
  }
  return ABCORE_OK;
}

abcore_status abcore_compute_static(abcore_graph h, uint32_t alpha, uint32_t beta,
                                    uint32_t *d_bitmask, void *stream) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (g && serving(*g)) return busy_error(__func__);
  if (!g || (!d_bitmask && g->n > 0)) {
    set_error("abcore_compute_static: null handle or bitmask");
    return ABCORE_EINVAL;
  }
  if (alpha < 1 || beta < 1) {
    set_error("abcore_compute_static: alpha and beta must be >= 1");
    return ABCORE_EINVAL;
  }
  CHK(hipSetDevice(g->device));
  TRY(check_abort(*g));
  if (g->n == 0) return ABCORE_OK;
  const StaticLayout L = static_layout(*g);
  if (L.total > kStaticScratchBytes) {
    set_error("abcore_compute_static: the working set needs %zu bytes, the static scratch "
              "holds %zu",
              L.total, kStaticScratchBytes);
    return ABCORE_EINVAL;
  }
  uint8_t *base = nullptr;
  TRY(scratch_base(g->device, &base));
  hipStream_t s = as_stream(stream);
  // the handle's working-set pointers point into the scratch for this call
  struct Swap {
    Graph &g;
    int32_t *deg, *queue;
    uint32_t *bits;
    PeelState *state;
    int64_t *part;
    int peel_mode;
    bool timing;
    ~Swap() {
      g.deg = deg;
      g.queue = queue;
      g.alive_bits = bits;
      g.state = state;
      g.part = part;
      g.peel_mode = peel_mode;
      g.timing = timing;
    }
  } restore{*g, g->deg, g->queue, g->alive_bits, g->state, g->part, g->peel_mode, g->timing};
  g->queue = reinterpret_cast<int32_t *>(base + L.queue);
  g->deg = reinterpret_cast<int32_t *>(base + L.deg);
  g->alive_bits = reinterpret_cast<uint32_t *>(base + L.bits);
  g->state = reinterpret_cast<PeelState *>(base + L.state);
  g->part = reinterpret_cast<int64_t *>(base + L.part);
  g->peel_mode = 3;     // the asynchronous worklist (no host reads)
  g->timing = false;    // event pairs would be created on demand
  const int64_t nqueue = (int64_t)kSub * g->qcap;
  const int64_t nzero = (int64_t)((L.total - L.bits) / sizeof(uint32_t));
  static_fill_kernel<<<std::min(g->cu_count * 8, kMaxBlocks), 256, 0, s>>>(
      reinterpret_cast<uint32_t *>(base + L.queue), nqueue,
      reinterpret_cast<uint32_t *>(base + L.bits), nzero);
  CHK(hipGetLastError());
  const int32_t thrU = clamp_thr(alpha), thrL = clamp_thr(beta);
  int64_t launches = 0;
  if (g->pull_mode != 1) {
    CHK(launch_scan_reset_gcc(*g, thrU, thrL, s));
    TRY(pull_peel_pack(*g, kGCC, thrU, thrL, true, d_bitmask, s, &launches, true));
  } else {
    CHK(launch_scan_gcc(*g, thrU, thrL, false, s));
    TRY(pull_peel_pack(*g, kGCC, thrU, thrL, false, d_bitmask, s, &launches));
  }
  return ABCORE_OK;
}

static abcore_status tune_mapping(Graph *g, uint32_t alpha, uint32_t beta, int32_t algo,
                                  void *stream, int *out_grid, int *out_claim, double *out_ms);

static abcore_status batch_thresholds(const uint32_t *h_alpha, const uint32_t *h_beta,
                                      int32_t q, std::vector<int32_t> &tu,
                                      std::vector<int32_t> &tl) {
  if (q < 0 || (q > 0 && (!h_alpha || !h_beta))) {
    set_error("batch: negative count or null threshold array");
    return ABCORE_EINVAL;
  }
  tu.resize(q);
  tl.resize(q);
  for (int32_t i = 0; i < q; ++i) {
    if (h_alpha[i] < 1 || h_beta[i] < 1) {
      set_error("batch: query %d has alpha or beta 0", i);
      return ABCORE_EINVAL;
    }
    tu[i] = clamp_thr(h_alpha[i]);
    tl[i] = clamp_thr(h_beta[i]);
  }
  return ABCORE_OK;
}

abcore_status abcore_batch_plan(const uint32_t *h_alpha, const uint32_t *h_beta, int32_t q,
                                int32_t *h_parent, int32_t *h_order, int32_t *out_states) {
  std::vector<int32_t> tu, tl;
  TRY(batch_thresholds(h_alpha, h_beta, q, tu, tl));
  BatchPlan plan = make_batch_plan(tu.data(), tl.data(), q);
  for (int32_t i = 0; i < q; ++i) {
    if (h_parent) h_parent[i] = plan.parent[i];
    if (h_order) h_order[i] = plan.order[i];
  }
  if (out_states) *out_states = plan.nslots;
  return ABCORE_OK;
}

abcore_status abcore_compute_batch(abcore_graph h, const uint32_t *h_alpha,
                                   const uint32_t *h_beta, int32_t q, uint32_t *d_bitmasks,
                                   void *stream) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (g && serving(*g)) return busy_error(__func__);
  if (!g || (q > 0 && g->n > 0 && !d_bitmasks)) {
    set_error("abcore_compute_batch: null handle or bitmask array");
    return ABCORE_EINVAL;
  }
  std::vector<int32_t> tu, tl;
  TRY(batch_thresholds(h_alpha, h_beta, q, tu, tl));
  if (q == 0 || g->n == 0) return ABCORE_OK;
  CHK(hipSetDevice(g->device));
  TRY(check_abort(*g));
  hipStream_t s = as_stream(stream);
  // the batch's mapping holds for this call only
  struct RestoreMapping {
    Graph &g;
    int grid, claim;
    bool active;
    ~RestoreMapping() {
      if (active) {
        g.grid = grid;
        g.claim = claim;
      }
    }
  } restore_mapping{*g, g->grid, g->claim, false};
  if (g->autotune && !g->tuned && g->peel_mode == 3) {
    // the asynchronous peel's mapping for this architecture and graph
    // shape: from the tuning cache, else tuned now on the batch's median
    // query (by alpha + beta) and cached
    TuneVal v{};
    if (!tune_find(*g, 1, &v)) {
      std::vector<int32_t> idx(q);
      for (int32_t i = 0; i < q; ++i) idx[i] = i;
      std::sort(idx.begin(), idx.end(),
                [&](int32_t x, int32_t y) { return tu[x] + tl[x] < tu[y] + tl[y]; });
      const int32_t r = idx[q / 2];
      TRY(tune_mapping(g, (uint32_t)tu[r], (uint32_t)tl[r], ABCORE_GCC, stream, &v.grid,
                       &v.claim, &v.ms));
      tune_store(*g, 1, v.grid, v.claim, v.ms);
    }
    restore_mapping.active = true;
    g->grid = v.grid;
    g->claim = v.claim;
  }
  BatchPlan plan = make_batch_plan(tu.data(), tl.data(), q);
  TRY(ensure_slots(*g, plan.nslots));
  // the sequence has no host reads in the asynchronous peel mode: it is
  // captured once into a HIP graph and replayed for the same batch
  if (g->peel_mode != 3) {
    TRY(run_batch(*g, plan, tu.data(), tl.data(), d_bitmasks, s));
    return read_state(*g, s);
  }
  std::vector<int32_t> key;
  key.reserve(2 * (size_t)q + 8);
  key.insert(key.end(), tu.begin(), tu.end());
  key.insert(key.end(), tl.begin(), tl.end());
  key.push_back(q);
  key.push_back(g->pull_mode);
  key.push_back(g->grid);
  key.push_back(g->claim);
  key.push_back(g->rank_order ? 1 : 0);
  key.push_back(g->delta.count > 0 ? 1 : 0);
  BatchCache &c = g->batch;
  if (!(c.exec && c.bits == d_bitmasks && c.version == g->version && c.key == key)) {
    drop_batch_cache(*g);
    if (!g->capture_stream) CHK(hipStreamCreateWithFlags(&g->capture_stream, hipStreamNonBlocking));
    const bool timing = g->timing;
    g->timing = false;
    if (pull_mode_allows_calibration(*g)) {
      abcore_status cst = calibrate_batch(*g, plan, tu.data(), tl.data(), d_bitmasks, s);
      if (cst != ABCORE_OK) {
        g->timing = timing;
        return cst;
      }
    }
    CHK(hipStreamBeginCapture(g->capture_stream, hipStreamCaptureModeThreadLocal));
    abcore_status st = run_batch(*g, plan, tu.data(), tl.data(), d_bitmasks, g->capture_stream);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(g->capture_stream, &graph);
    g->timing = timing;
    if (st != ABCORE_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    CHK(e);
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      CHK(e);
    }
    c.graph = graph;
    c.exec = exec;
    c.parity = g->rs_parity;
    c.bits = d_bitmasks;
    c.version = g->version;
    c.key = std::move(key);
  }
  // the replay uses the queue without passing through make_args, and the
  // state captured: make that one current again if queries in rank order
  // have exchanged the two since
  g->rs_ready = false;
  if (g->rs_parity != c.parity) {
    std::swap(g->state, g->state_alt);
    std::swap(g->part, g->part_alt);
    g->rs_parity ^= 1;
  }
  CHK(hipGraphLaunch(c.exec, s));
  return read_state(*g, s);
}

// abcore_query and abcore_query_set: the update, the component maintenance,
// the scoped peel, the answer and (d_set non-null) the vertex set.
static abcore_status query_impl(Graph *g, abcore_edge_update upd, uint32_t alpha, uint32_t beta,
                                int32_t *h_answer, uint32_t *h_endpoint_bits, uint32_t *d_set,
                                bool connected, int64_t *set_count, void *stream,
                                const char *fn) {
  if (g && serving(*g)) return busy_error(fn);
  if (!g || !h_answer) {
    set_error("%s: null handle or answer pointer", fn);
    return ABCORE_EINVAL;
  }
  if (upd.u < 0 || upd.u >= g->nU || upd.v < 0 || upd.v >= g->nL ||
      (upd.op != 1 && upd.op != -1)) {
    set_error("%s: update (%d, %d, op %d) out of range", fn, upd.u, upd.v, upd.op);
    return ABCORE_EINVAL;
  }
  if (alpha < 1 || beta < 1) {
    set_error("%s: alpha and beta must be >= 1", fn);
    return ABCORE_EINVAL;
  }
  CHK(hipSetDevice(g->device));
  TRY(check_abort(*g));
  hipStream_t s = as_stream(stream);
  TRY(compute_components(*g, s));
  TRY(ensure_delta(*g, s));
  if (d_set != nullptr && connected) {
    TRY(ensure(&g->list, g->n));
    TRY(ensure(&g->list2, g->n));
  }
  // 1. apply the update (validated on the device before any write)
  CHK(launch_init_state(*g, s));
  CHK(launch_update(*g, upd.u, upd.v, upd.op, g->delta.count, s));
  TRY(read_state(*g, s));
  const int32_t ustat = g->h_state->status;
  if (ustat == -(int32_t)ABCORE_EEXIST) {
    set_error("%s: edge (%d, %d) already present", fn, upd.u, upd.v);
    return ABCORE_EEXIST;
  }
  if (ustat == -(int32_t)ABCORE_ENOENT) {
    set_error("%s: edge (%d, %d) not present", fn, upd.u, upd.v);
    return ABCORE_ENOENT;
  }
  if (ustat == 1) g->delta.count += 1;
  g->m += upd.op;
  g->core_valid = false;
  g->version += 1;
  const int32_t cu = g->h_state->aux0, cv = g->h_state->aux1;
  const int32_t x = upd.u, y = g->nU + upd.v;
  // 2. component maintenance (Sec. V): merge on insertion, re-label the old
  //    component on deletion
  if (upd.op > 0) {
    if (cu != cv) CHK(launch_relabel(*g, std::max(cu, cv), std::min(cu, cv), s));
  } else {
    CHK(launch_cc(*g, cu, s));
  }
  // 3. scoped peel: Algorithm 1 on the component(s) of u and v only
  const int32_t thrU = clamp_thr(alpha), thrL = clamp_thr(beta);
  int64_t launches = 0;
  CHK(launch_init_state(*g, s));
  CHK(launch_scan_component_of(*g, thrU, thrL, x, y, s));
  // the first round in pull form when the frontier is heavy
  TRY(pull_peel_pack(*g, kGCC, thrU, thrL, g->pull_mode != 1, nullptr, s, &launches));
  CHK(launch_answer(*g, x, y, thrU, thrL, s));
  TRY(read_state(*g, s));
  const int32_t bits = g->h_state->aux0;
  *h_answer = (bits & 3) == 3 ? 1 : 0;
  if (h_endpoint_bits) *h_endpoint_bits = (uint32_t)bits;
  // 4. the vertex set (Remark of Sec. V): what the scoped peel left
  if (d_set != nullptr) TRY(scoped_set(*g, x, y, thrU, thrL, connected, d_set, set_count, s));
  return ABCORE_OK;
}

abcore_status abcore_query(abcore_graph h, abcore_edge_update upd, uint32_t alpha,
                           uint32_t beta, int32_t *h_answer, uint32_t *h_endpoint_bits,
                           void *stream) {
  return query_impl(reinterpret_cast<Graph *>(h), upd, alpha, beta, h_answer, h_endpoint_bits,
                    nullptr, false, nullptr, stream, __func__);
}

abcore_status abcore_query_set(abcore_graph h, abcore_edge_update upd, uint32_t alpha,
                               uint32_t beta, int32_t connected, int32_t *h_answer,
                               uint32_t *h_endpoint_bits, uint32_t *d_bitmask,
                               int64_t *out_count, void *stream) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (g && !d_bitmask && g->n > 0) {
    set_error("abcore_query_set: null bitmask");
    return ABCORE_EINVAL;
  }
  return query_impl(g, upd, alpha, beta, h_answer, h_endpoint_bits, d_bitmask, connected != 0,
                    out_count, stream, __func__);
}

// alpha_offset(alpha): the largest beta with a non-empty (alpha,beta)-core.
// Cores are nested (the (alpha,beta+1)-core lies inside the (alpha,beta)-
// core), so emptiness is monotone in beta and a binary search of GCC+
// queries finds it: non-empty at beta = delta when alpha <= delta (the
// (delta,delta)-core is inside), empty above the largest lower degree.
static abcore_status alpha_offset(Graph *g, uint32_t alpha, int32_t maxdeg_l, uint32_t *out,
                                  hipStream_t s) {
  auto nonempty = [&](uint32_t beta, bool *yes) -> abcore_status {
    TRY(abcore_compute(reinterpret_cast<abcore_graph>(g), alpha, beta, ABCORE_GCC_PLUS,
                       g->probe_bits, nullptr, s));
    int64_t c = 0;
    TRY(count_bits(*g, g->probe_bits, &c, s));
    *yes = c > 0;
    return ABCORE_OK;
  };
  bool yes = false;
  TRY(nonempty(1, &yes));
  if (!yes) {
    *out = 0;
    return ABCORE_OK;
  }
  uint64_t lo = 1, hi = (uint64_t)maxdeg_l + 1;  // non-empty at lo, empty at hi
  if (alpha <= (uint32_t)g->max_core && (uint64_t)g->max_core > lo)
    lo = std::min<uint64_t>((uint64_t)g->max_core, hi - 1);
  while (hi - lo > 1) {
    const uint64_t mid = lo + (hi - lo) / 2;
    TRY(nonempty((uint32_t)mid, &yes));
    (yes ? lo : hi) = mid;
  }
  *out = (uint32_t)lo;
  return ABCORE_OK;
}

abcore_status abcore_alpha_offsets(abcore_graph h, const uint32_t *h_alpha, int32_t q,
                                   uint32_t *h_offset, int32_t *out_delta, void *stream) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (g && serving(*g)) return busy_error(__func__);
  if (!g || q < 0 || (q > 0 && (!h_alpha || !h_offset))) {
    set_error("abcore_alpha_offsets: null handle or arrays, or q < 0");
    return ABCORE_EINVAL;
  }
  for (int32_t i = 0; i < q; ++i)
    if (h_alpha[i] < 1) {
      set_error("abcore_alpha_offsets: alpha %d is 0", i);
      return ABCORE_EINVAL;
    }
  CHK(hipSetDevice(g->device));
  TRY(check_abort(*g));
  hipStream_t s = as_stream(stream);
  TRY(compute_core(*g, s));
  if (out_delta) *out_delta = g->max_core;
  if (q == 0) return ABCORE_OK;
  TRY(ensure(&g->probe_bits, (g->n + 31) / 32 + 1));
  int32_t maxdeg_l = 0;
  TRY(max_degree(*g, g->nU, g->n, &maxdeg_l, s));
  for (int32_t i = 0; i < q; ++i) TRY(alpha_offset(g, h_alpha[i], maxdeg_l, &h_offset[i], s));
  return ABCORE_OK;
}

abcore_status abcore_default_query(abcore_graph h, uint32_t *alpha, uint32_t *beta,
                                   void *stream) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (!g || !alpha || !beta) {
    set_error("abcore_default_query: null pointer");
    return ABCORE_EINVAL;
  }
  int32_t delta = 0;
  TRY(abcore_alpha_offsets(h, nullptr, 0, nullptr, &delta, stream));
  const uint32_t a = std::max<uint32_t>(1, (uint32_t)((4 * (int64_t)delta) / 10));
  uint32_t off = 0;
  TRY(abcore_alpha_offsets(h, &a, 1, &off, nullptr, stream));
  *alpha = a;
  *beta = std::max<uint32_t>(1, (uint32_t)((6 * (uint64_t)off) / 10));
  return ABCORE_OK;
}

abcore_status abcore_community(abcore_graph h, int32_t q, uint32_t alpha, uint32_t beta,
                               int32_t connected, uint32_t *d_bitmask, int64_t *out_count,
                               void *stream) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (g && serving(*g)) return busy_error(__func__);
  if (!g || !d_bitmask) {
    set_error("abcore_community: null handle or bitmask");
    return ABCORE_EINVAL;
  }
  if (q < 0 || (int64_t)q >= g->n) {
    set_error("abcore_community: vertex %d out of range", q);
    return ABCORE_EINVAL;
  }
  if (alpha < 1 || beta < 1) {
    set_error("abcore_community: alpha and beta must be >= 1");
    return ABCORE_EINVAL;
  }
  CHK(hipSetDevice(g->device));
  TRY(check_abort(*g));
  hipStream_t s = as_stream(stream);
  TRY(compute_components(*g, s));
  if (connected) {
    TRY(ensure(&g->list, g->n));
    TRY(ensure(&g->list2, g->n));
  }
  // Algorithm 1 on q's connected component only, as GFQ scopes its peel
  const int32_t thrU = clamp_thr(alpha), thrL = clamp_thr(beta);
  int64_t launches = 0;
  CHK(launch_init_state(*g, s));
  CHK(launch_scan_component_of(*g, thrU, thrL, q, q, s));
  TRY(pull_peel_pack(*g, kGCC, thrU, thrL, g->pull_mode != 1, nullptr, s, &launches));
  return scoped_set(*g, q, q, thrU, thrL, connected != 0, d_bitmask, out_count, s);
}

abcore_status abcore_serve_start(abcore_graph h, int64_t max_inflight, int32_t device_slots,
                                 int32_t window) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (!g || max_inflight < 0 || device_slots < 0 || window < 0 || device_slots > 256) {
    set_error("abcore_serve_start: null handle or bad sizes");
    return ABCORE_EINVAL;
  }
  if (serving(*g)) return ABCORE_OK;
  CHK(hipSetDevice(g->device));
  TRY(check_abort(*g));
  hipStream_t s = nullptr;
  TRY(compute_components(*g, s));
  TRY(ensure_delta(*g, s));
  CHK(hipStreamSynchronize(s));
  return serve_start(*g, max_inflight > 0 ? max_inflight : 1024,
                     device_slots > 0 ? device_slots : 2, window > 0 ? window : kWindowMax);
}

abcore_status abcore_submit(abcore_graph h, abcore_edge_update upd, uint32_t alpha,
                            uint32_t beta, uint64_t *ticket) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (!g || !ticket) {
    set_error("abcore_submit: null handle or ticket");
    return ABCORE_EINVAL;
  }
  if (upd.u < 0 || upd.u >= g->nU || upd.v < 0 || upd.v >= g->nL ||
      (upd.op != 1 && upd.op != -1) || alpha < 1 || beta < 1) {
    set_error("abcore_submit: endpoint out of range, op not +1/-1, or alpha/beta 0");
    return ABCORE_EINVAL;
  }
  if (!serving(*g)) TRY(abcore_serve_start(h, 0, 0, 0));
  return serve_submit(*g, upd, clamp_thr(alpha), clamp_thr(beta), ticket);
}

abcore_status abcore_poll(abcore_graph h, uint64_t ticket, int32_t *answer,
                          uint32_t *endpoint_bits, uint64_t *t_done_ns) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (!g) {
    set_error("abcore_poll: null handle");
    return ABCORE_EINVAL;
  }
  return serve_poll(*g, ticket, answer, endpoint_bits, t_done_ns);
}

abcore_status abcore_serve_counters(abcore_graph h, int64_t *out, int32_t count) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (!g || !out || count < 0) {
    set_error("abcore_serve_counters: null handle or output");
    return ABCORE_EINVAL;
  }
  serve_counters(*g, out, count);
  return ABCORE_OK;
}

abcore_status abcore_serve_stop(abcore_graph h, int64_t *counters) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (!g) {
    set_error("abcore_serve_stop: null handle");
    return ABCORE_EINVAL;
  }
  abcore_status st = serve_stop(*g);
  if (counters) serve_counters(*g, counters, 3);
  return st;
}

// Times the query (alpha, beta) with algorithm algo (3 runs after a warm
// run, median) for every pair of asynchronous-peel grid size and claim size
// and returns the fastest pair; the handle's grid and claim are left as
// they were.
static abcore_status tune_mapping(Graph *g, uint32_t alpha, uint32_t beta, int32_t algo,
                                  void *stream, int *out_grid, int *out_claim, double *out_ms) {
  abcore_graph h = reinterpret_cast<abcore_graph>(g);
  hipStream_t s = as_stream(stream);
  const int64_t words = std::max<int64_t>(1, (g->n + 31) / 32);
  uint32_t *bits = nullptr;
  CHK(dev_malloc(&bits, sizeof(uint32_t) * words));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  const int saved_grid = g->grid, saved_claim = g->claim;
  const bool saved_timing = g->timing, saved_tuned = g->tuned;
  g->timing = false;
  g->tuned = true;  // the sweep's settings hold for its queries
  abcore_status st = he == hipSuccess ? ABCORE_OK : ABCORE_EDEVICE;
  const int cu = g->cu_count;
  const int grids[] = {cu / 2, (3 * cu) / 4, cu, (3 * cu) / 2, 2 * cu, 3 * cu};
  const int claims[] = {64, 32, 16};
  int best_grid = saved_grid, best_claim = saved_claim;
  double best = 1e30;
  for (int gi = 0; gi < 6 && st == ABCORE_OK; ++gi) {
    if (grids[gi] < 1 || (g->async_grid > 0 && grids[gi] > g->async_grid)) continue;
    for (int ci = 0; ci < 3 && st == ABCORE_OK; ++ci) {
      g->grid = grids[gi];
      g->claim = claims[ci];
      st = abcore_compute(h, alpha, beta, algo, bits, nullptr, stream);  // warm
      double t[3];
      for (int r = 0; r < 3 && st == ABCORE_OK; ++r) {
        if (hipEventRecord(e0, s) != hipSuccess) st = ABCORE_EDEVICE;
        if (st == ABCORE_OK) st = abcore_compute(h, alpha, beta, algo, bits, nullptr, stream);
        float ms = 0.f;
        if (st == ABCORE_OK && (hipEventRecord(e1, s) != hipSuccess ||
                                hipEventSynchronize(e1) != hipSuccess ||
                                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
          st = ABCORE_EDEVICE;
        t[r] = ms;
      }
      if (st != ABCORE_OK) break;
      std::sort(t, t + 3);
      if (t[1] < best) {
        best = t[1];
        best_grid = grids[gi];
        best_claim = claims[ci];
      }
    }
  }
  g->timing = saved_timing;
  g->tuned = saved_tuned;
  g->grid = saved_grid;
  g->claim = saved_claim;
  if (st == ABCORE_OK && read_state(*g, s) != ABCORE_OK) st = ABCORE_EDEVICE;
  if (st == ABCORE_OK) {
    *out_grid = best_grid;
    *out_claim = best_claim;
    *out_ms = best;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)dev_free(bits);
  return st;
}

abcore_status abcore_autotune(abcore_graph h, uint32_t alpha, uint32_t beta, int32_t algo,
                              int32_t *out_grid, int32_t *out_claim, double *out_ms,
                              void *stream) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (g && serving(*g)) return busy_error(__func__);
  if (!g || alpha < 1 || beta < 1 || (algo != ABCORE_GCC && algo != ABCORE_GCC_PLUS)) {
    set_error("abcore_autotune: null handle, threshold 0 or unknown algorithm");
    return ABCORE_EINVAL;
  }
  CHK(hipSetDevice(g->device));
  TRY(check_abort(*g));
  int grid = 0, claim = 0;
  double ms = 0;
  TRY(tune_mapping(g, alpha, beta, algo, stream, &grid, &claim, &ms));
  g->grid = grid;
  g->claim = claim;
  g->tuned = true;
  tune_store(*g, 0, grid, claim, ms);
  if (out_grid) *out_grid = grid;
  if (out_claim) *out_claim = claim;
  if (out_ms) *out_ms = ms;
  return ABCORE_OK;
}

abcore_status abcore_tuned(abcore_graph h, int32_t kind, int32_t *out_grid, int32_t *out_claim,
                           double *out_ms, int32_t *found) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (!g || !found || (kind != 0 && kind != 1)) {
    set_error("abcore_tuned: null handle or output, or unknown kind");
    return ABCORE_EINVAL;
  }
  TuneVal v{};
  *found = tune_find(*g, kind, &v) ? 1 : 0;
  if (*found) {
    if (out_grid) *out_grid = v.grid;
    if (out_claim) *out_claim = v.claim;
    if (out_ms) *out_ms = v.ms;
  }
  return ABCORE_OK;
}

abcore_status abcore_tune_cache(const char *path, int32_t mode) {
  if (mode == 2) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune.clear();
    return ABCORE_OK;
  }
  if (!path || (mode != 0 && mode != 1)) {
    set_error("abcore_tune_cache: null path or unknown mode %d", mode);
    return ABCORE_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_tune_mu);
  if (mode == 1) {
    FILE *f = fopen(path, "w");
    if (!f) {
      set_error("abcore_tune_cache: cannot write %s", path);
      return ABCORE_EINVAL;
    }
    for (const auto &kv : g_tune)
      fprintf(f, "%s %d %d %d %d %d %d %.6f\n", kv.first.arch.c_str(), kv.first.cu,
              kv.first.nlog, kv.first.elog, kv.first.kind, kv.second.grid, kv.second.claim,
              kv.second.ms);
    fclose(f);
    return ABCORE_OK;
  }
  FILE *f = fopen(path, "r");
  if (!f) {
    set_error("abcore_tune_cache: cannot read %s", path);
    return ABCORE_EINVAL;
  }
  char arch[64];
  TuneKey k;
  TuneVal v;
  int read = 0;
  while ((read = fscanf(f, "%63s %d %d %d %d %d %d %lf", arch, &k.cu, &k.nlog, &k.elog,
                        &k.kind, &v.grid, &v.claim, &v.ms)) == 8) {
    if (v.grid < 1 || v.grid > kMaxBlocks || v.claim < 1 || v.claim > kWave) continue;
    k.arch = arch;
    g_tune[k] = v;
  }
  fclose(f);
  if (read != EOF) {
    set_error("abcore_tune_cache: malformed line in %s", path);
    return ABCORE_EINVAL;
  }
  return ABCORE_OK;
}

}  // extern "C"
