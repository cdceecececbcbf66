// Serving loop for on-the-fly queries (GFQ, Sec. V) over a stream of edge
// updates: requests are admitted into a bounded set, grouped into windows,
// applied in stream order, and their scoped peels run concurrently, each on
// the graph version of its own update.
//
// Consistency: answer i is the one abcore_query would give after updates
// 1..i (the stream is cumulative).  The graph is updated in place and
// append-only while older queries still peel (deletion versions, pairs in
// insertion order), so every query reads exactly its version:
//   - degrees: the scan starts from the current degrees and undoes the later
//     updates of its window (updates of later windows are applied only after
//     this window's scans and pull rounds, ordered by events);
//   - edges: the versioned view of the peel;
//   - components: labels only merge while serving, so a query's scope is a
//     union of components of its version (stale, unsplit labels are exact).
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

#include <algorithm>
#include <string>
#include <vector>

#include "abcore_internal.h"

namespace abc {

abcore_status grow_delta(Graph &g, int64_t min_cap, hipStream_t s);

namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Request {
  uint64_t ticket;
  int32_t u, v, op;
  int32_t thrU, thrL;
  uint64_t t_submit;  // steady-clock nanoseconds at admission
};

struct Result {
  int32_t status;   // abcore_status
  int32_t answer;   // 1 if both endpoints are in the core
  uint32_t bits;    // bit0: u in the core, bit1: v in the core
  uint64_t t_done;  // steady-clock nanoseconds when the result was taken
};

// One device working set: degrees, frontier queues and state of one query.
struct Slot {
  hipStream_t stream = nullptr;
  int32_t *deg = nullptr;
  int32_t *queue = nullptr;
  PeelState *state = nullptr;
  int64_t *part = nullptr;
  uint32_t *bits = nullptr;   // survivors of the scan (pull round)
  int32_t *d_corr = nullptr;  // 2 * kCorrMax: vertices, then deltas
  int32_t *h_corr = nullptr;  // pinned staging of d_corr
  int32_t *h_out = nullptr;   // pinned: aux0, aux1, pulled, abort_flag of the state
  hipEvent_t scanned = nullptr, done = nullptr;
  bool busy = false;
  Request req{};
};

}  // namespace

struct Server {
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request> pending;
  std::unordered_map<uint64_t, Result> results;
  uint64_t next_ticket = 0;
  int64_t inflight = 0;  // admitted and not finished
  int64_t max_inflight = 1024;
  bool stop = false;
  bool running = false;
  std::string fail;  // non-empty once the engine has failed
  std::thread worker;
  std::vector<Slot> slots;
  int window_max = kWindowMax;
  hipStream_t main = nullptr;
  hipEvent_t applied = nullptr;
  int32_t *d_upd = nullptr, *h_upd = nullptr;  // 3 * kWindowMax
  WindowRecord *d_rec = nullptr, *h_rec = nullptr;
  std::vector<hipEvent_t> last_scans;  // scans of the previous window
  // Stale core-number pruning (Graph::serve_prune > 0): a snapshot of the
  // core numbers (Definition 2) and, per snapshot value c, how far the core
  // numbers of the vertices that had c may have moved since: they lie in
  // [c - dlo[c], c + dhi[c]].  An edge update changes only the core numbers
  // equal to K = min(core(u), core(v)), each by one (up on insertion, down
  // on deletion) -- the k-core maintenance property -- so an update widens
  // exactly the values whose interval meets K's possible range.  Lemma 1
  // with these intervals decides a request without a peel when both
  // endpoints are certainly in (lower end >= max(alpha,beta)) or certainly
  // out (upper end < min(alpha,beta)).
  std::vector<int32_t> core_h;
  std::vector<int64_t> dlo, dhi;
  int64_t since_refresh = 0;
  // counters
  int64_t windows = 0, served = 0, rejected = 0;
  int64_t decided = 0, refreshes = 0, timed_out = 0;
  double refresh_ms = 0;
  int64_t device_slots = 0;  // working sets in use (fewer under a memory budget)
};

namespace {

void free_slot(Slot &s) {
  if (s.stream) (void)hipStreamDestroy(s.stream);
  for (void *p : {(void *)s.deg, (void *)s.queue, (void *)s.state, (void *)s.part,
                  (void *)s.d_corr, (void *)s.bits})
    if (p) (void)dev_free(p);
  if (s.h_corr) (void)hipHostFree(s.h_corr);
  if (s.h_out) (void)hipHostFree(s.h_out);
  if (s.scanned) (void)hipEventDestroy(s.scanned);
  if (s.done) (void)hipEventDestroy(s.done);
  s = Slot();
}

void free_server_device(Server &S) {
  for (Slot &s : S.slots) free_slot(s);
  S.slots.clear();
  if (S.main) (void)hipStreamDestroy(S.main);
  if (S.applied) (void)hipEventDestroy(S.applied);
  if (S.d_upd) (void)dev_free(S.d_upd);
  if (S.h_upd) (void)hipHostFree(S.h_upd);
  if (S.d_rec) (void)dev_free(S.d_rec);
  if (S.h_rec) (void)hipHostFree(S.h_rec);
  S.main = nullptr;
  S.applied = nullptr;
  S.d_upd = S.h_upd = nullptr;
  S.d_rec = S.h_rec = nullptr;
  S.last_scans.clear();
}

hipError_t alloc_slot(Graph &g, Slot &s) {
  hipError_t e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = dev_malloc(&s.deg, sizeof(int32_t) * std::max<int64_t>(g.n, 1));
  if (e == hipSuccess) e = dev_malloc(&s.queue, sizeof(int32_t) * kSub * g.qcap);
  if (e == hipSuccess) e = hipMemset(s.queue, 0xFF, sizeof(int32_t) * kSub * g.qcap);
  if (e == hipSuccess) e = dev_malloc(&s.state, sizeof(PeelState));
  if (e == hipSuccess) e = hipMemset(s.state, 0, sizeof(PeelState));
  if (e == hipSuccess) e = dev_malloc(&s.part, sizeof(int64_t) * kMaxBlocks * kPartFields);
  if (e == hipSuccess) e = dev_malloc(&s.d_corr, sizeof(int32_t) * 2 * kCorrMax);
  if (e == hipSuccess)
    e = dev_malloc(&s.bits, sizeof(uint32_t) * std::max<int64_t>((g.n + 31) / 32, 1));
  if (e == hipSuccess) e = hipHostMalloc(&s.h_corr, sizeof(int32_t) * 2 * kCorrMax);
  if (e == hipSuccess) e = hipHostMalloc(&s.h_out, sizeof(int32_t) * 4);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s.scanned, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
  return e;
}

void finish(Server &S, uint64_t ticket, Result r) {
  std::lock_guard<std::mutex> lk(S.mu);
  S.results[ticket] = r;
  S.inflight -= 1;
  if (r.status == ABCORE_OK)
    S.served += 1;
  else if (r.status == ABCORE_ETIMEDOUT)
    S.timed_out += 1;
  else
    S.rejected += 1;
}

// Takes finished slots; with wait, blocks until every busy slot has finished.
bool reap(Server &S, bool wait) {
  bool any = false;
  for (Slot &s : S.slots) {
    if (!s.busy) continue;
    hipError_t e = wait ? hipEventSynchronize(s.done) : hipEventQuery(s.done);
    if (e == hipErrorNotReady) continue;
    Result r{};
    r.t_done = now_ns();
    if (e != hipSuccess) {
      r.status = ABCORE_EDEVICE;
      if (S.fail.empty()) S.fail = std::string("served query failed: ") + hipGetErrorString(e);
    } else if (s.h_out[3] != 0) {
      r.status = ABCORE_EDEVICE;
      if (S.fail.empty()) S.fail = "a served peel exceeded its spin limit";
    } else {
      r.status = ABCORE_OK;
      r.bits = (uint32_t)s.h_out[0];
      r.answer = r.bits == 3u ? 1 : 0;
    }
    s.busy = false;
    finish(S, s.req.ticket, r);
    any = true;
  }
  return any;
}

#define SCHK(x)                                                          \
  do {                                                                   \
    hipError_t e_ = (x);                                                 \
    if (e_ != hipSuccess) {                                              \
      S.fail = std::string(#x " failed: ") + hipGetErrorString(e_);      \
      return false;                                                      \
    }                                                                    \
  } while (0)

// A fresh snapshot of the core numbers of the current graph (every running
// query drained first, so nothing else uses the device meanwhile).
bool refresh_cores(Graph &g, Server &S) {
  reap(S, true);
  const auto t0 = std::chrono::steady_clock::now();
  g.core_valid = false;
  if (compute_core_numbers(g, S.main) != ABCORE_OK) {
    S.fail = "serving: core numbers for pruning failed";
    return false;
  }
  S.core_h.resize((size_t)g.n);
  if (g.n > 0)
    SCHK(hipMemcpyAsync(S.core_h.data(), g.core, sizeof(int32_t) * g.n, hipMemcpyDeviceToHost,
                        S.main));
  SCHK(hipStreamSynchronize(S.main));
  S.dlo.assign((size_t)g.max_core + 2, 0);
  S.dhi.assign((size_t)g.max_core + 2, 0);
  S.since_refresh = 0;
  S.refreshes += 1;
  S.refresh_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                      .count();
  return true;
}

// The interval that holds the current core number of vertex x.
inline void core_interval(const Server &S, int32_t x, int64_t *lo, int64_t *hi) {
  const int32_t c = S.core_h[(size_t)x];
  *lo = (int64_t)c - S.dlo[(size_t)c];
  *hi = (int64_t)c + S.dhi[(size_t)c];
}

// Widens the intervals an applied update (u, v, op) may have moved.
void widen_for_update(Server &S, int32_t x, int32_t y, int32_t op) {
  int64_t lx, hx, ly, hy;
  core_interval(S, x, &lx, &hx);
  core_interval(S, y, &ly, &hy);
  const int64_t klo = std::min(lx, ly), khi = std::min(hx, hy);
  const size_t nc = S.dlo.size();
  for (size_t c = 0; c < nc; ++c) {
    const int64_t lo = (int64_t)c - S.dlo[c], hi = (int64_t)c + S.dhi[c];
    if (hi >= klo && lo <= khi) (op > 0 ? S.dhi[c] : S.dlo[c]) += 1;
  }
}

// Lemma 1 on the intervals: 1 certainly in, 0 certainly out, -1 undecided.
inline int classify(const Server &S, int32_t x, int32_t dl, int32_t dq) {
  int64_t lo, hi;
  core_interval(S, x, &lo, &hi);
  if (lo >= dq) return 1;
  if (hi < dl) return 0;
  return -1;
}

// Applies one window of updates and launches its queries.
bool run_window(Graph &g, Server &S, const std::vector<Request> &win) {
  const int w = (int)win.size();
  if (g.delta.count + w > g.delta.cap || g.delta.count + w > g.pair_del_cap) {
    // growing moves the pair arrays that running peels read: drain first
    reap(S, true);
    if (grow_delta(g, g.delta.count + w, S.main) != ABCORE_OK) {
      S.fail = "serving: growing the inserted-edge storage failed";
      return false;
    }
  }
  for (hipEvent_t ev : S.last_scans) SCHK(hipStreamWaitEvent(S.main, ev, 0));
  S.last_scans.clear();
  for (int i = 0; i < w; ++i) {
    S.h_upd[3 * i] = win[i].u;
    S.h_upd[3 * i + 1] = win[i].v;
    S.h_upd[3 * i + 2] = win[i].op;
  }
  SCHK(hipMemcpyAsync(S.d_upd, S.h_upd, sizeof(int32_t) * 3 * w, hipMemcpyHostToDevice, S.main));
  SCHK(launch_update_window(g, S.d_upd, w, S.d_rec, S.main));
  SCHK(hipMemcpyAsync(S.h_rec, S.d_rec, sizeof(WindowRecord) * w, hipMemcpyDeviceToHost,
                      S.main));
  SCHK(hipStreamSynchronize(S.main));
  // merge the labels joined by the window's insertions (labels are the
  // smallest id of their component, so a merge keeps the smaller)
  std::unordered_map<int32_t, int32_t> up;
  auto find = [&](int32_t x) {
    while (true) {
      auto it = up.find(x);
      if (it == up.end() || it->second == x) return x;
      x = it->second;
    }
  };
  for (int i = 0; i < w; ++i) {
    const WindowRecord &r = S.h_rec[i];
    if (r.status != 0) continue;
    g.m += win[i].op;
    g.upd_version = r.version;
    g.delta.count = r.pairs_after;
    if (win[i].op > 0) {
      int32_t a = find(r.label_u), b = find(r.label_v);
      if (a != b) {
        if (a > b) std::swap(a, b);
        up[b] = a;
        if (!up.count(a)) up[a] = a;
      }
    }
  }
  for (auto &kv : up)
    if (find(kv.first) != kv.first) SCHK(launch_relabel(g, kv.first, find(kv.first), S.main));
  g.core_valid = false;
  g.version += 1;
  SCHK(hipEventRecord(S.applied, S.main));
  S.windows += 1;
  // the working sets share the co-resident capacity of the peel
  const int cap = g.async_grid > 0 ? g.async_grid : async_peel_grid(g);
  const int grid = std::max(1, cap / std::max<int>(1, (int)S.slots.size()));
  size_t next_slot = 0;
  for (int i = 0; i < w; ++i) {
    const WindowRecord &r = S.h_rec[i];
    if (r.status != 0) {
      Result res{};
      res.status = -r.status;
      res.t_done = now_ns();
      finish(S, win[i].ticket, res);
      continue;
    }
    if (!S.core_h.empty()) {
      // the snapshot's intervals, widened by this update and those before
      widen_for_update(S, win[i].u, g.nU + win[i].v, win[i].op);
      S.since_refresh += 1;
    }
    if (g.serve_deadline_us > 0 &&
        now_ns() > win[i].t_submit + (uint64_t)g.serve_deadline_us * 1000ull) {
      // past its deadline before its query started: the update stays
      // applied, the query is dropped
      Result res{};
      res.status = ABCORE_ETIMEDOUT;
      res.t_done = now_ns();
      finish(S, win[i].ticket, res);
      continue;
    }
    if (!S.core_h.empty()) {
      const int32_t x = win[i].u, y = g.nU + win[i].v;
      const int32_t dl = std::min(win[i].thrU, win[i].thrL);
      const int32_t dq = std::max(win[i].thrU, win[i].thrL);
      const int cu = classify(S, x, dl, dq), cv = classify(S, y, dl, dq);
      if (cu >= 0 && cv >= 0) {
        Result res{};
        res.status = ABCORE_OK;
        res.bits = (uint32_t)cu | ((uint32_t)cv << 1);
        res.answer = res.bits == 3u ? 1 : 0;
        res.t_done = now_ns();
        S.decided += 1;
        finish(S, win[i].ticket, res);
        continue;
      }
    }
    while (S.slots[next_slot].busy) ++next_slot;  // the window fits the free slots
    Slot &s = S.slots[next_slot];
    // the later updates of the window, undone for this query's view
    int c = 0;
    for (int j = i + 1; j < w; ++j) {
      if (S.h_rec[j].status != 0) continue;
      s.h_corr[c] = win[j].u;
      s.h_corr[kCorrMax + c] = -win[j].op;
      ++c;
      s.h_corr[c] = g.nU + win[j].v;
      s.h_corr[kCorrMax + c] = -win[j].op;
      ++c;
    }
    PeelArgs a = make_args(g, win[i].thrU, win[i].thrL);
    a.deg = s.deg;
    a.queue = s.queue;
    a.st = s.state;
    a.part = s.part;
    a.del_ver = g.del_ver;
    a.pair_del_ver = g.pair_del_ver;
    a.ver = r.version;
    a.pair_limit = r.pairs_after;
    a.ins_head = r.pairs_after > 0 ? g.delta.head : nullptr;
    a.abort_host = nullptr;  // a served abort is reported with its request
    const int32_t x = win[i].u, y = g.nU + win[i].v;
    SCHK(hipStreamWaitEvent(s.stream, S.applied, 0));
    if (c > 0)
      SCHK(hipMemcpyAsync(s.d_corr, s.h_corr, sizeof(int32_t) * 2 * kCorrMax,
                          hipMemcpyHostToDevice, s.stream));
    SCHK(launch_init_workspace(g, s.queue, s.state, s.part, s.stream));
    // the first round as a single query takes it: pulled when the device
    // finds it cheaper from the scan's sums (ABCORE_OPT_PULL 0), always (2)
    // or never (1)
    const bool pull = g.pull_mode != 1;
    SCHK(launch_scan_component_view(g, a, x, y, s.d_corr, s.d_corr + kCorrMax, c,
                                    pull ? s.bits : nullptr, s.stream));
    PeelArgs ap = a;
    if (pull) {
      // the pull round's completion runs in the peel's start phase
      SCHK(launch_pull_round_args(g, a, s.bits, s.d_corr, s.d_corr + kCorrMax, c, true,
                                  s.stream));
      ap.fix_rows = g.heavy_rows;
      ap.fix_bits = s.bits;
      ap.nfix = g.nheavy;
      ap.start_expect = grid;
    }
    // the scan and the pull round read the current degrees: the next
    // window's updates wait for them
    SCHK(hipEventRecord(s.scanned, s.stream));
    S.last_scans.push_back(s.scanned);
    SCHK(launch_peel_async_args(g, kGCC, ap, grid, s.stream));
    SCHK(launch_answer_view(a, x, y, s.stream));
    SCHK(hipMemcpyAsync(s.h_out, &s.state->aux0, sizeof(int32_t) * 4, hipMemcpyDeviceToHost,
                        s.stream));
    SCHK(hipEventRecord(s.done, s.stream));
    s.req = win[i];
    s.busy = true;
  }
  if (!S.core_h.empty() && g.serve_prune >= 2 && S.since_refresh >= g.serve_prune)
    return refresh_cores(g, S);
  return true;
}

void fail_all(Server &S) {
  // every admitted request ends with EDEVICE
  std::vector<Request> left;
  {
    std::lock_guard<std::mutex> lk(S.mu);
    left.assign(S.pending.begin(), S.pending.end());
    S.pending.clear();
  }
  for (Slot &s : S.slots)
    if (s.busy) {
      (void)hipEventSynchronize(s.done);
      s.busy = false;
      left.push_back(s.req);
    }
  for (const Request &r : left) {
    Result res{};
    res.status = ABCORE_EDEVICE;
    res.t_done = now_ns();
    finish(S, r.ticket, res);
  }
}

void worker_main(Graph *g) {
  Server &S = *g->server;
  (void)hipSetDevice(g->device);
  std::vector<Request> win;
  while (true) {
    bool progress = reap(S, false);
    int nfree = 0;
    for (const Slot &s : S.slots) nfree += s.busy ? 0 : 1;
    win.clear();
    {
      std::unique_lock<std::mutex> lk(S.mu);
      const int take = std::min(nfree, S.window_max);
      while ((int)win.size() < take && !S.pending.empty()) {
        win.push_back(S.pending.front());
        S.pending.pop_front();
      }
      if (win.empty() && !progress) {
        bool busy = false;
        for (const Slot &s : S.slots) busy = busy || s.busy;
        if (!busy && S.pending.empty()) {
          if (S.stop) break;
          S.cv.wait(lk, [&] { return S.stop || !S.pending.empty(); });
          continue;
        }
      }
    }
    if (!win.empty()) {
      if (!run_window(*g, S, win)) {
        // the window's requests are not in a slot yet: end them with the rest
        for (const Request &r : win) {
          bool in_slot = false;
          for (const Slot &s : S.slots) in_slot = in_slot || (s.busy && s.req.ticket == r.ticket);
          if (!in_slot) {
            Result res{};
            res.status = ABCORE_EDEVICE;
            res.t_done = now_ns();
            finish(S, r.ticket, res);
          }
        }
        fail_all(S);
        break;
      }
      progress = true;
    }
    if (!progress) std::this_thread::yield();
  }
  reap(S, true);
}

}  // namespace

bool serving(const Graph &g) { return g.server != nullptr && g.server->running; }

// Stops the engine after every admitted request has finished.
abcore_status serve_stop(Graph &g) {
  if (!serving(g)) return ABCORE_OK;
  Server &S = *g.server;
  {
    std::lock_guard<std::mutex> lk(S.mu);
    S.stop = true;
  }
  S.cv.notify_all();
  if (S.worker.joinable()) S.worker.join();
  (void)hipSetDevice(g.device);
  free_server_device(S);
  S.running = false;
  if (!S.fail.empty()) {
    set_error("%s", S.fail.c_str());
    return ABCORE_EDEVICE;
  }
  return ABCORE_OK;
}

void destroy_server(Graph &g) {
  if (!g.server) return;
  (void)serve_stop(g);
  delete g.server;
  g.server = nullptr;
}

abcore_status serve_start(Graph &g, int64_t max_inflight, int32_t slots, int32_t window) {
  if (serving(g)) return ABCORE_OK;
  if (!g.comp_valid || !g.comp) {
    set_error("serving: component labels missing");
    return ABCORE_EINVAL;
  }
  if (!g.server) g.server = new (std::nothrow) Server();
  if (!g.server) {
    set_error("serving: out of host memory");
    return ABCORE_ENOMEM;
  }
  Server &S = *g.server;
  S.stop = false;
  S.fail.clear();
  S.max_inflight = max_inflight;
  S.window_max = std::max(1, std::min(window, kWindowMax));
  S.slots.clear();
  hipError_t e = hipStreamCreateWithFlags(&S.main, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&S.applied, hipEventDisableTiming);
  if (e == hipSuccess) e = dev_malloc(&S.d_upd, sizeof(int32_t) * 3 * kWindowMax);
  if (e == hipSuccess) e = hipHostMalloc(&S.h_upd, sizeof(int32_t) * 3 * kWindowMax);
  if (e == hipSuccess) e = dev_malloc(&S.d_rec, sizeof(WindowRecord) * kWindowMax);
  if (e == hipSuccess) e = hipHostMalloc(&S.h_rec, sizeof(WindowRecord) * kWindowMax);
  if (e == hipSuccess && g.del_ver == nullptr) {
    e = dev_malloc(&g.del_ver, sizeof(int32_t) * std::max<int64_t>(2 * g.m_csr, 1));
    if (e == hipSuccess) e = hipMemset(g.del_ver, 0, sizeof(int32_t) * std::max<int64_t>(2 * g.m_csr, 1));
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_server_device(S);
    set_error("serving: allocation failed: %s", hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? ABCORE_ENOMEM : ABCORE_EDEVICE;
  }
  abcore_status st = grow_delta(g, g.delta.count + kWindowMax, S.main);
  if (st == ABCORE_OK && hipStreamSynchronize(S.main) != hipSuccess) st = ABCORE_EDEVICE;
  if (st != ABCORE_OK) {
    free_server_device(S);
    return st;
  }
  // Admission under a memory budget (abcore_set_memory_budget): as many
  // device working sets as fit, at least one; fewer working sets mean fewer
  // requests per window, and the rest wait in the admission queue (EBUSY
  // once max_inflight are admitted).
  for (int i = 0; i < slots; ++i) {
    S.slots.emplace_back();
    e = alloc_slot(g, S.slots.back());
    if (e != hipSuccess) {
      free_slot(S.slots.back());
      S.slots.pop_back();
      if (e == hipErrorOutOfMemory && !S.slots.empty()) e = hipSuccess;
      break;
    }
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_server_device(S);
    set_error("serving: working-set allocation failed: %s", hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? ABCORE_ENOMEM : ABCORE_EDEVICE;
  }
  S.device_slots = (int64_t)S.slots.size();
  S.core_h.clear();
  S.decided = S.refreshes = S.timed_out = 0;
  S.refresh_ms = 0;
  if (g.serve_prune > 0 && !refresh_cores(g, S)) {
    free_server_device(S);
    set_error("%s", S.fail.c_str());
    return ABCORE_EDEVICE;
  }
  S.running = true;
  try {
    S.worker = std::thread(worker_main, &g);
  } catch (...) {
    free_server_device(S);
    S.running = false;
    set_error("serving: cannot start the worker thread");
    return ABCORE_ENOMEM;
  }
  return ABCORE_OK;
}

abcore_status serve_submit(Graph &g, const abcore_edge_update &upd, int32_t thrU, int32_t thrL,
                           uint64_t *ticket) {
  Server &S = *g.server;
  std::lock_guard<std::mutex> lk(S.mu);
  if (!S.fail.empty()) {
    set_error("%s", S.fail.c_str());
    return ABCORE_EDEVICE;
  }
  if (S.inflight >= S.max_inflight) {
    set_error("abcore_submit: %lld requests in flight", (long long)S.inflight);
    return ABCORE_EBUSY;
  }
  Request r{};
  r.ticket = S.next_ticket++;
  r.u = upd.u;
  r.v = upd.v;
  r.op = upd.op;
  r.thrU = thrU;
  r.thrL = thrL;
  r.t_submit = now_ns();
  S.pending.push_back(r);
  S.inflight += 1;
  *ticket = r.ticket;
  S.cv.notify_one();
  return ABCORE_OK;
}

abcore_status serve_poll(Graph &g, uint64_t ticket, int32_t *answer, uint32_t *bits,
                         uint64_t *t_done) {
  if (!g.server) {
    set_error("abcore_poll: nothing was submitted");
    return ABCORE_EINVAL;
  }
  Server &S = *g.server;
  std::lock_guard<std::mutex> lk(S.mu);
  auto it = S.results.find(ticket);
  if (it == S.results.end()) {
    if (ticket >= S.next_ticket) {
      set_error("abcore_poll: unknown ticket %llu", (unsigned long long)ticket);
      return ABCORE_EINVAL;
    }
    return ABCORE_EAGAIN;  // admitted, not finished (or already polled)
  }
  const Result r = it->second;
  S.results.erase(it);
  if (answer) *answer = r.answer;
  if (bits) *bits = r.bits;
  if (t_done) *t_done = r.t_done;
  if (r.status == ABCORE_ETIMEDOUT)
    set_error("served request past its deadline: its update was applied, its query dropped");
  else if (r.status != ABCORE_OK)
    set_error("served update rejected or failed (status %d)", r.status);
  return (abcore_status)r.status;
}

void serve_counters(const Graph &g, int64_t *out, int count) {
  const Server *S = g.server;
  const int64_t v[8] = {S ? S->windows : 0,   S ? S->served : 0,    S ? S->rejected : 0,
                        S ? S->decided : 0,   S ? S->refreshes : 0,
                        S ? (int64_t)(S->refresh_ms * 1000.0) : 0,
                        S ? S->timed_out : 0, S ? S->device_slots : 0};
  for (int i = 0; i < count && i < 8; ++i) out[i] = v[i];
}

}  // namespace abc
