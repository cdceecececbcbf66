// C-ABI entry points of libabcore (declared in include/abcore.h).
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "abcore_internal.h"

namespace abc {

static thread_local char g_error[512] = "";

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

namespace {

#define CHK(x)                                                                     \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) {                                                        \
      set_error("%s: %s failed: %s", __func__, #x, hipGetErrorString(e_));         \
      return e_ == hipErrorOutOfMemory ? ABCORE_ENOMEM : ABCORE_EDEVICE;           \
    }                                                                              \
  } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline int32_t clamp_thr(uint32_t t) {
  return (int32_t)std::min<uint64_t>(t, (uint64_t)kMaxThreshold);
}

void free_graph(Graph *g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  for (auto &pr : g->events) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  for (hipEvent_t e : g->event_pool) (void)hipEventDestroy(e);
  void *bufs[] = {g->off,    g->cols,   g->deg0,       g->deg,        g->queue,
                  g->list,   g->list2,  g->state,      g->core,       g->comp,
                  g->parent, g->delta.head, g->delta.next, g->delta.other};
  for (void *p : bufs)
    if (p) (void)hipFree(p);
  if (g->h_state) (void)hipHostFree(g->h_state);
  delete g;
}

abcore_status ensure(int32_t **p, int64_t count) {
  if (*p) return ABCORE_OK;
  hipError_t e = hipMalloc(p, sizeof(int32_t) * std::max<int64_t>(count, 1));
  if (e != hipSuccess) {
    *p = nullptr;
    set_error("device allocation of %lld words failed: %s", (long long)count,
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

// Records an event pair around `launch` when timing is on.
template <class F>
hipError_t timed(Graph &g, hipStream_t s, int64_t nlaunch, F launch) {
  if (!g.timing) return launch();
  hipEvent_t a, b;
  hipError_t e = take_event(g, &a);
  if (e != hipSuccess) return e;
  if ((e = take_event(g, &b)) != hipSuccess) return e;
  if ((e = hipEventRecord(a, s)) != hipSuccess) return e;
  if ((e = launch()) != hipSuccess) return e;
  if ((e = hipEventRecord(b, s)) != hipSuccess) return e;
  g.events.emplace_back(a, b);
  g.timed_launches += nlaunch;
  return hipSuccess;
}

abcore_status read_state(Graph &g, hipStream_t s) {
  CHK(hipMemcpyAsync(g.h_state, g.state, sizeof(PeelState), hipMemcpyDeviceToHost, s));
  CHK(hipStreamSynchronize(s));
  return ABCORE_OK;
}

// Runs peel rounds until the frontier is empty.  Round kernels are enqueued
// in growing batches (4, 8, 16, ... up to rounds_per_sync); a launch after
// convergence returns immediately.
abcore_status run_rounds(Graph &g, PeelKind kind, int32_t thrU, int32_t thrL, hipStream_t s,
                         int64_t *launches) {
  // every non-empty round removes at least one vertex
  const int64_t max_launches = g.n + 4 * (int64_t)std::max(4, g.rounds_per_sync) + 8;
  int batch = 4;
  for (int64_t done = 0; done < max_launches; done += batch) {
    CHK(timed(g, s, batch, [&] { return launch_peel_rounds(g, kind, thrU, thrL, batch, s); }));
    *launches += batch;
    abcore_status st = read_state(g, s);
    if (st != ABCORE_OK) return st;
    if (g.h_state->lo >= g.h_state->hi) return ABCORE_OK;
    batch = std::min(batch * 2, std::max(4, g.rounds_per_sync));
  }
  set_error("peel did not converge");
  return ABCORE_EDEVICE;
}

abcore_status compute_core(Graph &g, hipStream_t s) {
  if (g.core_valid) return ABCORE_OK;
  abcore_status st;
  if ((st = ensure(&g.core, g.n)) != ABCORE_OK) return st;
  if ((st = ensure(&g.list, g.n)) != ABCORE_OK) return st;
  if ((st = ensure(&g.list2, g.n)) != ABCORE_OK) return st;
  CHK(launch_kcore_init(g, s));
  // each step either removes a vertex or raises the level past a live degree
  const int64_t max_steps = 3 * g.n + 256;
  int batch = 8;
  for (int64_t done = 0; done < max_steps; done += batch) {
    CHK(launch_kcore_steps(g, batch, s));
    if ((st = read_state(g, s)) != ABCORE_OK) return st;
    if (g.h_state->done) {
      g.max_core = g.h_state->max_core;
      g.core_valid = true;
      return ABCORE_OK;
    }
    batch = std::min(batch * 2, 64);
  }
  set_error("core decomposition did not converge");
  return ABCORE_EDEVICE;
}

abcore_status compute_components(Graph &g, hipStream_t s) {
  if (g.comp_valid) return ABCORE_OK;
  abcore_status st;
  if ((st = ensure(&g.comp, g.n)) != ABCORE_OK) return st;
  if ((st = ensure(&g.parent, g.n)) != ABCORE_OK) return st;
  if (g.n > 0) CHK(launch_cc(g, -1, s));
  CHK(hipStreamSynchronize(s));
  g.comp_valid = true;
  return ABCORE_OK;
}

abcore_status ensure_delta(Graph &g, hipStream_t s) {
  Delta &d = g.delta;
  if (d.head == nullptr) {
    abcore_status st = ensure(&d.head, g.n);
    if (st != ABCORE_OK) return st;
    CHK(hipMemsetAsync(d.head, 0xFF, sizeof(int32_t) * std::max<int64_t>(g.n, 1), s));
  }
  if (d.count < d.cap) return ABCORE_OK;
  const int64_t ncap = std::max<int64_t>(1024, d.cap * 2);
  int32_t *nn = nullptr, *no = nullptr;
  CHK(hipMalloc(&nn, sizeof(int32_t) * 2 * ncap));
  hipError_t e = hipMalloc(&no, sizeof(int32_t) * 2 * ncap);
  if (e != hipSuccess) {
    (void)hipFree(nn);
    set_error("delta growth failed: %s", hipGetErrorString(e));
    return ABCORE_ENOMEM;
  }
  if (d.count > 0) {
    CHK(hipMemcpyAsync(nn, d.next, sizeof(int32_t) * 2 * d.count, hipMemcpyDeviceToDevice, s));
    CHK(hipMemcpyAsync(no, d.other, sizeof(int32_t) * 2 * d.count, hipMemcpyDeviceToDevice, s));
  }
  CHK(hipStreamSynchronize(s));
  if (d.next) (void)hipFree(d.next);
  if (d.other) (void)hipFree(d.other);
  d.next = nn;
  d.other = no;
  d.cap = ncap;
  return ABCORE_OK;
}

}  // namespace
}  // namespace abc

using namespace abc;

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
  if (n_upper < 0 || n_lower < 0 || m < 0 || (int64_t)n_upper + n_lower >= 0x7FFFFFFFLL ||
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
  do {
    if (hipGetDevice(&g->device) != hipSuccess) {
      set_error("abcore_build_csr: no HIP device");
      st = ABCORE_EDEVICE;
      break;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, g->device) == hipSuccess && prop.multiProcessorCount > 0)
      g->cu_count = prop.multiProcessorCount;
    g->nU = n_upper;
    g->nL = n_lower;
    g->n = (int64_t)n_upper + n_lower;
    st = build_csr_device(*g, d_eu, d_ev, m, s);
    if (st != ABCORE_OK) break;
    if ((st = ensure(&g->deg, g->n)) != ABCORE_OK) break;
    if ((st = ensure(&g->queue, g->n + kLocalQueue)) != ABCORE_OK) break;
    hipError_t e = hipMalloc(&g->state, sizeof(PeelState));
    if (e == hipSuccess) e = hipHostMalloc(&g->h_state, sizeof(PeelState));
    if (e != hipSuccess) {
      set_error("abcore_build_csr: state allocation failed: %s", hipGetErrorString(e));
      st = ABCORE_ENOMEM;
      break;
    }
    memset(g->h_state, 0, sizeof(PeelState));
  } while (0);
  if (st != ABCORE_OK) {
    free_graph(g);
    return st;
  }
  if (out_m_distinct) *out_m_distinct = g->m;
  *out = reinterpret_cast<abcore_graph>(g);
  return ABCORE_OK;
}

abcore_status abcore_destroy(abcore_graph h) {
  free_graph(reinterpret_cast<Graph *>(h));
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
  if (!g || value < 0) {
    set_error("abcore_set_option: null handle or negative value");
    return ABCORE_EINVAL;
  }
  switch (option) {
    case ABCORE_OPT_PEEL_MODE:
      if (value > 1) {
        set_error("abcore_set_option: peel mode %lld not available", (long long)value);
        return ABCORE_EINVAL;
      }
      g->peel_mode = value == 0 ? 1 : (int)value;
      return ABCORE_OK;
    case ABCORE_OPT_GRID:
      g->grid = (int)std::min<int64_t>(value, 1 << 20);
      return ABCORE_OK;
    case ABCORE_OPT_TIMING:
      g->timing = value != 0;
      return ABCORE_OK;
    case ABCORE_OPT_ROUNDS_PER_SYNC:
      g->rounds_per_sync = value == 0 ? 16 : (int)std::min<int64_t>(value, 4096);
      return ABCORE_OK;
    default:
      set_error("abcore_set_option: unknown option %d", option);
      return ABCORE_EINVAL;
  }
}

abcore_status abcore_peel_timing(abcore_graph h, double *ms, int64_t *launches, int32_t reset) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (!g) {
    set_error("abcore_peel_timing: null handle");
    return ABCORE_EINVAL;
  }
  CHK(hipSetDevice(g->device));
  double total = 0.0;
  for (auto &pr : g->events) {
    CHK(hipEventSynchronize(pr.second));
    float t = 0.f;
    CHK(hipEventElapsedTime(&t, pr.first, pr.second));
    total += t;
  }
  if (ms) *ms = total;
  if (launches) *launches = g->timed_launches;
  if (reset) {
    for (auto &pr : g->events) {
      g->event_pool.push_back(pr.first);
      g->event_pool.push_back(pr.second);
    }
    g->events.clear();
    g->timed_launches = 0;
  }
  return ABCORE_OK;
}

abcore_status abcore_core_numbers(abcore_graph h, int32_t *d_core, int32_t *max_core,
                                  void *stream) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (!g) {
    set_error("abcore_core_numbers: null handle");
    return ABCORE_EINVAL;
  }
  CHK(hipSetDevice(g->device));
  hipStream_t s = as_stream(stream);
  abcore_status st = compute_core(*g, s);
  if (st != ABCORE_OK) return st;
  if (d_core && g->n > 0)
    CHK(hipMemcpyAsync(d_core, g->core, sizeof(int32_t) * g->n, hipMemcpyDeviceToDevice, s));
  CHK(hipStreamSynchronize(s));
  if (max_core) *max_core = g->max_core;
  return ABCORE_OK;
}

abcore_status abcore_components(abcore_graph h, int32_t *d_comp, void *stream) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (!g) {
    set_error("abcore_components: null handle");
    return ABCORE_EINVAL;
  }
  CHK(hipSetDevice(g->device));
  hipStream_t s = as_stream(stream);
  abcore_status st = compute_components(*g, s);
  if (st != ABCORE_OK) return st;
  if (d_comp && g->n > 0)
    CHK(hipMemcpyAsync(d_comp, g->comp, sizeof(int32_t) * g->n, hipMemcpyDeviceToDevice, s));
  CHK(hipStreamSynchronize(s));
  return ABCORE_OK;
}

abcore_status abcore_compute(abcore_graph h, uint32_t alpha, uint32_t beta, int32_t algo,
                             uint32_t *d_bitmask, abcore_stats *stats, void *stream) {
  Graph *g = reinterpret_cast<Graph *>(h);
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
  hipStream_t s = as_stream(stream);
  const int32_t thrU = clamp_thr(alpha), thrL = clamp_thr(beta);
  int64_t launches = 0, uncertain = 0;
  abcore_status st = ABCORE_OK;
  if (algo == ABCORE_GCC) {
    CHK(launch_init_state(g->state, s));
    CHK(launch_scan_gcc(*g, thrU, thrL, s));
    if ((st = run_rounds(*g, kGCC, thrU, thrL, s, &launches)) != ABCORE_OK) return st;
    CHK(launch_pack(*g, thrU, thrL, d_bitmask, s));
  } else {
    if ((st = compute_core(*g, s)) != ABCORE_OK) return st;
    const int32_t dl = std::min(thrU, thrL), dq = std::max(thrU, thrL);
    CHK(launch_init_state(g->state, s));
    if (dl == dq) {
      CHK(launch_pack_from_core(*g, dl, d_bitmask, s));
    } else {
      if ((st = ensure(&g->list, g->n)) != ABCORE_OK) return st;
      CHK(launch_classify(*g, thrU, thrL, dl, dq, s));
      CHK(launch_restricted_init(*g, thrU, thrL, dl, s));
      if ((st = run_rounds(*g, kGCCPlus, thrU, thrL, s, &launches)) != ABCORE_OK) return st;
      CHK(launch_pack(*g, thrU, thrL, d_bitmask, s));
    }
  }
  if (stats) {
    if ((st = read_state(*g, s)) != ABCORE_OK) return st;
    const PeelState &p = *g->h_state;
    if (algo == ABCORE_GCC_PLUS) uncertain = p.aux0;
    stats->removed = p.tail;
    stats->rounds = p.rounds;
    stats->entries_read = p.entries;
    stats->initial = p.first;
    stats->uncertain = uncertain;
    stats->launches = launches;
  }
  return ABCORE_OK;
}

abcore_status abcore_query(abcore_graph h, abcore_edge_update upd, uint32_t alpha,
                           uint32_t beta, int32_t *h_answer, uint32_t *h_endpoint_bits,
                           void *stream) {
  Graph *g = reinterpret_cast<Graph *>(h);
  if (!g || !h_answer) {
    set_error("abcore_query: null handle or answer pointer");
    return ABCORE_EINVAL;
  }
  if (upd.u < 0 || upd.u >= g->nU || upd.v < 0 || upd.v >= g->nL ||
      (upd.op != 1 && upd.op != -1)) {
    set_error("abcore_query: update (%d, %d, op %d) out of range", upd.u, upd.v, upd.op);
    return ABCORE_EINVAL;
  }
  if (alpha < 1 || beta < 1) {
    set_error("abcore_query: alpha and beta must be >= 1");
    return ABCORE_EINVAL;
  }
  CHK(hipSetDevice(g->device));
  hipStream_t s = as_stream(stream);
  abcore_status st;
  if ((st = compute_components(*g, s)) != ABCORE_OK) return st;
  if ((st = ensure_delta(*g, s)) != ABCORE_OK) return st;
  // 1. apply the update (validated on the device before any write)
  CHK(launch_init_state(g->state, s));
  CHK(launch_update(*g, upd.u, upd.v, upd.op, g->delta.count, s));
  if ((st = read_state(*g, s)) != ABCORE_OK) return st;
  const int32_t ustat = g->h_state->status;
  if (ustat == -(int32_t)ABCORE_EEXIST) {
    set_error("abcore_query: edge (%d, %d) already present", upd.u, upd.v);
    return ABCORE_EEXIST;
  }
  if (ustat == -(int32_t)ABCORE_ENOENT) {
    set_error("abcore_query: edge (%d, %d) not present", upd.u, upd.v);
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
  CHK(launch_init_state(g->state, s));
  CHK(launch_scan_component_of(*g, thrU, thrL, x, y, s));
  if ((st = run_rounds(*g, kGCC, thrU, thrL, s, &launches)) != ABCORE_OK) return st;
  CHK(launch_answer(*g, x, y, thrU, thrL, s));
  if ((st = read_state(*g, s)) != ABCORE_OK) return st;
  const int32_t bits = g->h_state->aux0;
  *h_answer = (bits & 3) == 3 ? 1 : 0;
  if (h_endpoint_bits) *h_endpoint_bits = (uint32_t)bits;
  return ABCORE_OK;
}

}  // extern "C"
