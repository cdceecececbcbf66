// On-the-fly query support (Sec. V, GFQ): connected components by parallel
// union-find, edge updates on the resident graph, and the scoped answer.
#include "prim.h"

#include <algorithm>

#include "abcore_internal.h"
#include "wave.h"

namespace abc {

namespace {

__device__ __forceinline__ int32_t aload(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void astore(int32_t *p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Union-find with parents that only ever point to smaller ids, so the root
// of every tree is the smallest id of its component (the canonical label).
// Reads are device-coherent atomics: a stale parent read could otherwise
// keep a thread retrying on an out-of-date root.
__device__ int32_t uf_find(int32_t *parent, int32_t x) {
  while (true) {
    const int32_t p = aload(&parent[x]);
    if (p == x) return x;
    const int32_t gp = aload(&parent[p]);
    if (gp == p) return p;
    astore(&parent[x], gp);  // path halving; gp is still an ancestor of x
    x = gp;
  }
}

__device__ void uf_union(int32_t *parent, int32_t a, int32_t b) {
  while (true) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a > b) {
      int32_t t = a;
      a = b;
      b = t;
    }
    const int32_t old = atomicCAS(&parent[b], b, a);
    if (old == b) return;
    b = old;
  }
}

__device__ __forceinline__ bool in_scope(const int32_t *comp, int32_t label, int64_t x) {
  return label < 0 || comp[x] == label;
}

__global__ void uf_init_kernel(int32_t *parent, const int32_t *comp, int32_t label, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride)
    if (in_scope(comp, label, x)) parent[x] = (int32_t)x;
}

// Sampling phase (the Afforest strategy of Sutton, Ben-Nun and Barak, 2018):
// every vertex in scope first unites with the first kSampleLinks entries of
// its row, which on skewed graphs already joins almost every vertex of the
// largest component into one tree.
constexpr int kSampleLinks = 2;

__global__ void uf_sample_link_kernel(const int64_t *__restrict__ off,
                                      const int32_t *__restrict__ cols, const int32_t *comp,
                                      int32_t label, int32_t *parent, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride) {
    if (!in_scope(comp, label, x)) continue;
    const int64_t s = off[x], e = off[x + 1];
    for (int64_t j = s; j < e && j < s + kSampleLinks; ++j) {
      const int32_t w = cols[j];
      if (w >= 0) uf_union(parent, (int32_t)x, w);
    }
  }
}

__global__ void uf_compress_kernel(int32_t *parent, const int32_t *comp, int32_t label,
                                   int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride)
    if (in_scope(comp, label, x)) astore(&parent[x], uf_find(parent, (int32_t)x));
}

// Roots of kRootSamples evenly spaced vertices (-1 when out of scope).
constexpr int kRootSamples = 1024;

__global__ void uf_sample_roots_kernel(const int32_t *parent, const int32_t *comp, int32_t label,
                                       int64_t n, int32_t *roots) {
  const int i = threadIdx.x;
  if (i >= kRootSamples) return;
  const int64_t x = (n * i) / kRootSamples;
  roots[i] = (x < n && in_scope(comp, label, x)) ? aload(&parent[x]) : -1;
}

// Completion: every vertex in scope outside the tree of root `big` unites
// with all of its neighbours (both layers' rows and inserted edges).  Edges
// with both ends in that tree need nothing: they are joined already.
__global__ __launch_bounds__(kBlock) void uf_rest_link_kernel(
    const int64_t *__restrict__ off, const int32_t *__restrict__ cols, const int32_t *comp,
    int32_t label, int32_t *parent, const int32_t *ins_head, const int32_t *ins_next,
    const int32_t *ins_other, int64_t n, int32_t big) {
  const int gw = blockIdx.x * kWavesPerBlock + wave_in_block();
  const int nw = gridDim.x * kWavesPerBlock;
  for (int64_t b = (int64_t)gw * kWave; b < n; b += (int64_t)nw * kWave) {
    const int64_t xi = b + lane_id();
    int32_t x = -1;
    if (xi < n && in_scope(comp, label, xi) && (big < 0 || uf_find(parent, (int32_t)xi) != big))
      x = (int32_t)xi;
    int64_t s = 0;
    int d = 0;
    if (x >= 0) {
      s = off[x];
      d = (int)(off[x + 1] - s);
    }
    const int incl = wave_incl_scan(d);
    const int total = __shfl(incl, kWave - 1, kWave);
    const int excl = incl - d;
    const int s_lo = (int)(uint32_t)(uint64_t)s;
    const int s_hi = (int)((uint64_t)s >> 32);
    for (int base = 0; base < total; base += kWave) {
      const int k = base + lane_id();
      const int kk = k < total ? k : total - 1;
      int j = 0;
#pragma unroll
      for (int step = 32; step > 0; step >>= 1) {
        int v = __shfl(incl, j + step - 1, kWave);
        if (v <= kk) j += step;
      }
      const int ex = __shfl(excl, j, kWave);
      const uint32_t lo32 = (uint32_t)__shfl(s_lo, j, kWave);
      const uint32_t hi32 = (uint32_t)__shfl(s_hi, j, kWave);
      const int32_t owner = __shfl(x, j, kWave);
      const int64_t start = (int64_t)(((uint64_t)hi32 << 32) | lo32);
      if (k < total) {
        const int32_t w = cols[start + (kk - ex)];
        if (w >= 0) uf_union(parent, owner, w);
      }
    }
    if (ins_head != nullptr && x >= 0) {
      for (int e = ins_head[x]; e >= 0; e = ins_next[e]) {
        const int32_t w = ins_other[e];
        if (w >= 0) uf_union(parent, x, w);
      }
    }
  }
}

__global__ void uf_label_kernel(int32_t *parent, int32_t *comp, int32_t label, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride)
    if (in_scope(comp, label, x)) comp[x] = uf_find(parent, (int32_t)x);
}

__global__ void relabel_kernel(int32_t *comp, int64_t n, int32_t from, int32_t to) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride)
    if (comp[x] == from) comp[x] = to;
}

// Position of `target` in the sorted CSR row [a, b) (entries compared after
// decoding tombstones ~c), or -1.
__device__ int64_t row_find(const int32_t *cols, int64_t a, int64_t b, int32_t target) {
  while (a < b) {
    const int64_t mid = a + (b - a) / 2;
    int32_t c = cols[mid];
    if (c < 0) c = ~c;
    if (c < target)
      a = mid + 1;
    else
      b = mid;
  }
  if (a < 0) return -1;
  return a;
}

// Applies one update on a single thread.  Validation precedes every write,
// so a rejected update leaves the graph untouched.  st->status: 0 applied,
// 1 applied using the new delta slot `slot`, -5 present (insertion),
// -4 absent (deletion).  aux0/aux1 receive the labels of u and v before the
// update.
__global__ void update_kernel(int64_t *off, int32_t *cols, int64_t m_csr, int32_t *deg0,
                              const int32_t *comp, int32_t *ins_head, int32_t *ins_next,
                              int32_t *ins_other, int64_t slot, int32_t nU, int32_t u,
                              int32_t v, int32_t op, PeelState *st) {
  const int32_t x = u, y = nU + v;
  st->aux0 = comp != nullptr ? comp[x] : -1;
  st->aux1 = comp != nullptr ? comp[y] : -1;
  // base CSR entry of the pair (row x holds y, row y holds x)
  int64_t jx = -1, jy = -1;
  {
    const int64_t a = off[x], b = off[x + 1];
    const int64_t p = row_find(cols, a, b, y);
    if (p < b) {
      int32_t c = cols[p];
      if ((c < 0 ? ~c : c) == y) jx = p;
    }
  }
  const bool csr_live = jx >= 0 && cols[jx] >= 0;
  if (jx >= 0) {
    const int64_t a = off[y], b = off[y + 1];
    jy = row_find(cols, a, b, x);
  }
  // inserted half-edge of the pair in row x (live or deleted)
  int32_t ex = -1;
  for (int32_t e = ins_head != nullptr ? ins_head[x] : -1; e >= 0; e = ins_next[e]) {
    const int32_t o = ins_other[e];
    if ((o < 0 ? ~o : o) == y) {
      ex = e;
      break;
    }
  }
  const bool delta_live = ex >= 0 && ins_other[ex] >= 0;
  const bool present = csr_live || delta_live;
  if (op > 0) {
    if (present) {
      st->status = -(int32_t)ABCORE_EEXIST;
      return;
    }
    if (jx >= 0) {  // revive the tombstoned CSR pair
      cols[jx] = y;
      cols[jy] = x;
      st->status = 0;
    } else if (ex >= 0) {  // revive the deleted inserted pair
      ins_other[ex] = y;
      ins_other[ex ^ 1] = x;
      st->status = 0;
    } else {
      const int32_t hx = (int32_t)(2 * slot), hy = (int32_t)(2 * slot + 1);
      ins_other[hx] = y;
      ins_other[hy] = x;
      ins_next[hx] = ins_head[x];
      ins_head[x] = hx;
      ins_next[hy] = ins_head[y];
      ins_head[y] = hy;
      st->status = 1;
    }
    deg0[x] += 1;
    deg0[y] += 1;
  } else {
    if (!present) {
      st->status = -(int32_t)ABCORE_ENOENT;
      return;
    }
    if (csr_live) {
      cols[jx] = ~y;
      cols[jy] = ~x;
    } else {
      ins_other[ex] = ~y;
      ins_other[ex ^ 1] = ~x;
    }
    deg0[x] -= 1;
    deg0[y] -= 1;
    st->status = 0;
  }
  (void)m_csr;
}

// A window of served updates, applied in order on a single thread (the order
// of the stream: each update is validated against the graph after the
// previous ones).  Append-only, so that queries of earlier versions still
// peeling see their own graph: a deleted base entry gets its deletion
// version in del_ver before it is tombstoned, a deleted inserted pair in
// pair_del_ver, and an insertion always takes a new pair (pairs are
// numbered in insertion order; a query sees pairs below its limit).  Each
// record: status (0, -EEXIST, -ENOENT), version (valid updates count up from
// ver_base), pairs after the update, labels of the endpoints before the
// window.
__global__ void update_window_kernel(const int64_t *off, int32_t *cols, int32_t *deg0,
                                     const int32_t *comp, int32_t *ins_head, int32_t *ins_next,
                                     int32_t *ins_other, int32_t *del_ver,
                                     int32_t *pair_del_ver, int32_t pair_base,
                                     int32_t ver_base, int32_t nU, const int32_t *upd, int w,
                                     WindowRecord *rec) {
  int32_t ver = ver_base, pairs = pair_base;
  for (int i = 0; i < w; ++i) {
    const int32_t x = upd[3 * i], y = nU + upd[3 * i + 1], op = upd[3 * i + 2];
    WindowRecord r;
    r.label_u = comp[x];
    r.label_v = comp[y];
    int64_t jx = -1, jy = -1;
    {
      const int64_t a = off[x], b = off[x + 1];
      const int64_t p = row_find(cols, a, b, y);
      if (p < b) {
        const int32_t c = cols[p];
        if ((c < 0 ? ~c : c) == y) jx = p;
      }
    }
    const bool csr_live = jx >= 0 && cols[jx] >= 0;
    if (csr_live) jy = row_find(cols, off[y], off[y + 1], x);
    int32_t ex = -1;  // live inserted half-edge of the pair in row x
    for (int32_t e = pairs > 0 ? ins_head[x] : -1; e >= 0; e = ins_next[e])
      if (ins_other[e] == y) {
        ex = e;
        break;
      }
    const bool present = csr_live || ex >= 0;
    r.status = 0;
    r.version = -1;
    if (op > 0 && present) {
      r.status = -(int32_t)ABCORE_EEXIST;
    } else if (op < 0 && !present) {
      r.status = -(int32_t)ABCORE_ENOENT;
    } else if (op > 0) {
      const int32_t v = ++ver;
      const int32_t hx = 2 * pairs, hy = 2 * pairs + 1;
      ins_other[hx] = y;
      ins_other[hy] = x;
      pair_del_ver[pairs] = 0x7FFFFFFF;
      ins_next[hx] = ins_head[x];
      ins_next[hy] = ins_head[y];
      __threadfence();  // the pair is complete before the lists point to it
      astore(&ins_head[x], hx);
      astore(&ins_head[y], hy);
      ++pairs;
      deg0[x] += 1;
      deg0[y] += 1;
      r.version = v;
    } else {
      const int32_t v = ++ver;
      if (csr_live) {
        del_ver[jx] = v;
        del_ver[jy] = v;
        __threadfence();  // the version is visible before the tombstone
        astore(&cols[jx], ~y);
        astore(&cols[jy], ~x);
      } else {
        pair_del_ver[ex >> 1] = v;
        __threadfence();
        astore(&ins_other[ex], ~y);
        astore(&ins_other[ex ^ 1], ~x);
      }
      deg0[x] -= 1;
      deg0[y] -= 1;
      r.version = v;
    }
    r.pairs_after = pairs;
    rec[i] = r;
  }
}

// Membership of the two endpoints after the scoped peel.
__global__ void answer_kernel(const int32_t *deg, int32_t x, int32_t y, int32_t thrU,
                              int32_t thrL, PeelState *st) {
  const int32_t bits = (deg[x] >= thrU ? 1 : 0) | (deg[y] >= thrL ? 2 : 0);
  st->aux0 = bits;
}

// Current-graph CSR export: degrees -> offsets are computed by the caller;
// each thread copies one row (live base entries, then inserted entries kept
// in ascending order by insertion).
__global__ void export_rows_kernel(const int64_t *off, const int32_t *cols,
                                   const int32_t *ins_head, const int32_t *ins_next,
                                   const int32_t *ins_other, const int64_t *out_off,
                                   int32_t *out_cols, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride) {
    int64_t o = out_off[x];
    const int64_t o0 = o;
    for (int64_t j = off[x]; j < off[x + 1]; ++j)
      if (cols[j] >= 0) out_cols[o++] = cols[j];
    if (ins_head != nullptr) {
      for (int32_t e = ins_head[x]; e >= 0; e = ins_next[e]) {
        const int32_t w = ins_other[e];
        if (w < 0) continue;
        int64_t p = o++;
        while (p > o0 && out_cols[p - 1] > w) {
          out_cols[p] = out_cols[p - 1];
          --p;
        }
        out_cols[p] = w;
      }
    }
  }
}

__global__ void widen_deg_kernel(const int32_t *deg, int64_t n, int64_t *out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += stride)
    out[i] = i < n ? (int64_t)deg[i] : 0;
}

int small_grid(const Graph &g, int64_t items) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((items + 255) / 256, g.cu_count * 8));
}

}  // namespace

// Component labels for the whole graph (label < 0) or re-labelling of the
// vertices currently labelled `label` (deletion may split that component).
// Synchronises the stream once (the largest tree's root is read on the
// host); uses the partial-sum buffers as scratch (they are reset before every
// computation).
hipError_t launch_cc(Graph &g, int32_t label, hipStream_t s) {
  static_assert(kRootSamples * sizeof(int32_t) <= kMaxBlocks * kPartFields * sizeof(int64_t),
                "root samples must fit the partial-sum buffer");
  const int32_t *head = g.delta.count > 0 ? g.delta.head : nullptr;
  int32_t *d_roots = reinterpret_cast<int32_t *>(g.part);
  int32_t *h_roots = reinterpret_cast<int32_t *>(g.h_part);
  uf_init_kernel<<<small_grid(g, g.n), 256, 0, s>>>(g.parent, g.comp, label, g.n);
  uf_sample_link_kernel<<<small_grid(g, g.n), 256, 0, s>>>(g.off, g.cols, g.comp, label,
                                                           g.parent, g.n);
  uf_compress_kernel<<<small_grid(g, g.n), 256, 0, s>>>(g.parent, g.comp, label, g.n);
  uf_sample_roots_kernel<<<1, kRootSamples, 0, s>>>(g.parent, g.comp, label, g.n, d_roots);
  hipError_t e = hipMemcpyAsync(h_roots, d_roots, sizeof(int32_t) * kRootSamples,
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  std::vector<int32_t> r(h_roots, h_roots + kRootSamples);
  std::sort(r.begin(), r.end());
  int32_t big = -1;
  int best = 0;
  for (size_t i = 0; i < r.size();) {
    size_t j = i;
    while (j < r.size() && r[j] == r[i]) ++j;
    if (r[i] >= 0 && (int)(j - i) > best) {
      best = (int)(j - i);
      big = r[i];
    }
    i = j;
  }
  uf_rest_link_kernel<<<wide_grid(g), kBlock, 0, s>>>(g.off, g.cols, g.comp, label, g.parent,
                                                      head, g.delta.next, g.delta.other, g.n,
                                                      big);
  uf_label_kernel<<<small_grid(g, g.n), 256, 0, s>>>(g.parent, g.comp, label, g.n);
  return hipGetLastError();
}

hipError_t launch_relabel(Graph &g, int32_t from, int32_t to, hipStream_t s) {
  relabel_kernel<<<small_grid(g, g.n), 256, 0, s>>>(g.comp, g.n, from, to);
  return hipGetLastError();
}

hipError_t launch_update(Graph &g, int32_t u, int32_t v, int32_t op, int64_t slot,
                         hipStream_t s) {
  update_kernel<<<1, 1, 0, s>>>(g.off, g.cols, g.m_csr, g.deg0, g.comp_valid ? g.comp : nullptr,
                                g.delta.head, g.delta.next, g.delta.other, slot, g.nU, u, v, op,
                                g.state);
  return hipGetLastError();
}

hipError_t launch_answer(Graph &g, int32_t x, int32_t y, int32_t thrU, int32_t thrL,
                         hipStream_t s) {
  answer_kernel<<<1, 1, 0, s>>>(g.deg, x, y, thrU, thrL, g.state);
  return hipGetLastError();
}

hipError_t launch_answer_view(const PeelArgs &a, int32_t x, int32_t y, hipStream_t s) {
  answer_kernel<<<1, 1, 0, s>>>(a.deg, x, y, a.thrU, a.thrL, a.st);
  return hipGetLastError();
}

hipError_t launch_update_window(Graph &g, const int32_t *d_upd, int w, WindowRecord *d_rec,
                                hipStream_t s) {
  update_window_kernel<<<1, 1, 0, s>>>(g.off, g.cols, g.deg0, g.comp, g.delta.head,
                                       g.delta.next, g.delta.other, g.del_ver, g.pair_del_ver,
                                       (int32_t)g.delta.count, g.upd_version, g.nU, d_upd, w,
                                       d_rec);
  return hipGetLastError();
}

// Writes the current CSR (n+1 offsets, 2m entries) to caller buffers.
hipError_t launch_export(Graph &g, int64_t *out_off, int32_t *out_cols, hipStream_t s) {
  int64_t *tmp64 = nullptr;
  void *temp = nullptr;
  size_t temp_bytes = 0;
  hipError_t e = dev_malloc_async(&tmp64, sizeof(int64_t) * (g.n + 1), s);
  if (e != hipSuccess) return e;
  widen_deg_kernel<<<small_grid(g, g.n + 1), 256, 0, s>>>(g.deg0, g.n, tmp64);
  e = prim::exclusive_sum(nullptr, temp_bytes, tmp64, out_off, (size_t)(g.n + 1), s);
  if (e == hipSuccess) e = dev_malloc_async(&temp, std::max<size_t>(temp_bytes, 16), s);
  if (e == hipSuccess)
    e = prim::exclusive_sum(temp, temp_bytes, tmp64, out_off, (size_t)(g.n + 1), s);
  if (e == hipSuccess && out_cols != nullptr) {
    const int32_t *head = g.delta.count > 0 ? g.delta.head : nullptr;
    export_rows_kernel<<<small_grid(g, g.n), 256, 0, s>>>(g.off, g.cols, head, g.delta.next,
                                                          g.delta.other, out_off, out_cols,
                                                          g.n);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (temp) (void)dev_free_async(temp, s);
  (void)dev_free_async(tmp64, s);
  return e;
}

}  // namespace abc
