// Scan, peel and pack kernels of GCC (Algorithm 1, Sec. IV-A) and GCC+
// (Algorithm 2, Sec. IV-B), and the level-synchronous k-core decomposition
// that provides GCC+'s core numbers (Definition 2).
//
// Mapping on gfx950: a wavefront takes 64 queued vertices at once (one per
// lane), prefix-sums their degrees and walks the concatenated adjacency 64
// entries per step, so a lane always owns one adjacency entry whatever the
// degree mix (coalesced CSR reads, no idle lanes on degree-1 vertices, hubs
// spread over the wave).  A neighbour is decremented with one device-scope
// atomic; the unique decrement that takes it from its threshold to one below
// enqueues it (every vertex enters the queue at most once).
#include <algorithm>

#include "abcore_internal.h"
#include "wave.h"

namespace abc {

// ---------------------------------------------------------------- state --

__global__ void init_state_kernel(PeelState *st) {
  PeelState z = {};
  z.min_alive = 0x7FFFFFFF;
  *st = z;
}

hipError_t launch_init_state(PeelState *st, hipStream_t s) {
  init_state_kernel<<<1, 1, 0, s>>>(st);
  return hipGetLastError();
}

int peel_grid(const Graph &g) {
  if (g.grid > 0) return g.grid;
  return g.cu_count * 8;  // 8 workgroups of 4 waves per CU: 32 waves per CU
}

// ----------------------------------------------------------- scan phase --
// Algorithm 1, scan phase: deg <- deg0 for every vertex and every vertex
// below its threshold (alpha for upper ids, beta for lower ids: a range check
// on the unified id) is appended to the frontier.  Four vertices per thread
// with 16-byte loads; one queue atomic per workgroup tile.

__global__ __launch_bounds__(kBlock) void scan_gcc_kernel(const int32_t *__restrict__ deg0,
                                                          int32_t *__restrict__ deg,
                                                          int32_t *__restrict__ q,
                                                          PeelState *st, int64_t n,
                                                          int32_t nU, int32_t thrU,
                                                          int32_t thrL) {
  __shared__ int s_wsum[kWavesPerBlock + 1];
  const int64_t tile = (int64_t)kBlock * 4;
  for (int64_t base = (int64_t)blockIdx.x * tile; base < n; base += (int64_t)gridDim.x * tile) {
    const int64_t x0 = base + (int64_t)threadIdx.x * 4;
    int32_t d[4] = {0, 0, 0, 0};
    bool p[4] = {false, false, false, false};
    if (x0 + 3 < n) {
      int4 v = *reinterpret_cast<const int4 *>(deg0 + x0);
      *reinterpret_cast<int4 *>(deg + x0) = v;
      d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
#pragma unroll
      for (int j = 0; j < 4; ++j) p[j] = d[j] < ((x0 + j) < nU ? thrU : thrL);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int64_t x = x0 + j;
        if (x < n) {
          d[j] = deg0[x];
          deg[x] = d[j];
          p[j] = d[j] < (x < nU ? thrU : thrL);
        }
      }
    }
    int cnt = (int)p[0] + (int)p[1] + (int)p[2] + (int)p[3];
    int pos = block_reserve(cnt, &st->tail, s_wsum);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (p[j]) q[pos++] = (int32_t)(x0 + j);
  }
  if (last_block_done(&st->finished)) {
    st->lo = 0;
    st->hi = atomicAdd(&st->tail, 0);
    st->first = st->hi;
    st->rounds = 0;
    st->finished = 0;
  }
}

hipError_t launch_scan_gcc(Graph &g, int32_t thrU, int32_t thrL, hipStream_t s) {
  int64_t tiles = (g.n + kBlock * 4 - 1) / (kBlock * 4);
  int grid = (int)std::min<int64_t>(std::max<int64_t>(tiles, 1), (int64_t)g.cu_count * 8);
  scan_gcc_kernel<<<grid, kBlock, 0, s>>>(g.deg0, g.deg, g.queue, g.state, g.n, g.nU, thrU,
                                          thrL);
  return hipGetLastError();
}

// GFQ (Sec. V): the scan restricted to the affected component(s); vertices of
// other components keep stale degrees and are never reached by the peel.
__global__ __launch_bounds__(kBlock) void scan_component_kernel(
    const int32_t *__restrict__ deg0, const int32_t *__restrict__ comp,
    int32_t *__restrict__ deg, int32_t *__restrict__ q, PeelState *st, int64_t n, int32_t nU,
    int32_t thrU, int32_t thrL, int32_t vx, int32_t vy) {
  __shared__ int s_wsum[kWavesPerBlock + 1];
  const int32_t c1 = comp[vx], c2 = comp[vy];
  const int64_t tile = (int64_t)kBlock * 4;
  for (int64_t base = (int64_t)blockIdx.x * tile; base < n; base += (int64_t)gridDim.x * tile) {
    const int64_t x0 = base + (int64_t)threadIdx.x * 4;
    bool p[4] = {false, false, false, false};
    if (x0 + 3 < n) {
      int4 c = *reinterpret_cast<const int4 *>(comp + x0);
      int cc[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (cc[j] == c1 || cc[j] == c2) {
          int32_t d = deg0[x0 + j];
          deg[x0 + j] = d;
          p[j] = d < ((x0 + j) < nU ? thrU : thrL);
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int64_t x = x0 + j;
        if (x < n && (comp[x] == c1 || comp[x] == c2)) {
          int32_t d = deg0[x];
          deg[x] = d;
          p[j] = d < (x < nU ? thrU : thrL);
        }
      }
    }
    int cnt = (int)p[0] + (int)p[1] + (int)p[2] + (int)p[3];
    int pos = block_reserve(cnt, &st->tail, s_wsum);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (p[j]) q[pos++] = (int32_t)(x0 + j);
  }
  if (last_block_done(&st->finished)) {
    st->lo = 0;
    st->hi = atomicAdd(&st->tail, 0);
    st->first = st->hi;
    st->rounds = 0;
    st->finished = 0;
  }
}

// Labels are read on the device from the endpoints x and y, after the
// component maintenance of the update has run on the same stream.
hipError_t launch_scan_component_of(Graph &g, int32_t thrU, int32_t thrL, int32_t x, int32_t y,
                                    hipStream_t s) {
  int64_t tiles = (g.n + kBlock * 4 - 1) / (kBlock * 4);
  int grid = (int)std::min<int64_t>(std::max<int64_t>(tiles, 1), (int64_t)g.cu_count * 8);
  scan_component_kernel<<<grid, kBlock, 0, s>>>(g.deg0, g.comp, g.deg, g.queue, g.state, g.n,
                                                g.nU, thrU, thrL, x, y);
  return hipGetLastError();
}

// ----------------------------------------------------------- peel phase --

// One decrement of Algorithm 1 (and Algorithm 2's filtered variant).
// The plain load is a filter: degrees only decrease, so a stale value is
// never below the true one, and a value below the threshold means the vertex
// is already removed or queued -- no atomic is needed.  GCC+ certain members
// (kDegIn) are skipped; certain non-members (kDegOut) fail the threshold test.
template <int KIND>
__device__ __forceinline__ bool peel_visit(const PeelArgs &a, int32_t w, int32_t thrU,
                                           int32_t thrL, int32_t level) {
  if (w < 0) return false;  // deleted edge
  const int32_t t = (KIND == kKCore) ? level + 1 : (w < a.nU ? thrU : thrL);
  const int32_t dw = a.deg[w];
  if (dw < t) return false;
  if (KIND == kGCCPlus && dw == kDegIn) return false;
  const int32_t old = atomicSub(&a.deg[w], 1);
  if (old != t) return false;
  if (KIND == kKCore) a.core[w] = level;
  return true;
}

// Processes up to 64 removed vertices (x < 0 marks an empty lane) with
// edge-balanced lanes: lane L of step s handles entry s*64+L of the
// concatenated adjacency lists.  The owner of an entry is found by a
// binary search over the wave's inclusive degree prefix (all in registers
// via cross-lane reads).
template <int KIND>
__device__ __forceinline__ void peel_batch(const PeelArgs &a, int32_t x, int32_t thrU,
                                           int32_t thrL, int32_t level, LocalQueue &lq,
                                           int64_t &entries) {
  int64_t s = 0;
  int d = 0;
  if (x >= 0) {
    s = a.off[x];
    d = (int)(a.off[x + 1] - s);
  }
  const int incl = wave_incl_scan(d);
  const int total = __shfl(incl, kWave - 1, kWave);
  const int excl = incl - d;
  const int s_lo = (int)(uint32_t)(uint64_t)s;
  const int s_hi = (int)((uint64_t)s >> 32);
  entries += d;
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
    const int64_t start = (int64_t)(((uint64_t)hi32 << 32) | lo32);
    bool push = false;
    int32_t w = -1;
    if (k < total) {
      w = a.cols[start + (kk - ex)];
      push = peel_visit<KIND>(a, w, thrU, thrL, level);
    }
    lq.push(push, w, a.queue, &a.st->tail);
  }
  if (a.ins_head != nullptr) {
    // edges inserted after the build: short per-vertex lists
    int e = x >= 0 ? a.ins_head[x] : -1;
    while (__ballot(e >= 0)) {
      bool push = false;
      int32_t w = -1;
      if (e >= 0) {
        w = a.ins_other[e];
        e = a.ins_next[e];
        entries += 1;
        push = peel_visit<KIND>(a, w, thrU, thrL, level);
      }
      lq.push(push, w, a.queue, &a.st->tail);
    }
  }
}

// Adds the workgroup's adjacency-entry count to the state (stats).
__device__ __forceinline__ void add_entries(int64_t entries, PeelState *st, int64_t *s_acc) {
  int64_t w = wave_sum64(entries);
  if (threadIdx.x == 0) *s_acc = 0;
  __syncthreads();
  if (lane_id() == 0 && w != 0) atomicAdd((unsigned long long *)s_acc, (unsigned long long)w);
  __syncthreads();
  if (threadIdx.x == 0 && *s_acc != 0)
    atomicAdd((unsigned long long *)&st->entries, (unsigned long long)*s_acc);
}

// One round: the vertices Q[lo, hi) are removed.  The last workgroup to
// finish advances the round to the items appended meanwhile.  Launched in
// batches; launches after convergence return at once.
template <int KIND>
__global__ __launch_bounds__(kBlock) void peel_round_kernel(PeelArgs a) {
  __shared__ int32_t s_lq[kWavesPerBlock][kLocalQueue];
  __shared__ int64_t s_acc;
  PeelState *st = a.st;
  const int32_t lo = st->lo, hi = st->hi;
  if (lo >= hi) return;
  const int32_t level = (KIND == kKCore) ? st->k : 0;
  LocalQueue lq{s_lq[wave_in_block()], 0};
  int64_t entries = 0;
  const int gw = blockIdx.x * kWavesPerBlock + wave_in_block();
  const int nw = gridDim.x * kWavesPerBlock;
  for (int64_t b = (int64_t)lo + (int64_t)gw * kWave; b < hi; b += (int64_t)nw * kWave) {
    const int64_t i = b + lane_id();
    const int32_t x = i < hi ? a.queue[i] : -1;
    peel_batch<KIND>(a, x, a.thrU, a.thrL, level, lq, entries);
  }
  lq.flush(a.queue, &st->tail);
  add_entries(entries, st, &s_acc);
  if (last_block_done(&st->finished)) {
    st->lo = hi;
    st->hi = atomicAdd(&st->tail, 0);
    st->rounds += 1;
    st->launches += 1;
    st->finished = 0;
  }
}

static PeelArgs make_args(Graph &g, int32_t thrU, int32_t thrL) {
  PeelArgs a;
  a.off = g.off;
  a.cols = g.cols;
  a.deg = g.deg;
  a.queue = g.queue;
  a.st = g.state;
  a.ins_head = g.delta.count > 0 ? g.delta.head : nullptr;
  a.ins_next = g.delta.next;
  a.ins_other = g.delta.other;
  a.core = g.core;
  a.nU = g.nU;
  a.thrU = thrU;
  a.thrL = thrL;
  return a;
}

hipError_t launch_peel_rounds(Graph &g, PeelKind kind, int32_t thrU, int32_t thrL, int rounds,
                              hipStream_t s) {
  PeelArgs a = make_args(g, thrU, thrL);
  const int grid = peel_grid(g);
  for (int r = 0; r < rounds; ++r) {
    if (kind == kGCC)
      peel_round_kernel<kGCC><<<grid, kBlock, 0, s>>>(a);
    else
      peel_round_kernel<kGCCPlus><<<grid, kBlock, 0, s>>>(a);
  }
  return hipGetLastError();
}

// ----------------------------------------------------------------- pack --
// Result of Algorithm 1 ("return V(G)"): a vertex is in the core iff its
// final degree is at least its threshold (a removed vertex went below its
// threshold once and only decreases afterwards).  One ballot per 64 ids.

__global__ __launch_bounds__(kBlock) void pack_kernel(const int32_t *__restrict__ deg,
                                                      int64_t n, int32_t nU, int32_t thrU,
                                                      int32_t thrL, uint32_t *__restrict__ bits,
                                                      int64_t nwords) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t base = ((int64_t)blockIdx.x * kWavesPerBlock + wave_in_block()) * kWave;
       base < nwords * 32; base += stride) {
    const int64_t x = base + lane_id();
    const bool p = x < n && deg[x] >= (x < nU ? thrU : thrL);
    const uint64_t mask = __ballot(p);
    const int64_t w0 = base / 32;
    if (lane_id() == 0) bits[w0] = (uint32_t)mask;
    if (lane_id() == 1 && w0 + 1 < nwords) bits[w0 + 1] = (uint32_t)(mask >> 32);
  }
}

hipError_t launch_pack(Graph &g, int32_t thrU, int32_t thrL, uint32_t *bits, hipStream_t s) {
  const int64_t nwords = (g.n + 31) / 32;
  if (nwords == 0) return hipSuccess;
  int64_t waves = (nwords * 32 + kWave - 1) / kWave;
  int grid = (int)std::min<int64_t>((waves + kWavesPerBlock - 1) / kWavesPerBlock,
                                    (int64_t)g.cu_count * 8);
  pack_kernel<<<grid, kBlock, 0, s>>>(g.deg, g.n, g.nU, thrU, thrL, bits, nwords);
  return hipGetLastError();
}

// GCC+ with alpha == beta: Lemma 1 decides every vertex (core >= k is in,
// core < k is out), so the result is a single scan of the core numbers.
__global__ __launch_bounds__(kBlock) void pack_from_core_kernel(const int32_t *__restrict__ core,
                                                                int64_t n, int32_t k,
                                                                uint32_t *__restrict__ bits,
                                                                int64_t nwords) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t base = ((int64_t)blockIdx.x * kWavesPerBlock + wave_in_block()) * kWave;
       base < nwords * 32; base += stride) {
    const int64_t x = base + lane_id();
    const bool p = x < n && core[x] >= k;
    const uint64_t mask = __ballot(p);
    const int64_t w0 = base / 32;
    if (lane_id() == 0) bits[w0] = (uint32_t)mask;
    if (lane_id() == 1 && w0 + 1 < nwords) bits[w0 + 1] = (uint32_t)(mask >> 32);
  }
}

hipError_t launch_pack_from_core(Graph &g, int32_t k, uint32_t *bits, hipStream_t s) {
  const int64_t nwords = (g.n + 31) / 32;
  if (nwords == 0) return hipSuccess;
  int64_t waves = (nwords * 32 + kWave - 1) / kWave;
  int grid = (int)std::min<int64_t>((waves + kWavesPerBlock - 1) / kWavesPerBlock,
                                    (int64_t)g.cu_count * 8);
  pack_from_core_kernel<<<grid, kBlock, 0, s>>>(g.core, g.n, k, bits, nwords);
  return hipGetLastError();
}

// ------------------------------------------------------------- GCC+ init --
// Algorithm 2's classification by Lemma 1 with delta_l = min(alpha,beta) and
// delta_q = max(alpha,beta): core < delta_l -> out, core >= delta_q -> in,
// otherwise uncertain (collected in g.list, count in st->aux0).

__global__ __launch_bounds__(kBlock) void classify_kernel(const int32_t *__restrict__ core,
                                                          int32_t *__restrict__ deg,
                                                          int32_t *__restrict__ unc,
                                                          PeelState *st, int64_t n, int32_t dl,
                                                          int32_t dq) {
  __shared__ int s_wsum[kWavesPerBlock + 1];
  const int64_t tile = (int64_t)kBlock * 4;
  for (int64_t base = (int64_t)blockIdx.x * tile; base < n; base += (int64_t)gridDim.x * tile) {
    const int64_t x0 = base + (int64_t)threadIdx.x * 4;
    bool p[4] = {false, false, false, false};
    int32_t c[4] = {0, 0, 0, 0};
    const bool full = x0 + 3 < n;
    if (full) {
      int4 v = *reinterpret_cast<const int4 *>(core + x0);
      c[0] = v.x; c[1] = v.y; c[2] = v.z; c[3] = v.w;
    } else {
      for (int j = 0; j < 4; ++j)
        if (x0 + j < n) c[j] = core[x0 + j];
    }
    int32_t dv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      dv[j] = c[j] < dl ? kDegOut : (c[j] >= dq ? kDegIn : 0);
      p[j] = (x0 + j < n) && c[j] >= dl && c[j] < dq;
    }
    if (full) {
      *reinterpret_cast<int4 *>(deg + x0) = make_int4(dv[0], dv[1], dv[2], dv[3]);
    } else {
      for (int j = 0; j < 4; ++j)
        if (x0 + j < n) deg[x0 + j] = dv[j];
    }
    int cnt = (int)p[0] + (int)p[1] + (int)p[2] + (int)p[3];
    int pos = block_reserve(cnt, &st->aux0, s_wsum);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (p[j]) unc[pos++] = (int32_t)(x0 + j);
  }
}

hipError_t launch_classify(Graph &g, int32_t thrU, int32_t thrL, int32_t dl, int32_t dq,
                           hipStream_t s) {
  (void)thrU;
  (void)thrL;
  int64_t tiles = (g.n + kBlock * 4 - 1) / (kBlock * 4);
  int grid = (int)std::min<int64_t>(std::max<int64_t>(tiles, 1), (int64_t)g.cu_count * 8);
  classify_kernel<<<grid, kBlock, 0, s>>>(g.core, g.deg, g.list, g.state, g.n, dl, dq);
  return hipGetLastError();
}

// Degree of every uncertain vertex inside G[{core >= delta_l}] -- the
// (alpha,beta)-core lies inside the (delta_l,delta_l)-core, so neighbours with
// smaller core numbers never count -- and the initial frontier of GCC+.
// Edge-balanced like the peel; per-vertex counts accumulate in LDS.
__global__ __launch_bounds__(kBlock) void restricted_init_kernel(PeelArgs a,
                                                                 const int32_t *__restrict__ unc,
                                                                 int32_t dl) {
  __shared__ int32_t s_lq[kWavesPerBlock][kLocalQueue];
  __shared__ int32_t s_cnt[kWavesPerBlock][kWave];
  __shared__ int64_t s_acc;
  PeelState *st = a.st;
  const int32_t nunc = st->aux0;
  LocalQueue lq{s_lq[wave_in_block()], 0};
  int32_t *cnt = s_cnt[wave_in_block()];
  int64_t entries = 0;
  const int gw = blockIdx.x * kWavesPerBlock + wave_in_block();
  const int nw = gridDim.x * kWavesPerBlock;
  for (int64_t b = (int64_t)gw * kWave; b < nunc; b += (int64_t)nw * kWave) {
    const int64_t i = b + lane_id();
    const int32_t x = i < nunc ? unc[i] : -1;
    int64_t s = 0;
    int d = 0;
    if (x >= 0) {
      s = a.off[x];
      d = (int)(a.off[x + 1] - s);
    }
    cnt[lane_id()] = 0;
    __builtin_amdgcn_wave_barrier();
    const int incl = wave_incl_scan(d);
    const int total = __shfl(incl, kWave - 1, kWave);
    const int excl = incl - d;
    const int s_lo = (int)(uint32_t)(uint64_t)s;
    const int s_hi = (int)((uint64_t)s >> 32);
    entries += d;
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
      const int64_t start = (int64_t)(((uint64_t)hi32 << 32) | lo32);
      if (k < total) {
        const int32_t w = a.cols[start + (kk - ex)];
        if (w >= 0 && a.core[w] >= dl) atomicAdd(&cnt[j], 1);
      }
    }
    int extra = 0;
    if (a.ins_head != nullptr && x >= 0) {
      for (int e = a.ins_head[x]; e >= 0; e = a.ins_next[e]) {
        const int32_t w = a.ins_other[e];
        if (w >= 0 && a.core[w] >= dl) ++extra;
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    bool push = false;
    if (x >= 0) {
      const int32_t dx = cnt[lane_id()] + extra;
      a.deg[x] = dx;
      push = dx < (x < a.nU ? a.thrU : a.thrL);
    }
    lq.push(push, x, a.queue, &st->tail);
    __builtin_amdgcn_wave_barrier();
  }
  lq.flush(a.queue, &st->tail);
  add_entries(entries, st, &s_acc);
  if (last_block_done(&st->finished)) {
    st->lo = 0;
    st->hi = atomicAdd(&st->tail, 0);
    st->first = st->hi;
    st->rounds = 0;
    st->finished = 0;
  }
}

hipError_t launch_restricted_init(Graph &g, int32_t thrU, int32_t thrL, int32_t dl,
                                  hipStream_t s) {
  PeelArgs a = make_args(g, thrU, thrL);
  restricted_init_kernel<<<peel_grid(g), kBlock, 0, s>>>(a, g.list, dl);
  return hipGetLastError();
}

// ------------------------------------------------------- core numbers --
// Level-synchronous k-core peeling (Definition 2; a (k,k)-core is the k-core
// of G taken as an ordinary graph).  Each launch performs one step:
//  - if the current round Q[lo,hi) is non-empty, it is peeled at level k
//    (threshold k+1; a vertex crossing to k gets core number k);
//  - otherwise a scan advances to the next level: every live vertex with
//    degree <= k' gets core k' and is queued, the alive list is compacted,
//    and when nothing was queued the smallest live degree gives the next
//    level directly (empty levels are skipped).

__global__ void kcore_init_kernel(const int32_t *__restrict__ deg0, int32_t *__restrict__ deg,
                                  int32_t *__restrict__ core, int32_t *__restrict__ alive,
                                  PeelState *st, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride) {
    deg[x] = deg0[x];
    core[x] = -1;
    alive[x] = (int32_t)x;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->alive_cur = (int32_t)n;
    st->next_k = 0;
    st->k = 0;
    st->max_core = 0;
    st->done = n == 0;
  }
}

hipError_t launch_kcore_init(Graph &g, hipStream_t s) {
  hipError_t e = launch_init_state(g.state, s);
  if (e != hipSuccess) return e;
  int grid = (int)std::min<int64_t>((g.n + kBlock - 1) / kBlock + 1, (int64_t)g.cu_count * 8);
  kcore_init_kernel<<<grid, kBlock, 0, s>>>(g.deg0, g.deg, g.core, g.list, g.state, g.n);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void kcore_step_kernel(PeelArgs a, int32_t *alive0,
                                                            int32_t *alive1) {
  __shared__ int32_t s_lq[kWavesPerBlock][kLocalQueue];
  __shared__ int64_t s_acc;
  __shared__ int s_wsum[kWavesPerBlock + 1];
  __shared__ int s_min;
  PeelState *st = a.st;
  if (st->done) return;
  const int32_t lo = st->lo, hi = st->hi;
  if (lo < hi) {
    const int32_t level = st->k;
    LocalQueue lq{s_lq[wave_in_block()], 0};
    int64_t entries = 0;
    const int gw = blockIdx.x * kWavesPerBlock + wave_in_block();
    const int nw = gridDim.x * kWavesPerBlock;
    for (int64_t b = (int64_t)lo + (int64_t)gw * kWave; b < hi; b += (int64_t)nw * kWave) {
      const int64_t i = b + lane_id();
      const int32_t x = i < hi ? a.queue[i] : -1;
      peel_batch<kKCore>(a, x, 0, 0, level, lq, entries);
    }
    lq.flush(a.queue, &st->tail);
    add_entries(entries, st, &s_acc);
    if (last_block_done(&st->finished)) {
      st->lo = hi;
      st->hi = atomicAdd(&st->tail, 0);
      st->rounds += 1;
      st->launches += 1;
      st->finished = 0;
    }
    return;
  }
  // scan step at level kn
  const int32_t kn = st->next_k;
  const int32_t cur = st->alive_cur;
  const int32_t *alive = st->alive_sel ? alive1 : alive0;
  int32_t *next = st->alive_sel ? alive0 : alive1;
  if (threadIdx.x == 0) s_min = 0x7FFFFFFF;
  __syncthreads();
  int local_min = 0x7FFFFFFF;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int64_t span = ((int64_t)cur + kBlock - 1) / kBlock * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < span; i += stride) {
    int32_t x = -1;
    bool push = false, keep = false;
    if (i < cur) {
      x = alive[i];
      if (a.core[x] < 0) {
        const int32_t d = a.deg[x];
        if (d <= kn) {
          a.core[x] = kn;
          push = true;
        } else {
          keep = true;
          local_min = min(local_min, d);
        }
      }
    }
    int pos = block_reserve((int)push, &st->tail, s_wsum);
    if (push) a.queue[pos] = x;
    pos = block_reserve((int)keep, &st->alive_next, s_wsum);
    if (keep) next[pos] = x;
  }
  local_min = wave_min(local_min);
  if (lane_id() == 0) atomicMin(&s_min, local_min);
  __syncthreads();
  if (threadIdx.x == 0 && s_min != 0x7FFFFFFF) atomicMin(&st->min_alive, s_min);
  if (last_block_done(&st->finished)) {
    const int32_t tail = atomicAdd(&st->tail, 0);
    const int32_t kept = atomicAdd(&st->alive_next, 0);
    const int32_t mn = atomicAdd(&st->min_alive, 0);
    const bool pushed = tail > hi;
    st->k = kn;
    st->lo = hi;
    st->hi = tail;
    if (pushed) st->max_core = kn;
    st->alive_cur = kept;
    st->alive_next = 0;
    st->alive_sel ^= 1;
    st->min_alive = 0x7FFFFFFF;
    st->next_k = pushed ? kn + 1 : max(kn + 1, mn);
    st->done = kept == 0;
    st->launches += 1;
    st->finished = 0;
  }
}

hipError_t launch_kcore_steps(Graph &g, int steps, hipStream_t s) {
  PeelArgs a = make_args(g, 0, 0);
  const int grid = peel_grid(g);
  for (int r = 0; r < steps; ++r)
    kcore_step_kernel<<<grid, kBlock, 0, s>>>(a, g.list, g.list2);
  return hipGetLastError();
}

}  // namespace abc
