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
//
// Rounds run either inside one cooperatively launched kernel separated by a
// grid barrier (no host involvement), or one kernel per round.  The first
// round of GCC may run in pull form: every vertex that survived the scan
// recounts its surviving neighbours from an LDS-staged bitmap, which replaces
// the scan frontier's atomic decrements (most of a power-law peel) by one
// streaming pass over the surviving rows.
//
// Same-address device-scope atomics and single-thread chains of coherent
// loads are the expensive operations here (about 11 ns and 1 us each), so
// appends are aggregated per workgroup, partial results live in per-workgroup
// slots, and round bookkeeping is done by a whole wave in parallel.
#include <algorithm>

#include <type_traits>

#include "abcore_internal.h"
#include "wave.h"

namespace abc {

constexpr int kScanBlock = 512;
constexpr int kScanChunk = 4096;  // vertices per workgroup chunk (4 per thread, 2 passes)

// ---------------------------------------------------------------- state --

// Queue slots not yet written hold kEmpty (the asynchronous peel waits on
// them); the previous computation's used prefixes [0, tail) are cleared
// before its state is reset.
constexpr int32_t kEmpty = -1;

// Returns the used prefixes [0, tail) of the sub-queues to kEmpty, this
// thread's share of them.  The cursors are read in one round trip (one lane
// each), then every prefix is cleared in turn.
__device__ __forceinline__ void clear_used_queue(int32_t *queue, int64_t qcap,
                                                 const PeelState *st, int64_t tid,
                                                 int64_t stride) {
  const int l = lane_id();
  const int32_t mine = l < kSub ? st->tail[l][0] : 0;
  for (int j = 0; j < kSub; ++j) {
    const int64_t t = min(max((int64_t)__shfl(mine, j, kWave), (int64_t)0), qcap);
    int32_t *q = queue + (int64_t)j * qcap;
    for (int64_t i = tid; i < t; i += stride) q[i] = kEmpty;
  }
}

// Both steps in one launch: every workgroup clears its share of the used
// queue prefixes and of the partial sums; the last one to finish (after
// every workgroup has read the append cursors) zeroes the state.
__global__ void reset_workspace_kernel(int32_t *queue, int64_t qcap, PeelState *st,
                                       int64_t *part, int nparts, int keep_word) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  clear_used_queue(queue, qcap, st, tid, stride);
  for (int64_t i = tid; i < nparts; i += stride) part[i] = 0;
  // no fence: the cursors were consumed (as loop bounds) before the arrival,
  // and the clearing stores need no order against the state's zeroing (the
  // next launch orders both)
  __syncthreads();
  if (wave_in_block() != 0) return;
  int last = 0;
  if (lane_id() == 0) last = arrive_on(&st->rst) ? 1 : 0;
  if (!__shfl(last, 0, kWave)) return;
  int32_t *words = reinterpret_cast<int32_t *>(st);
  constexpr int kRstBegin = (int)(offsetof(PeelState, rst) / 4);
  for (int i = lane_id(); i < kRstBegin; i += kWave)
    if (i != keep_word) words[i] = 0;
}

hipError_t launch_init_workspace(Graph &g, int32_t *queue, PeelState *state, int64_t *part,
                                  hipStream_t s, bool keep_abort) {
  static_assert(sizeof(PeelState) % 4 == 0, "state must be whole words");
  static_assert(offsetof(PeelState, abort_flag) % 4 == 0, "abort flag must be a word");
  const int keep = keep_abort ? (int)(offsetof(PeelState, abort_flag) / 4) : -1;
  reset_workspace_kernel<<<g.cu_count, 256, 0, s>>>(queue, g.qcap, state, part,
                                                    kMaxBlocks * kPartFields, keep);
  return hipGetLastError();
}

hipError_t launch_init_state(Graph &g, hipStream_t s, bool keep_abort) {
  return launch_init_workspace(g, g.queue, g.state, g.part, s, keep_abort);
}

int peel_grid(const Graph &g) {
  if (g.grid > 0) return std::min(g.grid, kMaxBlocks);
  return wide_grid(g);
}

int wide_grid(const Graph &g) {
  return std::min(g.cu_count * 4, kMaxBlocks);  // 4 workgroups of 8 waves per CU
}

// Asynchronous peel: one workgroup of 8 waves per CU unless set (measured
// best or near-best on power-law graphs of 20M-200M edges; abcore_autotune
// picks per graph).
int async_peel_grid(const Graph &g) {
  const int want = g.grid > 0 ? g.grid : g.cu_count;
  return std::max(1, std::min(want, g.async_grid > 0 ? g.async_grid : want));
}

static int flat_grid(const Graph &g, int64_t items, int per_block) {
  int64_t b = (items + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, std::min(g.cu_count * 8, kMaxBlocks)));
}

static int scan_grid(const Graph &g) {
  int64_t chunks = (g.n + kScanChunk - 1) / kScanChunk;
  return (int)std::max<int64_t>(1, std::min<int64_t>(chunks, std::min(g.cu_count * 4, kMaxBlocks)));
}

PeelArgs make_args(Graph &g, int32_t thrU, int32_t thrL) {
  PeelArgs a;
  a.off = g.off;
  a.cols = g.cols;
  a.deg = g.deg;
  a.queue = g.queue;
  a.qcap = g.qcap;
  a.st = g.state;
  a.part = g.part;
  a.ins_head = g.delta.count > 0 ? g.delta.head : nullptr;
  a.ins_next = g.delta.next;
  a.ins_other = g.delta.other;
  a.core = g.core;
  a.kdead = nullptr;
  a.piece_row = g.piece_row;
  a.piece_start = g.piece_start;
  a.piece_first = g.piece_first;
  a.del_ver = nullptr;
  a.pair_del_ver = nullptr;
  a.ver = 0x7FFFFFFF;
  a.pair_limit = 0x7FFFFFFF;
  a.claim = g.claim;
  a.fix_rows = nullptr;
  a.fix_bits = nullptr;
  a.nfix = 0;
  a.pack_bits = nullptr;
  a.start_expect = 0;
  a.alive0 = nullptr;
  a.f0_bits = nullptr;
  a.klim_u = -1;
  a.klim_l = -1;
  a.pack_vtx = nullptr;
  a.rs_mask = 0;
  a.rs_next_st = nullptr;
  a.rs_next_part = nullptr;
  a.rs_fail = nullptr;
  a.spin_limit = g.spin_limit > 0 ? g.spin_limit : kAsyncSpinLimit;
  a.abort_host = g.h_abort;
  a.append_sub = g.append_sub;
  a.dbg_enqueue = g.dbg_enqueue;
  // any launch but a query in rank order may leave the queue in use
  g.rs_ready = false;
  a.n = g.n;
  a.nU = g.nU;
  a.thrU = thrU;
  a.thrL = thrL;
  return a;
}

// Versioned view of an entry w loaded from position pos: an entry deleted
// after the query's version is still its edge.  Applied after a group of
// loads so that the loads stay in flight together (a.del_ver is uniform).
__device__ __forceinline__ int32_t view_col(const PeelArgs &a, bool valid, int64_t pos,
                                            int32_t w) {
  if (valid && w < 0 && ld_agent(&a.del_ver[pos]) > a.ver) return ~w;
  return w;
}

// Queue items: a vertex id x >= 0 (its whole row), or -(p + 2) for piece p
// of a split row (kPiece entries of it).
__device__ __forceinline__ int32_t piece_item(int32_t p) { return -(p + 2); }

// Row, entry range and "first piece" flag of an item (x < 0 with x != -1 is
// a piece; -1 is an empty lane).
// The degree slot of vertex (or, in rank order, rank) x.  In rank order
// consecutive ranks map to slots far apart (an odd multiplier is a bijection
// modulo a power of two).
constexpr uint32_t kRankMul = 0x9E3779B1u;
__device__ __forceinline__ int32_t deg_slot(const PeelArgs &a, int32_t x) {
  return a.rs_mask != 0 ? (int32_t)(((uint32_t)x * kRankMul) & a.rs_mask) : x;
}

__device__ __forceinline__ void decode_item(const PeelArgs &a, int32_t x, int32_t &row,
                                            int64_t &s, int &d, bool &first) {
  row = -1;
  s = 0;
  d = 0;
  first = false;
  if (x >= 0) {
    row = x;
    s = a.off[x];
    d = (int)(a.off[x + 1] - s);
    first = true;
  } else if (x < -1) {
    const int32_t p = -x - 2;
    row = a.piece_row[p];
    s = a.piece_start[p];
    const int64_t rs = a.off[row], re = a.off[row + 1];
    d = (int)(min(s + kPiece, re) - s);
    first = s == rs;
  }
}

// Appends removed vertices; a split row is appended as its pieces so that
// several waves share it.  Whole wave, uniform flow.
__device__ __forceinline__ void push_removed(const PeelArgs &a, LocalQueue &lq, bool pred,
                                             int32_t w) {
  const int32_t pf = pred ? a.piece_first[w] : -1;
  lq.push(pred && pf < 0, w);
  if (__ballot(pf >= 0)) {
    int np = 0;
    if (pf >= 0) np = (int)((a.off[w + 1] - a.off[w] + kPiece - 1) / kPiece);
    for (int k = 0; __ballot(k < np); ++k) lq.push(k < np, piece_item(pf + k));
  }
}

// Adds a workgroup total to its partial slot (block-exclusive, no atomics).
__device__ __forceinline__ void add_part(int64_t *part, int field, int64_t v, int64_t *s_acc) {
  const int64_t w = wave_sum64(v);
  if (threadIdx.x == 0) *s_acc = 0;
  __syncthreads();
  if (lane_id() == 0 && w != 0) atomicAdd((unsigned long long *)s_acc, (unsigned long long)w);
  __syncthreads();
  if (threadIdx.x == 0 && *s_acc != 0) part[(int64_t)blockIdx.x * kPartFields + field] += *s_acc;
}

// Collects a workgroup's appended vertices of one chunk in LDS and appends
// them to its sub-queue with one atomic.
struct ScanCollector {
  int32_t buf[kScanChunk];
  int count;
  int base;
  int rsub;

  // up to 4 items per thread; the whole workgroup calls in uniform flow
  __device__ __forceinline__ void append(const int32_t *items, int cnt) {
    const int incl = wave_incl_scan(cnt);
    int b = 0;
    if (lane_id() == kWave - 1 && incl > 0) b = atomicAdd(&count, incl);
    b = __shfl(b, kWave - 1, kWave);
    int pos = b + incl - cnt;
    for (int j = 0; j < cnt; ++j) buf[pos + j] = items[j];
  }

  // to a plain list with its own cursor
  __device__ __forceinline__ void flush(int32_t *q, int32_t *tail) {
    __syncthreads();
    const int c = count;
    if (threadIdx.x == 0) base = c > 0 ? atomicAdd(tail, c) : 0;
    __syncthreads();
    for (int i = threadIdx.x; i < c; i += blockDim.x) q[base + i] = buf[i];
    __syncthreads();
    if (threadIdx.x == 0) count = 0;
    __syncthreads();
  }

  // to the frontier queues, sub-queue `sub` first (reserve_slots)
  __device__ __forceinline__ void flush_queue(const PeelArgs &a, int sub) {
    __syncthreads();
    const int c = count;
    if (threadIdx.x == 0) {
      int2 r = make_int2(0, 0);
      if (c > 0) r = reserve_slots(a.st, a.queue, a.qcap, append_pref(a, sub), c, a.abort_host);
      base = r.y;
      rsub = r.x;
    }
    __syncthreads();
    if (rsub >= 0) {
      int32_t *q = a.queue + (int64_t)rsub * a.qcap + base;
      for (int i = threadIdx.x; i < c; i += blockDim.x) {
        q[i] = buf[i];
        ABC_COUNT_ENQUEUE(a.dbg_enqueue, buf[i]);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) count = 0;
    __syncthreads();
  }
};
static_assert(kScanChunk <= kMaxAppend, "a scan chunk is one append");

// ----------------------------------------------------------- scan phase --
// Algorithm 1, scan phase: deg <- deg0 for every vertex and every vertex
// below its threshold (alpha for upper ids, beta for lower ids: a range check
// on the unified id) is appended to the frontier.  Four vertices per thread
// with 16-byte loads.  Optionally writes the survivor bitmap used by a
// pull-form first round, and per-workgroup sums of the frontier size and
// degree (the push/pull decision).

__global__ __launch_bounds__(kScanBlock) void scan_gcc_kernel(PeelArgs a,
                                                              const int32_t *__restrict__ deg0,
                                                              uint32_t *__restrict__ bits,
                                                              int64_t n) {
  __shared__ ScanCollector col;
  __shared__ int64_t s_acc;
  if (threadIdx.x == 0) col.count = 0;
  __syncthreads();
  const int sub = blockIdx.x % kSub;
  int64_t f0 = 0, f0deg = 0;
  for (int64_t cb = (int64_t)blockIdx.x * kScanChunk; cb < n;
       cb += (int64_t)gridDim.x * kScanChunk) {
    for (int t = 0; t < kScanChunk; t += kScanBlock * 4) {
      const int64_t x0 = cb + t + (int64_t)threadIdx.x * 4;
      int32_t d[4] = {0, 0, 0, 0};
      bool p[4] = {false, false, false, false};
      uint32_t alive = 0;
      if (x0 + 3 < n) {
        int4 v = *reinterpret_cast<const int4 *>(deg0 + x0);
        *reinterpret_cast<int4 *>(a.deg + x0) = v;
        d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          p[j] = d[j] < ((x0 + j) < a.nU ? a.thrU : a.thrL);
          alive |= (uint32_t)(!p[j]) << j;
        }
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          int64_t x = x0 + j;
          if (x < n) {
            d[j] = deg0[x];
            a.deg[x] = d[j];
            p[j] = d[j] < (x < a.nU ? a.thrU : a.thrL);
            alive |= (uint32_t)(!p[j]) << j;
          }
        }
      }
      if (bits != nullptr) {
        // eight consecutive threads hold the 32 vertices of one bitmap word
        uint32_t w = alive << (4 * (lane_id() & 7));
        w |= __shfl_xor(w, 1, kWave);
        w |= __shfl_xor(w, 2, kWave);
        w |= __shfl_xor(w, 4, kWave);
        if ((lane_id() & 7) == 0 && x0 < n) bits[x0 / 32] = w;
      }
      int32_t items[4];
      int cnt = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (p[j]) {
          items[cnt++] = (int32_t)(x0 + j);
          f0deg += d[j];
        }
      }
      f0 += cnt;
      col.append(items, cnt);
    }
    col.flush_queue(a, sub);
  }
  add_part(a.part, kPartF0, f0, &s_acc);
  add_part(a.part, kPartF0Deg, f0deg, &s_acc);
  if (last_block_done<false>(a.st)) start_rounds_wave(a.st, a.qcap);
}

hipError_t launch_scan_gcc(Graph &g, int32_t thrU, int32_t thrL, bool want_bits,
                           hipStream_t s) {
  PeelArgs a = make_args(g, thrU, thrL);
  scan_gcc_kernel<<<scan_grid(g), kScanBlock, 0, s>>>(a, g.deg0,
                                                      want_bits ? g.alive_bits : nullptr, g.n);
  return hipGetLastError();
}

// The scan fused with the workspace reset, for the asynchronous peel after
// a pull round: the frontier is not queued here (the pull round counts it
// out of every surviving row, or queues it from the bitmap when it pushes
// instead).  Every workgroup first returns its share of the previous
// computation's queue prefixes to kEmpty and zeroes its partial slots; the
// last one to finish zeroes the state (all cursors were read by then).
__global__ __launch_bounds__(kScanBlock) void scan_reset_gcc_kernel(
    PeelArgs a, const int32_t *__restrict__ deg0, uint32_t *__restrict__ bits, int64_t n,
    int keep_word) {
  __shared__ int64_t s_acc;
  PeelState *st = a.st;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  clear_used_queue(a.queue, a.qcap, st, tid, stride);
  const int64_t nparts = (int64_t)kMaxBlocks * kPartFields;
  for (int64_t i = (int64_t)gridDim.x * kPartFields + tid; i < nparts; i += stride) a.part[i] = 0;
  if (threadIdx.x < kPartFields) a.part[(int64_t)blockIdx.x * kPartFields + threadIdx.x] = 0;
  __syncthreads();
  int64_t f0 = 0, f0deg = 0, alive_u = 0, alive_l = 0;
  for (int64_t cb = (int64_t)blockIdx.x * kScanChunk; cb < n;
       cb += (int64_t)gridDim.x * kScanChunk) {
    for (int t = 0; t < kScanChunk; t += kScanBlock * 4) {
      const int64_t x0 = cb + t + (int64_t)threadIdx.x * 4;
      int32_t d[4] = {0, 0, 0, 0};
      bool p[4] = {false, false, false, false};
      if (x0 + 3 < n) {
        const int4 v = *reinterpret_cast<const int4 *>(deg0 + x0);
        *reinterpret_cast<int4 *>(a.deg + x0) = v;
        d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
#pragma unroll
        for (int j = 0; j < 4; ++j) p[j] = d[j] < ((x0 + j) < a.nU ? a.thrU : a.thrL);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t x = x0 + j;
          if (x < n) {
            d[j] = deg0[x];
            a.deg[x] = d[j];
            p[j] = d[j] < (x < a.nU ? a.thrU : a.thrL);
          }
        }
      }
      uint32_t alive = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (x0 + j < n) {
          alive |= (uint32_t)(!p[j]) << j;
          if (!p[j]) {
            if (x0 + j < a.nU)
              ++alive_u;
            else
              ++alive_l;
          }
        }
        if (p[j]) {
          f0 += 1;
          f0deg += d[j];
        }
      }
      // eight consecutive threads hold the 32 vertices of one bitmap word
      uint32_t w = alive << (4 * (lane_id() & 7));
      w |= __shfl_xor(w, 1, kWave);
      w |= __shfl_xor(w, 2, kWave);
      w |= __shfl_xor(w, 4, kWave);
      if ((lane_id() & 7) == 0 && x0 < n) bits[x0 / 32] = w;
    }
  }
  add_part(a.part, kPartF0, f0, &s_acc);
  add_part(a.part, kPartF0Deg, f0deg, &s_acc);
  add_part(a.part, kPartAliveU, alive_u, &s_acc);
  add_part(a.part, kPartAliveL, alive_l, &s_acc);
  __syncthreads();
  if (wave_in_block() != 0) return;
  int last = 0;
  if (lane_id() == 0) last = arrive_on(&st->rst) ? 1 : 0;
  if (!__shfl(last, 0, kWave)) return;
  int32_t *words = reinterpret_cast<int32_t *>(st);
  constexpr int kRstBegin = (int)(offsetof(PeelState, rst) / 4);
  for (int i = lane_id(); i < kRstBegin; i += kWave)
    if (i != keep_word) words[i] = 0;
}

hipError_t launch_scan_reset_gcc(Graph &g, int32_t thrU, int32_t thrL, hipStream_t s,
                                  bool keep_abort) {
  PeelArgs a = make_args(g, thrU, thrL);
  const int keep = keep_abort ? (int)(offsetof(PeelState, abort_flag) / 4) : -1;
  scan_reset_gcc_kernel<<<scan_grid(g), kScanBlock, 0, s>>>(
      a, g.deg0, g.alive_bits, g.n, keep);
  return hipGetLastError();
}

// Scan of a nested query.  The working degrees hold the final state of a
// query (pU, pL) that the new query (thrU, thrL) dominates (pU <= thrU and
// pL <= thrL).  Its core contains the new core (the nesting of cores that
// Lemma 1's proof rests on), and a survivor's degree is exactly its degree
// inside it: every removed neighbour decremented it once (the filter never
// skips a vertex at or above its threshold).  Vertices the earlier query
// removed hold degrees below their old threshold and stay out; survivors
// below the new threshold form the frontier.  With bits, the scan also
// prepares a pull round: the bitmap of the survivors, the frontier's degree
// sum (what pushing it costs), the survivors' row entries (what pulling
// costs) and, for a surviving split row, the degree it leaves in place (its
// pieces recount the row from scratch and subtract that degree once; a
// pushed round keeps it).
__global__ __launch_bounds__(kScanBlock) void scan_nested_kernel(PeelArgs a, int32_t pU,
                                                                 int32_t pL, int64_t n,
                                                                 const int32_t *__restrict__ deg0,
                                                                 const int32_t *__restrict__ src,
                                                                 uint32_t *__restrict__ bits,
                                                                 uint32_t *__restrict__ fbits,
                                                                 int32_t *__restrict__ written) {
  __shared__ ScanCollector col;
  __shared__ int64_t s_acc;
  if (threadIdx.x == 0) col.count = 0;
  __syncthreads();
  const int sub = blockIdx.x % kSub;
  const int32_t *from = src != nullptr ? src : a.deg;
  int64_t f0 = 0, f0deg = 0, rest = 0;
  for (int64_t cb = (int64_t)blockIdx.x * kScanChunk; cb < n;
       cb += (int64_t)gridDim.x * kScanChunk) {
    for (int t = 0; t < kScanChunk; t += kScanBlock * 4) {
      const int64_t x0 = cb + t + (int64_t)threadIdx.x * 4;
      int32_t d[4] = {-1, -1, -1, -1};
      // whole degrees too when a pull round may follow: loaded with the
      // state, not behind it (one memory round trip per pass)
      int32_t w0[4] = {0, 0, 0, 0};
      if (x0 + 3 < n) {
        const int4 v = *reinterpret_cast<const int4 *>(from + x0);
        int4 v0 = make_int4(0, 0, 0, 0);
        if (bits != nullptr) v0 = *reinterpret_cast<const int4 *>(deg0 + x0);
        if (src != nullptr) *reinterpret_cast<int4 *>(a.deg + x0) = v;
        d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
        w0[0] = v0.x; w0[1] = v0.y; w0[2] = v0.z; w0[3] = v0.w;
      } else {
        for (int j = 0; j < 4; ++j)
          if (x0 + j < n) {
            d[j] = from[x0 + j];
            if (bits != nullptr) w0[j] = deg0[x0 + j];
            if (src != nullptr) a.deg[x0 + j] = d[j];
          }
      }
      int32_t items[4];
      int cnt = 0;
      uint32_t alive = 0, front = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool up = (x0 + j) < a.nU;
        const bool stays = x0 + j < n && d[j] >= (up ? a.thrU : a.thrL);
        if (x0 + j < n && d[j] >= (up ? pU : pL) && !stays) {
          items[cnt++] = (int32_t)(x0 + j);
          f0deg += d[j];
          front |= 1u << j;
        }
        alive |= (uint32_t)stays << j;
      }
      if (bits != nullptr) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if ((alive >> j) & 1u) {
            rest += w0[j];
            if (w0[j] > kPiece) written[a.piece_first[x0 + j]] = d[j];
          }
        }
        // eight consecutive threads hold the 32 vertices of one bitmap word
        uint32_t w = alive << (4 * (lane_id() & 7));
        w |= __shfl_xor(w, 1, kWave);
        w |= __shfl_xor(w, 2, kWave);
        w |= __shfl_xor(w, 4, kWave);
        if ((lane_id() & 7) == 0 && x0 < n) bits[x0 / 32] = w;
        if (fbits != nullptr) {
          uint32_t f = front << (4 * (lane_id() & 7));
          f |= __shfl_xor(f, 1, kWave);
          f |= __shfl_xor(f, 2, kWave);
          f |= __shfl_xor(f, 4, kWave);
          if ((lane_id() & 7) == 0 && x0 < n) fbits[x0 / 32] = f;
        }
      }
      f0 += cnt;
      // (with a frontier bitmap the pull kernel queues the frontier, and
      // only if it pushes)
      if (fbits == nullptr) col.append(items, cnt);
    }
    if (fbits == nullptr) col.flush_queue(a, sub);
  }
  add_part(a.part, kPartF0, f0, &s_acc);
  if (bits != nullptr) {
    add_part(a.part, kPartF0Deg, f0deg, &s_acc);
    add_part(a.part, kPartRest, rest, &s_acc);
  }
  if (last_block_done<false>(a.st)) start_rounds_wave(a.st, a.qcap);
}

hipError_t launch_scan_nested(Graph &g, int32_t pU, int32_t pL, int32_t thrU, int32_t thrL,
                              hipStream_t s, uint32_t *bits, const int32_t *src,
                              uint32_t *fbits) {
  PeelArgs a = make_args(g, thrU, thrL);
  scan_nested_kernel<<<scan_grid(g), kScanBlock, 0, s>>>(
      a, pU, pL, g.n, g.deg0, src, bits, bits != nullptr ? fbits : nullptr, g.split_written);
  return hipGetLastError();
}

// GFQ (Sec. V): the scan restricted to the affected component(s); vertices of
// other components keep stale degrees and are never reached by the peel.
// The labels are read on the device from the endpoints x and y, after the
// component maintenance of the update has run on the same stream.
// Served queries pass degree corrections (corr_x[i] gains corr_d[i]): the
// updates applied after the query's own, undone for its view.  They sit in
// an LDS hash table probed per scanned vertex.
constexpr int kCorrHash = 256;  // > 2 * kCorrMax, power of two

__global__ __launch_bounds__(kScanBlock) void scan_component_kernel(
    PeelArgs a, const int32_t *__restrict__ deg0, const int32_t *__restrict__ comp, int64_t n,
    int32_t vx, int32_t vy, const int32_t *__restrict__ corr_x,
    const int32_t *__restrict__ corr_d, int ncorr, uint32_t *__restrict__ bits) {
  __shared__ ScanCollector col;
  __shared__ int64_t s_acc;
  __shared__ int32_t h_key[kCorrHash];
  __shared__ int32_t h_val[kCorrHash];
  if (threadIdx.x == 0) col.count = 0;
  for (int i = threadIdx.x; i < kCorrHash; i += blockDim.x) h_key[i] = -1;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < ncorr; ++i) {
      const int32_t key = corr_x[i];
      uint32_t hsl = ((uint32_t)key * 2654435761u) >> 24;
      while (h_key[hsl & (kCorrHash - 1)] != -1 && h_key[hsl & (kCorrHash - 1)] != key) ++hsl;
      hsl &= kCorrHash - 1;
      if (h_key[hsl] == -1) {
        h_key[hsl] = key;
        h_val[hsl] = 0;
      }
      h_val[hsl] += corr_d[i];
    }
  }
  __syncthreads();
  const int32_t c1 = comp[vx], c2 = comp[vy];
  const int sub = blockIdx.x % kSub;
  int64_t f0 = 0, f0deg = 0;
  for (int64_t cb = (int64_t)blockIdx.x * kScanChunk; cb < n;
       cb += (int64_t)gridDim.x * kScanChunk) {
    for (int t = 0; t < kScanChunk; t += kScanBlock * 4) {
      const int64_t x0 = cb + t + (int64_t)threadIdx.x * 4;
      uint32_t alive = 0;
      int32_t cc[4] = {-1, -1, -1, -1};
      if (x0 + 3 < n) {
        int4 c = *reinterpret_cast<const int4 *>(comp + x0);
        cc[0] = c.x; cc[1] = c.y; cc[2] = c.z; cc[3] = c.w;
      } else {
        for (int j = 0; j < 4; ++j)
          if (x0 + j < n) cc[j] = comp[x0 + j];
      }
      int32_t items[4];
      int cnt = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (x0 + j < n && (cc[j] == c1 || cc[j] == c2)) {
          int32_t d = deg0[x0 + j];
          if (ncorr > 0) {
            const int32_t key = (int32_t)(x0 + j);
            uint32_t hsl = ((uint32_t)key * 2654435761u) >> 24;
            while (true) {
              const int32_t k = h_key[hsl & (kCorrHash - 1)];
              if (k == key) {
                d += h_val[hsl & (kCorrHash - 1)];
                break;
              }
              if (k == -1) break;
              ++hsl;
            }
          }
          a.deg[x0 + j] = d;
          if (d < ((x0 + j) < a.nU ? a.thrU : a.thrL)) {
            items[cnt++] = (int32_t)(x0 + j);
            f0deg += d;
          } else {
            alive |= 1u << j;
          }
        }
      }
      if (bits != nullptr) {
        // eight consecutive threads hold the 32 vertices of one bitmap word
        uint32_t wd = alive << (4 * (lane_id() & 7));
        wd |= __shfl_xor(wd, 1, kWave);
        wd |= __shfl_xor(wd, 2, kWave);
        wd |= __shfl_xor(wd, 4, kWave);
        if ((lane_id() & 7) == 0 && x0 < n) bits[x0 / 32] = wd;
      }
      f0 += cnt;
      col.append(items, cnt);
    }
    col.flush_queue(a, sub);
  }
  add_part(a.part, kPartF0, f0, &s_acc);
  add_part(a.part, kPartF0Deg, f0deg, &s_acc);
  if (last_block_done<false>(a.st)) start_rounds_wave(a.st, a.qcap);
}

hipError_t launch_scan_component_of(Graph &g, int32_t thrU, int32_t thrL, int32_t x, int32_t y,
                                    hipStream_t s) {
  PeelArgs a = make_args(g, thrU, thrL);
  scan_component_kernel<<<scan_grid(g), kScanBlock, 0, s>>>(
      a, g.deg0, g.comp, g.n, x, y, nullptr, nullptr, 0,
      g.pull_mode != 1 ? g.alive_bits : nullptr);
  return hipGetLastError();
}

hipError_t launch_scan_component_view(Graph &g, const PeelArgs &a, int32_t x, int32_t y,
                                      const int32_t *corr_x, const int32_t *corr_d, int ncorr,
                                      uint32_t *bits, hipStream_t s) {
  if (ncorr < 0 || ncorr > kCorrMax) return hipErrorInvalidValue;
  scan_component_kernel<<<scan_grid(g), kScanBlock, 0, s>>>(a, g.deg0, g.comp, g.n, x, y,
                                                            corr_x, corr_d, ncorr, bits);
  return hipGetLastError();
}

// ------------------------------------------------- edge-balanced walking --
// Lane L of step s of a wave batch handles entry s*64+L of the concatenated
// adjacency lists of the batch's vertices.  The owner of an entry is found
// by a binary search over the wave's inclusive degree prefix, in registers
// through cross-lane reads.
struct BatchWalk {
  int incl, excl, total;
  int s_lo, s_hi;

  __device__ __forceinline__ void init(int64_t s, int d) {
    incl = wave_incl_scan(d);
    total = __shfl(incl, kWave - 1, kWave);
    excl = incl - d;
    s_lo = (int)(uint32_t)(uint64_t)s;
    s_hi = (int)((uint64_t)s >> 32);
  }
  // For entry kk (< total): owner lane j and the entry's position in cols.
  __device__ __forceinline__ int64_t locate(int kk, int &j) const {
    j = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
      int v = __shfl(incl, j + step - 1, kWave);
      if (v <= kk) j += step;
    }
    const int ex = __shfl(excl, j, kWave);
    const uint32_t lo32 = (uint32_t)__shfl(s_lo, j, kWave);
    const uint32_t hi32 = (uint32_t)__shfl(s_hi, j, kWave);
    return (int64_t)(((uint64_t)hi32 << 32) | lo32) + (kk - ex);
  }
};

// Adds, for every owner lane, the number of its entries of this step whose
// flag is set (entries of one owner are contiguous lanes of the step).
__device__ __forceinline__ void segmented_count(int32_t *cnt, int j, bool act, bool ok,
                                                int nact) {
  const int jprev = __shfl_up(j, 1, kWave);
  const bool start = act && (lane_id() == 0 || jprev != j);
  const uint64_t starts = __ballot(start);
  const uint64_t okm = __ballot(ok);
  if (start) {
    const int L = lane_id();
    const uint64_t le = L == 63 ? ~0ull : ((1ull << (L + 1)) - 1);
    const uint64_t rest = starts & ~le;
    const int end = rest ? __builtin_ctzll(rest) : nact;
    const uint64_t upto = end >= 64 ? ~0ull : ((1ull << end) - 1);
    const uint64_t from = (1ull << L) - 1;
    cnt[j] += __popcll(okm & upto & ~from);
  }
  __builtin_amdgcn_wave_barrier();
}

// ----------------------------------------------------------- peel phase --

// One decrement of Algorithm 1 (and Algorithm 2's filtered variant): the
// vertex is queued iff the decrement takes its degree from the threshold to
// below it (the unique crossing: degrees only decrease).  GCC+ first loads
// the degree as a filter: a stale value is never below the true one, certain
// members (kDegIn) are skipped and certain non-members (kDegOut) fail the
// threshold test.
template <int KIND>
__device__ __forceinline__ bool peel_visit(const PeelArgs &a, int32_t w, int32_t level) {
  if (w < 0) return false;  // deleted edge
  const int32_t t = (KIND == kKCore) ? level + 1 : (w < a.nU ? a.thrU : a.thrL);
  if (KIND == kGCCPlus) {
    const int32_t dw = a.deg[w];
    if (dw < t || dw == kDegIn) return false;
  }
  return atomicSub(&a.deg[w], 1) == t;
}

// Steps of 64 entries whose loads a wave issues together: each step is a
// chain of dependent accesses (entry, degree, atomic), so independent steps
// are interleaved to keep several in flight per wave.
#ifndef ABC_UNROLL
#define ABC_UNROLL 4
#endif
#ifndef ABC_LEVEL_COMPACT_ALWAYS
#define ABC_LEVEL_COMPACT_ALWAYS 0
#endif
constexpr int kUnroll = ABC_UNROLL;

// Removes up to 64 queue items (vertices or pieces of split rows; -1 marks
// an empty lane).  LAZY (the asynchronous peel, which has no rounds): removed
// vertices are queued as plain ids, and a split row is expanded into its
// pieces when its item is taken -- the producer saves a dependent load per
// removal, the hub's walk moves one hop later.  Otherwise (round peels,
// whose round count is reported) split rows are queued as pieces at once.
template <int KIND, bool LAZY = false>
__device__ __forceinline__ void peel_batch(const PeelArgs &a, int32_t x, int32_t level,
                                           LocalQueue &lq, int64_t &entries) {
  int32_t row;
  int64_t s;
  int d;
  bool first;
  decode_item(a, x, row, s, d, first);
  if (KIND == kKCore && a.kdead != nullptr && x >= 0)
    atomicOr(&a.kdead[x >> 5], 1u << (x & 31));  // taken once: removed from here on
  if (LAZY && a.pack_vtx != nullptr && a.pack_bits != nullptr && x >= 0) {
    // rank order: the result bitmask holds the scan's survivors; a removed
    // vertex is taken here exactly once (its rank), so its bit is cleared
    // here, off the removal chain (no return value is waited for), and no
    // pack follows termination
    const int32_t v = a.pack_vtx[x];
    atomicAnd(&a.pack_bits[v >> 5], ~(1u << (v & 31)));
  }
  if (LAZY) {
    const bool split = x >= 0 && d > kPiece;
    if (__ballot(split)) {
      int np = 0;
      int32_t pf = 0;
      if (split) {
        // After a pull round a split row can be queued twice: by the
        // decrement that takes it below its threshold and by the start
        // phase's test of its pull-round count, which may read the degree
        // after that decrement.  The first consumer marks the degree (the
        // row is out of the core, its count no longer matters) and walks
        // the row; a later copy finds the mark and walks nothing.
        const bool mine = a.fix_bits == nullptr ||
                          atomicExch(&a.deg[x], kClaimedDeg) > kClaimedDeg / 2;
        if (mine) {
          pf = a.piece_first[x];
          np = (d + kPiece - 1) / kPiece;
        }
        d = 0;          // walked by its pieces
        first = false;  // the first piece walks the inserted edges
      }
      if (KIND == kKCore) {
        // core numbers: a level near the top removes a few hubs and little
        // else, and a hub's pieces kept local would be walked by one wave
        // (levels of 1,000 take 0.5 ms so); all but its first piece go to the
        // shared sub-queue at once, for the idle waves to take
        if (__ballot(np > 1)) {
          for (int k = 1; __ballot(k < np); ++k) lq.push(k < np, piece_item(pf + k));
          lq.flush();
        }
        lq.push(np > 0, piece_item(pf));
      } else {
        for (int k = 0; __ballot(k < np); ++k) lq.push(k < np, piece_item(pf + k));
      }
    }
  }
  BatchWalk bw;
  bw.init(s, d);
  entries += d;
  for (int base = 0; base < bw.total; base += kUnroll * kWave) {
    int32_t w[kUnroll];
    int64_t p[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int k = base + u * kWave + lane_id();
      int j;
      const int64_t pos = bw.locate(k < bw.total ? k : bw.total - 1, j);
      w[u] = k < bw.total ? a.cols[pos] : -1;
      p[u] = k < bw.total ? pos : -1;
    }
    if (a.del_ver != nullptr) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) w[u] = view_col(a, p[u] >= 0, p[u], w[u]);
    }
    int32_t t[kUnroll], dw[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      t[u] = (KIND == kKCore) ? level + 1 : (w[u] < a.nU ? a.thrU : a.thrL);
      // GCC+ loads the degree first: certain members (kDegIn) are never
      // decremented and certain non-members fail the threshold test.  The
      // other peels decrement unconditionally: the atomic returns the old
      // degree, which alone decides the crossing, and a removed vertex can
      // never cross again (its degree is already below the threshold) --
      // one round trip instead of a load followed by an atomic
      dw[u] = w[u] >= 0 ? (KIND == kGCCPlus ? a.deg[w[u]] : kMaxThreshold) : -1;
    }
    // core numbers: a neighbour removed before (at an earlier level, or
    // taken already at this one) needs no decrement; its bit is read from a
    // small bitmap, ahead of the atomics
    uint32_t gone[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      gone[u] = (KIND == kKCore && a.kdead != nullptr && w[u] >= 0)
                    ? (a.kdead[w[u] >> 5] >> (w[u] & 31)) & 1u
                    : 0u;
    bool push[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      // GCC+: the plain load is a filter (degrees only decrease, so a stale
      // value is never below the true one)
      bool live = w[u] >= 0 && dw[u] >= t[u];
      if (KIND == kGCCPlus) live = live && dw[u] != kDegIn;
      // the decrements are atomic-throughput bound: a vertex of the scan
      // frontier (a small, cache-resident bitmap) needs none
      if (KIND == kGCC && a.alive0 != nullptr && w[u] >= 0)
        live = live && ((a.alive0[w[u] >> 5] >> (w[u] & 31)) & 1u);
      // in rank order the scan's survivors are a prefix of each layer
      if (KIND == kGCC && a.klim_u >= 0)
        live = live && (w[u] < a.nU ? w[u] < a.klim_u : w[u] - a.nU < a.klim_l);
      if (KIND == kKCore) live = live && gone[u] == 0;
      push[u] = live && atomicSub(&a.deg[deg_slot(a, w[u])], 1) == t[u];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (KIND == kKCore && push[u]) st_agent(&a.core[w[u]], level);
      if (LAZY)
        lq.push(push[u], w[u]);
      else
        push_removed(a, lq, push[u], w[u]);
    }
  }
  if (a.ins_head != nullptr) {
    // edges inserted after the build: short per-vertex lists, walked once
    // per row (by its first piece)
    int e = (row >= 0 && first) ? a.ins_head[row] : -1;
    while (__ballot(e >= 0)) {
      bool push = false;
      int32_t w = -1;
      if (e >= 0) {
        if (a.del_ver == nullptr) {
          w = a.ins_other[e];
          e = a.ins_next[e];
        } else {
          // pairs at or past the limit were inserted after this query's
          // version, possibly while it runs: read coherently and skip them
          const int pair = e >> 1;
          if (pair >= a.pair_limit) {
            w = -1;
            e = ld_agent(&a.ins_next[e]);
          } else {
            w = a.ins_other[e];
            if (w < 0 && ld_agent(&a.pair_del_ver[pair]) > a.ver) w = ~w;
            e = a.ins_next[e];
          }
        }
        entries += 1;
        push = peel_visit<KIND>(a, w, level);
        if (KIND == kKCore && push) st_agent(&a.core[w], level);
      }
      if (LAZY)
        lq.push(push, w);
      else
        push_removed(a, lq, push, w);
    }
  }
}

// The work of one round over the current view; called by every thread.
template <int KIND>
__device__ __forceinline__ void peel_round_body(const PeelArgs &a, const RangeView &v,
                                                int32_t level, LocalQueue &lq,
                                                int64_t &entries) {
  const int32_t total = v.pre[kSub];
  const int waves = blockDim.x / kWave;
  const int gw = blockIdx.x * waves + wave_in_block();
  const int nw = gridDim.x * waves;
  for (int64_t b = (int64_t)gw * kWave; b < total; b += (int64_t)nw * kWave) {
    const int32_t i = (int32_t)(b + lane_id());
    const int32_t x = i < total ? view_item(v, a.queue, a.qcap, i) : -1;
    peel_batch<KIND>(a, x, level, lq, entries);
  }
}

// One round per launch; the last workgroup advances the round.  Launches
// after convergence return at once.
template <int KIND>
__global__ __launch_bounds__(kPeelBlock) void peel_round_kernel(PeelArgs a) {
  __shared__ int32_t s_lq[kPeelWaves][kLocalQueue];
  __shared__ RangeView s_view;
  __shared__ int s_cnt[kPeelWaves + 2];
  __shared__ int64_t s_acc;
  load_view(s_view, a.st);
  if (s_view.pre[kSub] == 0) return;
  LocalQueue lq = make_lq(s_lq[wave_in_block()], kLocalQueue, a);
  int64_t entries = 0;
  peel_round_body<KIND>(a, s_view, 0, lq, entries);
  block_flush(lq, s_cnt);
  add_part(a.part, kPartEntries, entries, &s_acc);
  if (last_block_done<false>(a.st)) {
    advance_round_wave(a.st, a.qcap);
    if (lane_id() == 0) atomicAdd((unsigned long long *)&a.st->launches, 1ull);
  }
}

// All rounds in one cooperative launch, separated by grid barriers.  Every
// non-empty round removes a vertex, so more than max_rounds rounds can only
// come from a fault; the loop then flags an abort instead of running on.
// Queue items cross workgroups through agent-scope stores and loads and the
// degrees only through atomics (plus stale-safe filter loads), so the
// barriers need no cache write-back or invalidation.
template <int KIND>
__global__ __launch_bounds__(kPeelBlock) void peel_persistent_kernel(PeelArgs a,
                                                                     int64_t max_rounds) {
  __shared__ int32_t s_lq[kPeelWaves][kLocalQueue];
  __shared__ RangeView s_view;
  __shared__ int s_cnt[kPeelWaves + 2];
  __shared__ int s_abort;
  __shared__ int64_t s_acc;
  LocalQueue lq = make_lq(s_lq[wave_in_block()], kLocalQueue, a);
  int64_t entries = 0;
  for (int64_t it = 0;; ++it) {
    if (threadIdx.x == 0) s_abort = ld_agent(&a.st->abort_flag);
    load_view(s_view, a.st);
    if (s_view.pre[kSub] == 0 || s_abort) break;
    if (it > max_rounds) {
      if (threadIdx.x == 0) st_agent(&a.st->abort_flag, 1);
      break;
    }
    peel_round_body<KIND>(a, s_view, 0, lq, entries);
    block_flush(lq, s_cnt);
    grid_sync<false>(a.st, [&] {
      advance_round_wave(a.st, a.qcap);
      if (lane_id() == 0) atomicAdd((unsigned long long *)&a.st->launches, 1ull);
    });
  }
  if (threadIdx.x == 0 && ld_agent(&a.st->abort_flag) != 0) report_abort(a);
  add_part(a.part, kPartEntries, entries, &s_acc);
}

hipError_t launch_peel_rounds(Graph &g, PeelKind kind, int32_t thrU, int32_t thrL, int rounds,
                              hipStream_t s) {
  PeelArgs a = make_args(g, thrU, thrL);
  const int grid = peel_grid(g);
  for (int r = 0; r < rounds; ++r) {
    if (kind == kGCC)
      peel_round_kernel<kGCC><<<grid, kPeelBlock, 0, s>>>(a);
    else
      peel_round_kernel<kGCCPlus><<<grid, kPeelBlock, 0, s>>>(a);
  }
  return hipGetLastError();
}

hipError_t launch_peel_persistent(Graph &g, PeelKind kind, int32_t thrU, int32_t thrL,
                                  hipStream_t s) {
  PeelArgs a = make_args(g, thrU, thrL);
  int64_t max_rounds = g.n + 2;
  void *args[] = {&a, &max_rounds};
  const void *fn = kind == kGCC ? reinterpret_cast<const void *>(&peel_persistent_kernel<kGCC>)
                                : reinterpret_cast<const void *>(&peel_persistent_kernel<kGCCPlus>);
  return hipLaunchCooperativeKernel(fn, dim3(g.persistent_grid), dim3(kPeelBlock), args, 0, s);
}

// --------------------------------------------------- asynchronous worklist --
// The peel without rounds: since the core does not depend on the order of
// removals (Definition 1 fixes a unique result), a removed vertex can be
// processed as soon as it is queued.  Each workgroup is bound to one
// sub-queue; its waves claim slots in groups, process the items as they
// are written (a slot holds kEmpty until then) and append what they remove to
// the same sub-queue, whose claimed-but-unwritten slots always belong to a
// waiting wave of that sub-queue.  Termination: every queued item has been
// processed, read as sum(done) == sum(tail) with all `done` read before any
// `tail` (an item's appends precede its `done` increment), which means no item
// was in flight and none can be appended any more.  Wave 0 of a waiting
// workgroup also steals: it claims exactly the appended-but-unclaimed slots
// of another sub-queue (compare-and-swap on that head, never past its tail),
// so items never wait for a workgroup of their own sub-queue to be
// resident, and several peels can share the device without any co-residency
// assumption.  Only wave 0 of a workgroup reads the shared termination words
// (same-address reads serialise like atomics); it tells the other waves
// through LDS.  Claims are 32 slots by default (a.claim).

__device__ __forceinline__ bool quiescent(PeelState *st, int32_t start_expect, int64_t qcap) {
  const int j = lane_id();
  int32_t d = 0, t = 0;
  if (start_expect > 0) {
    // every workgroup has queued its start-phase items
    const int32_t sv = j < kGroups ? ld_agent(&st->started[j][0]) : 0;
    if (wave_sum(sv) < start_expect) return false;
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  }
  if (j < kSub) d = ld_agent(&st->consumed[j][0]);
  const int dsum = wave_sum(d);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  if (j < kSub) t = phys_tail(st, j, qcap);
  const int tsum = wave_sum(t);
  return dsum == tsum;
}

#ifndef ABC_QMASK
#define ABC_QMASK 3
#endif
#ifndef ABC_BACKOFF
#define ABC_BACKOFF 16
#endif
#ifndef ABC_SLEEP
#define ABC_SLEEP 4
#endif
#ifndef ABC_STEAL_EVERY
#define ABC_STEAL_EVERY 1
#endif

// Removes one batch of up to 64 items and, last in first out, everything
// the batch removes while it fits the wave's local buffer (local
// continuation: no round trip through the sub-queue; only an overflowing
// buffer shares work), then appends the rest and counts the batch as
// processed.  The count follows the appends, so termination cannot be
// declared while any of this is in flight.
template <int KIND>
__device__ __forceinline__ void async_batch(const PeelArgs &a, int32_t item, int nitems,
                                            LocalQueue &lq, int32_t *consumed,
                                            int64_t &entries, int32_t level) {
  peel_batch<KIND, true>(a, item, level, lq, entries);
  while (lq.count > 0) {
    const int take = min(lq.count, kWave);
    __builtin_amdgcn_wave_barrier();
    const int32_t xi = lane_id() < take ? lq.buf[lq.count - take + lane_id()] : -1;
    __builtin_amdgcn_wave_barrier();
    lq.count -= take;
    peel_batch<KIND, true>(a, xi, level, lq, entries);
  }
  lq.flush();
  __builtin_amdgcn_s_waitcnt(0);
  if (lane_id() == 0) atomicAdd(consumed, nitems);
}

// Claims up to 64 appended, unclaimed slots of sub-queue v (none past its
// tail); returns the count claimed, base in *base.  Wave-uniform.
__device__ __forceinline__ int steal_claim(PeelState *st, int v, int max_take, int64_t qcap,
                                           int *base) {
  int b = 0, c = 0;
  if (lane_id() == 0) {
    const int h = ld_agent(&st->head[v][0]);
    const int t = phys_tail(st, v, qcap);
    if (h < t) {
      const int want = min(t - h, max_take);
      if (atomicCAS(&st->head[v][0], h, h + want) == h) {
        b = h;
        c = want;
      }
    }
  }
  *base = __shfl(b, 0, kWave);
  return __shfl(c, 0, kWave);
}

template <int KIND>
__global__ __launch_bounds__(kPeelBlock) void peel_async_kernel(PeelArgs a) {
  __shared__ int32_t s_lq[kPeelWaves][kLocalQueue];
  __shared__ int64_t s_acc;
  __shared__ int s_cnt[kPeelWaves + 2];
  __shared__ int s_stop;
  // rank order after an aborted query: the queue may hold stale items
  if (a.rs_fail != nullptr && ld_agent(a.rs_fail) != 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st_agent(&a.st->abort_flag, 1);
      report_abort(a);
    }
    return;
  }
  if (threadIdx.x == 0) s_stop = 0;
  __syncthreads();
  LocalQueue lq = make_lq(s_lq[wave_in_block()], kLocalQueue, a);
  const int waves = blockDim.x / kWave;
  const int gw = blockIdx.x * waves + wave_in_block();
  const int nw = gridDim.x * waves;
  int64_t fixed = 0;  // split rows the start phase queued
  if (a.start_expect > 0) {
    // start phase: after a pull round, the split rows below their threshold
    // (their pieces' counts are complete at the kernel boundary)
    if (a.fix_bits != nullptr && ld_agent(&a.st->pulled) != 0) {
      for (int64_t b = (int64_t)gw * kWave; b < a.nfix; b += (int64_t)nw * kWave) {
        const int64_t i = b + lane_id();
        bool push = false;
        int32_t x = -1;
        if (i < a.nfix) x = a.fix_rows[i];
        if (x >= 0 && ((a.fix_bits[x >> 5] >> (x & 31)) & 1u))
          push = a.deg[x] < (x < a.nU ? a.thrU : a.thrL);
        fixed += push ? 1 : 0;
        lq.push(push, x);
      }
    }
    block_flush(lq, s_cnt);
    // the appended items (agent-scope stores) are complete before the start
    // count, so a termination test that sees the count sees them
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(&a.st->started[blockIdx.x % kGroups][0], 1);
  }
  const int j = blockIdx.x % kSub;
  int32_t *head = &a.st->head[j][0];
  int32_t *consumed = &a.st->consumed[j][0];
  // core decomposition: the level set by the preceding scan (nothing to do
  // once every vertex has its core number)
  if (KIND == kKCore && ld_agent(&a.st->done) != 0) return;
  const int32_t level = KIND == kKCore ? ld_agent(&a.st->k) : 0;
  int64_t entries = 0;
  uint32_t idle = 0, victim = 0;
  bool finished = false;
  const int claim = a.claim;
  while (!finished) {
    int base = 0;
    if (lane_id() == 0) base = atomicAdd(head, claim);
    base = __shfl(base, 0, kWave);
    const int64_t slot = (int64_t)base + lane_id();
    // slots past the capacity are never written and never read: such a lane
    // stays pending, so its wave ends through the termination test
    bool pending = lane_id() < claim;
    while (__ballot(pending)) {
      int32_t item = kEmpty;
      if (pending && slot < a.qcap) item = ld_agent(&lq.q[slot]);
      const bool ready = pending && item != kEmpty;
      // rank order: a slot is claimed once and read once, so it returns to
      // empty as soon as its item is taken (the next query finds it so)
      if (a.rs_next_st != nullptr && ready) lq.q[slot] = kEmpty;
      const uint64_t rmask = __ballot(ready);
      if (rmask) {
        async_batch<KIND>(a, ready && item != kSkipItem ? item : -1, (int)__popcll(rmask), lq,
                          consumed, entries, level);
        pending = pending && !ready;
        idle = 0;
        continue;
      }
      // nothing in the own slots: wave 0 steals from another sub-queue (one
      // victim per poll, in rotation; one wave per workgroup keeps the
      // polls of the shared cursors few)
      victim = victim % (kSub - 1) + 1;
      int sbase = 0;
      const int taken = (wave_in_block() == 0 && (idle % ABC_STEAL_EVERY) == 0)
                            ? steal_claim(a.st, (j + (int)victim) % kSub, claim, a.qcap, &sbase)
                            : 0;
      if (taken > 0) {
        const int32_t *vq = a.queue + (int64_t)((j + (int)victim) % kSub) * a.qcap;
        // the slots are reserved by appenders that are running: wait for
        // their stores (bounded like every other wait)
        int32_t sitem = -1;
        if (lane_id() < taken) {
          uint32_t spin = 0;
          do {
            sitem = ld_agent(&vq[sbase + lane_id()]);
          } while (sitem == kEmpty && ++spin < a.spin_limit);
          if (sitem == kEmpty) {
            st_agent(&a.st->abort_flag, 1);
            sitem = -1;
          } else if (a.rs_next_st != nullptr) {
            const_cast<int32_t *>(vq)[sbase + lane_id()] = kEmpty;
          }
          if (sitem == kSkipItem) sitem = -1;
        }
        async_batch<KIND>(a, sitem, taken, lq, consumed, entries, level);
        idle = 0;
        continue;
      }
      // waiting: poll with growing back-off and give up after the spin
      // limit (an abort, reported).  Only wave 0 of a workgroup polls the
      // shared words (same-address reads serialise like atomics): its
      // group's copy of `fin` every poll, and every fourth poll the
      // termination test, whose first success sets every copy.  It passes
      // the verdict to the other waves through LDS.
      ++idle;
      int stop = 0;
      if (wave_in_block() == 0) {
        if (lane_id() == 0) stop = ld_agent(&a.st->fin[blockIdx.x % kGroups][0]);
        stop = __shfl(stop, 0, kWave);
        if (!stop && (idle & ABC_QMASK) == 0) {
          if (quiescent(a.st, a.start_expect, a.qcap)) {
            if (lane_id() < kGroups) st_agent(&a.st->fin[lane_id()][0], 1);
            stop = 1;
          } else {
            if (lane_id() == 0) stop = ld_agent(&a.st->abort_flag);
            stop = __shfl(stop, 0, kWave);
          }
        }
        if (stop && lane_id() == 0) __hip_atomic_store(&s_stop, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      } else {
        stop = __hip_atomic_load(&s_stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      if (stop) {
        finished = true;
        break;
      }
      if (idle > a.spin_limit) {
        if (lane_id() == 0) {
          st_agent(&a.st->abort_flag, 1);
          __hip_atomic_store(&s_stop, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        finished = true;
        break;
      }
      for (uint32_t k = 0; k < min(idle, (uint32_t)ABC_BACKOFF); ++k) __builtin_amdgcn_s_sleep(ABC_SLEEP);
    }
  }
  add_part(a.part, kPartEntries, entries, &s_acc);
  add_part(a.part, kPartF1, fixed, &s_acc);
  if (KIND == kKCore && threadIdx.x < kSub) {
    // everything appended so far is processed: the next level's scan starts
    // its range here (every workgroup writes the same final cursors)
    st_agent(&a.st->hi[threadIdx.x], phys_tail(a.st, threadIdx.x, a.qcap));
  }
  const bool aborted = ld_agent(&a.st->abort_flag) != 0;
  if (aborted && threadIdx.x == 0) report_abort(a);
  if (a.rs_next_st != nullptr && aborted) {
    // ended by an abort: other workgroups may still use the queue
    if (threadIdx.x == 0) st_agent(a.rs_fail, 1);
  } else if (a.rs_next_st != nullptr) {
    // rank order: the next query's workspace.  Termination means every
    // queued slot was taken, and each was returned to empty when it was; the
    // other state and partial sums (not this launch's) are zeroed
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < (int64_t)kMaxBlocks * kPartFields; i += stride)
      a.rs_next_part[i] = 0;
    int32_t *words = reinterpret_cast<int32_t *>(a.rs_next_st);
    for (int64_t i = tid; i < (int64_t)(sizeof(PeelState) / 4); i += stride) words[i] = 0;
  }
  if (a.pack_bits != nullptr && a.pack_vtx == nullptr && !aborted) {
    // the result (Algorithm 1's V(G)): termination means every decrement
    // is done; degrees are read at device scope (they changed by atomics)
    // kPackSpan consecutive vertices per lane pass, all loads issued before
    // the first test, so a wave has that many reads in flight
    const int64_t n = a.n;
    constexpr int kPackSpan = 8;
    for (int64_t b = (int64_t)gw * kWave * kPackSpan; b < n;
         b += (int64_t)nw * kWave * kPackSpan) {
      int32_t dv[kPackSpan];
#pragma unroll
      for (int u = 0; u < kPackSpan; ++u) {
        const int64_t x = b + u * kWave + lane_id();
        dv[u] = x < n ? ld_agent(&a.deg[x]) : 0;
      }
#pragma unroll
      for (int u = 0; u < kPackSpan; ++u) {
        const int64_t b64 = b + u * kWave;
        const int64_t x = b64 + lane_id();
        const uint64_t m = __ballot(x < n && dv[u] >= (x < a.nU ? a.thrU : a.thrL));
        if (lane_id() < 2 && b64 + 32 * lane_id() < n)
          a.pack_bits[(b64 >> 5) + lane_id()] = (uint32_t)(m >> (32 * lane_id()));
      }
    }
  }
}

hipError_t launch_peel_async_args(Graph &g, PeelKind kind, const PeelArgs &a, int grid,
                                  hipStream_t s) {
  (void)g;
  grid = std::max(1, grid);
  if (kind == kGCC)
    peel_async_kernel<kGCC><<<grid, kPeelBlock, 0, s>>>(a);
  else
    peel_async_kernel<kGCCPlus><<<grid, kPeelBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_peel_async_fused(Graph &g, PeelKind kind, int32_t thrU, int32_t thrL,
                                   const uint32_t *fix_bits, uint32_t *pack_bits,
                                   hipStream_t s, bool split_done) {
  PeelArgs a = make_args(g, thrU, thrL);
  const int grid = async_peel_grid(g);
  if (split_done) {
    a.alive0 = fix_bits;  // the filter only: the pull round queued its split rows
  } else if (fix_bits != nullptr) {
    a.fix_rows = g.heavy_rows;
    a.fix_bits = fix_bits;
    a.nfix = g.nheavy;
    a.start_expect = grid;
    a.alive0 = fix_bits;
  }
  a.pack_bits = pack_bits;
  return launch_peel_async_args(g, kind, a, grid, s);
}

hipError_t launch_peel_async(Graph &g, PeelKind kind, int32_t thrU, int32_t thrL,
                             hipStream_t s) {
  PeelArgs a = make_args(g, thrU, thrL);
  return launch_peel_async_args(g, kind, a, async_peel_grid(g), s);
}

// ------------------------------------------------------ pull first round --
// The first peel round in pull form.  After the scan, every vertex that
// survived it counts its neighbours that survived it (bitmap lookups), which
// is exactly its degree after the removal of the scan frontier; those now
// below their threshold form the second frontier.  The frontier of the scan
// itself is then never walked.  Upper rows look up lower vertices and lower
// rows upper vertices, so each phase stages one layer's bitmap in LDS when
// it fits.  Rows longer than kPiece are counted piece by piece (balanced
// batches); a row's pieces add their counts to its degree atomically, the
// first piece also removing the degree the scan wrote, and a separate fixup
// kernel queues the split rows that end below their threshold.  Chosen on
// the device from the scan's frontier degree sum.

// Rows of at most kLightRow entries are counted thread per row (up to
// kLightRow independent loads in flight per lane); longer rows of at most
// kPiece entries and the pieces of split rows are counted by 16-lane groups,
// each group four chunks of up to 64 entries at a time (16 loads per lane in
// flight, each load 64 contiguous bytes per group).
constexpr int kLightRow = 16;

struct ChunkDesc {
  int64_t s;      // first entry
  int32_t d;      // entries
  int32_t owner;  // lane that receives the count
};

struct PullShared {
  int32_t lq[kPullWaves][kPullLocalQueue];
  int32_t cnt[kPullWaves][kWave];
  ChunkDesc desc[kPullWaves][kWave];
  int s_cnt[kPullWaves + 2];
  int decide;
  int next_row, next_piece;  // the workgroup's next unclaimed row / piece
  int32_t k_alive[2];        // rank mode: survivors of the upper / lower layer
  int64_t acc;
};

// Bit of neighbour v (0 for v < 0: padding or a deleted entry), branch-free
// so that a group of lookups issues together.
// Entry tests in two steps, so that a batch issues all its word loads
// before it uses any (one wait for the batch instead of one per entry):
// word(v) loads what the test needs, pass(word, v) decides.  Deleted and
// padding entries (negative) never pass.
struct BitTest {  // v's bit in a bitmap of words from base_word (global)
  const uint32_t *w;
  int64_t base_word;
  uint32_t zero;  // (unused)
  __device__ __forceinline__ uint32_t word(int32_t v) const {
    return w[v >= 0 ? (int64_t)(v >> 5) - base_word : 0];
  }
  __device__ __forceinline__ uint32_t pass(uint32_t wd, int32_t v) const {
    return v >= 0 ? (wd >> (v & 31)) & 1u : 0u;
  }
};
// The same for a bitmap staged in LDS with a zero word at index `zero`
// (just past the staged words): a negative entry's word index, computed
// signed, is negative and clamps (as unsigned) to the zero word, so neither
// the index nor the result needs a test of the sign; ubfe takes the bit
// position from the low five bits of v.
struct BitTestLds {
  const uint32_t *w;
  int64_t base_word;
  uint32_t zero;
  __device__ __forceinline__ uint32_t word(int32_t v) const {
    const uint32_t idx = (uint32_t)((v >> 5) - (int32_t)base_word);
    return w[min(idx, zero)];
  }
  __device__ __forceinline__ uint32_t pass(uint32_t wd, int32_t v) const {
    return __builtin_amdgcn_ubfe(wd, (uint32_t)v, 1u);
  }
};
struct BelowTest {  // v below a bound (the rank copy's surviving prefix)
  int32_t kb;
  __device__ __forceinline__ uint32_t word(int32_t) const { return 0; }
  __device__ __forceinline__ uint32_t pass(uint32_t, int32_t v) const {
    return (uint32_t)(v >= 0 && v < kb);
  }
};

// Row entries that pass `test` in [s, s+d) of `src` (the adjacency with the
// bitmap test, deleted entries negative and never counting, or the rank
// copy with a rank bound), d <= kLightRow.
template <class Test>
__device__ __forceinline__ int count_row_thread(const PeelArgs &a, const int32_t *src, int64_t s,
                                                int d, Test test) {
  int32_t w[kLightRow];
#pragma unroll
  for (int j = 0; j < kLightRow; ++j) w[j] = j < d ? src[s + j] : -1;
  if (a.del_ver != nullptr) {
#pragma unroll
    for (int j = 0; j < kLightRow; ++j) w[j] = view_col(a, j < d, s + j, w[j]);
  }
  uint32_t wd[kLightRow];
#pragma unroll
  for (int j = 0; j < kLightRow; ++j) wd[j] = test.word(w[j]);
  int c = 0;
#pragma unroll
  for (int j = 0; j < kLightRow; ++j) c += (int)test.pass(wd[j], w[j]);
  return c;
}

// Counts, for every lane with pred, the entries of its chunk [s, s+d) of
// `src` (d <= 64) that pass `test`; the count lands in cnt[lane].  Whole wave.
template <class Test>
__device__ __forceinline__ void count_chunks(const PeelArgs &a, const int32_t *src, bool pred,
                                             int64_t s, int d, ChunkDesc *desc, int32_t *cnt,
                                             Test test) {
  const uint64_t m = __ballot(pred);
  const int total = __popcll(m);
  if (total == 0) return;
  if (pred) {
    ChunkDesc &cd = desc[__popcll(m & lanemask_lt())];
    cd.s = s;
    cd.d = d;
    cd.owner = lane_id();
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const int grp = lane_id() >> 4, l = lane_id() & 15;
  for (int base = 0; base < total; base += 16) {
    int64_t cs[4];
    int cdn[4], own[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = base + grp * 4 + r;
      const bool ok = i < total;
      cs[r] = ok ? desc[i].s : 0;
      cdn[r] = ok ? desc[i].d : 0;
      own[r] = ok ? desc[i].owner : -1;
    }
    int32_t w[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = l + 16 * j;
        w[r][j] = k < cdn[r] ? src[cs[r] + k] : -1;
      }
    if (a.del_ver != nullptr) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          w[r][j] = view_col(a, l + 16 * j < cdn[r], cs[r] + l + 16 * j, w[r][j]);
    }
    uint32_t wd[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int j = 0; j < 4; ++j) wd[r][j] = test.word(w[r][j]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int c = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) c += (int)test.pass(wd[r][j], w[r][j]);
      c += __shfl_xor(c, 8, 16);
      c += __shfl_xor(c, 4, 16);
      c += __shfl_xor(c, 2, 16);
      c += __shfl_xor(c, 1, 16);
      if (l == 0 && own[r] >= 0) cnt[own[r]] = c;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Inserted neighbours of x with their bit set (versioned view as in the
// peel: pairs from the limit on are skipped, pairs deleted after the
// query's version still count).
__device__ __forceinline__ int delta_alive(const PeelArgs &a, const uint32_t *gbits, int32_t x,
                                           int64_t &entries) {
  int extra = 0;
  for (int e = a.ins_head[x]; e >= 0;) {
    int32_t w, next;
    if (a.del_ver == nullptr) {
      w = a.ins_other[e];
      next = a.ins_next[e];
    } else if ((e >> 1) >= a.pair_limit) {
      w = -1;
      next = ld_agent(&a.ins_next[e]);
    } else {
      w = a.ins_other[e];
      if (w < 0 && ld_agent(&a.pair_del_ver[e >> 1]) > a.ver) w = ~w;
      next = a.ins_next[e];
    }
    if (w >= 0) {
      ++entries;
      extra += (gbits[w >> 5] >> (w & 31)) & 1u;
    }
    e = next;
  }
  return extra;
}

// kLds: the neighbour layer's bitmap is staged in LDS (a compile-time
// choice, so that lookups are LDS reads and not generic-address loads).
// kRank: the rank form (rows of the degree-rank copy, rcols non-null),
// compiled apart from the vertex form (each form has its own tests).
template <bool kLds, bool kRank>
__global__ __launch_bounds__(kPullBlock) void pull_round_kernel(
    PeelArgs a, const uint32_t *__restrict__ gbits, const int32_t *__restrict__ deg0, int64_t n,
    int scan_blocks, int mode, int use_lds, int64_t total_entries, int64_t npieces,
    int64_t npieces_upper, const int32_t *__restrict__ corr_x,
    const int32_t *__restrict__ corr_d, int ncorr, int advance,
    const int32_t *__restrict__ bounds, int queue_f0, const uint32_t *__restrict__ rowbits,
    int rest_part, const int32_t *__restrict__ written_snap, const int32_t *__restrict__ rcols,
    const int32_t *__restrict__ rank_vtx, const int64_t *__restrict__ roff, int64_t nheavy,
    int64_t nheavy_upper, int rspace, int64_t rk_u, int64_t rk_l, uint32_t *__restrict__ rs_bits) {
  static_assert(!(kLds && kRank), "the rank form looks nothing up in a bitmap");
  extern __shared__ __align__(16) uint32_t s_bits[];
  __shared__ PullShared sh;
  if (rspace && a.rs_fail != nullptr && ld_agent(a.rs_fail) != 0) {
    // rank order after an aborted query: the queue may hold stale items
    if (blockIdx.x == 0 && threadIdx.x == 0) st_agent(&a.st->abort_flag, 1);
    return;
  }
  // Each phase walks one layer's rows; its bitmap of the other layer is
  // staged in LDS (kLds) from the 16-byte boundary at or below its first
  // word.  Phase 0
  // (upper rows) is staged while wave 0 makes the push/pull decision.
  auto stage_base = [&](int phase) -> int64_t { return ((phase == 0 ? a.nU : 0) >> 5) & ~3LL; };
  auto stage = [&](int phase) {
    const int64_t nb_lo = phase == 0 ? a.nU : 0, nb_hi = phase == 0 ? n : a.nU;
    const int64_t w1 = nb_hi > nb_lo ? ((nb_hi - 1) >> 5) : (nb_lo >> 5);
    const int64_t a0 = stage_base(phase);
    const int64_t n4 = (w1 + 1 - a0) / 4;  // whole 16-byte groups up to w1
    // direct global-to-LDS loads (lane l fills bytes [16 l, 16 l + 16) of
    // its wave's 1 KiB chunk), all in flight at once and holding no
    // registers; every workgroup reads the same words, so each starts at its
    // own chunk to spread the grid's requests over the cache channels
    const int64_t nchunks = (n4 + kWave - 1) / kWave;
    const int64_t rot = nchunks > 0 ? (int64_t)blockIdx.x * nchunks / gridDim.x : 0;
    for (int64_t c = wave_in_block(); c < nchunks; c += blockDim.x / kWave) {
      const int64_t cc = c + rot < nchunks ? c + rot : c + rot - nchunks;
      const int64_t i = cc * kWave + lane_id();
      if (i < n4)
        __builtin_amdgcn_global_load_lds(
            (const __attribute__((address_space(1))) void *)(gbits + a0 + 4 * i),
            (__attribute__((address_space(3))) void *)(s_bits + 4 * cc * kWave), 16, 0, 0);
    }
    for (int64_t i = a0 + 4 * n4 + threadIdx.x; i <= w1; i += blockDim.x) s_bits[i - a0] = gbits[i];
    // the zero word just past the staged ones (the dynamic size holds four
    // words more than a layer's bitmap, and a0 lies at most three below it)
    if (threadIdx.x == 0) s_bits[w1 + 1 - a0] = 0;
    __builtin_amdgcn_s_waitcnt(0);  // the loads have landed in LDS (the caller then syncs)
  };
  auto zero_word = [&](int phase) -> uint32_t {
    const int64_t nb_lo = phase == 0 ? a.nU : 0, nb_hi = phase == 0 ? n : a.nU;
    const int64_t w1 = nb_hi > nb_lo ? ((nb_hi - 1) >> 5) : (nb_lo >> 5);
    return (uint32_t)(w1 + 1 - stage_base(phase));
  };
  if (threadIdx.x == 0) {
    sh.next_row = 0;
    sh.next_piece = 0;
  }
  if (wave_in_block() == 0) {
    // the scan's frontier degree sum, from its per-workgroup slots
    const int64_t f0deg = wave_sum_strided(a.part + kPartF0Deg, scan_blocks, kPartFields);
    const int64_t rest = rest_part ? wave_sum_strided(a.part + kPartRest, scan_blocks, kPartFields)
                                   : total_entries - f0deg;
    // pull pays one streaming read per surviving entry instead of one atomic
    // per frontier entry: worth it when the frontier carries a sizeable share
    // (a random 4-byte atomic moves about 100 bytes of lines to and from
    // HBM; a pulled entry about 18 with its bitmap lookup in L2 or the
    // Infinity Cache, hence the factor 6 when the bitmap is not in LDS, and
    // 16 when it is); with the rank copy a pull round reads about a line per
    // surviving row (a few per split row): worth it once the frontier's
    // atomics are about half as many as the survivors
    int64_t ku = 0, kl = 0;
    if (kRank) {
      // (known in advance for a query in rank order)
      ku = rk_u >= 0 ? rk_u : wave_sum_strided(a.part + kPartAliveU, scan_blocks, kPartFields);
      kl = rk_l >= 0 ? rk_l : wave_sum_strided(a.part + kPartAliveL, scan_blocks, kPartFields);
      if (lane_id() == 0) {
        sh.k_alive[0] = (int32_t)ku;
        sh.k_alive[1] = (int32_t)kl;
      }
    }
    const bool pull =
        mode == 2 ||
        (mode == 0 && f0deg > 0 &&
         (kRank ? f0deg * 2 >= ku + kl
                           : (use_lds ? f0deg * 16 >= rest : f0deg * 6 >= rest)));
    if (lane_id() == 0) sh.decide = pull ? 1 : 0;
  }
  if (kLds) stage(0);
  __syncthreads();
  if (!sh.decide) {
    if (queue_f0) {
      // the first round is pushed and the scan did not queue its frontier:
      // queue every vertex of the scan's frontier (bit clear), 32 per lane;
      // each wave appends its 64 words to a sub-queue of its own choice, so
      // that the sub-queues receive even shares
      const int64_t nwords = (n + 31) >> 5;
      const int waves = blockDim.x / kWave;
      for (int64_t w0 = ((int64_t)blockIdx.x * waves + wave_in_block()) * kWave; w0 < nwords;
           w0 += (int64_t)gridDim.x * waves * kWave) {
        const int64_t w = w0 + lane_id();
        uint32_t dead = 0;
        if (w < nwords) {
          dead = a.f0_bits != nullptr ? a.f0_bits[w] : ~gbits[w];
          const int64_t valid = n - (w << 5);
          if (valid < 32) dead &= (1u << valid) - 1u;
        }
        const int cnt = __popc(dead);
        const int incl = wave_incl_scan(cnt);
        const int sub = (int)((w0 / kWave) % kSub);
        int2 r = make_int2(0, 0);
        if (lane_id() == kWave - 1 && incl > 0)
          r = reserve_slots(a.st, a.queue, a.qcap, append_pref(a, sub), incl, a.abort_host);
        const int rs = __shfl(r.x, kWave - 1, kWave);
        int pos = __shfl(r.y, kWave - 1, kWave) + incl - cnt;
        int32_t *q = a.queue + (int64_t)rs * a.qcap;
        while (rs >= 0 && dead != 0) {
          const int32_t x = (int32_t)((w << 5) + (__ffs(dead) - 1));
          q[pos++] = x;
          ABC_COUNT_ENQUEUE(a.dbg_enqueue, x);
          dead &= dead - 1;
        }
      }
    }
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st_agent(&a.st->pulled, 1);
  LocalQueue lq = make_lq(sh.lq[wave_in_block()], kPullLocalQueue, a);
  int32_t *cnt = sh.cnt[wave_in_block()];
  ChunkDesc *desc = sh.desc[wave_in_block()];
  int64_t entries = 0, f1 = 0;
  for (int phase = 0; phase < 2; ++phase) {
    // phase 0: upper rows (neighbours are lower ids), phase 1: lower rows
    const int64_t lo = phase == 0 ? 0 : a.nU, hi = phase == 0 ? a.nU : n;
    const int64_t plo = phase == 0 ? 0 : npieces_upper, phi = phase == 0 ? npieces_upper : npieces;
    if (phase == 1) {
      // every wave is done with phase 0 before its bitmap and counters go
      __syncthreads();
      if (threadIdx.x == 0) {
        sh.next_row = 0;
        sh.next_piece = 0;
      }
      if (kLds) stage(1);
      __syncthreads();
    }
    if (lo >= hi) continue;
    const uint32_t *lk = gbits;
    int64_t lk_base = 0;
    uint32_t lk_zero = 0;
    if (kLds) {
      lk = s_bits;
      lk_base = stage_base(phase);
      lk_zero = zero_word(phase);
    }
    using RowTest = typename std::conditional<kLds, BitTestLds, BitTest>::type;
    // This workgroup's rows (a range of equal weight, else an equal share)
    // and pieces; its waves claim 64 of them at a time through LDS.
    const int G = (int)gridDim.x, k = (int)blockIdx.x;
    const int64_t r0 = bounds != nullptr ? bounds[phase * (G + 1) + k] : lo + (hi - lo) * k / G;
    const int64_t r1 = bounds != nullptr ? bounds[phase * (G + 1) + k + 1]
                                         : lo + (hi - lo) * (k + 1) / G;
    const int64_t p0 = plo + (phi - plo) * k / G, p1 = plo + (phi - plo) * (k + 1) / G;
    if (kRank) {
      // Rank form: the surviving rows of this layer are its ranks below
      // kself, split rows (more than kPiece entries) first; a row's
      // surviving neighbours are its rank row's prefix below kb.  Chunks of
      // 64 ranks are dealt to the workgroups in turn (workgroup k takes
      // chunks k, k + G, ...), its waves claiming them through LDS.
      // (rank order, rspace: the rank rows are the rows, a row's degree is
      // written at its rank and a removed row is queued as its rank)
      const int64_t base = phase == 0 ? 0 : a.nU;
      const int64_t kself = sh.k_alive[phase];
      // neighbours are global ranks: an upper row's lie past nU
      const int32_t kb = sh.k_alive[phase ^ 1] + (phase == 0 ? a.nU : 0);
      const int64_t nh = phase == 0 ? nheavy_upper : nheavy - nheavy_upper;
      const int64_t hend = base + min(nh, kself), lend = base + kself;
      const BelowTest below{kb};
      for (;;) {
        int claim = 0;
        if (lane_id() == 0) claim = atomicAdd(&sh.next_row, 1);
        const int64_t b = hend + ((int64_t)k + (int64_t)__shfl(claim, 0, kWave) * G) * kWave;
        if (b >= lend) break;
        const int64_t r = b + lane_id();
        const bool alive = r < lend;
        int32_t x = -1;
        int64_t s = 0;
        int d = 0;
        if (alive) {
          x = rspace ? (int32_t)r : rank_vtx[r];
          s = roff[r];
          d = (int)(roff[r + 1] - s);
        }
        int c = 0;
        const bool grouped = alive && d > kLightRow;
        if (alive && d <= kLightRow) c = count_row_thread(a, rcols, s, d, below);
        count_chunks(a, rcols, grouped, s, d, desc, cnt, below);
        if (grouped) c = cnt[lane_id()];
        bool push = false;
        if (alive) {
          entries += d;
          a.deg[deg_slot(a, x)] = c;
          push = c < (x < a.nU ? a.thrU : a.thrL);
          f1 += push ? 1 : 0;
        }
        lq.push(push, x);
        __builtin_amdgcn_wave_barrier();
      }
      // split rows: a 16-lane group per row finds the end of the row's
      // prefix below kb, 16 probes per step (a 50,000-entry row takes three
      // steps and a final one), so the row is complete at once (no pieces,
      // no completion in the peel's start phase)
      const int grp = lane_id() >> 4, l = lane_id() & 15;
      for (;;) {
        int claim = 0;
        if (lane_id() == 0) claim = atomicAdd(&sh.next_piece, 1);
        const int64_t hb = base + ((int64_t)k + (int64_t)__shfl(claim, 0, kWave) * G) * 4;
        if (hb >= hend) break;
        const int64_t r = hb + grp;
        int32_t x = -1;
        int64_t s = 0;
        const bool alive = r < hend;
        int lo = 0, hi = 0;
        if (alive) {
          x = rspace ? (int32_t)r : rank_vtx[r];
          s = roff[r];
          hi = (int)(roff[r + 1] - s);
        }
        while (__ballot(hi - lo > 16)) {
          const bool act = hi - lo > 16;
          const int span = hi - lo;
          const int p = lo + (int)(((int64_t)span * l) / 16);
          const bool t = act && rcols[s + p] < kb;
          const int cc = __popcll((__ballot(t) >> (16 * grp)) & 0xFFFFull);
          if (act) {
            // the end lies in (p_{cc-1}, p_cc]
            const int pprev = lo + (int)(((int64_t)span * (cc - 1)) / 16);
            const int pcur = lo + (int)(((int64_t)span * cc) / 16);
            const int nlo = cc == 0 ? lo : pprev + 1;
            hi = cc == 16 ? hi : pcur;
            lo = nlo;
          }
        }
        const bool t = lo + l < hi && rcols[s + lo + l] < kb;
        const int cnt_row = lo + __popcll((__ballot(t) >> (16 * grp)) & 0xFFFFull);
        bool push = false;
        if (alive && l == 0) {
          a.deg[deg_slot(a, x)] = cnt_row;
          push = cnt_row < (x < a.nU ? a.thrU : a.thrL);
          f1 += push ? 1 : 0;
          entries += 64;
        }
        lq.push(push, x);
        __builtin_amdgcn_wave_barrier();
      }
      continue;
    }
    // rows of at most kPiece entries, 64 consecutive vertices per claim; the
    // offsets and survivor bits of the next claim are loaded before this one
    // is counted (one memory round trip per claim instead of two)
    auto claim_rows = [&]() -> int64_t {
      int claim = 0;
      if (lane_id() == 0) claim = atomicAdd(&sh.next_row, kWave);
      return r0 + __shfl(claim, 0, kWave);
    };
    int64_t s_next = 0, e_next = 0;
    uint32_t w_next = 0;
    auto fetch_rows = [&](int64_t bb) {
      const int64_t xi = bb + lane_id();
      if (xi < r1) {
        w_next = rowbits[xi >> 5];
        s_next = a.off[xi];
        e_next = a.off[xi + 1];
      }
    };
    int64_t b = claim_rows();
    fetch_rows(b);
    while (b < r1) {
      const int64_t xi = b + lane_id();
      const int32_t x = xi < r1 ? (int32_t)xi : -1;
      const int64_t s = s_next;
      const int d = (int)(e_next - s_next);
      // split rows are counted by their pieces
      const bool alive = x >= 0 && ((w_next >> (xi & 31)) & 1u) && d <= kPiece;
      const int64_t bn = claim_rows();
      fetch_rows(bn);
      b = bn;
      int c = 0;
      const bool grouped = alive && d > kLightRow;
      const RowTest bit{lk, lk_base, lk_zero};
      if (alive && d <= kLightRow) c = count_row_thread(a, a.cols, s, d, bit);
      count_chunks(a, a.cols, grouped, s, d, desc, cnt, bit);
      if (grouped) c = cnt[lane_id()];
      bool push = false;
      if (alive) {
        entries += d;
        if (a.ins_head != nullptr) c += delta_alive(a, gbits, x, entries);
        a.deg[x] = c;
        push = c < (x < a.nU ? a.thrU : a.thrL);
        f1 += push ? 1 : 0;
      }
      lq.push(push, x);
      __builtin_amdgcn_wave_barrier();
    }
    // pieces of longer rows: per-piece counts summed per row inside the
    // wave (a row's pieces are consecutive), one atomic per row and wave
    for (;;) {
      int claim = 0;
      if (lane_id() == 0) claim = atomicAdd(&sh.next_piece, kWave);
      const int64_t b = p0 + __shfl(claim, 0, kWave);
      if (b >= p1) break;
      const int64_t pi = b + lane_id();
      int32_t row = -1;
      int64_t s = 0;
      int d = 0;
      bool first = false, alive = false;
      if (pi < p1) {
        row = a.piece_row[pi];
        s = a.piece_start[pi];
        const int64_t rs = a.off[row], re = a.off[row + 1];
        alive = (rowbits[row >> 5] >> (row & 31)) & 1u;
        d = (int)(min(s + kPiece, re) - s);
        first = s == rs;
      }
      count_chunks(a, a.cols, alive, s, d, desc, cnt, RowTest{lk, lk_base, lk_zero});
      int c = 0;
      if (alive) {
        entries += d;
        c = cnt[lane_id()];
        if (first) {
          if (a.ins_head != nullptr) c += delta_alive(a, gbits, row, entries);
          // the scan wrote deg[row] = deg0[row] (plus the view's correction),
          // or a nested scan left the degree recorded at the first piece
          int32_t written = written_snap != nullptr ? written_snap[pi] : deg0[row];
          for (int i = 0; i < ncorr; ++i)
            if (corr_x[i] == row) written += corr_d[i];
          c -= written;
        }
      }
      // segmented sum over lanes of equal rows (dead rows contribute 0)
      const int32_t key = alive ? row : -1;
      const int incl = wave_incl_scan(c);
      const int32_t prev_key = __shfl_up(key, 1, kWave);
      const int32_t next_key = __shfl_down(key, 1, kWave);
      const bool head = lane_id() == 0 || prev_key != key;
      const bool tail = lane_id() == kWave - 1 || next_key != key;
      const uint64_t heads = __ballot(head);
      const uint64_t le = lane_id() == kWave - 1 ? ~0ull : ((1ull << (lane_id() + 1)) - 1);
      const int start = 63 - __builtin_clzll(heads & le);
      const int before = __shfl(incl, start > 0 ? start - 1 : 0, kWave);
      const int total = incl - (start > 0 ? before : 0);
      if (tail && key >= 0 && total != 0) atomicAdd(&a.deg[key], total);
      __builtin_amdgcn_wave_barrier();
    }
  }
  block_flush(lq, sh.s_cnt);
  add_part(a.part, kPartEntries, entries, &sh.acc);
  add_part(a.part, kPartF1, f1, &sh.acc);
  if (rs_bits != nullptr) {
    // rank order: the scan's survivors (degree >= threshold) into the result
    // bitmask, from which the peel clears the vertices it removes.  Each lane
    // tests 4 consecutive vertices; 8 lanes assemble one 32-bit word.
    const int64_t step = (int64_t)gridDim.x * blockDim.x * 4;
    for (int64_t b = ((int64_t)blockIdx.x * blockDim.x + wave_in_block() * kWave) * 4; b < n;
         b += step) {
      const int64_t x0 = b + 4 * lane_id();
      int32_t d[4] = {0, 0, 0, 0};
      if (x0 + 3 < n) {
        const int4 v = *reinterpret_cast<const int4 *>(deg0 + x0);
        d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
      } else {
        for (int k2 = 0; k2 < 4; ++k2)
          if (x0 + k2 < n) d[k2] = deg0[x0 + k2];
      }
      uint32_t alive = 0;
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) {
        const int64_t x = x0 + k2;
        alive |= (uint32_t)(x < n && d[k2] >= (x < a.nU ? a.thrU : a.thrL)) << k2;
      }
      uint32_t w = alive << (4 * (lane_id() & 7));
      w |= __shfl_xor(w, 1, kWave);
      w |= __shfl_xor(w, 2, kWave);
      w |= __shfl_xor(w, 4, kWave);
      if ((lane_id() & 7) == 0 && x0 < n) rs_bits[x0 >> 5] = w;
    }
  }
  if (advance && last_block_done<false>(a.st)) {
    advance_round_wave(a.st, a.qcap);
    if (lane_id() == 0) atomicAdd((unsigned long long *)&a.st->launches, 1ull);
  }
}

// After a pull round: queues the split rows that ended below their threshold
// and starts the next round.  Does nothing when the first round was pushed.
__global__ __launch_bounds__(kPeelBlock) void pull_fixup_kernel(
    PeelArgs a, const uint32_t *__restrict__ gbits, const int32_t *__restrict__ heavy_rows,
    int64_t nheavy) {
  __shared__ int32_t s_lq[kPeelWaves][kLocalQueue];
  __shared__ int s_cnt[kPeelWaves + 2];
  if (ld_agent(&a.st->pulled) == 0) return;
  LocalQueue lq = make_lq(s_lq[wave_in_block()], kLocalQueue, a);
  const int waves = blockDim.x / kWave;
  const int gw = blockIdx.x * waves + wave_in_block();
  const int nw = gridDim.x * waves;
  for (int64_t b = (int64_t)gw * kWave; b < nheavy; b += (int64_t)nw * kWave) {
    const int64_t i = b + lane_id();
    bool push = false;
    int32_t x = -1;
    if (i < nheavy) x = heavy_rows[i];
    if (x >= 0 && ((gbits[x >> 5] >> (x & 31)) & 1u))
      push = a.deg[x] < (x < a.nU ? a.thrU : a.thrL);
    push_removed(a, lq, push, x);
  }
  block_flush(lq, s_cnt);
  if (last_block_done<false>(a.st)) {
    advance_round_wave(a.st, a.qcap);
    if (lane_id() == 0) atomicAdd((unsigned long long *)&a.st->launches, 1ull);
  }
}

// Allows the pull kernel to stage a layer bitmap as large as the device's
// per-workgroup LDS permits.
hipError_t prepare_pull_kernel(Graph &g) {
  // (256 bytes left for the alignment of the dynamic part)
  const int dyn = (int)std::max<int64_t>(
      0, (int64_t)g.lds_per_block - (int64_t)sizeof(PullShared) - 256);
  return hipFuncSetAttribute(reinterpret_cast<const void *>(&pull_round_kernel<true, false>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
}

bool pull_uses_lds(const Graph &g) {
  const int64_t words_upper = g.nU > 0 ? ((int64_t)g.nU - 1) / 32 + 1 : 0;
  const int64_t words_lower = g.nL > 0 ? ((g.n - 1) >> 5) - (g.nU >> 5) + 1 : 0;
  const int64_t need = 4 * (std::max(words_upper, words_lower) + 4);
  return (size_t)need + sizeof(PullShared) + 1024 <= g.lds_per_block;
}

hipError_t launch_pull_round_args(Graph &g, const PeelArgs &a, const uint32_t *bits,
                                  const int32_t *corr_x, const int32_t *corr_d, int ncorr,
                                  bool advance, hipStream_t s, bool queue_f0,
                                  const uint32_t *rowbits, bool force, bool rest_part,
                                  bool rank) {
  if (g.pull_mode == 1 && !force) return hipSuccess;
  const int mode = force ? 2 : g.pull_mode;
  if (rowbits == nullptr) rowbits = bits;
  rank = rank && g.rcols != nullptr;
  const int64_t words_upper = g.nU > 0 ? ((int64_t)g.nU - 1) / 32 + 1 : 0;
  const int64_t words_lower = g.nL > 0 ? ((g.n - 1) >> 5) - (g.nU >> 5) + 1 : 0;
  // the rank form looks nothing up: no bitmap in LDS
  const bool use_lds = !rank && pull_uses_lds(g);
  const size_t dyn = use_lds ? (size_t)(4 * (std::max(words_upper, words_lower) + 4)) : 0;
  const int64_t total_entries = 2 * g.m;
  const int grid = g.cu_count;
  const int32_t *bounds = g.pull_bounds_grid == grid ? g.pull_bounds : nullptr;
  const int32_t *rcols = rank ? g.rcols : nullptr;
  if (use_lds)
    pull_round_kernel<true, false><<<grid, kPullBlock, dyn, s>>>(
        a, bits, g.deg0, g.n, scan_grid(g), mode, 1, total_entries, g.npieces,
        g.npieces_upper, corr_x, corr_d, ncorr, advance ? 1 : 0, bounds, queue_f0 ? 1 : 0,
        rowbits, rest_part ? 1 : 0, rest_part ? g.split_written : nullptr, nullptr, g.rank_vtx,
        g.roff, g.nheavy, g.nheavy_upper, 0, -1, -1, nullptr);
  else if (rcols != nullptr)
    pull_round_kernel<false, true><<<grid, kPullBlock, dyn, s>>>(
        a, bits, g.deg0, g.n, scan_grid(g), mode, 0, total_entries, g.npieces,
        g.npieces_upper, corr_x, corr_d, ncorr, advance ? 1 : 0, bounds, queue_f0 ? 1 : 0,
        rowbits, rest_part ? 1 : 0, rest_part ? g.split_written : nullptr, rcols, g.rank_vtx,
        g.roff, g.nheavy, g.nheavy_upper, 0, -1, -1, nullptr);
  else
    pull_round_kernel<false, false><<<grid, kPullBlock, dyn, s>>>(
        a, bits, g.deg0, g.n, scan_grid(g), mode, 0, total_entries, g.npieces,
        g.npieces_upper, corr_x, corr_d, ncorr, advance ? 1 : 0, bounds, queue_f0 ? 1 : 0,
        rowbits, rest_part ? 1 : 0, rest_part ? g.split_written : nullptr, nullptr, g.rank_vtx,
        g.roff, g.nheavy, g.nheavy_upper, 0, -1, -1, nullptr);
  return hipGetLastError();
}

hipError_t launch_pull_round(Graph &g, int32_t thrU, int32_t thrL, hipStream_t s,
                             bool advance, bool queue_f0, const uint32_t *rowbits, bool force,
                             bool rest_part, bool rank, const uint32_t *f0bits) {
  PeelArgs a = make_args(g, thrU, thrL);
  a.f0_bits = f0bits;
  return launch_pull_round_args(g, a, g.alive_bits, nullptr, nullptr, 0, advance, s, queue_f0,
                                rowbits, force, rest_part, rank);
}

// A query in rank order (unchanged graph): part 0, the first round pulled on
// the rank rows, whose survivors are ranks [0, ku) and [nU, nU + kl), which
// also writes their bitmap into the result; part 1, the asynchronous peel on
// the rank rows, which clears the result bit of each vertex it removes and,
// after termination, leaves the other workspace state ready for the next
// query.  g.state must be a zeroed state and the queue empty.
hipError_t launch_rank_query(Graph &g, int32_t thrU, int32_t thrL, int64_t ku, int64_t kl,
                             uint32_t *pack_bits, hipStream_t s, int part) {
  if (part == 0) {
    PeelArgs a = make_args(g, thrU, thrL);
    a.ins_head = nullptr;
    a.deg = g.rdeg;
    a.rs_mask = g.rdeg_mask;
    a.rs_fail = g.rs_fail;
    const int grid = g.cu_count;
    pull_round_kernel<false, true><<<grid, kPullBlock, 0, s>>>(
        a, g.alive_bits, g.deg0, g.n, scan_grid(g), 2, 0, 2 * g.m, g.npieces, g.npieces_upper,
        nullptr, nullptr, 0, 0, nullptr, 0, g.alive_bits, 0, nullptr, g.rcols, g.rank_vtx, g.roff,
        g.nheavy, g.nheavy_upper, 1, ku, kl, pack_bits);
    return hipGetLastError();
  }
  PeelArgs a = make_args(g, thrU, thrL);
  a.off = g.roff;
  a.cols = g.rcols;
  a.piece_row = g.rp_row;
  a.piece_start = g.rp_start;
  a.piece_first = g.rp_first;
  a.ins_head = nullptr;
  a.klim_u = (int32_t)ku;
  a.klim_l = (int32_t)kl;
  a.pack_vtx = g.rank_vtx;
  a.pack_bits = pack_bits;
  a.deg = g.rdeg;
  a.rs_mask = g.rdeg_mask;
  a.rs_next_st = g.state_alt;
  a.rs_next_part = g.part_alt;
  a.rs_fail = g.rs_fail;
  return launch_peel_async_args(g, kGCC, a, async_peel_grid(g), s);
}

__global__ void rank_prep_kernel(int32_t *queue, int64_t qcap, const PeelState *st,
                                 PeelState *next_st, int64_t *next_part, int nparts,
                                 int32_t *rs_fail) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid == 0) *rs_fail = 0;
  clear_used_queue(queue, qcap, st, tid, stride);
  for (int64_t i = tid; i < nparts; i += stride) next_part[i] = 0;
  int32_t *words = reinterpret_cast<int32_t *>(next_st);
  for (int64_t i = tid; i < (int64_t)(sizeof(PeelState) / 4); i += stride) words[i] = 0;
}

hipError_t launch_rank_prep(Graph &g, hipStream_t s) {
  rank_prep_kernel<<<g.cu_count, 256, 0, s>>>(g.queue, g.qcap, g.state, g.state_alt, g.part_alt,
                                              kMaxBlocks * kPartFields, g.rs_fail);
  return hipGetLastError();
}

// Must follow the pull round on the same stream (it completes that round).
hipError_t launch_pull_fixup_args(Graph &g, const PeelArgs &a, const uint32_t *bits,
                                  hipStream_t s) {
  if (g.pull_mode == 1) return hipSuccess;
  pull_fixup_kernel<<<flat_grid(g, std::max<int64_t>(g.nheavy, 1), kPeelBlock), kPeelBlock, 0, s>>>(
      a, bits, g.heavy_rows, g.nheavy);
  return hipGetLastError();
}

hipError_t launch_pull_fixup(Graph &g, int32_t thrU, int32_t thrL, hipStream_t s) {
  return launch_pull_fixup_args(g, make_args(g, thrU, thrL), g.alive_bits, s);
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
  pack_kernel<<<flat_grid(g, nwords * 32, kBlock), kBlock, 0, s>>>(g.deg, g.n, g.nU, thrU, thrL,
                                                                  bits, nwords);
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
  pack_from_core_kernel<<<flat_grid(g, nwords * 32, kBlock), kBlock, 0, s>>>(g.core, g.n, k, bits,
                                                                            nwords);
  return hipGetLastError();
}

// ------------------------------------------------------------- GCC+ init --
// Algorithm 2's classification by Lemma 1 with delta_l = min(alpha,beta) and
// delta_q = max(alpha,beta): core < delta_l -> out, core >= delta_q -> in,
// otherwise uncertain.  Uncertain vertices are appended to the queues; the
// next kernel consumes them as its items.

__global__ __launch_bounds__(kScanBlock) void classify_kernel(PeelArgs a, int64_t n, int32_t dl,
                                                              int32_t dq) {
  __shared__ ScanCollector col;
  if (threadIdx.x == 0) col.count = 0;
  __syncthreads();
  const int sub = blockIdx.x % kSub;
  for (int64_t cb = (int64_t)blockIdx.x * kScanChunk; cb < n;
       cb += (int64_t)gridDim.x * kScanChunk) {
    for (int t = 0; t < kScanChunk; t += kScanBlock * 4) {
      const int64_t x0 = cb + t + (int64_t)threadIdx.x * 4;
      int32_t c[4] = {0, 0, 0, 0};
      const bool full = x0 + 3 < n;
      if (full) {
        int4 v = *reinterpret_cast<const int4 *>(a.core + x0);
        c[0] = v.x; c[1] = v.y; c[2] = v.z; c[3] = v.w;
      } else {
        for (int j = 0; j < 4; ++j)
          if (x0 + j < n) c[j] = a.core[x0 + j];
      }
      int32_t dv[4];
      int32_t items[4];
      int cnt = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        dv[j] = c[j] < dl ? kDegOut : (c[j] >= dq ? kDegIn : 0);
        if ((x0 + j < n) && c[j] >= dl && c[j] < dq) items[cnt++] = (int32_t)(x0 + j);
      }
      if (full) {
        *reinterpret_cast<int4 *>(a.deg + x0) = make_int4(dv[0], dv[1], dv[2], dv[3]);
      } else {
        for (int j = 0; j < 4; ++j)
          if (x0 + j < n) a.deg[x0 + j] = dv[j];
      }
      col.append(items, cnt);
    }
    col.flush_queue(a, sub);
  }
  if (last_block_done<false>(a.st)) {
    start_rounds_wave(a.st, a.qcap);
    if (lane_id() == 0) st_agent(&a.st->aux0, ld_agent(&a.st->first));  // uncertain count
  }
}

hipError_t launch_classify(Graph &g, int32_t dl, int32_t dq, hipStream_t s) {
  PeelArgs a = make_args(g, 0, 0);
  classify_kernel<<<scan_grid(g), kScanBlock, 0, s>>>(a, g.n, dl, dq);
  return hipGetLastError();
}

// The same classification for the asynchronous peel, fused with the
// workspace reset (as the GCC scan): nothing is queued.  An uncertain vertex
// whose whole degree is already below its threshold is out as well
// (Algorithm 1's scan).  It writes the degrees the pull round starts from
// (out, in, or deg0 for an uncertain vertex, whose row the pull round
// recounts), the bitmap of the vertices not known to be out ({core >=
// delta_l} less the scan frontier: Algorithm 2's uncertain vertices count
// only neighbours with core >= delta_l, and a neighbour below its threshold
// is removed at once), the bitmap of the remaining uncertain vertices (the
// rows the pull round counts) and the number of uncertain vertices (Lemma
// 1's classes) per workgroup.
__global__ __launch_bounds__(kScanBlock) void classify_reset_kernel(
    PeelArgs a, const int32_t *__restrict__ deg0, uint32_t *__restrict__ hbits,
    uint32_t *__restrict__ ubits, int64_t n, int32_t dl, int32_t dq) {
  __shared__ int64_t s_acc;
  PeelState *st = a.st;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  clear_used_queue(a.queue, a.qcap, st, tid, stride);
  const int64_t nparts = (int64_t)kMaxBlocks * kPartFields;
  for (int64_t i = (int64_t)gridDim.x * kPartFields + tid; i < nparts; i += stride) a.part[i] = 0;
  if (threadIdx.x < kPartFields) a.part[(int64_t)blockIdx.x * kPartFields + threadIdx.x] = 0;
  __syncthreads();
  int64_t nunc = 0;
  for (int64_t cb = (int64_t)blockIdx.x * kScanChunk; cb < n;
       cb += (int64_t)gridDim.x * kScanChunk) {
    for (int t = 0; t < kScanChunk; t += kScanBlock * 4) {
      const int64_t x0 = cb + t + (int64_t)threadIdx.x * 4;
      int32_t c[4] = {0, 0, 0, 0}, d0[4] = {0, 0, 0, 0};
      const bool full = x0 + 3 < n;
      if (full) {
        const int4 v = *reinterpret_cast<const int4 *>(a.core + x0);
        const int4 e = *reinterpret_cast<const int4 *>(deg0 + x0);
        c[0] = v.x; c[1] = v.y; c[2] = v.z; c[3] = v.w;
        d0[0] = e.x; d0[1] = e.y; d0[2] = e.z; d0[3] = e.w;
      } else {
        for (int j = 0; j < 4; ++j)
          if (x0 + j < n) {
            c[j] = a.core[x0 + j];
            d0[j] = deg0[x0 + j];
          }
      }
      int32_t dv[4];
      uint32_t h = 0, u = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool valid = x0 + j < n;
        const int32_t th = (x0 + j) < a.nU ? a.thrU : a.thrL;
        const bool unc = valid && c[j] >= dl && c[j] < dq;
        const bool counted = unc && d0[j] >= th;
        // (a certain member has deg0 >= core >= delta_q >= its threshold)
        dv[j] = c[j] >= dq ? kDegIn : (counted ? d0[j] : kDegOut);
        h |= (uint32_t)(valid && c[j] >= dl && d0[j] >= th) << j;
        u |= (uint32_t)counted << j;
        nunc += unc ? 1 : 0;
      }
      if (full) {
        *reinterpret_cast<int4 *>(a.deg + x0) = make_int4(dv[0], dv[1], dv[2], dv[3]);
      } else {
        for (int j = 0; j < 4; ++j)
          if (x0 + j < n) a.deg[x0 + j] = dv[j];
      }
      // eight consecutive threads hold the 32 vertices of one bitmap word
      h <<= 4 * (lane_id() & 7);
      u <<= 4 * (lane_id() & 7);
      h |= __shfl_xor(h, 1, kWave);
      u |= __shfl_xor(u, 1, kWave);
      h |= __shfl_xor(h, 2, kWave);
      u |= __shfl_xor(u, 2, kWave);
      h |= __shfl_xor(h, 4, kWave);
      u |= __shfl_xor(u, 4, kWave);
      if ((lane_id() & 7) == 0 && x0 < n) {
        hbits[x0 / 32] = h;
        ubits[x0 / 32] = u;
      }
    }
  }
  add_part(a.part, kPartF0, nunc, &s_acc);
  __syncthreads();
  if (wave_in_block() != 0) return;
  int last = 0;
  if (lane_id() == 0) last = arrive_on(&st->rst) ? 1 : 0;
  if (!__shfl(last, 0, kWave)) return;
  int32_t *words = reinterpret_cast<int32_t *>(st);
  constexpr int kRstBegin = (int)(offsetof(PeelState, rst) / 4);
  for (int i = lane_id(); i < kRstBegin; i += kWave) words[i] = 0;
}

hipError_t launch_classify_reset(Graph &g, int32_t thrU, int32_t thrL, int32_t dl, int32_t dq,
                                  hipStream_t s) {
  PeelArgs a = make_args(g, thrU, thrL);
  classify_reset_kernel<<<scan_grid(g), kScanBlock, 0, s>>>(a, g.deg0, g.alive_bits, g.row_bits,
                                                            g.n, dl, dq);
  return hipGetLastError();
}

// Degree of every uncertain vertex inside G[{core >= delta_l}] -- the
// (alpha,beta)-core lies inside the (delta_l,delta_l)-core, so neighbours with
// smaller core numbers never count -- and the initial frontier of GCC+.
__global__ __launch_bounds__(kPeelBlock) void restricted_init_kernel(PeelArgs a, int32_t dl) {
  __shared__ int32_t s_lq[kPeelWaves][kLocalQueue];
  __shared__ int32_t s_cnt_own[kPeelWaves][kWave];
  __shared__ RangeView s_view;
  __shared__ int s_cnt[kPeelWaves + 2];
  __shared__ int64_t s_acc;
  load_view(s_view, a.st);
  LocalQueue lq = make_lq(s_lq[wave_in_block()], kLocalQueue, a);
  int32_t *cnt = s_cnt_own[wave_in_block()];
  int64_t entries = 0;
  const int32_t total = s_view.pre[kSub];
  const int waves = blockDim.x / kWave;
  const int gw = blockIdx.x * waves + wave_in_block();
  const int nw = gridDim.x * waves;
  for (int64_t b = (int64_t)gw * kWave; b < total; b += (int64_t)nw * kWave) {
    const int32_t i = (int32_t)(b + lane_id());
    const int32_t x = i < total ? view_item(s_view, a.queue, a.qcap, i) : -1;
    int64_t s = 0;
    int d = 0;
    if (x >= 0) {
      s = a.off[x];
      d = (int)(a.off[x + 1] - s);
    }
    cnt[lane_id()] = 0;
    __builtin_amdgcn_wave_barrier();
    BatchWalk bw;
    bw.init(s, d);
    entries += d;
    for (int base = 0; base < bw.total; base += kUnroll * kWave) {
      int32_t w[kUnroll], cw[kUnroll];
      int jj[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int k = base + u * kWave + lane_id();
        const int64_t pos = bw.locate(k < bw.total ? k : bw.total - 1, jj[u]);
        w[u] = k < bw.total ? a.cols[pos] : -1;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) cw[u] = w[u] >= 0 ? a.core[w[u]] : -1;
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int k = base + u * kWave + lane_id();
        segmented_count(cnt, jj[u], k < bw.total, w[u] >= 0 && cw[u] >= dl,
                        min(kWave, bw.total - base - u * kWave));
      }
    }
    int extra = 0;
    if (a.ins_head != nullptr && x >= 0) {
      for (int e = a.ins_head[x]; e >= 0; e = a.ins_next[e]) {
        const int32_t w = a.ins_other[e];
        if (w >= 0 && a.core[w] >= dl) ++extra;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    bool push = false;
    if (x >= 0) {
      const int32_t dx = cnt[lane_id()] + extra;
      a.deg[x] = dx;
      push = dx < (x < a.nU ? a.thrU : a.thrL);
    }
    lq.push(push, x);
    __builtin_amdgcn_wave_barrier();
  }
  block_flush(lq, s_cnt);
  add_part(a.part, kPartEntries, entries, &s_acc);
  if (last_block_done<false>(a.st)) {
    advance_round_wave(a.st, a.qcap);
    // the uncertain list is not a round: the frontier starts the count
    const int j = lane_id();
    int32_t f = 0;
    if (j < kSub) f = ld_agent(&a.st->hi[j]) - ld_agent(&a.st->lo[j]);
    f = wave_sum(f);
    if (j == 0) {
      st_agent(&a.st->first, f);
      st_agent(&a.st->rounds, 0);
    }
  }
}

hipError_t launch_restricted_init(Graph &g, int32_t thrU, int32_t thrL, int32_t dl,
                                  hipStream_t s) {
  PeelArgs a = make_args(g, thrU, thrL);
  restricted_init_kernel<<<wide_grid(g), kPeelBlock, 0, s>>>(a, dl);
  return hipGetLastError();
}

// ------------------------------------------------------- core numbers --
// Level-synchronous k-core peeling (Definition 2; a (k,k)-core is the k-core
// of G taken as an ordinary graph).  Phases:
//  - round: the current frontier is peeled at level k (threshold k+1; a
//    vertex crossing to k gets core number k);
//  - scan (frontier empty): every live vertex of the alive list with degree
//    <= k' gets core k' and is queued; when nothing was queued the smallest
//    live degree gives the next level directly (empty levels are skipped);
//  - compaction (right after a scan that left under half the list alive):
//    the list is rewritten without dead vertices, each workgroup at the
//    offset given by the kept counts of the workgroups before it.
// The persistent kernel loops over phases with grid barriers; the step
// kernel performs one phase per launch.

__global__ void kcore_init_kernel(const int32_t *__restrict__ deg0, int32_t *__restrict__ deg,
                                  int32_t *__restrict__ core, int32_t *__restrict__ alive,
                                  uint32_t *__restrict__ dead, PeelState *st, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride) {
    deg[x] = deg0[x];
    core[x] = -1;
    alive[x] = (int32_t)x;
  }
  if (dead != nullptr) {
    const int64_t words = (n + 31) / 32;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride)
      dead[i] = 0;
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
  hipError_t e = launch_init_state(g, s);
  if (e != hipSuccess) return e;
  kcore_init_kernel<<<flat_grid(g, g.n, kBlock), kBlock, 0, s>>>(g.deg0, g.deg, g.core, g.list,
                                                                 g.kdead, g.state, g.n);
  return hipGetLastError();
}

struct KCoreShared {
  int32_t lq[kPeelWaves][kLocalQueue];
  RangeView view;
  int s_cnt[kPeelWaves + 2];
  int s_wsum[kPeelWaves + 1];
  int phase;   // 0 done, 1 round, 2 scan, 3 compaction
  int level, next_k, cur, sel;
  int s_min;
  int64_t acc;
  int64_t offset;
};

// Reads the phase from the state (all threads).  Written only when a phase
// completes, i.e. before the barrier (or kernel boundary) preceding this.
__device__ __forceinline__ void kcore_read_phase(KCoreShared &sh, PeelState *st) {
  load_view(sh.view, st);
  if (threadIdx.x == 0) {
    const bool abort = ld_agent(&st->abort_flag) != 0;
    // a compaction runs right after its scan, before any round of the new
    // level can change which vertices are live: its offsets come from the
    // scan's kept counts
    if (abort || st->done)
      sh.phase = 0;
    else if (st->compact)
      sh.phase = 3;
    else if (sh.view.pre[kSub] > 0)
      sh.phase = 1;
    else
      sh.phase = 2;
    sh.level = st->k;
    sh.next_k = st->next_k;
    sh.cur = st->alive_cur;
    sh.sel = st->alive_sel;
  }
  __syncthreads();
}

// Work of one phase (whole grid).
__device__ void kcore_phase(const PeelArgs &a, KCoreShared &sh, LocalQueue &lq,
                            int32_t *alive0, int32_t *alive1, int64_t &entries) {
  if (sh.phase == 1) {
    peel_round_body<kKCore>(a, sh.view, sh.level, lq, entries);
    block_flush(lq, sh.s_cnt);
    return;
  }
  const int32_t cur = sh.cur;
  const int32_t *A = sh.sel ? alive1 : alive0;
  int32_t *N = sh.sel ? alive0 : alive1;
  const int64_t chunk = ((int64_t)cur + gridDim.x - 1) / gridDim.x;
  const int64_t c0 = std::min<int64_t>((int64_t)blockIdx.x * chunk, cur);
  const int64_t c1 = std::min<int64_t>(c0 + chunk, cur);
  const int64_t span = (c1 - c0 + blockDim.x - 1) / blockDim.x * blockDim.x;
  if (sh.phase == 2) {
    const int32_t kn = sh.next_k;
    int kept = 0, mn = 0x7FFFFFFF;
    for (int64_t t = threadIdx.x; t < span; t += blockDim.x) {
      const int64_t i = c0 + t;
      bool push = false;
      int32_t x = -1;
      if (i < c1) {
        x = A[i];
        if (a.core[x] < 0) {
          const int32_t d = a.deg[x];
          if (d <= kn) {
            a.core[x] = kn;
            push = true;
          } else {
            ++kept;
            mn = min(mn, d);
          }
        }
      }
      lq.push(push, x);
    }
    block_flush(lq, sh.s_cnt);
    const int wk = wave_sum(kept);
    const int wm = wave_min(mn);
    if (threadIdx.x == 0) {
      sh.acc = 0;
      sh.s_min = 0x7FFFFFFF;
    }
    __syncthreads();
    if (lane_id() == 0) {
      atomicAdd((unsigned long long *)&sh.acc, (unsigned long long)wk);
      atomicMin(&sh.s_min, wm);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      a.part[(int64_t)blockIdx.x * kPartFields + kPartKept] = sh.acc;
      a.part[(int64_t)blockIdx.x * kPartFields + kPartMin] = sh.s_min;
    }
    return;
  }
  // compaction: offset = kept counts of the preceding workgroups
  if (wave_in_block() == 0) {
    const int64_t o = wave_sum_strided(a.part + kPartKept, (int)blockIdx.x, kPartFields);
    if (lane_id() == 0) sh.offset = o;
  }
  __syncthreads();
  int64_t o = sh.offset;
  for (int64_t t = threadIdx.x; t < span; t += blockDim.x) {
    const int64_t i = c0 + t;
    int32_t x = -1;
    bool keep = false;
    if (i < c1) {
      x = A[i];
      keep = a.core[x] < 0;
    }
    int incl = wave_incl_scan((int)keep);
    if (lane_id() == kWave - 1) sh.s_wsum[wave_in_block()] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
        int v = sh.s_wsum[w];
        sh.s_wsum[w] = tot;
        tot += v;
      }
      sh.s_wsum[kPeelWaves] = tot;
    }
    __syncthreads();
    if (keep) N[o + sh.s_wsum[wave_in_block()] + incl - 1] = x;
    o += sh.s_wsum[kPeelWaves];
    __syncthreads();
  }
}

// Completes a phase: the 64 lanes of one wave, with every write of the phase
// visible.
__device__ void kcore_complete(const PeelArgs &a, int phase, int nblocks) {
  PeelState *st = a.st;
  const int lane = lane_id();
  if (phase == 1) {
    advance_round_wave(st, a.qcap);
  } else if (phase == 2) {
    const int32_t kn = st->next_k;
    const int64_t kept = wave_sum_strided(a.part + kPartKept, nblocks, kPartFields);
    const int32_t mn =
        (int32_t)wave_min_strided(a.part + kPartMin, nblocks, kPartFields, 0x7FFFFFFF);
    int32_t after = 0;
    if (lane < kSub) after = phys_tail(st, lane, a.qcap) - ld_agent(&st->hi[lane]);
    after = wave_sum(after);
    advance_round_wave(st, a.qcap);  // the scan's pushes become the level's first round
    if (lane == 0) {
      const bool pushed = after > 0;
      st->k = kn;
      if (pushed) st->max_core = kn;
      st->next_k = pushed ? kn + 1 : max(kn + 1, mn);
      st->kept = (int32_t)kept;
      if (kept == 0) {
        st->alive_cur = 0;
        st->done = 1;
      } else {
        st->compact = kept * 2 < st->alive_cur ? 1 : 0;
      }
    }
  } else if (phase == 3) {
    if (lane == 0) {
      st->alive_sel ^= 1;
      st->alive_cur = st->kept;
      st->compact = 0;
    }
  }
  if (lane == 0) atomicAdd((unsigned long long *)&st->launches, 1ull);
}

// Each phase removes a vertex, raises the level past a live degree, or
// compacts the list after a scan, so max_phases (4n + 1024) bounds a correct
// run; beyond it the loop flags an abort.
__global__ __launch_bounds__(kPeelBlock) void kcore_persistent_kernel(PeelArgs a, int32_t *alive0,
                                                                      int32_t *alive1,
                                                                      int64_t max_phases) {
  __shared__ KCoreShared sh;
  LocalQueue lq = make_lq(sh.lq[wave_in_block()], kLocalQueue, a);
  int64_t entries = 0;
  for (int64_t it = 0;; ++it) {
    kcore_read_phase(sh, a.st);
    const int phase = sh.phase;
    if (phase == 0) break;
    if (it > max_phases) {
      if (threadIdx.x == 0) st_agent(&a.st->abort_flag, 1);
      break;
    }
    kcore_phase(a, sh, lq, alive0, alive1, entries);
    grid_sync(a.st, [&] { kcore_complete(a, phase, (int)gridDim.x); });
  }
  add_part(a.part, kPartEntries, entries, &sh.acc);
}

__global__ __launch_bounds__(kPeelBlock) void kcore_step_kernel(PeelArgs a, int32_t *alive0,
                                                                int32_t *alive1) {
  __shared__ KCoreShared sh;
  LocalQueue lq = make_lq(sh.lq[wave_in_block()], kLocalQueue, a);
  int64_t entries = 0;
  kcore_read_phase(sh, a.st);
  const int phase = sh.phase;
  if (phase == 0) return;
  kcore_phase(a, sh, lq, alive0, alive1, entries);
  // the completion reads other workgroups' kept counts: release them first
  if (last_block_done<true>(a.st)) kcore_complete(a, phase, (int)gridDim.x);
}

hipError_t launch_kcore_persistent(Graph &g, hipStream_t s) {
  PeelArgs a = make_args(g, 0, 0);
  int32_t *l0 = g.list, *l1 = g.list2;
  int64_t max_phases = 4 * g.n + 1024;
  void *args[] = {&a, &l0, &l1, &max_phases};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&kcore_persistent_kernel),
                                    dim3(g.kcore_grid), dim3(kPeelBlock), args, 0, s);
}

// ---------------------------------------------- core numbers by levels --
// Level k of the decomposition (Definition 2: core(x) = the largest k with x
// in the k-core) as one scan and one asynchronous peel.  The scan takes the
// live vertices of degree <= k (core k), queues them, and appends the others
// to the next alive list (the vertices live when the scan ran); the
// peel then gives core k to every vertex whose degree falls to k, in any
// order (the k-core is unique).  A level that queues nothing jumps to the
// smallest live degree.  No grid barrier: two launches per level.
__global__ __launch_bounds__(kScanBlock) void kcore_level_scan_kernel(PeelArgs a,
                                                                      int32_t *list0,
                                                                      int32_t *list1) {
  __shared__ ScanCollector col;   // queued vertices
  __shared__ ScanCollector keep;  // live vertices for the next level
  __shared__ int32_t s_min;
  __shared__ int32_t s_kept, s_dead;
  PeelState *st = a.st;
  if (st->done) return;  // written by an earlier launch
  const int32_t kn = st->next_k;
  const int32_t cur = st->alive_cur;
  const int sel = st->alive_sel;
  // the list is rewritten without its removed entries only when enough of
  // it was found removed before (rewriting costs a write per kept entry;
  // a removed entry left in place costs a read per scan, and the degree
  // tells it apart at any later level too)
  const bool compact = ABC_LEVEL_COMPACT_ALWAYS || st->compact != 0;
  const int32_t *A = sel ? list1 : list0;
  int32_t *N = sel ? list0 : list1;
  if (threadIdx.x == 0) {
    col.count = 0;
    keep.count = 0;
    s_min = 0x7FFFFFFF;
    s_kept = 0;
    s_dead = 0;
  }
  __syncthreads();
  const int sub = blockIdx.x % kSub;
  int32_t mn = 0x7FFFFFFF;
  int kept_here = 0, dead_here = 0;
  for (int64_t cb = (int64_t)blockIdx.x * kScanChunk; cb < cur;
       cb += (int64_t)gridDim.x * kScanChunk) {
    for (int t = 0; t < kScanChunk; t += kScanBlock * 4) {
      const int64_t i0 = cb + t + (int64_t)threadIdx.x * 4;
      int32_t items[4], kept[4];
      int cnt = 0, kc = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (i0 + j < cur) {
          // the list held live vertices of degree > the previous level when
          // that level's scan wrote it; its peel left the survivors at
          // degree >= kn and the removed ones below, so the degree alone
          // tells them apart (no read of core[])
          const int32_t x = A[i0 + j];
          const int32_t d = a.deg[x];
          if (d == kn) {
            a.core[x] = kn;
            items[cnt++] = x;
          } else if (d > kn) {
            kept[kc++] = x;
            mn = min(mn, d);
          } else {
            ++dead_here;
          }
        }
      }
      col.append(items, cnt);
      kept_here += kc;
      dead_here += cnt;  // queued now: removed for the next scan
      if (compact) keep.append(kept, kc);
    }
    col.flush_queue(a, sub);
    if (compact) keep.flush(N, &a.st->kept);
  }
  mn = wave_min(mn);
  kept_here = wave_sum(kept_here);
  dead_here = wave_sum(dead_here);
  if (lane_id() == 0) {
    atomicMin(&s_min, mn);
    atomicAdd(&s_kept, kept_here);
    atomicAdd(&s_dead, dead_here);
  }
  __syncthreads();
  if (!compact && threadIdx.x == 0 && s_kept > 0) atomicAdd(&st->kept, s_kept);
  if (threadIdx.x == 0 && s_dead > 0) atomicAdd(&st->dead, s_dead);
  if (threadIdx.x == 0) a.part[(int64_t)blockIdx.x * kPartFields + kPartMin] = s_min;
  if (last_block_done<false>(st)) {
    const int lane = lane_id();
    int32_t after = 0;
    if (lane < kSub) after = phys_tail(st, lane, a.qcap) - ld_agent(&st->hi[lane]);
    after = wave_sum(after);
    const int32_t gmin =
        (int32_t)wave_min_strided(a.part + kPartMin, (int)gridDim.x, kPartFields, 0x7FFFFFFF);
    advance_round_wave(st, a.qcap);  // the queued vertices start the level's peel
    if (lane < kGroups) st->fin[lane][0] = 0;  // the level's peel detects its own end
    if (lane == 0) {
      const int32_t kept_n = ld_agent(&st->kept);  // live entries
      const int32_t dead_n = ld_agent(&st->dead);
      st->k = kn;
      if (after > 0) st->max_core = kn;
      st->next_k = after > 0 ? kn + 1 : max(kn + 1, gmin);
      if (compact) {
        st->alive_cur = kept_n;
        st->alive_sel = sel ^ 1;
      }
      // the next scan rewrites the list once a quarter of it is removed
      const int32_t len = compact ? kept_n : cur;
      st->compact = (int64_t)(compact ? 0 : dead_n) * 4 > len ? 1 : 0;
      st->live = kept_n;
      st->kept = 0;
      st->dead = 0;
      if (kept_n == 0) st->done = 1;
      atomicAdd((unsigned long long *)&st->launches, 1ull);
    }
  }
}

#ifndef ABC_KCORE_DEAD_BITS
#define ABC_KCORE_DEAD_BITS 1
#endif
hipError_t launch_kcore_levels(Graph &g, int levels, hipStream_t s) {
  PeelArgs a = make_args(g, 0, 0);
  if (ABC_KCORE_DEAD_BITS) a.kdead = g.kdead;
  const int sgrid = std::min(g.cu_count * 4, kMaxBlocks);
  const int agrid = async_peel_grid(g);
  for (int l = 0; l < levels; ++l) {
    kcore_level_scan_kernel<<<sgrid, kScanBlock, 0, s>>>(a, g.list, g.list2);
    peel_async_kernel<kKCore><<<agrid, kPeelBlock, 0, s>>>(a);
  }
  return hipGetLastError();
}

hipError_t launch_kcore_steps(Graph &g, int steps, hipStream_t s) {
  PeelArgs a = make_args(g, 0, 0);
  const int grid = peel_grid(g);
  for (int r = 0; r < steps; ++r) kcore_step_kernel<<<grid, kPeelBlock, 0, s>>>(a, g.list, g.list2);
  return hipGetLastError();
}

// Co-resident workgroup counts for the cooperative kernels.
hipError_t query_persistent_grids(Graph &g) {
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, reinterpret_cast<const void *>(&peel_persistent_kernel<kGCC>), kPeelBlock, 0);
  if (e != hipSuccess) return e;
  int per_cu2 = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu2, reinterpret_cast<const void *>(&peel_persistent_kernel<kGCCPlus>), kPeelBlock, 0);
  if (e != hipSuccess) return e;
  int per_cu3 = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu3, reinterpret_cast<const void *>(&kcore_persistent_kernel), kPeelBlock, 0);
  if (e != hipSuccess) return e;
  int per_cu4 = 0, per_cu5 = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu4, reinterpret_cast<const void *>(&peel_async_kernel<kGCC>), kPeelBlock, 0);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu5, reinterpret_cast<const void *>(&peel_async_kernel<kGCCPlus>), kPeelBlock, 0);
  if (e != hipSuccess) return e;
  g.async_grid = std::min(kMaxBlocks, g.cu_count * std::max(1, std::min({per_cu4, per_cu5, 4})));
  const int pc = std::max(1, std::min({per_cu, per_cu2, 2}));
  g.persistent_grid = std::min(kMaxBlocks, g.cu_count * pc);
  g.kcore_grid = std::min(kMaxBlocks, g.cu_count * std::max(1, std::min(per_cu3, 2)));
  return hipSuccess;
}

}  // namespace abc
