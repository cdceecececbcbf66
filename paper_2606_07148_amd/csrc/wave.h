// Wavefront- and grid-level primitives for gfx950 (64-lane waves).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "abcore_internal.h"

namespace abc {

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }
__device__ __forceinline__ int wave_in_block() { return (int)(threadIdx.x / kWave); }
__device__ __forceinline__ uint64_t lanemask_lt() {
  return (uint64_t(1) << lane_id()) - 1;
}

__device__ __forceinline__ int32_t ld_agent(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_agent(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(int32_t *p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Tells the host that a computation ended by a spin-limit abort: one store
// at system scope into the handle's pinned, coherent word (if any).
__device__ __forceinline__ void report_abort(const PeelArgs &a) {
  if (a.abort_host != nullptr)
    __hip_atomic_store(a.abort_host, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Inclusive prefix sum across the 64 lanes (all lanes must be active).
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int t = __shfl_up(v, o, kWave);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
  return v;
}

// Reserves `cnt` consecutive slots for one append; called by one thread.
// The sub-queues share one bound instead of each holding the worst case:
// a computation appends at most 2n + pieces + kLocalQueue items, and each
// sub-queue holds a 16th of that plus kMaxAppend (the largest single append).
// Sub-queue `pref` is tried first.  An append that does not fit fills the
// rest of that sub-queue with kSkipItem (consumers take such a slot and
// count it as processed) and tries the next sub-queue; the slots past qcap
// that its failed reservation counted are never written or claimed (every
// range end, every steal and the termination test use min(tail, qcap)).
// A sub-queue that rejects an append is full from then on with fewer than
// kMaxAppend skips, so if all kSub rejected, more than kSub * (qcap -
// kMaxAppend) >= the bound real items would have been appended: the loop
// always ends with a reservation.  Should the bound ever be broken anyway,
// the computation aborts (nothing is written past qcap).  Returns the
// sub-queue in .x (-1 on that abort) and the first slot in .y.
__device__ __forceinline__ int2 reserve_slots(PeelState *st, int32_t *queue, int64_t qcap,
                                              int pref, int cnt, int *abort_host) {
  int s = pref;
  for (int tries = 0; tries < kSub; ++tries) {
    // a full sub-queue stays full: after the first attempt, skip such ones
    // without counting more slots past their capacity
    if (tries > 0 && ld_agent(&st->tail[s][0]) >= qcap) {
      s = (s + 1) % kSub;
      continue;
    }
    const int base = atomicAdd(&st->tail[s][0], cnt);
    if ((int64_t)base + cnt <= qcap) return make_int2(s, base);
    int32_t *q = queue + (int64_t)s * qcap;
    for (int64_t i = base; i < qcap; ++i) st_agent(&q[i], kSkipItem);
    s = (s + 1) % kSub;
  }
  st_agent(&st->abort_flag, 1);
  if (abort_host != nullptr)
    __hip_atomic_store(abort_host, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  return make_int2(-1, 0);
}

// Debug builds (ABC_DEBUG_ENQUEUE) count every vertex that enters the
// frontier (a wave's local queue or a sub-queue), per vertex, so that tests
// can check that each removal is queued exactly once (the crossing rule);
// release builds emit nothing.
#ifdef ABC_DEBUG_ENQUEUE
#define ABC_COUNT_ENQUEUE(counts, x)                                   \
  do {                                                                 \
    if ((counts) != nullptr && (x) >= 0) atomicAdd(&(counts)[(x)], 1); \
  } while (0)
#else
#define ABC_COUNT_ENQUEUE(counts, x) \
  do {                               \
  } while (0)
#endif

// The sub-queue an append tries first.
__device__ __forceinline__ int append_pref(const PeelArgs &a, int own) {
  return a.append_sub >= 0 ? a.append_sub : own;
}

// End of sub-queue j's written range: its tail, less the slots a rejected
// append counted past the capacity.
__device__ __forceinline__ int32_t phys_tail(PeelState *st, int j, int64_t qcap) {
  return (int32_t)min((int64_t)ld_agent(&st->tail[j][0]), qcap);
}

// Per-wave frontier buffer in LDS, flushed to the workgroup's sub-queue (or
// the next with room, see reserve_slots).
// Every call must be made by the whole wave in uniform control flow.
struct LocalQueue {
  int32_t *buf;
  int cap;
  int count;      // wave-uniform
  int32_t *q;     // this workgroup's sub-queue (its consumers read it)
  int32_t *queue; // every sub-queue
  int64_t qcap;
  PeelState *st;
  int *abort_host;
  int32_t *dbg;   // debug builds: per-vertex enqueue counts
  int sub;

  __device__ __forceinline__ void flush() {
    if (count == 0) return;
    __builtin_amdgcn_wave_barrier();
    int2 r = make_int2(0, 0);
    if (lane_id() == 0) r = reserve_slots(st, queue, qcap, sub, count, abort_host);
    const int s = __shfl(r.x, 0, kWave);
    const int base = __shfl(r.y, 0, kWave);
    if (s >= 0) {
      int32_t *dst = queue + (int64_t)s * qcap + base;
      for (int i = lane_id(); i < count; i += kWave) st_agent(&dst[i], buf[i]);
    }
    __builtin_amdgcn_wave_barrier();
    count = 0;
  }

  __device__ __forceinline__ void push(bool pred, int32_t val) {
    uint64_t mask = __ballot(pred);
    int c = __popcll(mask);
    if (c == 0) return;
    if (count + c > cap) flush();
    if (pred) {
      buf[count + __popcll(mask & lanemask_lt())] = val;
      // counted on entry: a wave may process its own removals without
      // ever sharing them
      ABC_COUNT_ENQUEUE(dbg, val);
    }
    count += c;
  }
};

__device__ __forceinline__ LocalQueue make_lq(int32_t *buf, int cap, const PeelArgs &a) {
  const int sub = blockIdx.x % kSub;
  LocalQueue lq;
  lq.buf = buf;
  lq.cap = cap;
  lq.count = 0;
  lq.q = a.queue + (int64_t)sub * a.qcap;
  lq.queue = a.queue;
  lq.qcap = a.qcap;
  lq.st = a.st;
  lq.abort_host = a.abort_host;
  lq.dbg = a.dbg_enqueue;
  lq.sub = append_pref(a, sub);
  return lq;
}

// Flushes every wave's local queue of the workgroup with a single append.
// s_cnt: LDS, at least (waves + 2) ints.  Whole workgroup, uniform flow.
__device__ __forceinline__ void block_flush(LocalQueue &lq, int *s_cnt) {
  const int waves = blockDim.x / kWave;
  if (lane_id() == 0) s_cnt[wave_in_block()] = lq.count;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int w = 0; w < waves; ++w) {
      int t = s_cnt[w];
      s_cnt[w] = tot;
      tot += t;
    }
    int2 r = make_int2(0, 0);
    if (tot > 0) r = reserve_slots(lq.st, lq.queue, lq.qcap, lq.sub, tot, lq.abort_host);
    s_cnt[waves] = r.y;
    s_cnt[waves + 1] = r.x;
  }
  __syncthreads();
  const int s = s_cnt[waves + 1];
  if (s >= 0) {
    int32_t *dst = lq.queue + (int64_t)s * lq.qcap + s_cnt[waves] + s_cnt[wave_in_block()];
    for (int i = lane_id(); i < lq.count; i += kWave) st_agent(&dst[i], lq.buf[i]);
  }
  lq.count = 0;
  __syncthreads();
}

// A round's items: the sub-queue ranges [lo[j], hi[j]) seen as one
// concatenated index space (loaded into LDS by load_view).
struct RangeView {
  int32_t pre[kSub + 1];
  int32_t lo[kSub];
};

__device__ __forceinline__ void load_view(RangeView &v, PeelState *st) {
  if (threadIdx.x < kSub) {
    v.lo[threadIdx.x] = ld_agent(&st->lo[threadIdx.x]);
    v.pre[threadIdx.x + 1] = ld_agent(&st->hi[threadIdx.x]) - v.lo[threadIdx.x];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    v.pre[0] = 0;
    for (int j = 0; j < kSub; ++j) v.pre[j + 1] += v.pre[j];
  }
  __syncthreads();
}

__device__ __forceinline__ int32_t view_item(const RangeView &v, const int32_t *queue,
                                             int64_t qcap, int32_t i) {
  int j = 0;
#pragma unroll
  for (int s = kSub / 2; s > 0; s >>= 1)
    if (v.pre[j + s] <= i) j += s;
  const int32_t x = ld_agent(&queue[(int64_t)j * qcap + v.lo[j] + (i - v.pre[j])]);
  return x == kSkipItem ? -1 : x;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Single-writer increment of a state counter (only the thread completing a
// round writes it).
__device__ __forceinline__ void bump(int32_t *p) { st_agent(p, ld_agent(p) + 1); }

// Advances the round: the items appended since the last snapshot become the
// next round.  Called by the 64 lanes of one wave (lane j < kSub handles
// sub-queue j) once every append of the round is complete.
__device__ __forceinline__ void advance_round_wave(PeelState *st, int64_t qcap) {
  const int j = lane_id();
  int32_t h = 0, l = 0, t = 0;
  if (j < kSub) {
    h = ld_agent(&st->hi[j]);
    l = ld_agent(&st->lo[j]);
    t = phys_tail(st, j, qcap);
  }
  const int prev = wave_sum(h - l);
  if (j < kSub) {
    st_agent(&st->lo[j], h);
    st_agent(&st->hi[j], t);
    st_agent(&st->head[j][0], h);  // the asynchronous peel starts at lo
    st_agent(&st->consumed[j][0], h);
  }
  if (j == 0 && prev > 0) bump(&st->rounds);
}

// Sets lo to 0 and hi to the tails: the first round after a scan.  One wave.
__device__ __forceinline__ void start_rounds_wave(PeelState *st, int64_t qcap) {
  const int j = lane_id();
  int32_t t = 0;
  if (j < kSub) {
    t = phys_tail(st, j, qcap);
    st_agent(&st->lo[j], 0);
    st_agent(&st->hi[j], t);
    st_agent(&st->head[j][0], 0);
    st_agent(&st->consumed[j][0], 0);
  }
  const int tot = wave_sum(t);
  if (j == 0) {
    st_agent(&st->first, tot);
    st_agent(&st->rounds, 0);
  }
}

// Arrival on the group/top lines; true in lane 0 for the last arrival.
__device__ __forceinline__ bool arrive_on(Arrival *arr) {
  const int ng = min((int)gridDim.x, kGroups);
  const int grp = blockIdx.x % kGroups;
  const int gsize = ((int)gridDim.x - grp + kGroups - 1) / kGroups;
  const uint32_t c = atomicAdd(&arr->group[grp][0], 1u);
  if ((int)c != gsize - 1) return false;
  st_agent(&arr->group[grp][0], 0u);
  const uint32_t t = atomicAdd(&arr->top[0], 1u);
  if ((int)t != ng - 1) return false;
  st_agent(&arr->top[0], 0u);
  return true;
}

__device__ __forceinline__ bool arrive(PeelState *st) { return arrive_on(&st->arr); }

// Last-workgroup detection.  Returns true in every lane of wave 0 of the
// workgroup that arrives last.  With kRelease, each workgroup first makes
// its plain stores visible (needed when the last workgroup reads data other
// than the atomic append cursors).
template <bool kRelease>
__device__ __forceinline__ bool last_block_done(PeelState *st) {
  __syncthreads();
  if (wave_in_block() != 0) return false;
  int last = 0;
  if (lane_id() == 0) {
    if (kRelease) __threadfence();
    last = arrive(st) ? 1 : 0;
  }
  last = __shfl(last, 0, kWave);
  if (last && kRelease) __threadfence();
  return last != 0;
}

// Grid-wide barrier for co-resident (cooperatively launched) workgroups.
// Wave 0 of the last arrival runs `on_last` (a snapshot of the round state,
// all 64 lanes) before releasing everyone.  A workgroup that waits longer
// than the spin limit sets abort_flag and leaves; callers stop at their next
// check of the flag.  kFence = false omits the release/acquire fences (each
// writes back or invalidates the L2): correct only when every value passed
// between workgroups across the barrier goes through agent-scope atomic
// loads/stores or atomic read-modify-writes.
constexpr uint32_t kSpinLimit = 1u << 24;

template <bool kFence = true, class F>
__device__ __forceinline__ void grid_sync(PeelState *st, F on_last) {
  // every wave's stores of the round are acknowledged before the arrival
  if (!kFence) __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (wave_in_block() == 0) {
    uint32_t g = 0;
    int last = 0;
    if (lane_id() == 0) {
      g = __hip_atomic_load(&st->arr.gen[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (kFence) __threadfence();
      last = arrive(st) ? 1 : 0;
    }
    last = __shfl(last, 0, kWave);
    g = __shfl(g, 0, kWave);
    if (last) {
      if (kFence) __threadfence();
      on_last();
      if (kFence) __threadfence();
      __builtin_amdgcn_s_waitcnt(0);  // the snapshot's stores land before the release
      __builtin_amdgcn_wave_barrier();
      if (lane_id() == 0)
        __hip_atomic_store(&st->arr.gen[0], g + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane_id() == 0) {
      // relaxed polling: an acquire load would invalidate the L2 on every poll
      uint32_t spins = 0;
      while (__hip_atomic_load(&st->arr.gen[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) {
          st_agent(&st->abort_flag, 1);
          break;
        }
      }
    }
    if (kFence) __threadfence();
  }
  __syncthreads();
}

// Sum over lanes of v[i * stride] for i in [0, count): plain loads spread
// over the wave (values written before the caller's last acquire).
// Eight loads per lane are issued before any is added, so the sum takes
// one memory round trip per 512 values.
__device__ __forceinline__ int64_t wave_sum_strided(const int64_t *v, int count, int stride) {
  constexpr int kU = 8;
  int64_t acc = 0;
  for (int i0 = 0; i0 < count; i0 += kU * kWave) {
    int64_t t[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = i0 + u * kWave + lane_id();
      t[u] = i < count ? v[(int64_t)i * stride] : 0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) acc += t[u];
  }
  return wave_sum64(acc);
}

__device__ __forceinline__ int64_t wave_min_strided(const int64_t *v, int count, int stride,
                                                    int64_t init) {
  int64_t acc = init;
  for (int i = lane_id(); i < count; i += kWave) acc = min(acc, v[(int64_t)i * stride]);
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) acc = min(acc, (int64_t)__shfl_xor(acc, o, kWave));
  return acc;
}

}  // namespace abc
