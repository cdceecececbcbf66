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

// Per-wave frontier buffer in LDS, flushed to the workgroup's sub-queue.
// Every call must be made by the whole wave in uniform control flow.
struct LocalQueue {
  int32_t *buf;
  int cap;
  int count;     // wave-uniform
  int32_t *q;    // this workgroup's sub-queue
  int32_t *tail; // its append cursor

  __device__ __forceinline__ void flush() {
    if (count == 0) return;
    __builtin_amdgcn_wave_barrier();
    int base = 0;
    if (lane_id() == 0) base = atomicAdd(tail, count);
    base = __shfl(base, 0, kWave);
    for (int i = lane_id(); i < count; i += kWave) st_agent(&q[base + i], buf[i]);
    __builtin_amdgcn_wave_barrier();
    count = 0;
  }

  __device__ __forceinline__ void push(bool pred, int32_t val) {
    uint64_t mask = __ballot(pred);
    int c = __popcll(mask);
    if (c == 0) return;
    if (count + c > cap) flush();
    if (pred) buf[count + __popcll(mask & lanemask_lt())] = val;
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
  lq.tail = &a.st->tail[sub][0];
  return lq;
}

// Flushes every wave's local queue of the workgroup with a single append.
// s_cnt: LDS, at least (waves + 1) ints.  Whole workgroup, uniform flow.
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
    s_cnt[waves] = tot > 0 ? atomicAdd(lq.tail, tot) : 0;
  }
  __syncthreads();
  const int base = s_cnt[waves] + s_cnt[wave_in_block()];
  for (int i = lane_id(); i < lq.count; i += kWave) st_agent(&lq.q[base + i], lq.buf[i]);
  lq.count = 0;
  __syncthreads();
}

// Workgroup-aggregated append of `cnt` items per thread to this workgroup's
// sub-queue; returns the thread's first position.  Whole workgroup.
__device__ __forceinline__ int block_reserve(int cnt, int32_t *tail, int *s_wsum) {
  const int waves = blockDim.x / kWave;
  int incl = wave_incl_scan(cnt);
  if (lane_id() == kWave - 1) s_wsum[wave_in_block()] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int w = 0; w < waves; ++w) {
      int t = s_wsum[w];
      s_wsum[w] = tot;
      tot += t;
    }
    s_wsum[waves] = tot > 0 ? atomicAdd(tail, tot) : 0;
  }
  __syncthreads();
  int pos = s_wsum[waves] + s_wsum[wave_in_block()] + incl - cnt;
  __syncthreads();
  return pos;
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
  return ld_agent(&queue[(int64_t)j * qcap + v.lo[j] + (i - v.pre[j])]);
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
__device__ __forceinline__ void advance_round_wave(PeelState *st) {
  const int j = lane_id();
  int32_t h = 0, l = 0, t = 0;
  if (j < kSub) {
    h = ld_agent(&st->hi[j]);
    l = ld_agent(&st->lo[j]);
    t = ld_agent(&st->tail[j][0]);
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
__device__ __forceinline__ void start_rounds_wave(PeelState *st) {
  const int j = lane_id();
  int32_t t = 0;
  if (j < kSub) {
    t = ld_agent(&st->tail[j][0]);
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
