// Wavefront-level primitives for gfx950 (64-lane waves).
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

// Per-wave frontier buffer in LDS (the wavefront-local queue of Algorithm 1),
// flushed to the global queue with one atomic per flush.  Every call must be
// made by the whole wave in uniform control flow.
struct LocalQueue {
  int32_t *buf;
  int count;  // wave-uniform

  __device__ __forceinline__ void flush(int32_t *q, int32_t *tail) {
    if (count == 0) return;
    __builtin_amdgcn_wave_barrier();
    int base = 0;
    if (lane_id() == 0) base = atomicAdd(tail, count);
    base = __shfl(base, 0, kWave);
    for (int i = lane_id(); i < count; i += kWave) q[base + i] = buf[i];
    __builtin_amdgcn_wave_barrier();
    count = 0;
  }

  __device__ __forceinline__ void push(bool pred, int32_t val, int32_t *q, int32_t *tail) {
    uint64_t mask = __ballot(pred);
    int c = __popcll(mask);
    if (c == 0) return;
    if (count + c > kLocalQueue) flush(q, tail);
    if (pred) buf[count + __popcll(mask & lanemask_lt())] = val;
    count += c;
  }
};

// Workgroup-aggregated append: each thread contributes `cnt` items; returns
// the position of the thread's first item in the global array whose cursor
// is *tail.  One global atomic per workgroup call.  Must be called by every
// thread of the workgroup.
__device__ __forceinline__ int block_reserve(int cnt, int32_t *tail, int *s_wsum) {
  int incl = wave_incl_scan(cnt);
  if (lane_id() == kWave - 1) s_wsum[wave_in_block()] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) {
      int t = s_wsum[w];
      s_wsum[w] = tot;
      tot += t;
    }
    s_wsum[kWavesPerBlock] = tot > 0 ? atomicAdd(tail, tot) : 0;
  }
  __syncthreads();
  int pos = s_wsum[kWavesPerBlock] + s_wsum[wave_in_block()] + incl - cnt;
  __syncthreads();
  return pos;
}

// Last-workgroup detection: returns true in thread 0 of the workgroup that
// finishes a launch last; all prior global writes of every workgroup are
// visible to it.
__device__ __forceinline__ bool last_block_done(uint32_t *finished) {
  __syncthreads();
  bool last = false;
  if (threadIdx.x == 0) {
    __threadfence();
    uint32_t t = atomicAdd(finished, 1u);
    last = (t == gridDim.x - 1);
    if (last) __threadfence();
  }
  return last;
}

}  // namespace abc
