// Vertex sets around a query (Remark of Sec. V): after a peel scoped to the
// component(s) of one or two vertices -- GFQ's Algorithm 1 on the affected
// component, or the same for a static query vertex -- the result is either
// every survivor of that scope (the vertices the scoped peel leaves) or only
// those connected to the query vertices through survivors (the connected
// part of the (alpha,beta)-core that holds them, found by a breadth-first
// search over the core's induced subgraph).
#include "abcore_internal.h"
#include "wave.h"

namespace abc {

// Bit x of `bits`: x lies in the component of vx or of vy (labels read from
// comp, which the scoped scan used) and its final working degree reached its
// threshold.  Every word is written.
__global__ __launch_bounds__(kBlock) void pack_scope_kernel(const int32_t *__restrict__ deg,
                                                            const int32_t *__restrict__ comp,
                                                            int32_t vx, int32_t vy, int64_t n,
                                                            int32_t nU, int32_t thrU,
                                                            int32_t thrL,
                                                            uint32_t *__restrict__ bits,
                                                            int64_t nwords) {
  const int32_t c1 = comp[vx], c2 = comp[vy];
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t base = ((int64_t)blockIdx.x * kWavesPerBlock + wave_in_block()) * kWave;
       base < nwords * 32; base += stride) {
    const int64_t x = base + lane_id();
    bool p = false;
    if (x < n) {
      const int32_t c = comp[x];
      p = (c == c1 || c == c2) && ld_agent(&deg[x]) >= (x < nU ? thrU : thrL);
    }
    const uint64_t mask = __ballot(p);
    const int64_t w0 = base / 32;
    if (lane_id() == 0) bits[w0] = (uint32_t)mask;
    if (lane_id() == 1 && w0 + 1 < nwords) bits[w0 + 1] = (uint32_t)(mask >> 32);
  }
}

__global__ void zero_words_kernel(uint32_t *__restrict__ w, int64_t nwords) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += stride)
    w[i] = 0u;
}

// Search seeds: each of the (up to two) seed vertices that is a member
// starts the search (marked visited, put in the first frontier).
__global__ void bfs_seed_kernel(const uint32_t *__restrict__ member, uint32_t *visited,
                                int32_t sx, int32_t sy, int32_t *front, int32_t *count) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int c = 0;
  const int32_t seeds[2] = {sx, sy};
  for (int i = 0; i < 2; ++i) {
    const int32_t x = seeds[i];
    if (x < 0 || !((member[x >> 5] >> (x & 31)) & 1u)) continue;
    const uint32_t bit = 1u << (x & 31);
    if (visited[x >> 5] & bit) continue;
    visited[x >> 5] |= bit;
    front[c++] = x;
  }
  count[0] = c;
  count[1] = 0;
}

// Claims w for the search: a member not visited yet (the atomic OR decides
// which lane of the grid takes it, exactly once).
__device__ __forceinline__ bool bfs_claim(const uint32_t *__restrict__ member, uint32_t *visited,
                                          int32_t w) {
  const uint32_t bit = 1u << (w & 31);
  if (!(member[w >> 5] & bit)) return false;
  if (ld_agent(&visited[w >> 5]) & bit) return false;
  return (atomicOr(&visited[w >> 5], bit) & bit) == 0u;
}

// One level of the search: a wave per frontier vertex walks its CSR row
// (tombstoned entries, stored as ~col, skipped) 64 entries at a time, then
// lane 0 its inserted edges; newly claimed vertices form the next frontier
// (one append counter increment per wave and step).
__global__ __launch_bounds__(kBlock) void bfs_level_kernel(
    const int64_t *__restrict__ off, const int32_t *__restrict__ cols,
    const int32_t *__restrict__ ins_head, const int32_t *__restrict__ ins_next,
    const int32_t *__restrict__ ins_other, const uint32_t *__restrict__ member,
    uint32_t *visited, const int32_t *__restrict__ front, const int32_t *count,
    int32_t *next) {
  const int32_t nfront = count[0];
  int32_t *nnext = const_cast<int32_t *>(count) + 1;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + wave_in_block();
  const int64_t nw = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t i = gw; i < nfront; i += nw) {
    const int32_t x = front[i];
    const int64_t b = off[x], e = off[x + 1];
    for (int64_t j0 = b; j0 < e; j0 += kWave) {
      const int64_t j = j0 + lane_id();
      int32_t w = -1;
      bool take = false;
      if (j < e) {
        w = cols[j];
        take = w >= 0 && bfs_claim(member, visited, w);
      }
      const uint64_t mask = __ballot(take);
      if (mask) {
        int base = 0;
        if (lane_id() == 0) base = atomicAdd(nnext, (int)__popcll(mask));
        base = __shfl(base, 0, kWave);
        if (take) next[base + (int)__popcll(mask & lanemask_lt())] = w;
      }
    }
    if (ins_head != nullptr && lane_id() == 0) {
      for (int h = ins_head[x]; h >= 0; h = ins_next[h]) {
        const int32_t w = ins_other[h];
        if (w >= 0 && bfs_claim(member, visited, w)) next[atomicAdd(nnext, 1)] = w;
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void popcount_kernel(const uint32_t *__restrict__ w,
                                                          int64_t nwords,
                                                          unsigned long long *out) {
  __shared__ unsigned long long s;
  if (threadIdx.x == 0) s = 0;
  __syncthreads();
  unsigned long long c = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += stride)
    c += (unsigned long long)__popc(w[i]);
  atomicAdd(&s, c);
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, s);
}

// The largest degree over ids [lo, hi) into *out (which must start at 0).
__global__ __launch_bounds__(kBlock) void max_deg_kernel(const int32_t *__restrict__ deg0,
                                                         int64_t lo, int64_t hi, int32_t *out) {
  __shared__ int32_t s;
  if (threadIdx.x == 0) s = 0;
  __syncthreads();
  int32_t m = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi; i += stride)
    m = max(m, deg0[i]);
  atomicMax(&s, m);
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(out, s);
}

static int grid_for(const Graph &g, int64_t items, int per_block) {
  const int64_t b = (items + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, std::min(g.cu_count * 8, kMaxBlocks)));
}

// The vertex set after a peel scoped to the components of vx and vy (their
// labels in g.comp): every survivor of the scope, or with `connected` the
// survivors reachable from vx or vy through survivors.  Writes every word of
// d_bits; *count (nullable) receives the set's size.  Synchronous.
abcore_status scoped_set(Graph &g, int32_t vx, int32_t vy, int32_t thrU, int32_t thrL,
                         bool connected, uint32_t *d_bits, int64_t *count, hipStream_t s) {
  const int64_t nwords = (g.n + 31) / 32;
  if (g.aux == nullptr) {
    if (dev_malloc(&g.aux, sizeof(int64_t) * 4) != hipSuccess) {
      g.aux = nullptr;
      set_error("community: allocation of counters failed");
      return ABCORE_ENOMEM;
    }
  }
  uint32_t *member = connected ? g.row_bits : d_bits;
  pack_scope_kernel<<<grid_for(g, nwords * 32, kBlock), kBlock, 0, s>>>(
      g.deg, g.comp, vx, vy, g.n, g.nU, thrU, thrL, member, nwords);
  if (hipGetLastError() != hipSuccess) goto fail;
  if (connected) {
    int32_t *front = g.list, *next = g.list2;
    int32_t *cnt = reinterpret_cast<int32_t *>(g.aux);
    int32_t h_cnt[2] = {0, 0};
    zero_words_kernel<<<grid_for(g, nwords, 256), 256, 0, s>>>(d_bits, nwords);
    bfs_seed_kernel<<<1, 64, 0, s>>>(member, d_bits, vx, vy == vx ? -1 : vy, front, cnt);
    if (hipGetLastError() != hipSuccess) goto fail;
    if (hipMemcpyAsync(h_cnt, cnt, sizeof(h_cnt), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      goto fail;
    // every level claims at least one new vertex, so at most n levels run
    for (int64_t level = 0; h_cnt[0] > 0 && level <= g.n; ++level) {
      bfs_level_kernel<<<grid_for(g, (int64_t)h_cnt[0] * kWave, kBlock), kBlock, 0, s>>>(
          g.off, g.cols, g.delta.count > 0 ? g.delta.head : nullptr, g.delta.next,
          g.delta.other, member, d_bits, front, cnt, next);
      if (hipGetLastError() != hipSuccess) goto fail;
      // the next frontier's size becomes the current one; its counter restarts
      if (hipMemcpyAsync(h_cnt, cnt, sizeof(h_cnt), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        goto fail;
      const int32_t reset[2] = {h_cnt[1], 0};
      if (hipMemcpyAsync(cnt, reset, sizeof(reset), hipMemcpyHostToDevice, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        goto fail;
      h_cnt[0] = h_cnt[1];
      std::swap(front, next);
    }
  }
  if (count != nullptr) {
    unsigned long long h = 0;
    unsigned long long *dc = reinterpret_cast<unsigned long long *>(g.aux) + 2;
    if (hipMemsetAsync(dc, 0, sizeof(unsigned long long), s) != hipSuccess) goto fail;
    popcount_kernel<<<grid_for(g, nwords, kBlock), kBlock, 0, s>>>(d_bits, nwords, dc);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&h, dc, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      goto fail;
    *count = (int64_t)h;
  } else if (hipStreamSynchronize(s) != hipSuccess) {
    goto fail;
  }
  return ABCORE_OK;
fail:
  set_error("community: a device call failed");
  return ABCORE_EDEVICE;
}

abcore_status max_degree(Graph &g, int64_t lo, int64_t hi, int32_t *out, hipStream_t s) {
  if (g.aux == nullptr && dev_malloc(&g.aux, sizeof(int64_t) * 4) != hipSuccess) {
    g.aux = nullptr;
    set_error("offsets: allocation of counters failed");
    return ABCORE_ENOMEM;
  }
  int32_t *d = reinterpret_cast<int32_t *>(g.aux);
  int32_t h = 0;
  if (hipMemsetAsync(d, 0, sizeof(int32_t), s) != hipSuccess) goto fail;
  if (hi > lo) {
    max_deg_kernel<<<grid_for(g, hi - lo, kBlock), kBlock, 0, s>>>(g.deg0, lo, hi, d);
    if (hipGetLastError() != hipSuccess) goto fail;
  }
  if (hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    goto fail;
  *out = h;
  return ABCORE_OK;
fail:
  set_error("offsets: a device call failed");
  return ABCORE_EDEVICE;
}

abcore_status count_bits(Graph &g, const uint32_t *bits, int64_t *out, hipStream_t s) {
  if (g.aux == nullptr && dev_malloc(&g.aux, sizeof(int64_t) * 4) != hipSuccess) {
    g.aux = nullptr;
    set_error("allocation of counters failed");
    return ABCORE_ENOMEM;
  }
  const int64_t nwords = (g.n + 31) / 32;
  unsigned long long h = 0;
  unsigned long long *dc = reinterpret_cast<unsigned long long *>(g.aux) + 2;
  if (hipMemsetAsync(dc, 0, sizeof(unsigned long long), s) != hipSuccess) goto fail;
  if (nwords > 0) {
    popcount_kernel<<<grid_for(g, nwords, kBlock), kBlock, 0, s>>>(bits, nwords, dc);
    if (hipGetLastError() != hipSuccess) goto fail;
  }
  if (hipMemcpyAsync(&h, dc, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    goto fail;
  *out = (int64_t)h;
  return ABCORE_OK;
fail:
  set_error("counting bits: a device call failed");
  return ABCORE_EDEVICE;
}

}  // namespace abc
