// Core numbers of the deepest part of the graph by an h-index fixpoint.
//
// The level-by-level peel (Definition 2 via Batagelj and Zaversnik's order)
// pays one dependent step per cascade round, and on skewed graphs most of
// those rounds fall in the few thousand levels above a hundred, where only a
// small, dense part of the graph is left.  Once every vertex of core number
// below k0 has its value, the live vertices H are exactly the k0-core, and
// the core numbers of H in G are its core numbers as a graph of its own (the
// k-core of G for k >= k0 lies inside H).  They are also the fixpoint of
//   est(x) <- min(est(x), h-index of { est(w) : w neighbour of x in H }),
// started from the degrees in H (Lu, Zhou, Zhang and Stanley, 2016; the
// h-index of a multiset is the largest h with at least h members >= h): the
// iterates stay upper bounds of the core numbers and reach them.  Each sweep
// is a fully parallel pass over H's adjacency, and the number of sweeps is
// small where the number of cascade rounds is large.
//
// Here H's adjacency is compacted (local ids, live-live entries only), the
// sweeps update the values in place (Gauss-Seidel: a vertex may already see
// values its neighbours lowered in the same sweep; every value read is still
// an upper bound of its core number, so every value computed is too), a
// sweep that changes nothing ends the iteration, and the values are written
// back as core numbers.
#include "abcore_internal.h"
#include "prim.h"
#include "wave.h"

namespace abc {

namespace {

// Live vertices of the alive list (core < 0) into hv, their local ids into
// lid; *count receives their number.  One append counter increment per wave.
__global__ __launch_bounds__(kBlock) void top_select_kernel(const int32_t *__restrict__ alive,
                                                            int64_t cnt,
                                                            const int32_t *__restrict__ core,
                                                            int32_t *__restrict__ hv,
                                                            int32_t *__restrict__ lid,
                                                            int32_t *count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < cnt; base += stride) {
    const int64_t i = base + threadIdx.x;
    int32_t x = -1;
    bool live = false;
    if (i < cnt) {
      x = alive[i];
      live = core[x] < 0;
    }
    const uint64_t mask = __ballot(live);
    int at = 0;
    if (lane_id() == 0 && mask) at = atomicAdd(count, (int)__popcll(mask));
    at = __shfl(at, 0, kWave);
    if (live) {
      const int32_t j = at + (int)__popcll(mask & lanemask_lt());
      hv[j] = x;
      lid[x] = j;
    }
  }
}

// Walks the live neighbours of x (CSR entries, tombstones ~col skipped, then
// inserted edges) 64 at a time; f(w, rank) gets each live neighbour and its
// rank among them, in row order.  Wave-uniform; returns the count.
template <class F>
__device__ __forceinline__ int64_t walk_live(const int64_t *__restrict__ off,
                                             const int32_t *__restrict__ cols,
                                             const int32_t *__restrict__ ins_head,
                                             const int32_t *__restrict__ ins_next,
                                             const int32_t *__restrict__ ins_other,
                                             const int32_t *__restrict__ core, int32_t x, F f) {
  const int64_t b = off[x], e = off[x + 1];
  int64_t done = 0;
  for (int64_t j0 = b; j0 < e; j0 += kWave) {
    const int64_t j = j0 + lane_id();
    int32_t w = -1;
    bool live = false;
    if (j < e) {
      w = cols[j];
      live = w >= 0 && core[w] < 0;
    }
    const uint64_t mask = __ballot(live);
    if (live) f(w, done + (int64_t)__popcll(mask & lanemask_lt()));
    done += (int64_t)__popcll(mask);
  }
  if (ins_head != nullptr) {
    // inserted edges: lane 0 walks the list, the rest of the wave waits
    int64_t extra = 0;
    if (lane_id() == 0) {
      for (int h = ins_head[x]; h >= 0; h = ins_next[h]) {
        const int32_t w = ins_other[h];
        if (w >= 0 && core[w] < 0) f(w, done + extra++);
      }
    }
    done += __shfl(extra, 0, kWave);
  }
  return done;
}

// Degrees in H: hlen[j] = live neighbours of hv[j]; est[j] starts there.
__global__ __launch_bounds__(kBlock) void top_count_kernel(
    const int64_t *__restrict__ off, const int32_t *__restrict__ cols,
    const int32_t *__restrict__ ins_head, const int32_t *__restrict__ ins_next,
    const int32_t *__restrict__ ins_other, const int32_t *__restrict__ core,
    const int32_t *__restrict__ hv, int64_t h, int64_t *__restrict__ hlen,
    int32_t *__restrict__ est) {
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + wave_in_block();
  const int64_t nw = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t j = gw; j < h; j += nw) {
    const int64_t d = walk_live(off, cols, ins_head, ins_next, ins_other, core, hv[j],
                                [](int32_t, int64_t) {});
    if (lane_id() == 0) {
      hlen[j] = d;
      est[j] = (int32_t)d;
    }
  }
}

// H's adjacency in local ids: row j at hoff[j], its live neighbours in order.
__global__ __launch_bounds__(kBlock) void top_fill_kernel(
    const int64_t *__restrict__ off, const int32_t *__restrict__ cols,
    const int32_t *__restrict__ ins_head, const int32_t *__restrict__ ins_next,
    const int32_t *__restrict__ ins_other, const int32_t *__restrict__ core,
    const int32_t *__restrict__ hv, const int32_t *__restrict__ lid, int64_t h,
    const int64_t *__restrict__ hoff, int32_t *__restrict__ hcols) {
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + wave_in_block();
  const int64_t nw = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t j = gw; j < h; j += nw) {
    int32_t *row = hcols + hoff[j];
    walk_live(off, cols, ins_head, ins_next, ins_other, core, hv[j],
              [&](int32_t w, int64_t r) { row[r] = lid[w]; });
  }
}

// Rows of at most kRegSpan * 64 entries keep their neighbours' values in
// registers through a binary search; longer rows count their neighbours'
// values once into a per-wave LDS histogram of [k0, min(cur, k0 + kBins))
// (values above go to a wave-level count); only an h-index above that
// window needs a binary search that rereads the row per probe.
// Loads are issued kUnroll at a time per lane, so a long row keeps many
// in flight.
constexpr int kRegSpan = 8;

// A neighbour's value, which other waves may be lowering: a relaxed load
// that may be served by this compute unit's cache (a stale value is an
// older, larger one, still an upper bound; a sweep that changes nothing
// reads only values written before it began, after the caches were
// invalidated at the kernel boundary).
__device__ __forceinline__ int32_t ld_near(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
constexpr int kBins = 2048;
constexpr int kUnroll = 8;

// One sweep in place: est[j] <- largest h <= est[j] with at least h
// neighbours whose value is >= h (>= k0 always: the iterates bound the core
// numbers, all >= k0, from above).  Values are written at device scope, so
// a vertex may see what other waves lowered so far.  Only vertices
// marked in dirty_now are computed (a vertex none of whose neighbours
// changed would get its value again); each vertex this sweep lowers marks its
// neighbours in dirty_next (also those already computed in this sweep with
// its older value).  A sweep that lowers nothing read only values written
// before it began, so est is then the fixpoint; the sweeps after it return
// at once.  changed[t] counts the vertices sweep t lowered.
__global__ __launch_bounds__(kBlock) void hindex_sweep_kernel(
    const int64_t *__restrict__ hoff, const int32_t *__restrict__ hcols, int64_t h,
    int32_t k0, int32_t *est, int32_t *changed, int t, uint8_t *__restrict__ dirty_now,
    uint8_t *__restrict__ dirty_next) {
  __shared__ int32_t s_bins[kWavesPerBlock][kBins];
  if (t > 0 && ld_agent(&changed[t - 1]) == 0) return;
  int32_t *bins = s_bins[wave_in_block()];
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + wave_in_block();
  const int64_t nw = (int64_t)gridDim.x * kWavesPerBlock;
  int lowered = 0;
  for (int64_t j = gw; j < h; j += nw) {
    // no neighbour changed in the previous sweep: its value stands
    if (!dirty_now[j]) continue;
    const int32_t cur = ld_agent(&est[j]);
    __builtin_amdgcn_wave_barrier();
    if (lane_id() == 0) dirty_now[j] = 0;  // cleared for the marks of the next sweep but one
    const int64_t b = hoff[j], e = hoff[j + 1], d = e - b;
    int32_t res = cur;
    if (d <= (int64_t)kRegSpan * kWave) {
      int32_t v[kRegSpan];
#pragma unroll
      for (int u = 0; u < kRegSpan; ++u) {
        const int64_t k = b + u * kWave + lane_id();
        v[u] = k < e ? ld_near(&est[hcols[k]]) : -1;
      }
      auto count_ge = [&](int32_t th) -> int64_t {
        int64_t c = 0;
#pragma unroll
        for (int u = 0; u < kRegSpan; ++u) c += (int64_t)__popcll(__ballot(v[u] >= th));
        return c;
      };
      if (count_ge(cur) < cur) {
        // the predicate count_ge(x) >= x holds at k0 and fails at cur
        int32_t lo = k0, hi = cur - 1;
        while (lo < hi) {
          const int32_t mid = lo + (hi - lo + 1) / 2;
          if (count_ge(mid) >= mid)
            lo = mid;
          else
            hi = mid - 1;
        }
        res = lo;
      }
    } else {
      // bins[v - k0] counts the neighbours of value v in [k0, cap), where
      // cap = min(cur, k0 + kBins); `top` those of value >= cap
      const int32_t cap = cur - k0 < kBins ? cur : k0 + kBins;
      const int nb = cap - k0;
      for (int i = lane_id(); i < nb; i += kWave) bins[i] = 0;
      __builtin_amdgcn_wave_barrier();
      int64_t top = 0;
      for (int64_t k0i = b; k0i < e; k0i += (int64_t)kUnroll * kWave) {
        int32_t w[kUnroll], v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int64_t k = k0i + u * kWave + lane_id();
          w[u] = k < e ? hcols[k] : -1;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = w[u] >= 0 ? ld_near(&est[w[u]]) : -1;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          top += (int64_t)__popcll(__ballot(v[u] >= cap));
          if (v[u] >= k0 && v[u] < cap) atomicAdd(&bins[v[u] - k0], 1);
        }
      }
      __builtin_amdgcn_wave_barrier();
      if (top >= cap && cap < cur) {
        // the h-index is at least cap: search [cap, cur) rereading the row
        auto count_ge = [&](int32_t th) -> int64_t {
          int64_t c = 0;
          for (int64_t k0i = b; k0i < e; k0i += (int64_t)kUnroll * kWave) {
            int32_t w[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
              const int64_t k = k0i + u * kWave + lane_id();
              w[u] = k < e ? hcols[k] : -1;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
              c += (int64_t)__popcll(__ballot(w[u] >= 0 && ld_near(&est[w[u]]) >= th));
          }
          return c;
        };
        if (count_ge(cur) < cur) {
          int32_t lo = cap, hi = cur - 1;
          while (lo < hi) {
            const int32_t mid = lo + (hi - lo + 1) / 2;
            if (count_ge(mid) >= mid)
              lo = mid;
            else
              hi = mid - 1;
          }
          res = lo;
        }
      } else if (top < cap) {
        // count(>= x) for x = cap - 1, cap - 2, ... down to k0: the first x
        // (from the top) with count >= x is the h-index; 64 bins a step,
        // lane L at x = hi - L, the counts by an inclusive wave scan
        int64_t acc = top;
        int32_t found = k0;
        for (int32_t hi = cap - 1; hi >= k0; hi -= kWave) {
          const int32_t x = hi - lane_id();
          const int64_t c = x >= k0 ? (int64_t)bins[x - k0] : 0;
          int64_t incl = c;
#pragma unroll
          for (int o = 1; o < kWave; o <<= 1) {
            const int64_t tt = __shfl_up(incl, o, kWave);
            if (lane_id() >= o) incl += tt;
          }
          const uint64_t ok = __ballot(x >= k0 && acc + incl >= (int64_t)x);
          if (ok) {
            found = hi - (int32_t)(__ffsll((unsigned long long)ok) - 1);
            break;
          }
          acc += __shfl(incl, kWave - 1, kWave);
        }
        res = found;
      }
      __builtin_amdgcn_wave_barrier();
    }
    if (res != cur) {
      if (lane_id() == 0) st_agent(&est[j], res);
      // its neighbours are recomputed in the next sweep
      ++lowered;
      for (int64_t k = b + lane_id(); k < e; k += kWave) dirty_next[hcols[k]] = 1;
    }
  }
  if (lane_id() == 0 && lowered > 0) atomicAdd(&changed[t], lowered);
}

// core[hv[j]] = est[j]; *vmax receives the largest value.
__global__ __launch_bounds__(kBlock) void top_write_kernel(const int32_t *__restrict__ hv,
                                                           const int32_t *__restrict__ est,
                                                           int64_t h, int32_t *__restrict__ core,
                                                           int32_t *vmax) {
  __shared__ int32_t s;
  if (threadIdx.x == 0) s = 0;
  __syncthreads();
  int32_t m = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < h; j += stride) {
    core[hv[j]] = est[j];
    m = max(m, est[j]);
  }
  atomicMax(&s, m);
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(vmax, s);
}

int grid_of(const Graph &g, int64_t items, int per_block) {
  const int64_t b = (items + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, std::min(g.cu_count * 8, kMaxBlocks)));
}

}  // namespace

// After the levels below k0 (every vertex of core < k0 has its value; the
// live ones of the alive list, `cnt` entries, are the k0-core): the core
// numbers of the live vertices by the h-index fixpoint.  *finished = false
// (and nothing changed) if it did not converge within max_sweeps, so the
// caller can go on level by level.  Synchronous.
abcore_status kcore_top(Graph &g, const int32_t *alive, int64_t cnt, int32_t k0,
                        int max_sweeps, bool *finished, int32_t *top_max, hipStream_t s) {
  *finished = false;
  int32_t *lid = nullptr, *hv = nullptr, *hcols = nullptr, *est = nullptr, *ctr = nullptr;
  uint8_t *dirty = nullptr;
  int64_t *hlen = nullptr, *hoff = nullptr;
  void *temp = nullptr;
  size_t temp_bytes = 0;
  int32_t h32 = 0;
  int64_t h = 0, eh = 0;
  abcore_status st = ABCORE_EDEVICE;
  const int32_t *ih = g.delta.count > 0 ? g.delta.head : nullptr;
  const int sweeps_per_check = 16;
  const int nctr = max_sweeps + 1;
  auto ok = [](hipError_t e) { return e == hipSuccess; };
  do {
    if (!ok(dev_malloc_async(&lid, sizeof(int32_t) * std::max<int64_t>(g.n, 1), s)) ||
        !ok(dev_malloc_async(&hv, sizeof(int32_t) * std::max<int64_t>(cnt, 1), s)) ||
        !ok(dev_malloc_async(&ctr, sizeof(int32_t) * (nctr + 1), s))) {
      st = ABCORE_ENOMEM;
      break;
    }
    if (!ok(hipMemsetAsync(ctr, 0, sizeof(int32_t) * (nctr + 1), s))) break;
    if (cnt > 0) {
      top_select_kernel<<<grid_of(g, cnt, kBlock), kBlock, 0, s>>>(alive, cnt, g.core, hv, lid,
                                                                   ctr + nctr);
      if (!ok(hipGetLastError())) break;
    }
    if (!ok(hipMemcpyAsync(&h32, ctr + nctr, sizeof(int32_t), hipMemcpyDeviceToHost, s)) ||
        !ok(hipStreamSynchronize(s)))
      break;
    h = h32;
    if (!ok(dev_malloc_async(&hlen, sizeof(int64_t) * (h + 1), s)) ||
        !ok(dev_malloc_async(&hoff, sizeof(int64_t) * (h + 1), s)) ||
        !ok(dev_malloc_async(&est, sizeof(int32_t) * std::max<int64_t>(h, 1), s))) {
      st = ABCORE_ENOMEM;
      break;
    }
    if (!ok(hipMemsetAsync(hlen + h, 0, sizeof(int64_t), s))) break;
    if (h > 0) {
      top_count_kernel<<<grid_of(g, h * kWave, kBlock), kBlock, 0, s>>>(
          g.off, g.cols, ih, g.delta.next, g.delta.other, g.core, hv, h, hlen, est);
      if (!ok(hipGetLastError())) break;
    }
    if (!ok(prim::exclusive_sum(nullptr, temp_bytes, hlen, hoff, (size_t)(h + 1), s))) break;
    if (!ok(dev_malloc_async(&temp, std::max<size_t>(temp_bytes, 16), s))) {
      st = ABCORE_ENOMEM;
      break;
    }
    if (!ok(prim::exclusive_sum(temp, temp_bytes, hlen, hoff, (size_t)(h + 1), s))) break;
    if (!ok(hipMemcpyAsync(&eh, hoff + h, sizeof(int64_t), hipMemcpyDeviceToHost, s)) ||
        !ok(hipStreamSynchronize(s)))
      break;
    if (!ok(dev_malloc_async(&hcols, sizeof(int32_t) * std::max<int64_t>(eh, 1), s))) {
      st = ABCORE_ENOMEM;
      break;
    }
    if (h > 0) {
      top_fill_kernel<<<grid_of(g, h * kWave, kBlock), kBlock, 0, s>>>(
          g.off, g.cols, ih, g.delta.next, g.delta.other, g.core, hv, lid, h, hoff, hcols);
      if (!ok(hipGetLastError())) break;
    }
    // which vertices a sweep recomputes: all in the first, then those with a
    // neighbour lowered by the sweep before (two byte arrays, alternating)
    if (!ok(dev_malloc_async(&dirty, sizeof(uint8_t) * 2 * std::max<int64_t>(h, 1), s))) {
      st = ABCORE_ENOMEM;
      break;
    }
    if (h > 0 && (!ok(hipMemsetAsync(dirty, 1, sizeof(uint8_t) * h, s)) ||
                  !ok(hipMemsetAsync(dirty + h, 0, sizeof(uint8_t) * h, s))))
      break;
    // sweeps in place, checked every sweeps_per_check
    int t = 0, fixed_at = -1;
    std::vector<int32_t> hc(sweeps_per_check);
    bool failed = false;
    while (t < max_sweeps && fixed_at < 0 && h > 0) {
      const int t0 = t;
      for (int r = 0; r < sweeps_per_check && t < max_sweeps; ++r, ++t) {
        hindex_sweep_kernel<<<grid_of(g, h * kWave, kBlock), kBlock, 0, s>>>(
            hoff, hcols, h, k0, est, ctr, t, dirty + (t % 2) * h, dirty + ((t + 1) % 2) * h);
      }
      if (!ok(hipGetLastError()) ||
          !ok(hipMemcpyAsync(hc.data(), ctr + t0, sizeof(int32_t) * (t - t0),
                             hipMemcpyDeviceToHost, s)) ||
          !ok(hipStreamSynchronize(s))) {
        failed = true;
        break;
      }
      for (int r = 0; r < t - t0; ++r)
        if (hc[r] == 0) {
          fixed_at = t0 + r;
          break;
        }
    }
    if (failed) break;
    if (h > 0 && fixed_at < 0) {
      st = ABCORE_OK;  // not converged: the caller continues level by level
      break;
    }
    g.top_stats[0] = k0;
    g.top_stats[1] = h;
    g.top_stats[2] = eh;
    g.top_stats[3] = fixed_at + 1;
    const int32_t *fin = est;
    int32_t *dmax = ctr + nctr;
    int32_t hmax = 0;
    if (!ok(hipMemsetAsync(dmax, 0, sizeof(int32_t), s))) break;
    if (h > 0) {
      top_write_kernel<<<grid_of(g, h, kBlock), kBlock, 0, s>>>(hv, fin, h, g.core, dmax);
      if (!ok(hipGetLastError())) break;
    }
    if (!ok(hipMemcpyAsync(&hmax, dmax, sizeof(int32_t), hipMemcpyDeviceToHost, s)) ||
        !ok(hipStreamSynchronize(s)))
      break;
    *top_max = hmax;
    *finished = true;
    st = ABCORE_OK;
  } while (0);
  for (void *p : {(void *)lid, (void *)hv, (void *)hcols, (void *)est, (void *)ctr, (void *)hlen,
                  (void *)hoff, (void *)dirty, temp})
    if (p) (void)dev_free_async(p, s);
  if (st != ABCORE_OK) set_error("core numbers: the h-index phase failed");
  return st;
}

}  // namespace abc
