// Core numbers of the deepest part of the graph by an h-index fixpoint.
//
// The level-by-level peel (Definition 2 via Batagelj and Zaversnik's order)
// pays one dependent step per cascade round, and on skewed graphs most of
// those rounds fall in the few thousand levels above a hundred, where only a
// small, dense part of the graph is left.  Once every vertex of core number
// below k0 has its value, the live vertices H are exactly the k0-core, and
// the core numbers of H in G are its core numbers as a graph of its own (the
// k-core of G for k >= k0 lies inside H).  They are also the fixpoint of
//   est(x) <- h-index of { est(w) : w neighbour of x in H },
// started from the degrees in H (Lu, Zhou, Zhang and Stanley, 2016; the
// h-index of a multiset is the largest h with at least h members >= h): the
// iterates stay upper bounds of the core numbers and reach them.
//
// Schedule.  H is bipartite, so the layers take turns ("half sweeps"): a
// half recomputes vertices of one layer against the other layer's values,
// which stay fixed during it -- Gauss-Seidel order with no race.  A vertex
// is recomputed only when its value must drop: c(x) counts the neighbours
// whose value is >= est(x), and x is due exactly when c(x) < est(x).  A
// vertex a half lowers from `old` to `new` decrements c(y) of each
// neighbour y with old >= est(y) > new, and the next half lists the due
// vertices of its layer from the counts.  Past the first few halves only a
// few thousand vertices drop per half, while a dense core's every row has
// one of them as neighbour, so this does a fraction of the work of sweeps
// that recompute every row with a changed neighbour.
//
// Layout.  H's vertices get local ids by layer, then by decreasing degree,
// so the most referenced values of a layer come first: each workgroup keeps
// the first 63,488 values of the layer a half reads in LDS (16 bits each,
// offsets from k0), and only entries past them read the values array.  Rows
// are written at offsets given by the vertices' degrees in G (an upper
// bound of their degrees in H), so the adjacency is built in one pass over
// the rows (long rows by id ranges of the other layer, one range per XCD);
// a neighbour's local id comes from its rank among the live vertices in id
// order (a live bitmap with per-word prefix counts) through a permutation.
// The phase's buffers stay with the handle for the next decomposition.
#include <algorithm>
#include <vector>

#include "abcore_internal.h"
#include "prim.h"
#include "wave.h"

namespace abc {

namespace {

constexpr int kHalfBlock = 1024;
constexpr int kHalfWaves = kHalfBlock / kWave;
constexpr int kCache = 63488;  // LDS values per workgroup (124 KB)
constexpr int kFine = 256;     // unit bins just below the upper end of the search range
constexpr int kCoarse = 256;   // equal-width bins over the rest of the range
constexpr int kRegSpan = 8;    // rows of at most 8 x 64 entries keep their values in registers
#ifndef ABC_TOP_UNROLL
#define ABC_TOP_UNROLL 8
#endif
#ifndef ABC_TOP_LONG_ROW
#define ABC_TOP_LONG_ROW 2048
#endif
#ifndef ABC_TOP_FILL_PARTS
#define ABC_TOP_FILL_PARTS 1
#endif
#ifndef ABC_TOP_UNROLL_BLOCK
#define ABC_TOP_UNROLL_BLOCK 4
#endif
constexpr int kUnroll = ABC_TOP_UNROLL;             // row entries in flight per lane
constexpr int kLongRow = ABC_TOP_LONG_ROW;          // longer rows: walked by a whole workgroup
constexpr int kUnrollBlock = ABC_TOP_UNROLL_BLOCK;  // the same for those walks
// summed decrement targets: 16-bit sums, two to a word, in the bins of
// waves 1..15 (a sum counts rows of one workgroup: at most one decrement
// of a target per row, far fewer rows than 65536 per workgroup and half)
constexpr int kAgg = 2 * (kHalfBlock / kWave - 1) * (kFine + kCoarse);

// Live vertices of the alive list (core < 0) into hv and their bits into
// live; count[0] receives their number, count[1] the number in the upper
// layer.  One append counter increment per wave.
__global__ __launch_bounds__(kBlock) void top_select_kernel(const int32_t *__restrict__ alive,
                                                            int64_t cnt,
                                                            const int32_t *__restrict__ core,
                                                            int32_t nU, int32_t *__restrict__ hv,
                                                            uint32_t *__restrict__ live,
                                                            int32_t *count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < cnt; base += stride) {
    const int64_t i = base + threadIdx.x;
    int32_t x = -1;
    bool on = false;
    if (i < cnt) {
      x = alive[i];
      on = core[x] < 0;
    }
    const uint64_t mask = __ballot(on);
    const uint64_t upper = __ballot(on && x < nU);
    int at = 0;
    if (lane_id() == 0 && mask) {
      at = atomicAdd(&count[0], (int)__popcll(mask));
      if (upper) atomicAdd(&count[1], (int)__popcll(upper));
    }
    at = __shfl(at, 0, kWave);
    if (on) {
      hv[at + (int)__popcll(mask & lanemask_lt())] = x;
      atomicOr(&live[x >> 5], 1u << (x & 31));
    }
  }
}

// Sort keys: layer, then decreasing degree in G, then id.
__global__ void top_keys_kernel(const int32_t *__restrict__ hv, int64_t h,
                                const int32_t *__restrict__ deg0, int32_t nU,
                                uint64_t *__restrict__ keys) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < h; j += stride) {
    const int32_t x = hv[j];
    keys[j] = ((uint64_t)(x >= nU) << 63) | ((uint64_t)(0x7FFFFFFF - deg0[x]) << 32) |
              (uint64_t)(uint32_t)x;
  }
}

// Live vertices per 32-id word of the live bitmap (words entries; one more
// zero for the exclusive sum).
__global__ void top_word_count_kernel(const uint32_t *__restrict__ live, int64_t words,
                                      int64_t *__restrict__ wcount) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= words; i += stride)
    wcount[i] = i < words ? __popc(live[i]) : 0;
}

// rk[i] = {live bits of word i, live vertices in the words before it}: the
// rank of a live vertex among the live ones in id order is a single 8-byte
// read, next to its liveness bit.
__global__ void top_word_pack_kernel(const uint32_t *__restrict__ live,
                                     const int64_t *__restrict__ wpre, int64_t words,
                                     uint2 *__restrict__ rk) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride)
    rk[i] = make_uint2(live[i], (uint32_t)wpre[i]);
}

__device__ __forceinline__ int32_t id_rank(const uint2 word, int32_t w) {
  return (int32_t)(word.y + (uint32_t)__popc(word.x & ((1u << (w & 31)) - 1u)));
}

// hv[j], perm[rank of hv[j] in id order] = j (the local id), and the row
// capacity deg0 (the exclusive sum of which places the rows) from the
// sorted keys.
__global__ void top_place_kernel(const uint64_t *__restrict__ keys, int64_t h,
                                 const int32_t *__restrict__ deg0, const uint2 *__restrict__ rk,
                                 int32_t *__restrict__ hv, int32_t *__restrict__ perm,
                                 int64_t *__restrict__ cap) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < h; j += stride) {
    const int32_t x = (int32_t)(uint32_t)keys[j];
    hv[j] = x;
    perm[id_rank(rk[x >> 5], x)] = (int32_t)j;
    cap[j] = deg0[x];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) cap[h] = 0;
}

// Row j of H: the live neighbours of hv[j] (CSR entries, tombstones ~col
// skipped, then inserted edges) as local ids, in row order, from hoff[j];
// hlen[j] and est[j] receive their number.  *overflow is set if a row has
// more live neighbours than its capacity (its degree in G): never, unless
// the degrees are inconsistent with the rows.  One wave per row.
__global__ __launch_bounds__(kBlock) void top_fill_kernel(
    const int64_t *__restrict__ off, const int32_t *__restrict__ cols,
    const int32_t *__restrict__ ins_head, const int32_t *__restrict__ ins_next,
    const int32_t *__restrict__ ins_other, const uint2 *__restrict__ rk,
    const int32_t *__restrict__ hv, const int32_t *__restrict__ perm, int64_t h,
    const int64_t *__restrict__ hoff, int32_t *__restrict__ hcols, int32_t *__restrict__ hlen,
    int32_t *__restrict__ est, int32_t *overflow) {
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + wave_in_block();
  const int64_t nw = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t j = gw; j < h; j += nw) {
    const int32_t x = hv[j];
    const int64_t cap = hoff[j + 1] - hoff[j];
    int32_t *row = hcols + hoff[j];
    const int64_t b = off[x], e = off[x + 1];
    int64_t done = 0;
    for (int64_t j0 = b; j0 < e; j0 += (int64_t)kUnroll * kWave) {
      int32_t w[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int64_t k = j0 + u * kWave + lane_id();
        w[u] = k < e ? cols[k] : -1;
      }
      uint2 word[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) word[u] = w[u] >= 0 ? rk[w[u] >> 5] : make_uint2(0, 0);
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const bool on = w[u] >= 0 && ((word[u].x >> (w[u] & 31)) & 1u);
        const uint64_t mask = __ballot(on);
        const int64_t r = done + (int64_t)__popcll(mask & lanemask_lt());
        if (on && r < cap) row[r] = perm[id_rank(word[u], w[u])];
        done += (int64_t)__popcll(mask);
      }
    }
    if (ins_head != nullptr) {
      // inserted edges: lane 0 walks the list
      int64_t extra = 0;
      if (lane_id() == 0) {
        for (int q = ins_head[x]; q >= 0; q = ins_next[q]) {
          const int32_t w = ins_other[q];
          const uint2 word = w >= 0 ? rk[w >> 5] : make_uint2(0, 0);
          if (w >= 0 && ((word.x >> (w & 31)) & 1u)) {
            if (done + extra < cap) row[done + extra] = perm[id_rank(word, w)];
            ++extra;
          }
        }
      }
      done += __shfl(extra, 0, kWave);
    }
    if (lane_id() == 0) {
      if (done > cap) atomicExch(overflow, 1);
      const int32_t d = (int32_t)std::min<int64_t>(done, cap);
      hlen[j] = d;
      est[j] = d;
    }
  }
}

// The same rows built in id ranges of the other layer, one range per XCD.
// A neighbour's rank word and local id are random reads; in one walk every
// XCD reads all of rk and perm (17.5 MB and 3 MB at 10^9 edges), more than
// its 4 MB L2, while a range's slice of each fits.  Workgroup b takes range
// b % kParts (the dispatcher deals workgroups to the XCDs in turn; any
// other placement is still correct, only slower).  Needs rows sorted by
// neighbour id with no tombstones and no inserted edges: a graph unchanged
// since the build.
constexpr int kParts = 8;
// Rows of fewer entries on average are filled by one walk each: a range of
// a short row is a few entries behind a chain of dependent loads (at 48
// entries per row the ranges took 3.4 ms where the row walk took 0.6 ms;
// at 1,190 they took 8.9 ms where it took 11.6 ms).
constexpr int kPartsMinRow = 512;

// pos[j * (kParts + 1) + p]: the CSR position of row j's first entry in
// range p (ranges of span ids over the other layer; entry kParts is the
// row's end).  One wave per row; lane p binary-searches range p's start.
__global__ __launch_bounds__(kBlock) void top_bounds_kernel(
    const int64_t *__restrict__ off, const int32_t *__restrict__ cols,
    const int32_t *__restrict__ hv, int64_t h, int32_t nU, int32_t spanU, int32_t spanL,
    int64_t *__restrict__ pos) {
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + wave_in_block();
  const int64_t nw = (int64_t)gridDim.x * kWavesPerBlock;
  const int lane = lane_id();
  for (int64_t j = gw; j < h; j += nw) {
    if (lane > kParts) continue;
    const int32_t x = hv[j];
    const int64_t b = off[x], e = off[x + 1];
    int64_t lo = b;
    if (lane == kParts) {
      lo = e;
    } else if (lane > 0) {
      // upper rows hold lower ids [nU, n), lower rows upper ids [0, nU)
      const int64_t first = x < nU ? (int64_t)nU + (int64_t)lane * spanL : (int64_t)lane * spanU;
      int64_t hi = e;
      while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if ((int64_t)cols[mid] < first)
          lo = mid + 1;
        else
          hi = mid;
      }
    }
    pos[j * (kParts + 1) + lane] = lo;
  }
}

// Row j's live neighbours in range p as local ids, appended to the row in
// any order (the h-index phase reads a row as a set): one reservation on
// hlen[j] per step of kUnroll x 64 entries.  hlen starts at zero; the
// entries past the row's capacity are counted, not written.
__global__ __launch_bounds__(kBlock) void top_fill_parts_kernel(
    const int32_t *__restrict__ cols, const uint2 *__restrict__ rk,
    const int32_t *__restrict__ perm, int64_t h, const int64_t *__restrict__ pos,
    const int64_t *__restrict__ hoff, int32_t *__restrict__ hcols, int32_t *__restrict__ hlen) {
  const int part = (int)(blockIdx.x % kParts);
  const int64_t gw = (int64_t)(blockIdx.x / kParts) * kWavesPerBlock + wave_in_block();
  const int64_t nw = (int64_t)(gridDim.x / kParts) * kWavesPerBlock;
  for (int64_t j = gw; j < h; j += nw) {
    const int64_t b = pos[j * (kParts + 1) + part], e = pos[j * (kParts + 1) + part + 1];
    const int64_t r0 = hoff[j], cap = hoff[j + 1] - r0;
    int32_t *row = hcols + r0;
    for (int64_t j0 = b; j0 < e; j0 += (int64_t)kUnroll * kWave) {
      int32_t w[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int64_t k = j0 + u * kWave + lane_id();
        w[u] = k < e ? cols[k] : -1;
      }
      uint2 word[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) word[u] = w[u] >= 0 ? rk[w[u] >> 5] : make_uint2(0, 0);
      uint64_t mask[kUnroll];
      int total = 0;
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        mask[u] = __ballot(w[u] >= 0 && ((word[u].x >> (w[u] & 31)) & 1u));
        total += (int)__popcll(mask[u]);
      }
      if (total == 0) continue;
      int at = 0;
      if (lane_id() == 0) at = atomicAdd(&hlen[j], total);
      int64_t r = __shfl(at, 0, kWave);
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const bool on = (mask[u] >> lane_id()) & 1ull;
        const int64_t q = r + (int64_t)__popcll(mask[u] & lanemask_lt());
        if (on && q < cap) row[q] = perm[id_rank(word[u], w[u])];
        r += (int64_t)__popcll(mask[u]);
      }
    }
  }
}

// Row lengths after top_fill_parts_kernel: clamped to the capacity (a
// longer row sets *overflow), and the starting values.
__global__ void top_len_kernel(const int64_t *__restrict__ hoff, int64_t h,
                               int32_t *__restrict__ hlen, int32_t *__restrict__ est,
                               int32_t *overflow) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < h; j += stride) {
    const int64_t cap = hoff[j + 1] - hoff[j];
    int32_t d = hlen[j];
    if (d > cap) {
      atomicExch(overflow, 1);
      d = (int32_t)cap;
    }
    hlen[j] = d;
    est[j] = d;
  }
}

struct HalfArgs {
  const int64_t *hoff;
  const int32_t *hlen;
  const int32_t *hcols;
  int32_t *est;  // current values, by local id
  int32_t *cnt;  // c(x): neighbours whose value is >= est(x)
  int32_t k0;
  int32_t tgt_base, tgt_cnt;  // the layer the rows read (fixed during the half)
  // the vertices to recompute, in their layer's buffer of cap_in slots:
  // rows of at most kLongRow entries from the front (len_in[0] of them),
  // longer rows from the back (len_in[1])
  const int32_t *q_in;
  const int32_t *len_in;
  int32_t cap_in;
  int propagate;  // lowered vertices decrement their neighbours' counts
  int spec;       // every listed vertex is due (it drops): see hindex_wave
};

#ifndef ABC_TOP_LDS_BARRIER
#define ABC_TOP_LDS_BARRIER 1
#endif
// A workgroup barrier that orders LDS only: the half kernel's barriers
// guard LDS words, and its global writes (decrements, values) are read by
// later kernels only, so no wave waits here for its global memory traffic.
__device__ __forceinline__ void lds_barrier() {
#if ABC_TOP_LDS_BARRIER
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
#else
  __syncthreads();
#endif
}

// Decrements of c(w).  Many rows that drop in one half share their most
// referenced neighbours, whose counts would take every one of those
// decrements on one address in turn; the long-row phase sums them per
// workgroup in LDS (agg, 16-bit sums for the first nagg local ids of the
// layer the rows read) and adds each sum once.
struct Dec {
  int32_t *cnt;
  int32_t base;
  uint32_t *agg;
  int nagg;
  __device__ __forceinline__ void operator()(int32_t w) const {
    const uint32_t r = (uint32_t)(w - base);
    if (r < (uint32_t)nagg)
      atomicAdd(&agg[r >> 1], 1u << ((r & 1) * 16));
    else
      (void)__hip_atomic_fetch_add(&cnt[w], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};

// x lowered from cur to h: its neighbour w valued v with cur >= v > h no
// longer counts toward c(w).  No value is returned (nothing waits): which
// vertices became due is read from the counts before the next half.
__device__ __forceinline__ void uncount(const Dec &dec, int32_t w, int32_t v, int32_t cur,
                                        int32_t h) {
  if (v <= cur && v > h) dec(w);
}

// One pass of the binned h-index search over [lo, hi]: values above hi are
// counted, the kFine integers just below hi get one bin each, the rest of
// the range [lo, fine_lo) kCoarse equal-width bins.
struct Pass {
  int32_t lo, hi, fine_lo, width;
  int nb;
};

__device__ __forceinline__ Pass pass_of(int32_t lo, int32_t hi) {
  Pass p;
  p.lo = lo;
  p.hi = hi;
  p.fine_lo = max(lo, hi - kFine + 1);
  const int64_t nco = (int64_t)p.fine_lo - lo;
  p.width = nco > 0 ? (int32_t)((nco + kCoarse - 1) / kCoarse) : 1;
  p.nb = nco > 0 ? (int)((nco + p.width - 1) / p.width) : 0;
  return p;
}

__device__ __forceinline__ void bin_value(const Pass &p, int32_t v, uint32_t *bins) {
  if (v <= p.hi && v >= p.fine_lo)
    atomicAdd(&bins[v - p.fine_lo], 1u);
  else if (v < p.fine_lo && v >= p.lo)
    atomicAdd(&bins[kFine + (v - p.lo) / p.width], 1u);
}

// After a pass (one wave): true and *res = the largest h in [lo, hi] with
// count_ge(h) >= h if it lies among the unit bins, else false and the
// highest coarse bin whose lower edge e has count_ge(e) >= e: the answer's
// range [*res, *nhi] for the next pass (count_ge(lo) >= lo must hold, which
// makes some bin qualify).  *c receives count_ge(*res).
__device__ bool scan_bins(const Pass &p, const uint32_t *bins, int64_t above, int32_t *res,
                          int32_t *nhi, int64_t *c) {
  const uint32_t *fine = bins, *coarse = bins + kFine;
  // unit bins from hi down: lane L at t = top - L; counts by an inclusive
  // wave scan; the first t (from the top) with count >= t wins
  int64_t acc = above;
  for (int32_t top = p.hi; top >= p.fine_lo; top -= kWave) {
    const int32_t t = top - lane_id();
    int64_t incl = t >= p.fine_lo ? (int64_t)fine[t - p.fine_lo] : 0;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int64_t y = __shfl_up(incl, o, kWave);
      if (lane_id() >= o) incl += y;
    }
    const uint64_t ok = __ballot(t >= p.fine_lo && acc + incl >= (int64_t)t);
    if (ok) {
      const int l = __ffsll((unsigned long long)ok) - 1;
      *res = top - l;
      *nhi = *res;
      *c = acc + __shfl(incl, l, kWave);
      return true;
    }
    acc += __shfl(incl, kWave - 1, kWave);
  }
  // coarse bins from the top: bin i covers [lo + i * width, lo + (i + 1) * width)
  for (int topb = p.nb - 1; topb >= 0; topb -= kWave) {
    const int bi = topb - lane_id();
    int64_t incl = bi >= 0 ? (int64_t)coarse[bi] : 0;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int64_t y = __shfl_up(incl, o, kWave);
      if (lane_id() >= o) incl += y;
    }
    const int64_t edge = (int64_t)p.lo + (int64_t)bi * p.width;
    const uint64_t ok = __ballot(bi >= 0 && acc + incl >= edge);
    if (ok) {
      const int l = __ffsll((unsigned long long)ok) - 1;
      *res = p.lo + (topb - l) * p.width;
      *nhi = min(*res + p.width - 1, p.fine_lo - 1);
      *c = acc + __shfl(incl, l, kWave);
      return *res == *nhi;
    }
    acc += __shfl(incl, kWave - 1, kWave);
  }
  *res = p.lo;  // not reached while count_ge(lo) >= lo
  *nhi = p.lo;
  *c = acc;
  return true;
}

// The search for a row walked by one wave, in passes that reread the row.
// Two passes cover ranges up to kFine + kFine * kCoarse; more take more.
// spec (a vertex known to drop, below cur = hi): the first pass already
// takes it out of the counts of its neighbours valued exactly cur.
template <class V>
__device__ int32_t hindex_wave(const int32_t *__restrict__ hcols, int64_t b, int64_t e,
                               int32_t lo, int32_t hi, uint32_t *bins, V val, int64_t *c,
                               const Dec *spec) {
  const int32_t cur = hi;
  for (bool first = true;; first = false) {
    const Pass p = pass_of(lo, hi);
    for (int i = lane_id(); i < kFine + kCoarse; i += kWave) bins[i] = 0;
    __builtin_amdgcn_wave_barrier();
    int64_t above = 0;
    for (int64_t k0i = b; k0i < e; k0i += (int64_t)kUnroll * kWave) {
      int32_t w[kUnroll], v[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int64_t k = k0i + u * kWave + lane_id();
        w[u] = k < e ? hcols[k] : -1;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) v[u] = w[u] >= 0 ? val(w[u]) : INT32_MIN;
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        above += (int64_t)__popcll(__ballot(v[u] > p.hi));
        bin_value(p, v[u], bins);
        if (first && spec != nullptr && v[u] == cur) (*spec)(w[u]);
      }
    }
    __builtin_amdgcn_wave_barrier();
    int32_t res, nhi;
    const bool exact = scan_bins(p, bins, above, &res, &nhi, c);
    __builtin_amdgcn_wave_barrier();
    if (exact) return res;
    lo = res;
    hi = nhi;
  }
}

struct BlockShared {
  uint32_t above;
  int32_t res, nhi;
  int exact;
  int64_t c;
};

// The same search for a long row walked by the whole workgroup (bins shared
// by its waves, scanned by wave 0; spec as above).  Every thread calls it.
template <class V>
__device__ int32_t hindex_block(const int32_t *__restrict__ hcols, int64_t b, int64_t e,
                                int32_t lo, int32_t hi, uint32_t *bins, BlockShared &sh, V val,
                                int64_t *c, const Dec *spec) {
  const int32_t cur = hi;
  for (bool first = true;; first = false) {
    const Pass p = pass_of(lo, hi);
    for (int i = threadIdx.x; i < kFine + kCoarse; i += blockDim.x) bins[i] = 0;
    if (threadIdx.x == 0) sh.above = 0;
    lds_barrier();
    uint32_t above = 0;
    for (int64_t k0i = b; k0i < e; k0i += (int64_t)kUnrollBlock * kHalfBlock) {
      int32_t w[kUnrollBlock], v[kUnrollBlock];
#pragma unroll
      for (int u = 0; u < kUnrollBlock; ++u) {
        const int64_t k = k0i + u * kHalfBlock + threadIdx.x;
        w[u] = k < e ? hcols[k] : -1;
      }
#pragma unroll
      for (int u = 0; u < kUnrollBlock; ++u) v[u] = w[u] >= 0 ? val(w[u]) : INT32_MIN;
#pragma unroll
      for (int u = 0; u < kUnrollBlock; ++u) {
        above += (uint32_t)__popcll(__ballot(v[u] > p.hi));
        bin_value(p, v[u], bins);
        if (first && spec != nullptr && v[u] == cur) (*spec)(w[u]);
      }
    }
    if (lane_id() == 0 && above) atomicAdd(&sh.above, above);
    lds_barrier();
    if (wave_in_block() == 0) {
      int32_t res, nhi;
      int64_t cc;
      const bool exact = scan_bins(p, bins, (int64_t)sh.above, &res, &nhi, &cc);
      if (lane_id() == 0) {
        sh.res = res;
        sh.nhi = nhi;
        sh.exact = exact;
        sh.c = cc;
      }
    }
    lds_barrier();
    const bool exact = sh.exact != 0;
    const int32_t res = sh.res, nhi = sh.nhi;
    const int64_t cc = sh.c;
    lds_barrier();  // the next pass rewrites the shared words
    if (exact) {
      *c = cc;
      return res;
    }
    lo = res;
    hi = nhi;
  }
}

// One half sweep (see the file comment).  One workgroup per compute unit
// (the LDS holds the value cache and the bins): first the long rows, one
// per workgroup at a time, then the others, one per wave.
__global__ __launch_bounds__(kHalfBlock) void hindex_half_kernel(HalfArgs a) {
  __shared__ uint16_t cache[kCache];
  __shared__ uint32_t s_bins[kHalfWaves][kFine + kCoarse];
  __shared__ BlockShared sh;
  const int64_t n_short = a.len_in[0], n_long = a.len_in[1];
  if (blockIdx.x >= n_long && (int64_t)blockIdx.x * kHalfWaves >= n_short) return;  // idle
  const int kc = min(kCache, a.tgt_cnt);
  for (int i = threadIdx.x; i < kc; i += blockDim.x)
    cache[i] = (uint16_t)min(a.est[a.tgt_base + i] - a.k0, 65535);
  lds_barrier();
  const int32_t k0 = a.k0;
  // cached values are offsets from k0 saturated at 65535: exact for every
  // comparison with thresholds <= cur while cur - k0 < 65535
  auto make_val = [&](int32_t cur) {
    const int kcr = cur - k0 < 65535 ? kc : 0;
    return [&, kcr](int32_t w) -> int32_t {
      const uint32_t r = (uint32_t)(w - a.tgt_base);
      return r < (uint32_t)kcr ? (int32_t)cache[r] + k0 : a.est[w];
    };
  };
  // long rows: decrements of the first kAgg ids summed in the bins of
  // waves 1.. (wave 0's bins serve the search), flushed before the short rows
  const bool have_long = blockIdx.x < n_long;
  uint32_t *agg = s_bins[1];
  // (a 16-bit sum cannot wrap: at most 65535 rows per workgroup, else no sums)
  const int nagg = n_long <= (int64_t)65535 * gridDim.x ? min(kAgg, a.tgt_cnt) : 0;
  if (have_long) {
    for (int i = threadIdx.x; i < (nagg + 1) / 2; i += blockDim.x) agg[i] = 0;
    lds_barrier();
  }
  const Dec dec_long{a.cnt, a.tgt_base, agg, nagg};
  const Dec dec_short{a.cnt, a.tgt_base, nullptr, 0};
  // a row's vertex, value and extent are loaded one row ahead (the vertex
  // two ahead), off the chain of dependent loads of the row in hand
  auto long_vertex = [&](int64_t i) { return i < n_long ? a.q_in[a.cap_in - 1 - i] : 0; };
  const int64_t step = gridDim.x;
  int32_t x_next = long_vertex(blockIdx.x);
  int32_t x_after = long_vertex(blockIdx.x + step);
  int32_t cur_next = a.est[x_next];
  int64_t b_next = a.hoff[x_next], d_next = a.hlen[x_next];
  for (int64_t i = blockIdx.x; i < n_long; i += step) {
    const int32_t x = x_next, cur = cur_next;
    const int64_t b = b_next, e = b + d_next;
    x_next = x_after;
    x_after = long_vertex(i + 2 * step);
    cur_next = a.est[x_next];
    b_next = a.hoff[x_next];
    d_next = a.hlen[x_next];
    const auto val = make_val(cur);
    int64_t c = 0;
    const Dec *spec = a.spec ? &dec_long : nullptr;
    const int32_t h = hindex_block(a.hcols, b, e, k0, cur, s_bins[0], sh, val, &c, spec);
    // the neighbours valued cur are done if the first pass took them out
    const int32_t top = spec ? cur - 1 : cur;
    if (a.propagate && h < top) {
      for (int64_t k0i = b; k0i < e; k0i += (int64_t)kUnrollBlock * kHalfBlock) {
        int32_t w[kUnrollBlock], v[kUnrollBlock];
#pragma unroll
        for (int u = 0; u < kUnrollBlock; ++u) {
          const int64_t k = k0i + u * kHalfBlock + threadIdx.x;
          w[u] = k < e ? a.hcols[k] : -1;
        }
#pragma unroll
        for (int u = 0; u < kUnrollBlock; ++u) v[u] = w[u] >= 0 ? val(w[u]) : INT32_MIN;
#pragma unroll
        for (int u = 0; u < kUnrollBlock; ++u) uncount(dec_long, w[u], v[u], top, h);
      }
    }
    if (threadIdx.x == 0) {
      a.cnt[x] = (int32_t)min<int64_t>(c, 0x7FFFFFFF);
      if (h < cur) a.est[x] = h;
    }
  }
  if (have_long) {
    lds_barrier();
    for (int i = threadIdx.x; i < nagg; i += blockDim.x) {
      const uint32_t sum = (agg[i >> 1] >> ((i & 1) * 16)) & 0xFFFFu;
      if (sum != 0)
        (void)__hip_atomic_fetch_add(&a.cnt[a.tgt_base + i], -(int32_t)sum, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
    }
    lds_barrier();  // the short rows' bins reuse the sums' words
  }
  uint32_t *bins = s_bins[wave_in_block()];
  const int64_t nw = (int64_t)gridDim.x * kHalfWaves;
  for (int64_t i = (int64_t)blockIdx.x * kHalfWaves + wave_in_block(); i < n_short; i += nw) {
    const int32_t x = a.q_in[i];
    const int32_t cur = a.est[x];
    const int64_t b = a.hoff[x], d = a.hlen[x], e = b + d;
    const auto val = make_val(cur);
    int32_t h = cur;
    int64_t c = 0;
    if (d <= (int64_t)kRegSpan * kWave) {
      int32_t w[kRegSpan], v[kRegSpan];
#pragma unroll
      for (int u = 0; u < kRegSpan; ++u) {
        const int64_t k = b + u * kWave + lane_id();
        w[u] = k < e ? a.hcols[k] : -1;
      }
#pragma unroll
      for (int u = 0; u < kRegSpan; ++u) v[u] = w[u] >= 0 ? val(w[u]) : INT32_MIN;
      auto count_ge = [&](int32_t th) -> int64_t {
        int64_t n = 0;
#pragma unroll
        for (int u = 0; u < kRegSpan; ++u) n += (int64_t)__popcll(__ballot(v[u] >= th));
        return n;
      };
      c = count_ge(cur);
      if (c < cur) {
        // count_ge(x) >= x holds at k0 (H is the k0-core) and fails at cur
        int32_t lo = k0, hi = cur - 1;
        while (lo < hi) {
          const int32_t mid = lo + (hi - lo + 1) / 2;
          if (count_ge(mid) >= mid)
            lo = mid;
          else
            hi = mid - 1;
        }
        h = lo;
        c = count_ge(h);
      }
      if (a.propagate && h < cur) {
#pragma unroll
        for (int u = 0; u < kRegSpan; ++u) uncount(dec_short, w[u], v[u], cur, h);
      }
    } else {
      // the first pass also settles a row that does not drop (its answer
      // is cur, among the unit bins)
      const Dec *spec = a.spec ? &dec_short : nullptr;
      h = hindex_wave(a.hcols, b, e, k0, cur, bins, val, &c, spec);
      const int32_t top = spec ? cur - 1 : cur;
      if (a.propagate && h < top) {
        for (int64_t k0i = b; k0i < e; k0i += (int64_t)kUnroll * kWave) {
          int32_t w[kUnroll], v[kUnroll];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            const int64_t k = k0i + u * kWave + lane_id();
            w[u] = k < e ? a.hcols[k] : -1;
          }
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) v[u] = w[u] >= 0 ? val(w[u]) : INT32_MIN;
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) uncount(dec_short, w[u], v[u], top, h);
        }
      }
    }
    if (lane_id() == 0) {
      a.cnt[x] = (int32_t)min<int64_t>(c, 0x7FFFFFFF);
      if (h < cur) a.est[x] = h;
    }
  }
}

// The list of half t: the vertices of the layer [base, base + count) that
// are due (c(x) < est(x); c starts at 0, so the first half of each layer
// takes all), short rows from the front of the layer's buffer, long rows
// from its back; len[0] and len[1] receive their numbers.
__global__ __launch_bounds__(kBlock) void top_due_kernel(const int32_t *__restrict__ est,
                                                         const int32_t *__restrict__ cnt,
                                                         const int32_t *__restrict__ hlen,
                                                         int32_t base, int32_t count,
                                                         int32_t *__restrict__ list,
                                                         int32_t *len) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x; o < count; o += stride) {
    const int64_t i = o + threadIdx.x;
    const int32_t j = base + (int32_t)i;
    const bool due = i < count && cnt[j] < est[j];
    const bool lg = due && hlen[j] > kLongRow;
    const uint64_t ms = __ballot(due && !lg), ml = __ballot(lg);
    int bs = 0, bl = 0;
    if (lane_id() == 0) {
      if (ms) bs = atomicAdd(&len[0], (int)__popcll(ms));
      if (ml) bl = atomicAdd(&len[1], (int)__popcll(ml));
    }
    bs = __shfl(bs, 0, kWave);
    bl = __shfl(bl, 0, kWave);
    if (due) {
      // the two ends never meet: at most count vertices are due
      if (lg)
        list[count - 1 - (bl + (int)__popcll(ml & lanemask_lt()))] = j;
      else
        list[bs + (int)__popcll(ms & lanemask_lt())] = j;
    }
  }
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

// The phase's buffers stay with the handle for the next decomposition and
// grow when short, so a repeated decomposition allocates and frees nothing
// (freeing the gigabytes of one call cost about 4 ms at 10^9 edges).  A
// buffer that must grow is freed first; hipFree waits for the device.
template <class T>
hipError_t keep(Graph &g, int slot, T **p, size_t bytes) {
  bytes = std::max<size_t>(bytes, 16);
  if (g.top_cap[slot] < bytes) {
    if (g.top_buf[slot] != nullptr) {
      (void)dev_free(g.top_buf[slot]);
      g.top_buf[slot] = nullptr;
      g.top_cap[slot] = 0;
    }
    void *q = nullptr;
    const hipError_t e = dev_malloc_bytes(&q, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();  // the caller falls back; later checks must not see it
      *p = nullptr;
      return e;
    }
    g.top_buf[slot] = q;
    g.top_cap[slot] = bytes;
  }
  *p = static_cast<T *>(g.top_buf[slot]);
  return hipSuccess;
}

}  // namespace

// After the levels below k0 (every vertex of core < k0 has its value; the
// live ones of the alive list, `cnt` entries, are the k0-core): the core
// numbers of the live vertices by the h-index fixpoint.  *finished = false
// (and nothing changed) if it did not converge within max_halves half
// sweeps, so the caller can go on level by level.  Synchronous.
abcore_status kcore_top(Graph &g, const int32_t *alive, int64_t cnt, int32_t k0,
                        int max_halves, bool *finished, int32_t *top_max, hipStream_t s) {
  *finished = false;
  int32_t *perm = nullptr, *hv = nullptr, *hcols = nullptr, *est = nullptr, *ctr = nullptr;
  int64_t *wcount = nullptr, *wpre = nullptr;
  uint2 *rk = nullptr;
  int32_t *hlen = nullptr, *cntv = nullptr, *lists = nullptr, *list_len = nullptr;
  uint32_t *live = nullptr;
  uint64_t *keys = nullptr, *keys2 = nullptr;
  int64_t *cap = nullptr, *hoff = nullptr, *pos = nullptr;
  void *temp = nullptr;
  size_t temp_bytes = 0;
  int32_t hc[3] = {0, 0, 0};
  int64_t h = 0, eh = 0;
  abcore_status st = ABCORE_EDEVICE;
  const char *why = "core numbers: the h-index phase failed";
  const int32_t *ih = g.delta.count > 0 ? g.delta.head : nullptr;
  const int halves_per_check = 16;
  const int64_t words = (g.n + 31) / 32;
  auto ok = [](hipError_t e) { return e == hipSuccess; };
  do {
    // ctr: [0] live count, [1] upper-layer count, [2] overflow, [3] maximum
    if (!ok(keep(g, 0, &wcount, sizeof(int64_t) * (words + 1))) ||
        !ok(keep(g, 1, &wpre, sizeof(int64_t) * (words + 1))) ||
        !ok(keep(g, 2, &rk, sizeof(uint2) * std::max<int64_t>(words, 1))) ||
        !ok(keep(g, 3, &hv, sizeof(int32_t) * std::max<int64_t>(cnt, 1))) ||
        !ok(keep(g, 4, &live, sizeof(uint32_t) * std::max<int64_t>(words, 1))) ||
        !ok(keep(g, 5, &ctr, sizeof(int32_t) * 4)) ||
        !ok(keep(g, 6, &list_len, sizeof(int32_t) * 2 * (max_halves + 2)))) {
      st = ABCORE_ENOMEM;
      break;
    }
    if (!ok(hipMemsetAsync(ctr, 0, sizeof(int32_t) * 4, s)) ||
        !ok(hipMemsetAsync(list_len, 0, sizeof(int32_t) * 2 * (max_halves + 2), s)) ||
        !ok(hipMemsetAsync(live, 0, sizeof(uint32_t) * std::max<int64_t>(words, 1), s)))
      break;
    if (cnt > 0) {
      top_select_kernel<<<grid_of(g, cnt, kBlock), kBlock, 0, s>>>(alive, cnt, g.core, g.nU,
                                                                   hv, live, ctr);
      if (!ok(hipGetLastError())) break;
    }
    if (!ok(hipMemcpyAsync(hc, ctr, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, s)) ||
        !ok(hipStreamSynchronize(s)))
      break;
    h = hc[0];
    const int32_t hU = hc[1];
    if (!ok(keep(g, 7, &keys, sizeof(uint64_t) * std::max<int64_t>(h, 1))) ||
        !ok(keep(g, 8, &keys2, sizeof(uint64_t) * std::max<int64_t>(h, 1))) ||
        !ok(keep(g, 9, &cap, sizeof(int64_t) * (h + 1))) ||
        !ok(keep(g, 10, &hoff, sizeof(int64_t) * (h + 1))) ||
        !ok(keep(g, 11, &hlen, sizeof(int32_t) * std::max<int64_t>(h, 1))) ||
        !ok(keep(g, 12, &est, sizeof(int32_t) * std::max<int64_t>(h, 1))) ||
        !ok(keep(g, 13, &cntv, sizeof(int32_t) * std::max<int64_t>(h, 1))) ||
        !ok(keep(g, 14, &lists, sizeof(int32_t) * std::max<int64_t>(h, 1)))) {
      st = ABCORE_ENOMEM;
      break;
    }
    if (!ok(keep(g, 15, &perm, sizeof(int32_t) * std::max<int64_t>(h, 1)))) {
      st = ABCORE_ENOMEM;
      break;
    }
    // local ids: layer, then decreasing degree
    if (h > 0) {
      top_keys_kernel<<<grid_of(g, h, kBlock), kBlock, 0, s>>>(hv, h, g.deg0, g.nU, keys);
      if (!ok(hipGetLastError())) break;
    }
    size_t sort_bytes = 0, scan_bytes = 0, wscan_bytes = 0;
    if (!ok(prim::sort_keys(nullptr, sort_bytes, keys, keys2, (size_t)h, 0, 64, s)) ||
        !ok(prim::exclusive_sum(nullptr, scan_bytes, cap, hoff, (size_t)(h + 1), s)) ||
        !ok(prim::exclusive_sum(nullptr, wscan_bytes, wcount, wpre, (size_t)(words + 1), s)))
      break;
    temp_bytes = std::max<size_t>({sort_bytes, scan_bytes, wscan_bytes, 16});
    if (!ok(keep(g, 16, &temp, temp_bytes))) {
      st = ABCORE_ENOMEM;
      break;
    }
    // ranks of the live vertices in id order, read next to their bits
    top_word_count_kernel<<<grid_of(g, words + 1, kBlock), kBlock, 0, s>>>(live, words, wcount);
    size_t tb = temp_bytes;
    if (!ok(hipGetLastError()) ||
        !ok(prim::exclusive_sum(temp, tb, wcount, wpre, (size_t)(words + 1), s)))
      break;
    if (words > 0) {
      top_word_pack_kernel<<<grid_of(g, words, kBlock), kBlock, 0, s>>>(live, wpre, words, rk);
      if (!ok(hipGetLastError())) break;
    }
    tb = temp_bytes;
    if (h > 0 && !ok(prim::sort_keys(temp, tb, keys, keys2, (size_t)h, 0, 64, s))) break;
    top_place_kernel<<<grid_of(g, h + 1, kBlock), kBlock, 0, s>>>(keys2, h, g.deg0, rk, hv, perm,
                                                                   cap);
    if (!ok(hipGetLastError())) break;
    tb = temp_bytes;
    if (!ok(prim::exclusive_sum(temp, tb, cap, hoff, (size_t)(h + 1), s))) break;
    if (!ok(hipMemcpyAsync(&eh, hoff + h, sizeof(int64_t), hipMemcpyDeviceToHost, s)) ||
        !ok(hipStreamSynchronize(s)))
      break;
    if (!ok(keep(g, 17, &hcols, sizeof(int32_t) * std::max<int64_t>(eh, 1)))) {
      st = ABCORE_ENOMEM;
      break;
    }
    // rows by id ranges, one per XCD, on a graph unchanged since the build
    // (sorted rows) whose deep core's rows are long; otherwise, or without
    // room for the range bounds, one walk per row
    bool parts = false;
    if (ABC_TOP_FILL_PARTS && h > 0 && g.version == 0 && g.delta.count == 0 &&
        eh >= (int64_t)kPartsMinRow * h) {
      parts = ok(keep(g, 18, &pos, sizeof(int64_t) * h * (kParts + 1)));
      if (!parts) (void)hipGetLastError();  // the fallback needs no memory
    }
    if (parts) {
      const int64_t nU = g.nU, nL = g.n - g.nU;
      const int32_t spanU = (int32_t)(((nU + kParts - 1) / kParts + 31) / 32 * 32);
      const int32_t spanL = (int32_t)(((nL + kParts - 1) / kParts + 31) / 32 * 32);
      top_bounds_kernel<<<grid_of(g, h * kWave, kBlock), kBlock, 0, s>>>(
          g.off, g.cols, hv, h, g.nU, spanU, spanL, pos);
      if (!ok(hipGetLastError()) || !ok(hipMemsetAsync(hlen, 0, sizeof(int32_t) * h, s))) break;
      const int pg = std::max(kParts, grid_of(g, h * kWave * kParts, kBlock) / kParts * kParts);
      top_fill_parts_kernel<<<pg, kBlock, 0, s>>>(g.cols, rk, perm, h, pos, hoff, hcols, hlen);
      top_len_kernel<<<grid_of(g, h, kBlock), kBlock, 0, s>>>(hoff, h, hlen, est, ctr + 2);
      if (!ok(hipGetLastError())) break;
    } else if (h > 0) {
      top_fill_kernel<<<grid_of(g, h * kWave, kBlock), kBlock, 0, s>>>(
          g.off, g.cols, ih, g.delta.next, g.delta.other, rk, hv, perm, h, hoff, hcols, hlen,
          est, ctr + 2);
      if (!ok(hipGetLastError())) break;
    }
    // half sweeps: the upper layer first (all of it, no counts to keep yet),
    // then the lower layer (all of it, decrementing the upper layer's
    // counts), then the due vertices of each layer in turn; list_len[2t] and
    // list_len[2t + 1] count half t's short and long rows
    const int32_t hL = (int32_t)h - hU;
    if (h > 0 && !ok(hipMemsetAsync(cntv, 0, sizeof(int32_t) * h, s))) break;
    const int grid = std::max(1, std::min(g.cu_count, kMaxBlocks));
    int t = 0, fixed_at = -1;
    std::vector<int32_t> hq(2 * halves_per_check);
    bool failed = false;
    while (t < max_halves && fixed_at < 0 && h > 0) {
      const int t0 = t;
      for (int r = 0; r < halves_per_check && t < max_halves; ++r, ++t) {
        const bool upper = (t % 2) == 0;
        const int32_t self_base = upper ? 0 : hU, self_cnt = upper ? hU : hL;
        top_due_kernel<<<grid_of(g, self_cnt, kBlock), kBlock, 0, s>>>(
            est, cntv, hlen, self_base, self_cnt, lists + self_base, list_len + 2 * t);
        HalfArgs a{};
        a.hoff = hoff;
        a.hlen = hlen;
        a.hcols = hcols;
        a.est = est;
        a.cnt = cntv;
        a.k0 = k0;
        a.tgt_base = upper ? hU : 0;
        a.tgt_cnt = upper ? hL : hU;
        a.q_in = lists + self_base;
        a.len_in = list_len + 2 * t;
        a.cap_in = self_cnt;
        a.propagate = t >= 1;
        a.spec = t >= 2;  // from the third half on, a listed vertex is due
        hindex_half_kernel<<<grid, kHalfBlock, 0, s>>>(a);
      }
      if (!ok(hipGetLastError()) ||
          !ok(hipMemcpyAsync(hq.data(), list_len + 2 * t0, sizeof(int32_t) * 2 * (t - t0),
                             hipMemcpyDeviceToHost, s)) ||
          !ok(hipStreamSynchronize(s))) {
        failed = true;
        break;
      }
      // a half with nothing due after the first two: the fixpoint
      for (int r = 0; r < t - t0 && fixed_at < 0; ++r)
        if (t0 + r >= 2 && hq[2 * r] + hq[2 * r + 1] == 0) fixed_at = t0 + r - 1;
    }
    if (failed) break;
    int32_t flags[2] = {0, 0};
    if (!ok(hipMemcpyAsync(flags, ctr + 2, sizeof(int32_t), hipMemcpyDeviceToHost, s)) ||
        !ok(hipStreamSynchronize(s)))
      break;
    if (flags[0] != 0) {
      why = "core numbers: a row of the deep core exceeded its capacity";
      break;
    }
    if (h > 0 && fixed_at < 0) {
      st = ABCORE_OK;  // not converged: the caller continues level by level
      break;
    }
    g.top_stats[0] = k0;
    g.top_stats[1] = h;
    g.top_stats[2] = eh;
    g.top_stats[3] = fixed_at + 1;
    int32_t *dmax = ctr + 3;
    int32_t hmax = 0;
    if (h > 0) {
      top_write_kernel<<<grid_of(g, h, kBlock), kBlock, 0, s>>>(hv, est, h, g.core, dmax);
      if (!ok(hipGetLastError())) break;
    }
    if (!ok(hipMemcpyAsync(&hmax, dmax, sizeof(int32_t), hipMemcpyDeviceToHost, s)) ||
        !ok(hipStreamSynchronize(s)))
      break;
    *top_max = hmax;
    *finished = true;
    st = ABCORE_OK;
  } while (0);
  if (st == ABCORE_ENOMEM) set_error("core numbers: the h-index phase is out of memory");
  else if (st != ABCORE_OK) set_error("%s", why);
  return st;
}

}  // namespace abc
