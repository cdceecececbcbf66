// Device construction of the unified CSR (Sec. III: CSR storage; Sec. IV-A:
// contiguous ids, upper first).  Pairs are keyed (u*nL + v), radix-sorted
// and deduplicated (E is a set); the sorted keys give the upper rows
// directly, a second sort on (v*nU + u) gives the lower rows.  Both sorts are
// rocPRIM's device radix sort, called directly (prim.h); the build is
// preprocessing and is not part of the timed peel.
#include "prim.h"

#include <algorithm>

#include "abcore_internal.h"

namespace abc {

namespace {

__global__ void validate_kernel(const int32_t *__restrict__ eu, const int32_t *__restrict__ ev,
                                int64_t m, int32_t nU, int32_t nL, int32_t *bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int found = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    const int32_t u = eu[i], v = ev[i];
    found |= (u < 0 || u >= nU || v < 0 || v >= nL);
  }
  if (__ballot(found) != 0 && (threadIdx.x & 63) == 0) atomicOr(bad, 1);
}

__global__ void make_keys_kernel(const int32_t *__restrict__ eu, const int32_t *__restrict__ ev,
                                 int64_t m, int32_t nL, uint64_t *__restrict__ keys) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride)
    keys[i] = (uint64_t)(uint32_t)eu[i] * (uint64_t)nL + (uint64_t)(uint32_t)ev[i];
}

// Counts one per valid lane into deg[row] where the lanes of a wave hold
// sorted rows (the valid lanes a prefix of the wave): one atomic per run of
// equal rows, so that a hub's entries do not queue on one address.
__device__ __forceinline__ void add_row_runs(int32_t *deg, int32_t row, bool ok) {
  const int lane = (int)(threadIdx.x % kWave);
  const int32_t prev = __shfl_up(row, 1, kWave);
  const bool start = ok && (lane == 0 || prev != row);
  const uint64_t starts = __ballot(start);
  const int nvalid = __popcll(__ballot(ok));
  if (start) {
    const uint64_t above = lane == kWave - 1 ? 0ull : (starts >> (lane + 1)) << (lane + 1);
    const int end = above ? __builtin_ctzll(above) : nvalid;
    atomicAdd(&deg[row], end - lane);
  }
}

// Upper side: unique key i = (u, v) -> cols[i] = nU + v; upper degrees; and
// the transposed key (v*nU + u) for the lower rows.  (Wave-uniform loop.)
__global__ void upper_rows_kernel(const uint64_t *__restrict__ ukeys, int64_t md, int32_t nU,
                                  int32_t nL, int32_t *__restrict__ cols,
                                  int32_t *__restrict__ deg, uint64_t *__restrict__ tkeys) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x / kWave) * kWave; b < md;
       b += stride) {
    const int64_t i = b + (int64_t)(threadIdx.x % kWave);
    const bool ok = i < md;
    int32_t u = 0;
    if (ok) {
      const uint64_t k = ukeys[i];
      u = (int32_t)(k / (uint64_t)nL);
      const int32_t v = (int32_t)(k % (uint64_t)nL);
      cols[i] = nU + v;
      tkeys[i] = (uint64_t)(uint32_t)v * (uint64_t)nU + (uint64_t)(uint32_t)u;
    }
    add_row_runs(deg, u, ok);
  }
}

// Lower side: keys sorted by (v, u) -> cols[md + i] = u; lower degrees.
__global__ void lower_rows_kernel(const uint64_t *__restrict__ lkeys, int64_t md, int32_t nU,
                                  int32_t *__restrict__ cols, int32_t *__restrict__ deg) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x / kWave) * kWave; b < md;
       b += stride) {
    const int64_t i = b + (int64_t)(threadIdx.x % kWave);
    const bool ok = i < md;
    int32_t v = 0;
    if (ok) {
      const uint64_t k = lkeys[i];
      cols[md + i] = (int32_t)(k % (uint64_t)nU);
      v = (int32_t)(k / (uint64_t)nU);
    }
    add_row_runs(deg + nU, v, ok);
  }
}

__global__ void widen_kernel(const int32_t *__restrict__ deg, int64_t n,
                             int64_t *__restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += stride)
    out[i] = i < n ? (int64_t)deg[i] : 0;
}

// Piece counts of every row (rows longer than kPiece entries are split) and
// split-row flags, each followed by a zero so an exclusive scan yields the
// totals in the last slot.
__global__ void count_pieces_kernel(const int64_t *__restrict__ off, int64_t n,
                                    int64_t *__restrict__ np, int64_t *__restrict__ hv) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= n; x += stride) {
    const int64_t d = x < n ? off[x + 1] - off[x] : 0;
    np[x] = d > kPiece ? (d + kPiece - 1) / kPiece : 0;
    hv[x] = d > kPiece ? 1 : 0;
  }
}

__global__ void fill_pieces_kernel(const int64_t *__restrict__ off, int64_t n,
                                   const int64_t *__restrict__ first,
                                   const int64_t *__restrict__ hfirst,
                                   int32_t *__restrict__ piece_row,
                                   int64_t *__restrict__ piece_start,
                                   int32_t *__restrict__ piece_first,
                                   int32_t *__restrict__ heavy_rows) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride) {
    const int64_t d = off[x + 1] - off[x];
    if (d > kPiece) {
      const int64_t f = first[x];
      const int64_t np = (d + kPiece - 1) / kPiece;
      piece_first[x] = (int32_t)f;
      heavy_rows[hfirst[x]] = (int32_t)x;
      for (int64_t k = 0; k < np; ++k) {
        piece_row[f + k] = (int32_t)x;
        piece_start[f + k] = off[x] + k * kPiece;
      }
    } else {
      piece_first[x] = -1;
    }
  }
}

// Weight of a row in the pull round: its entries when it is walked as a row
// (a split row is walked by its pieces) plus a fixed cost per row.
constexpr int64_t kRowCost = 4;
__global__ void row_weight_kernel(const int64_t *__restrict__ off, int64_t n,
                                  int64_t *__restrict__ w) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= n; x += stride) {
    const int64_t d = x < n ? off[x + 1] - off[x] : 0;
    w[x] = x < n ? (d <= kPiece ? d : 0) + kRowCost : 0;
  }
}

// Bound k of layer p (0 upper, 1 lower): the first row of the layer whose
// exclusive weight prefix reaches k/G of the layer's weight.  The prefix is
// strictly increasing (every row costs at least kRowCost), so bound 0 and
// bound G are the layer's first row and its end.
__global__ void pull_bounds_kernel(const int64_t *__restrict__ pre, int64_t nU, int64_t n, int G,
                                   int32_t *__restrict__ bounds) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * (G + 1)) return;
  const int p = t / (G + 1), k = t % (G + 1);
  int64_t lo = p == 0 ? 0 : nU, hi = p == 0 ? nU : n;
  const int64_t base = pre[lo];
  const int64_t target = base + (pre[hi] - base) * k / G;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (pre[mid] >= target)
      hi = mid;
    else
      lo = mid + 1;
  }
  bounds[t] = (int32_t)lo;
}

int bits_for(uint64_t maxkey) {
  int b = 0;
  while (b < 64 && (maxkey >> b) != 0) ++b;
  return std::max(b, 1);
}

}  // namespace

// Builds off/cols/deg0 of g (already sized: g.nU, g.nL, g.n set; arrays not
// yet allocated).  Returns a status and sets the error message.
abcore_status build_csr_device(Graph &g, const int32_t *eu, const int32_t *ev, int64_t m,
                               hipStream_t s) {
#define BCHK(x)                                                                     \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) {                                                         \
      set_error("CSR build: %s failed: %s", #x, hipGetErrorString(e_));             \
      status = (e_ == hipErrorOutOfMemory) ? ABCORE_ENOMEM : ABCORE_EDEVICE;        \
      goto done;                                                                    \
    }                                                                               \
  } while (0)
  abcore_status status = ABCORE_OK;
  const int grid = std::max(1, std::min(g.cu_count * 8, (int)((m + 255) / 256)));
  int32_t *d_bad = nullptr;
  uint64_t *k0 = nullptr, *k1 = nullptr;
  int *d_nsel = nullptr;
  void *temp = nullptr;
  size_t temp_bytes = 0, need = 0;
  int64_t *deg64 = nullptr;
  int32_t h_bad = 0;
  int h_nsel = 0;
  int64_t md = 0;
  const int ubits = bits_for((uint64_t)std::max(g.nU, 1) * (uint64_t)std::max(g.nL, 1) - 1);
  const int lbits = ubits;

  BCHK(dev_malloc(&g.off, sizeof(int64_t) * (g.n + 1)));
  BCHK(dev_malloc(&g.deg0, sizeof(int32_t) * std::max<int64_t>(g.n, 1)));
  BCHK(hipMemsetAsync(g.deg0, 0, sizeof(int32_t) * std::max<int64_t>(g.n, 1), s));
  if (m > 0) {
    BCHK(dev_malloc_async(&d_bad, sizeof(int32_t), s));
    BCHK(hipMemsetAsync(d_bad, 0, sizeof(int32_t), s));
    validate_kernel<<<grid, 256, 0, s>>>(eu, ev, m, g.nU, g.nL, d_bad);
    BCHK(hipGetLastError());
    BCHK(hipMemcpyAsync(&h_bad, d_bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BCHK(hipStreamSynchronize(s));
    if (h_bad) {
      set_error("abcore_build_csr: edge endpoint out of range");
      status = ABCORE_EINVAL;
      goto done;
    }
    BCHK(dev_malloc_async(&k0, sizeof(uint64_t) * m, s));
    BCHK(dev_malloc_async(&k1, sizeof(uint64_t) * m, s));
    BCHK(dev_malloc_async(&d_nsel, sizeof(int), s));
    make_keys_kernel<<<grid, 256, 0, s>>>(eu, ev, m, g.nL, k0);
    BCHK(hipGetLastError());
    // temp storage large enough for the sort and the unique selection
    BCHK(prim::sort_keys(nullptr, need, k0, k1, (size_t)m, 0, ubits, s));
    temp_bytes = std::max(temp_bytes, need);
    BCHK(prim::unique(nullptr, need, k1, k0, d_nsel, (size_t)m, s));
    temp_bytes = std::max(temp_bytes, need);
    BCHK(dev_malloc_async(&temp, std::max<size_t>(temp_bytes, 16), s));
    BCHK(prim::sort_keys(temp, temp_bytes, k0, k1, (size_t)m, 0, ubits, s));
    BCHK(prim::unique(temp, temp_bytes, k1, k0, d_nsel, (size_t)m, s));
    BCHK(hipMemcpyAsync(&h_nsel, d_nsel, sizeof(int), hipMemcpyDeviceToHost, s));
    BCHK(hipStreamSynchronize(s));
    md = h_nsel;
  }
  g.m_csr = md;
  g.m = md;
  BCHK(dev_malloc(&g.cols, sizeof(int32_t) * std::max<int64_t>(2 * md, 1)));
  if (md > 0) {
    const int gridm = std::max(1, std::min(g.cu_count * 8, (int)((md + 255) / 256)));
    upper_rows_kernel<<<gridm, 256, 0, s>>>(k0, md, g.nU, g.nL, g.cols, g.deg0, k1);
    BCHK(hipGetLastError());
    BCHK(prim::sort_keys(temp, temp_bytes, k1, k0, (size_t)md, 0, lbits, s));
    lower_rows_kernel<<<gridm, 256, 0, s>>>(k0, md, g.nU, g.cols, g.deg0);
    BCHK(hipGetLastError());
  }
  BCHK(dev_malloc_async(&deg64, sizeof(int64_t) * (g.n + 1), s));
  {
    const int gridn = std::max(1, std::min(g.cu_count * 8, (int)((g.n + 256) / 256)));
    widen_kernel<<<gridn, 256, 0, s>>>(g.deg0, g.n, deg64);
    BCHK(hipGetLastError());
    need = 0;
    BCHK(prim::exclusive_sum(nullptr, need, deg64, g.off, (size_t)(g.n + 1), s));
    if (need > temp_bytes) {
      BCHK(dev_free_async(temp, s));
      temp = nullptr;
      temp_bytes = need;
      BCHK(dev_malloc_async(&temp, temp_bytes, s));
    }
    BCHK(prim::exclusive_sum(temp, temp_bytes, deg64, g.off, (size_t)(g.n + 1), s));
  }
  BCHK(hipStreamSynchronize(s));
done:
  for (void *p : {(void *)d_bad, (void *)k0, (void *)k1, (void *)d_nsel, temp, (void *)deg64})
    if (p) (void)dev_free_async(p, s);
  return status;
#undef BCHK
}

// Splits rows longer than kPiece entries into pieces (see Graph).
abcore_status build_pieces(Graph &g, hipStream_t s) {
#define PCHK(x)                                                                     \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) {                                                         \
      set_error("piece build: %s failed: %s", #x, hipGetErrorString(e_));           \
      status = (e_ == hipErrorOutOfMemory) ? ABCORE_ENOMEM : ABCORE_EDEVICE;        \
      goto done;                                                                    \
    }                                                                               \
  } while (0)
  abcore_status status = ABCORE_OK;
  int64_t *np = nullptr, *hv = nullptr, *first = nullptr, *hfirst = nullptr;
  void *temp = nullptr;
  size_t temp_bytes = 0;
  int64_t h_tot[4] = {0, 0, 0, 0};
  const int grid = std::max(1, std::min(g.cu_count * 8, (int)((g.n + 256) / 256)));
  PCHK(dev_malloc_async(&np, sizeof(int64_t) * (g.n + 1), s));
  PCHK(dev_malloc_async(&hv, sizeof(int64_t) * (g.n + 1), s));
  PCHK(dev_malloc_async(&first, sizeof(int64_t) * (g.n + 1), s));
  PCHK(dev_malloc_async(&hfirst, sizeof(int64_t) * (g.n + 1), s));
  count_pieces_kernel<<<grid, 256, 0, s>>>(g.off, g.n, np, hv);
  PCHK(hipGetLastError());
  PCHK(prim::exclusive_sum(nullptr, temp_bytes, np, first, (size_t)(g.n + 1), s));
  PCHK(dev_malloc_async(&temp, std::max<size_t>(temp_bytes, 16), s));
  PCHK(prim::exclusive_sum(temp, temp_bytes, np, first, (size_t)(g.n + 1), s));
  PCHK(prim::exclusive_sum(temp, temp_bytes, hv, hfirst, (size_t)(g.n + 1), s));
  PCHK(hipMemcpyAsync(&h_tot[0], first + g.n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  PCHK(hipMemcpyAsync(&h_tot[1], first + g.nU, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  PCHK(hipMemcpyAsync(&h_tot[2], hfirst + g.n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  PCHK(hipMemcpyAsync(&h_tot[3], hfirst + g.nU, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  PCHK(hipStreamSynchronize(s));
  g.npieces = h_tot[0];
  g.npieces_upper = h_tot[1];
  g.nheavy = h_tot[2];
  g.nheavy_upper = h_tot[3];
  PCHK(dev_malloc(&g.piece_row, sizeof(int32_t) * std::max<int64_t>(g.npieces, 1)));
  PCHK(dev_malloc(&g.piece_start, sizeof(int64_t) * std::max<int64_t>(g.npieces, 1)));
  PCHK(dev_malloc(&g.piece_first, sizeof(int32_t) * std::max<int64_t>(g.n, 1)));
  PCHK(dev_malloc(&g.heavy_rows, sizeof(int32_t) * std::max<int64_t>(g.nheavy, 1)));
  PCHK(dev_malloc(&g.split_written, sizeof(int32_t) * std::max<int64_t>(g.npieces, 1)));
  fill_pieces_kernel<<<grid, 256, 0, s>>>(g.off, g.n, first, hfirst, g.piece_row, g.piece_start,
                                          g.piece_first, g.heavy_rows);
  PCHK(hipGetLastError());
  // pull round work split (np and hv are free again: weights and prefix)
  g.pull_bounds_grid = g.cu_count;
  PCHK(dev_malloc(&g.pull_bounds, sizeof(int32_t) * 2 * (g.pull_bounds_grid + 1)));
  row_weight_kernel<<<grid, 256, 0, s>>>(g.off, g.n, np);
  PCHK(hipGetLastError());
  PCHK(prim::exclusive_sum(temp, temp_bytes, np, hv, (size_t)(g.n + 1), s));
  pull_bounds_kernel<<<(2 * (g.pull_bounds_grid + 1) + 255) / 256, 256, 0, s>>>(
      hv, g.nU, g.n, g.pull_bounds_grid, g.pull_bounds);
  PCHK(hipGetLastError());
  PCHK(hipStreamSynchronize(s));
done:
  for (void *p : {(void *)np, (void *)hv, (void *)first, (void *)hfirst, temp})
    if (p) (void)dev_free_async(p, s);
  return status;
#undef PCHK
}

namespace {

// (layer-local key) decreasing degree, then id: 64-bit keys whose order is
// the rank order of one layer.
__global__ void rank_keys_kernel(const int64_t *__restrict__ off, int64_t lo, int64_t hi,
                                 uint64_t *__restrict__ keys) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < hi; x += stride) {
    const uint64_t d = (uint64_t)(off[x + 1] - off[x]);
    keys[x - lo] = ((0x7FFFFFFFull - d) << 32) | (uint64_t)(x - lo);
  }
}

__global__ void rank_scatter_kernel(const uint64_t *__restrict__ sorted, int64_t cnt, int64_t lo,
                                    const int64_t *__restrict__ off, int32_t *__restrict__ rank,
                                    int32_t *__restrict__ rank_vtx, int64_t *__restrict__ rdeg) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride) {
    const int64_t x = lo + (int64_t)(uint32_t)sorted[i];
    rank[x] = (int32_t)i;
    rank_vtx[lo + i] = (int32_t)x;
    rdeg[lo + i] = off[x + 1] - off[x];
  }
}

// Entry keys (global rank of the row, neighbour's rank): sorted, the rows
// come out in rank order and each row's ranks ascending.  A wave per row
// (rows in turn), its lanes over the row's entries, so that hubs do not
// serialise on one thread.
__global__ void entry_keys_kernel(const int64_t *__restrict__ off, const int32_t *__restrict__ cols,
                                  const int32_t *__restrict__ rank, int64_t n, int64_t nU, int rbits,
                                  uint64_t *__restrict__ keys) {
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  const int64_t w0 = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = (int)(threadIdx.x % kWave);
  for (int64_t x = w0; x < n; x += waves) {
    const uint64_t r = (uint64_t)rank[x] + (x < nU ? 0 : (uint64_t)nU);
    const int64_t e1 = off[x + 1];
    for (int64_t e = off[x] + lane; e < e1; e += kWave)
      keys[e] = (r << rbits) | (uint64_t)rank[cols[e]];
  }
}

// The neighbour's global rank: a lower neighbour (of an upper row) is its
// layer rank past nU, so that the rank rows form a CSR graph of their own.
__global__ void entry_unkey_kernel(const uint64_t *__restrict__ keys, int64_t cnt, int rbits,
                                   int64_t nU, int32_t *__restrict__ rcols) {
  const uint64_t mask = (1ull << rbits) - 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride) {
    const bool upper_row = (int64_t)(keys[i] >> rbits) < nU;
    rcols[i] = (int32_t)((int64_t)(keys[i] & mask) + (upper_row ? nU : 0));
  }
}

// Degree counts by threshold, from the rank order (degrees decrease along a
// layer's ranks): at the last rank of each run of equal degrees d, the
// layer's vertices of degree >= d and their entries.
__global__ void rank_table_kernel(const int64_t *__restrict__ roff, int64_t lo, int64_t hi,
                                  int64_t *__restrict__ ge_cnt, int64_t *__restrict__ ge_ent) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < hi; r += stride) {
    const int64_t d = roff[r + 1] - roff[r];
    const int64_t dn = r + 1 < hi ? roff[r + 2] - roff[r + 1] : -1;
    if (d != dn) {
      ge_cnt[d] = r + 1 - lo;
      ge_ent[d] = roff[r + 1] - roff[lo];
    }
  }
}

}  // namespace

abcore_status build_ranks(Graph &g, hipStream_t s) {
  const int64_t ent = 2 * g.m_csr;
  if (g.n == 0) return ABCORE_OK;
  // 2^31 items is the sort's limit; larger graphs keep the bitmap pull
  if (ent >= 0x7FFFFFFFLL) return ABCORE_OK;
  uint64_t *k0 = nullptr, *k1 = nullptr;
  void *temp = nullptr;
  size_t temp_bytes = 0, need = 0;
  bool ok = true;
  const int grid = std::max(1, std::min(g.cu_count * 8, (int)((g.n + 255) / 256)));
  const int64_t nmax = std::max<int64_t>(std::max<int64_t>(g.nU, g.nL), 1);
  const int rbits = bits_for((uint64_t)nmax - 1);
  const int xbits = bits_for((uint64_t)std::max<int64_t>(g.n, 1) - 1);
  const int64_t items = std::max<int64_t>(ent, nmax);
  auto fail = [&](hipError_t e) {
    if (e != hipSuccess) ok = false;
    return e != hipSuccess;
  };
  do {
    if (fail(dev_malloc(&g.rank, sizeof(int32_t) * g.n))) break;
    if (fail(dev_malloc(&g.rank_vtx, sizeof(int32_t) * g.n))) break;
    if (fail(dev_malloc(&g.roff, sizeof(int64_t) * (g.n + 1)))) break;
    if (fail(dev_malloc(&g.rcols, sizeof(int32_t) * std::max<int64_t>(ent, 1)))) break;
    g.rdeg_mask = (uint32_t)((1ull << xbits) - 1);
    if (fail(dev_malloc(&g.rdeg, sizeof(int32_t) * ((size_t)g.rdeg_mask + 1)))) break;
    // k0 also holds the degrees by rank (n + 1 values after n + 1 slots)
    if (fail(dev_malloc_async(&k0, sizeof(uint64_t) * std::max<int64_t>(items, 2 * (g.n + 1)), s))) break;
    if (fail(dev_malloc_async(&k1, sizeof(uint64_t) * items, s))) break;
    // temporary storage for the largest sort, and the offsets' scan
    if (fail(prim::sort_keys(nullptr, need, k0, k1, (size_t)items, 0, 64, s)))
      break;
    temp_bytes = std::max<size_t>(need, 16);
    need = 0;
    if (fail(prim::exclusive_sum(nullptr, need, reinterpret_cast<int64_t *>(k0),
                                              g.roff, (size_t)(g.n + 1), s)))
      break;
    temp_bytes = std::max(temp_bytes, need);
    if (fail(dev_malloc_async(&temp, temp_bytes, s))) break;
    // ranks, one layer at a time
    for (int layer = 0; layer < 2 && ok; ++layer) {
      const int64_t lo = layer == 0 ? 0 : g.nU, hi = layer == 0 ? g.nU : g.n;
      if (hi <= lo) continue;
      rank_keys_kernel<<<grid, 256, 0, s>>>(g.off, lo, hi, k0);
      if (fail(hipGetLastError())) break;
      size_t tb = temp_bytes;
      if (fail(prim::sort_keys(temp, tb, k0, k1, (size_t)(hi - lo), 0, 64, s)))
        break;
      // (k0 holds no keys any more past the sort: its tail collects the
      // degrees by rank, the offsets' scan input)
      rank_scatter_kernel<<<grid, 256, 0, s>>>(k1, hi - lo, lo, g.off, g.rank, g.rank_vtx,
                                               reinterpret_cast<int64_t *>(k0) + g.n + 1);
      if (fail(hipGetLastError())) break;
    }
    if (!ok) break;
    {
      int64_t *rdeg = reinterpret_cast<int64_t *>(k0) + g.n + 1;
      if (fail(hipMemsetAsync(rdeg + g.n, 0, sizeof(int64_t), s))) break;
      size_t tb = temp_bytes;
      if (fail(prim::exclusive_sum(temp, tb, rdeg, g.roff, (size_t)(g.n + 1), s))) break;
    }
    if (ent > 0) {
      entry_keys_kernel<<<grid, 256, 0, s>>>(g.off, g.cols, g.rank, g.n, g.nU, rbits, k0);
      if (fail(hipGetLastError())) break;
      size_t tb = temp_bytes;
      if (fail(prim::sort_keys(temp, tb, k0, k1, (size_t)ent, 0, rbits + xbits, s)))
        break;
      entry_unkey_kernel<<<grid, 256, 0, s>>>(k1, ent, rbits, g.nU, g.rcols);
      if (fail(hipGetLastError())) break;
    }
    // the rank rows' pieces (the same lengths as the vertex rows', in rank
    // order; k0 and k1 serve as the counts and their scans)
    {
      int64_t *np = reinterpret_cast<int64_t *>(k0), *hv = np + (g.n + 1);
      int64_t *hfirst = nullptr;
      if (fail(dev_malloc_async(&hfirst, sizeof(int64_t) * 2 * (g.n + 1), s))) break;
      int32_t *hrows = nullptr;
      bool pok = false;
      do {
        int64_t *fcopy = hfirst + (g.n + 1);
        count_pieces_kernel<<<grid, 256, 0, s>>>(g.roff, g.n, np, hv);
        if (fail(hipGetLastError())) break;
        size_t tb = temp_bytes;
        if (fail(prim::exclusive_sum(temp, tb, np, fcopy, (size_t)(g.n + 1), s))) break;
        tb = temp_bytes;
        if (fail(prim::exclusive_sum(temp, tb, hv, hfirst, (size_t)(g.n + 1), s))) break;
        if (fail(dev_malloc(&g.rp_row, sizeof(int32_t) * std::max<int64_t>(g.npieces, 1)))) break;
        if (fail(dev_malloc(&g.rp_start, sizeof(int64_t) * std::max<int64_t>(g.npieces, 1))))
          break;
        if (fail(dev_malloc(&g.rp_first, sizeof(int32_t) * g.n))) break;
        if (fail(dev_malloc_async(&hrows, sizeof(int32_t) * std::max<int64_t>(g.nheavy, 1), s))) break;
        fill_pieces_kernel<<<grid, 256, 0, s>>>(g.roff, g.n, fcopy, hfirst, g.rp_row, g.rp_start,
                                                g.rp_first, hrows);
        if (fail(hipGetLastError())) break;
        pok = true;
      } while (0);
      if (fail(hipStreamSynchronize(s))) pok = false;
      if (hrows) (void)dev_free_async(hrows, s);
      (void)dev_free_async(hfirst, s);
      if (!pok) {
        ok = false;
        break;
      }
    }
    // per layer and threshold t: the vertices of degree >= t (ranks [0, K))
    // and their entries, kept on the host
    for (int layer = 0; layer < 2 && ok; ++layer) {
      const int64_t lo = layer == 0 ? 0 : g.nU, hi = layer == 0 ? g.nU : g.n;
      g.rk_cnt[layer].assign(1, 0);
      g.rk_ent[layer].assign(1, 0);
      if (hi <= lo) continue;
      int64_t r01[2] = {0, 0};
      if (fail(hipMemcpyAsync(r01, g.roff + lo, sizeof(int64_t) * 2, hipMemcpyDeviceToHost, s)))
        break;
      if (fail(hipStreamSynchronize(s))) break;
      const int64_t maxdeg = r01[1] - r01[0];
      // (k0 and k1 are free again and hold at least n + 1 values each)
      int64_t *gc = reinterpret_cast<int64_t *>(k0), *ge = reinterpret_cast<int64_t *>(k1);
      if (maxdeg + 1 > g.n + 1) {
        ok = false;
        break;
      }
      if (fail(hipMemsetAsync(gc, 0xFF, sizeof(int64_t) * (maxdeg + 1), s))) break;
      rank_table_kernel<<<grid, 256, 0, s>>>(g.roff, lo, hi, gc, ge);
      if (fail(hipGetLastError())) break;
      std::vector<int64_t> hc(maxdeg + 1), he(maxdeg + 1);
      if (fail(hipMemcpyAsync(hc.data(), gc, sizeof(int64_t) * (maxdeg + 1),
                              hipMemcpyDeviceToHost, s)))
        break;
      if (fail(hipMemcpyAsync(he.data(), ge, sizeof(int64_t) * (maxdeg + 1),
                              hipMemcpyDeviceToHost, s)))
        break;
      if (fail(hipStreamSynchronize(s))) break;
      // a degree no vertex has takes the counts of the next larger one
      std::vector<int64_t> &kc = g.rk_cnt[layer], &ke = g.rk_ent[layer];
      kc.assign(maxdeg + 2, 0);
      ke.assign(maxdeg + 2, 0);
      for (int64_t t = maxdeg; t >= 0; --t) {
        kc[t] = hc[t] >= 0 ? hc[t] : kc[t + 1];
        ke[t] = hc[t] >= 0 ? he[t] : ke[t + 1];
      }
    }
    if (!ok) break;
    if (fail(hipStreamSynchronize(s))) break;
  } while (0);
  for (void *p : {(void *)k0, (void *)k1, temp})
    if (p) (void)dev_free_async(p, s);
  if (!ok) {
    (void)hipGetLastError();
    if (g.rank) (void)dev_free(g.rank);
    if (g.rank_vtx) (void)dev_free(g.rank_vtx);
    if (g.roff) (void)dev_free(g.roff);
    if (g.rcols) (void)dev_free(g.rcols);
    if (g.rdeg) (void)dev_free(g.rdeg);
    g.rdeg = nullptr;
    g.rdeg_mask = 0;
    if (g.rp_row) (void)dev_free(g.rp_row);
    if (g.rp_start) (void)dev_free(g.rp_start);
    if (g.rp_first) (void)dev_free(g.rp_first);
    g.rank = nullptr;
    g.rank_vtx = nullptr;
    g.roff = nullptr;
    g.rcols = nullptr;
    g.rp_row = nullptr;
    g.rp_start = nullptr;
    g.rp_first = nullptr;
    for (int layer = 0; layer < 2; ++layer) {
      g.rk_cnt[layer].clear();
      g.rk_ent[layer].clear();
    }
  }
  return ABCORE_OK;
}

}  // namespace abc
