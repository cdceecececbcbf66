// Seeded synthetic bipartite-graph generators shared by the oracle and the
// device library.  This file holds no (alpha,beta)-core arithmetic: it only
// produces edge lists, query parameters and update streams.
//
// Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014) used in counter mode: the
// i-th value of stream s is mix64(key(seed, s) + (i + 1) * GAMMA), which is
// exactly the i-th output of a SplitMix64 generator whose state starts at
// key(seed, s).  Bounded integers use Lemire's multiply-high reduction
// ("Fast random integer generation in an interval", TOMACS 2019) without the
// rejection step.  Weighted endpoint choice uses Vose's alias method
// ("A linear algorithm for generating random numbers with a given
// distribution", IEEE TSE 1991).
//
// Every function is deterministic for a given argument list; OpenMP only
// splits independent counter ranges and per-row sorts.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <unordered_map>
#include <unordered_set>
#include <parallel/algorithm>
#include <omp.h>

namespace {

constexpr uint64_t GAMMA = 0x9E3779B97F4A7C15ULL;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Stream tags keep the purposes of the random numbers independent.
enum : uint64_t {
  TAG_EDGES = 1, TAG_PERM_U = 2, TAG_PERM_L = 3, TAG_QUERIES = 4,
  TAG_UPDATES = 5, TAG_ARRIVALS = 6
};

inline uint64_t stream_key(uint64_t seed, uint64_t tag) {
  return mix64(seed * GAMMA + tag * 0xD1B54A32D192ED03ULL);
}
inline uint64_t draw(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * GAMMA); }
inline uint64_t bounded(uint64_t r, uint64_t n) {
  return (uint64_t)(((unsigned __int128)r * n) >> 64);
}
inline double unit(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

struct Alias {
  std::vector<double> prob;
  std::vector<int32_t> alias;
  std::vector<int32_t> perm;  // rank -> vertex id
  int64_t n = 0;
  inline int32_t sample(uint64_t r_idx, uint64_t r_coin) const {
    int64_t i = (int64_t)bounded(r_idx, (uint64_t)n);
    int32_t rank = unit(r_coin) < prob[i] ? (int32_t)i : alias[i];
    return perm[rank];
  }
};

// Chung-Lu expected degrees for one layer: w_r proportional to
// r^(-1/(gamma-1)) for rank r = 1..n (gamma is the exponent of the degree
// distribution), scaled so the weights sum to m, capped at `cap`, with the
// uncapped weights rescaled until the cap holds everywhere.
static bool chung_lu_weights(int64_t n, int64_t m, double gamma, double cap,
                             std::vector<double>& w) {
  w.assign(n, 0.0);
  const double e = -1.0 / (gamma - 1.0);
  for (int64_t r = 0; r < n; ++r) w[r] = std::pow((double)(r + 1), e);
  // suffix sums of the raw weights
  std::vector<double> suf(n + 1, 0.0);
  for (int64_t r = n - 1; r >= 0; --r) suf[r] = suf[r + 1] + w[r];
  if ((double)n * cap < (double)m) return false;
  int64_t k = 0;  // number of capped ranks (a prefix, raw weights decrease)
  double scale = (double)m / suf[0];
  while (k < n && w[k] * scale > cap) {
    ++k;
    double rest = (double)m - (double)k * cap;
    if (rest <= 0.0 || suf[k] <= 0.0) return false;
    scale = rest / suf[k];
  }
  for (int64_t r = 0; r < n; ++r) w[r] = r < k ? cap : w[r] * scale;
  return true;
}

static void build_alias(const std::vector<double>& w, Alias& a) {
  const int64_t n = (int64_t)w.size();
  a.n = n;
  a.prob.assign(n, 0.0);
  a.alias.assign(n, 0);
  double total = 0.0;
  for (double x : w) total += x;
  std::vector<double> p(n);
  for (int64_t i = 0; i < n; ++i) p[i] = w[i] * (double)n / total;
  std::vector<int32_t> small, large;
  small.reserve(n);
  large.reserve(n);
  for (int64_t i = 0; i < n; ++i) (p[i] < 1.0 ? small : large).push_back((int32_t)i);
  while (!small.empty() && !large.empty()) {
    int32_t s = small.back(); small.pop_back();
    int32_t l = large.back(); large.pop_back();
    a.prob[s] = p[s];
    a.alias[s] = l;
    p[l] = (p[l] + p[s]) - 1.0;
    (p[l] < 1.0 ? small : large).push_back(l);
  }
  for (int32_t l : large) { a.prob[l] = 1.0; a.alias[l] = l; }
  for (int32_t s : small) { a.prob[s] = 1.0; a.alias[s] = s; }
}

// Seeded Fisher-Yates permutation so that heavy ranks land on scattered ids.
static void permutation(int64_t n, uint64_t key, std::vector<int32_t>& perm) {
  perm.resize(n);
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)bounded(draw(key, (uint64_t)i), (uint64_t)(i + 1));
    std::swap(perm[i], perm[j]);
  }
}

// Keeps the first m distinct pairs of the draw sequence pair(0), pair(1), ...
// Writes them sorted by (u, v).  Returns m on success, a negative value when
// the sequence could not supply m distinct pairs within the attempt limit.
template <class PairFn>
static int64_t first_distinct(int32_t nU, int64_t m, PairFn pair_of, int64_t d0,
                              int32_t* eu, int32_t* ev) {
  if (m == 0) return 0;
  int64_t D = d0;
  for (int attempt = 0; attempt < 12; ++attempt) {
    if (D > (int64_t)0xFFFFFFFFLL) return -2;  // draw index must fit 32 bits
    std::vector<int32_t> U(D), V(D);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < D; ++i) {
      int32_t u, v;
      pair_of((uint64_t)i, u, v);
      U[i] = u;
      V[i] = v;
    }
    // bucket draws by upper endpoint; each entry packs (v, draw index)
    std::vector<int64_t> start(nU + 1, 0);
    {
      std::vector<int64_t> cnt(nU, 0);
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < D; ++i) __atomic_fetch_add(&cnt[U[i]], 1, __ATOMIC_RELAXED);
      for (int32_t u = 0; u < nU; ++u) start[u + 1] = start[u] + cnt[u];
    }
    std::vector<uint64_t> ent(D);
    {
      std::vector<int64_t> cur(start.begin(), start.end() - 1);
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < D; ++i) {
        int64_t pos = __atomic_fetch_add(&cur[U[i]], 1, __ATOMIC_RELAXED);
        ent[pos] = ((uint64_t)(uint32_t)V[i] << 32) | (uint64_t)(uint32_t)i;
      }
    }
    std::vector<int32_t>().swap(U);
    std::vector<int32_t>().swap(V);
    std::vector<uint8_t> fresh(D, 0);
#pragma omp parallel for schedule(dynamic, 256)
    for (int32_t u = 0; u < nU; ++u) {
      uint64_t* b = ent.data() + start[u];
      int64_t len = start[u + 1] - start[u];
      std::sort(b, b + len);
      for (int64_t j = 0; j < len; ++j)
        if (j == 0 || (b[j] >> 32) != (b[j - 1] >> 32)) fresh[b[j] & 0xFFFFFFFFULL] = 1;
    }
    // D* = one past the draw index of the m-th fresh pair
    int64_t seen = 0, dstar = -1;
    for (int64_t i = 0; i < D; ++i) {
      seen += fresh[i];
      if (seen == m) { dstar = i + 1; break; }
    }
    if (dstar < 0) {
      if (seen == 0) return -3;
      double grow = (double)m / (double)seen;
      int64_t next = (int64_t)((double)D * grow * 1.05) + 4096;
      if (next <= D) next = D + 4096;
      D = next;
      continue;
    }
    std::vector<int64_t> outcnt(nU + 1, 0);
#pragma omp parallel for schedule(dynamic, 256)
    for (int32_t u = 0; u < nU; ++u) {
      int64_t c = 0;
      for (int64_t j = start[u]; j < start[u + 1]; ++j) {
        uint64_t idx = ent[j] & 0xFFFFFFFFULL;
        c += (fresh[idx] && (int64_t)idx < dstar);
      }
      outcnt[u + 1] = c;
    }
    for (int32_t u = 0; u < nU; ++u) outcnt[u + 1] += outcnt[u];
#pragma omp parallel for schedule(dynamic, 256)
    for (int32_t u = 0; u < nU; ++u) {
      int64_t o = outcnt[u];
      for (int64_t j = start[u]; j < start[u + 1]; ++j) {
        uint64_t idx = ent[j] & 0xFFFFFFFFULL;
        if (fresh[idx] && (int64_t)idx < dstar) {
          eu[o] = u;
          ev[o] = (int32_t)(ent[j] >> 32);
          ++o;
        }
      }
    }
    return m;
  }
  return -4;
}

struct ChungLuTables {
  Alias up, lo;
};

static bool make_tables(int32_t nU, int32_t nL, int64_t m, double gU, double gL,
                        double cap, uint64_t seed, ChungLuTables& t) {
  std::vector<double> w;
  if (!chung_lu_weights(nU, m, gU, cap, w)) return false;
  build_alias(w, t.up);
  if (!chung_lu_weights(nL, m, gL, cap, w)) return false;
  build_alias(w, t.lo);
  permutation(nU, stream_key(seed, TAG_PERM_U), t.up.perm);
  permutation(nL, stream_key(seed, TAG_PERM_L), t.lo.perm);
  return true;
}

}  // namespace

extern "C" {

int bg_num_threads(void) { return omp_get_max_threads(); }

uint64_t bg_splitmix_draw(uint64_t seed, uint64_t tag, uint64_t i) {
  return draw(stream_key(seed, tag), i);
}

// Uniform bipartite graph: the first m distinct pairs of a stream of pairs
// with u uniform in [0,nU) and v uniform in [0,nL).
int64_t bg_uniform(int32_t nU, int32_t nL, int64_t m, uint64_t seed, int32_t* eu,
                   int32_t* ev) {
  if (nU <= 0 || nL <= 0 || m < 0 || (double)m > 0.5 * (double)nU * (double)nL) return -1;
  const uint64_t key = stream_key(seed, TAG_EDGES);
  auto pair_of = [&](uint64_t i, int32_t& u, int32_t& v) {
    u = (int32_t)bounded(draw(key, 2 * i), (uint64_t)nU);
    v = (int32_t)bounded(draw(key, 2 * i + 1), (uint64_t)nL);
  };
  return first_distinct(nU, m, pair_of, m + m / 4 + 4096, eu, ev);
}

// Chung-Lu bipartite graph: each draw picks u and v independently with
// probability proportional to their expected degrees (power law with
// degree-distribution exponents gU and gL, capped at `cap`); the graph is the
// first m distinct pairs of the draw sequence.
int64_t bg_chung_lu(int32_t nU, int32_t nL, int64_t m, double gU, double gL, double cap,
                    uint64_t seed, int32_t* eu, int32_t* ev) {
  if (nU <= 0 || nL <= 0 || m < 0 || gU <= 1.0 || gL <= 1.0 || cap < 1.0) return -1;
  ChungLuTables t;
  if (!make_tables(nU, nL, m, gU, gL, cap, seed, t)) return -1;
  const uint64_t key = stream_key(seed, TAG_EDGES);
  auto pair_of = [&](uint64_t i, int32_t& u, int32_t& v) {
    u = t.up.sample(draw(key, 4 * i), draw(key, 4 * i + 1));
    v = t.lo.sample(draw(key, 4 * i + 2), draw(key, 4 * i + 3));
  };
  return first_distinct(nU, m, pair_of, m + m / 3 + 4096, eu, ev);
}

// q query pairs with alpha and beta drawn independently and log-uniformly:
// floor(exp(ln lo + U * (ln(hi + 1) - ln lo))) clamped to [lo, hi].
void bg_loguniform_pairs(int32_t q, int32_t lo, int32_t hi, uint64_t seed, int32_t* alpha,
                         int32_t* beta) {
  const uint64_t key = stream_key(seed, TAG_QUERIES);
  const double a = std::log((double)lo), b = std::log((double)hi + 1.0);
  for (int32_t i = 0; i < q; ++i) {
    for (int k = 0; k < 2; ++k) {
      double x = std::floor(std::exp(a + unit(draw(key, 2 * (uint64_t)i + k)) * (b - a)));
      int32_t y = (int32_t)std::min(std::max(x, (double)lo), (double)hi);
      (k == 0 ? alpha : beta)[i] = y;
    }
  }
}

// Update stream over a graph given as m distinct edges.  Each update is an
// insertion with probability ins_permille/1000, drawn from the same Chung-Lu
// tables as the graph and redrawn while the pair is present, and otherwise a
// deletion chosen uniformly among the currently present edges.  Every update
// also carries (alpha, beta) log-uniform in [qlo, qhi] and an exponential
// inter-arrival gap of mean 1 (scaled by the caller to a rate).
// op: +1 insert, -1 delete.  Returns the number of updates written or < 0.
int64_t bg_update_stream(int32_t nU, int32_t nL, int64_t m, const int32_t* eu,
                         const int32_t* ev, double gU, double gL, double cap,
                         uint64_t graph_seed, uint64_t seed, int64_t count,
                         int32_t ins_permille, int32_t qlo, int32_t qhi, int32_t* out_u,
                         int32_t* out_v, int32_t* out_op, int32_t* out_alpha,
                         int32_t* out_beta, double* out_gap) {
  if (nU <= 0 || nL <= 0 || m <= 0 || count < 0) return -1;
  ChungLuTables t;
  // the tables depend only on the graph parameters, so inserts follow the
  // graph's own degree weights
  if (!make_tables(nU, nL, m, gU, gL, cap, graph_seed, t)) return -1;
  // present: the current edge keys (deletions draw a uniform position and
  // swap the last key into it).  Membership: the sorted base keys, minus the
  // deleted base keys, plus the inserted keys still present.
  std::vector<uint64_t> present(m);
  for (int64_t i = 0; i < m; ++i) present[i] = (uint64_t)eu[i] * (uint64_t)nL + (uint64_t)ev[i];
  std::vector<uint64_t> base(present);
  __gnu_parallel::sort(base.begin(), base.end());
  std::unordered_set<uint64_t> base_deleted, inserted;
  auto is_present = [&](uint64_t k) {
    if (inserted.count(k)) return true;
    return std::binary_search(base.begin(), base.end(), k) && !base_deleted.count(k);
  };
  const uint64_t key = stream_key(seed, TAG_UPDATES);
  const uint64_t akey = stream_key(seed, TAG_ARRIVALS);
  const double la = std::log((double)qlo), lb = std::log((double)qhi + 1.0);
  uint64_t ctr = 0;
  for (int64_t j = 0; j < count; ++j) {
    bool ins = bounded(draw(key, ctr++), 1000) < (uint64_t)ins_permille || present.empty();
    if (ins) {
      uint64_t k;
      int32_t u, v;
      int guard = 0;
      do {
        u = t.up.sample(draw(key, ctr), draw(key, ctr + 1));
        v = t.lo.sample(draw(key, ctr + 2), draw(key, ctr + 3));
        ctr += 4;
        k = (uint64_t)u * (uint64_t)nL + (uint64_t)v;
        if (++guard > 1000000) return -5;
      } while (is_present(k));
      inserted.insert(k);
      present.push_back(k);
      out_u[j] = u; out_v[j] = v; out_op[j] = 1;
    } else {
      int64_t pos = (int64_t)bounded(draw(key, ctr++), (uint64_t)present.size());
      uint64_t k = present[pos];
      present[pos] = present.back();
      present.pop_back();
      if (!inserted.erase(k)) base_deleted.insert(k);
      out_u[j] = (int32_t)(k / (uint64_t)nL);
      out_v[j] = (int32_t)(k % (uint64_t)nL);
      out_op[j] = -1;
    }
    for (int c = 0; c < 2; ++c) {
      double x = std::floor(std::exp(la + unit(draw(key, ctr++)) * (lb - la)));
      int32_t y = (int32_t)std::min(std::max(x, (double)qlo), (double)qhi);
      (c == 0 ? out_alpha : out_beta)[j] = y;
    }
    out_gap[j] = -std::log1p(-unit(draw(akey, (uint64_t)j)));
  }
  return count;
}

}  // extern "C"
