/*
 * TEST INFRASTRUCTURE -- the CPU oracle for (alpha,beta)-core computation.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * use it.  It shares no code with the device library.
 *
 * Plain, sequential, single-threaded C.  Every routine writes out a
 * definition from the paper (Feng et al., "Efficient (alpha,beta)-core
 * Computation and On-the-fly Query at Billion Scale with GPUs"):
 *
 *   - Graph model (Sec. III): G = (U u L, E), E a set of (upper, lower)
 *     pairs.  Vertices get unified ids, upper 0..nU-1, lower nU..nU+nL-1
 *     (the contiguous-id layout of Sec. IV-A).
 *   - (alpha,beta)-core (Definition 1): the maximal subgraph in which every
 *     upper vertex has degree >= alpha and every lower vertex >= beta.  It is
 *     computed by the peeling procedure of Sec. III-A (the Online method):
 *     remove violators with their edges until none is left.
 *   - Core number (Definition 2): the largest delta with the vertex in the
 *     (delta,delta)-core, i.e. the k-core number of G taken as an ordinary
 *     graph; computed with the bucket algorithm of Batagelj and Zaversnik
 *     (the paper's reference for the definition).
 *   - Connected components (Sec. V preprocessing): breadth-first search,
 *     label = smallest unified id in the component.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ CSR --
 * Builds the adjacency of both layers as one unified CSR (Sec. III: CSR
 * storage; Sec. IV-A: contiguous ids).  Row u (upper) lists nU+v for every
 * edge (u,v); row nU+v lists u.  Rows are sorted ascending.  Duplicate pairs
 * are removed (E is a set).  Two stable counting sorts (by v, then by u)
 * order the pairs; a third (by v) orders the lower rows.
 * Returns the number of distinct edges, or -1 for an out-of-range id / OOM.
 * off has n+1 entries, cols room for 2m entries. */
int64_t or_build_csr(int32_t nU, int32_t nL, int64_t m, const int32_t *eu,
                     const int32_t *ev, int64_t *off, int32_t *cols) {
  int64_t n = (int64_t)nU + nL;
  for (int64_t i = 0; i < m; ++i)
    if (eu[i] < 0 || eu[i] >= nU || ev[i] < 0 || ev[i] >= nL) return -1;
  int32_t *tu = malloc(sizeof(int32_t) * (m ? m : 1));
  int32_t *tv = malloc(sizeof(int32_t) * (m ? m : 1));
  int32_t *su = malloc(sizeof(int32_t) * (m ? m : 1));
  int32_t *sv = malloc(sizeof(int32_t) * (m ? m : 1));
  int64_t *cnt = calloc((size_t)(n + 1), sizeof(int64_t));
  if (!tu || !tv || !su || !sv || !cnt) {
    free(tu); free(tv); free(su); free(sv); free(cnt);
    return -1;
  }
  /* pass 1: stable counting sort by v */
  for (int64_t i = 0; i < m; ++i) cnt[ev[i] + 1]++;
  for (int32_t v = 0; v < nL; ++v) cnt[v + 1] += cnt[v];
  for (int64_t i = 0; i < m; ++i) {
    int64_t p = cnt[ev[i]]++;
    tu[p] = eu[i];
    tv[p] = ev[i];
  }
  /* pass 2: stable counting sort by u -> pairs ordered by (u, v) */
  memset(cnt, 0, sizeof(int64_t) * (size_t)(n + 1));
  for (int64_t i = 0; i < m; ++i) cnt[tu[i] + 1]++;
  for (int32_t u = 0; u < nU; ++u) cnt[u + 1] += cnt[u];
  for (int64_t i = 0; i < m; ++i) {
    int64_t p = cnt[tu[i]]++;
    su[p] = tu[i];
    sv[p] = tv[i];
  }
  /* drop duplicates */
  int64_t md = 0;
  for (int64_t i = 0; i < m; ++i) {
    if (md > 0 && su[md - 1] == su[i] && sv[md - 1] == sv[i]) continue;
    su[md] = su[i];
    sv[md] = sv[i];
    ++md;
  }
  /* degrees */
  int64_t *deg = calloc((size_t)n, sizeof(int64_t));
  if (!deg) {
    free(tu); free(tv); free(su); free(sv); free(cnt);
    return -1;
  }
  for (int64_t i = 0; i < md; ++i) {
    deg[su[i]]++;
    deg[(int64_t)nU + sv[i]]++;
  }
  off[0] = 0;
  for (int64_t x = 0; x < n; ++x) off[x + 1] = off[x] + deg[x];
  /* upper rows: off[u] counts the pairs with a smaller u, so in (u, v) order
   * pair i lands at position i */
  for (int64_t i = 0; i < md; ++i) cols[i] = nU + sv[i];
  /* lower rows: scanning pairs in (u, v) order keeps each row ascending */
  int64_t *cur = cnt; /* reuse: write cursor per lower vertex */
  for (int32_t v = 0; v < nL; ++v) cur[v] = off[(int64_t)nU + v];
  for (int64_t i = 0; i < md; ++i) cols[cur[sv[i]]++] = su[i];
  free(tu); free(tv); free(su); free(sv); free(cnt); free(deg);
  return md;
}

/* ----------------------------------------------------------------- peel --
 * The (alpha,beta)-core of Definition 1 by sequential peeling (Sec. III-A).
 * deg(x) starts at |N(x)|.  Every vertex below its threshold (alpha for
 * upper, beta for lower) is marked removed and queued; popping x lowers the
 * degree of each neighbour that is still present, and a neighbour that falls
 * below its threshold is marked and queued in turn.  Survivors are the core.
 *
 * member[x] = 1 for core vertices.  stats (nullable, 4 entries):
 *   [0] |R| removed vertices, [1] sum of |N(x)| over removed x,
 *   [2] m_peeled = m - |E(core)|, [3] number of FIFO generations (rounds).
 * order (nullable, room for n entries): the removed vertices in the order
 *   they were marked, i.e. the FIFO contents; order[0..|R|) is written.
 * Returns 0, or -1 on allocation failure. */
int or_peel_order(int32_t nU, int32_t nL, const int64_t *off, const int32_t *cols,
                  int64_t alpha, int64_t beta, uint8_t *member, int64_t *stats,
                  int64_t *order) {
  int64_t n = (int64_t)nU + nL;
  int64_t *deg = malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
  int64_t *queue = malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
  uint8_t *removed = calloc((size_t)(n ? n : 1), 1);
  if (!deg || !queue || !removed) {
    free(deg); free(queue); free(removed);
    return -1;
  }
  int64_t head = 0, tail = 0;
  for (int64_t x = 0; x < n; ++x) {
    deg[x] = off[x + 1] - off[x];
    int64_t thr = x < nU ? alpha : beta;
    if (deg[x] < thr) {
      removed[x] = 1;
      queue[tail++] = x;
    }
  }
  int64_t rounds = 0, gen_end = tail, sum_deg = 0;
  if (tail > 0) rounds = 1;
  while (head < tail) {
    if (head == gen_end) { /* a new generation of removals starts */
      gen_end = tail;
      ++rounds;
    }
    int64_t x = queue[head++];
    sum_deg += off[x + 1] - off[x];
    for (int64_t j = off[x]; j < off[x + 1]; ++j) {
      int64_t w = cols[j];
      if (removed[w]) continue;
      deg[w] -= 1;
      int64_t thr = w < nU ? alpha : beta;
      if (deg[w] < thr) {
        removed[w] = 1;
        queue[tail++] = w;
      }
    }
  }
  /* edges inside the core: count from the upper side */
  int64_t m_total = off[nU] - off[0], m_core = 0;
  for (int64_t x = 0; x < nU; ++x) {
    if (removed[x]) continue;
    for (int64_t j = off[x]; j < off[x + 1]; ++j) m_core += !removed[cols[j]];
  }
  for (int64_t x = 0; x < n; ++x) member[x] = !removed[x];
  if (stats) {
    stats[0] = tail;
    stats[1] = sum_deg;
    stats[2] = m_total - m_core;
    stats[3] = rounds;
  }
  if (order) memcpy(order, queue, sizeof(int64_t) * (size_t)tail);
  free(deg); free(queue); free(removed);
  return 0;
}

int or_peel(int32_t nU, int32_t nL, const int64_t *off, const int32_t *cols,
            int64_t alpha, int64_t beta, uint8_t *member, int64_t *stats) {
  return or_peel_order(nU, nL, off, cols, alpha, beta, member, stats, NULL);
}

/* ---------------------------------------------------------- core number --
 * Definition 2 via the O(m) bucket algorithm of Batagelj and Zaversnik: keep
 * vertices sorted by current degree in bins; repeatedly take a vertex v of
 * least degree, fix core(v) = deg(v), and move every neighbour u with
 * deg(u) > deg(v) down one bin.  Isolated vertices get core 0. */
int or_core_numbers(int32_t nU, int32_t nL, const int64_t *off, const int32_t *cols,
                    int32_t *core) {
  int64_t n = (int64_t)nU + nL;
  if (n == 0) return 0;
  int64_t md = 0;
  int64_t *deg = malloc(sizeof(int64_t) * (size_t)n);
  int64_t *pos = malloc(sizeof(int64_t) * (size_t)n);
  int64_t *vert = malloc(sizeof(int64_t) * (size_t)n);
  if (!deg || !pos || !vert) {
    free(deg); free(pos); free(vert);
    return -1;
  }
  for (int64_t x = 0; x < n; ++x) {
    deg[x] = off[x + 1] - off[x];
    if (deg[x] > md) md = deg[x];
  }
  int64_t *bin = calloc((size_t)(md + 1), sizeof(int64_t));
  if (!bin) {
    free(deg); free(pos); free(vert);
    return -1;
  }
  for (int64_t x = 0; x < n; ++x) bin[deg[x]]++;
  int64_t start = 0;
  for (int64_t d = 0; d <= md; ++d) {
    int64_t num = bin[d];
    bin[d] = start;
    start += num;
  }
  for (int64_t x = 0; x < n; ++x) {
    pos[x] = bin[deg[x]];
    vert[pos[x]] = x;
    bin[deg[x]]++;
  }
  for (int64_t d = md; d >= 1; --d) bin[d] = bin[d - 1];
  bin[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t v = vert[i];
    for (int64_t j = off[v]; j < off[v + 1]; ++j) {
      int64_t u = cols[j];
      if (deg[u] > deg[v]) {
        int64_t du = deg[u], pu = pos[u];
        int64_t pw = bin[du], w = vert[pw];
        if (u != w) {
          pos[u] = pw; vert[pu] = w;
          pos[w] = pu; vert[pw] = u;
        }
        bin[du]++;
        deg[u]--;
      }
    }
  }
  for (int64_t x = 0; x < n; ++x) core[x] = (int32_t)deg[x];
  free(deg); free(pos); free(vert); free(bin);
  return 0;
}

/* ----------------------------------------------------------- components --
 * Connected components by breadth-first search (Sec. V preprocessing).
 * Starting searches in increasing id order labels every component with its
 * smallest unified id. */
int or_components(int32_t nU, int32_t nL, const int64_t *off, const int32_t *cols,
                  int32_t *comp) {
  int64_t n = (int64_t)nU + nL;
  if (n == 0) return 0;
  int64_t *queue = malloc(sizeof(int64_t) * (size_t)n);
  if (!queue) return -1;
  for (int64_t x = 0; x < n; ++x) comp[x] = -1;
  for (int64_t s = 0; s < n; ++s) {
    if (comp[s] >= 0) continue;
    int64_t head = 0, tail = 0;
    comp[s] = (int32_t)s;
    queue[tail++] = s;
    while (head < tail) {
      int64_t x = queue[head++];
      for (int64_t j = off[x]; j < off[x + 1]; ++j) {
        int64_t w = cols[j];
        if (comp[w] < 0) {
          comp[w] = (int32_t)s;
          queue[tail++] = w;
        }
      }
    }
  }
  free(queue);
  return 0;
}
