/*
 * Multithreaded CPU peel of the (alpha,beta)-core -- the CPU comparison
 * point of the benchmark (the Online baseline of Sec. III-A and Table II,
 * peeling on the host), run on all host threads.  Not used by the device
 * library.
 *
 * The frontier peeling of Sec. III-A, round by round with OpenMP: a round's
 * frontier is split across the threads; each removed vertex lowers the
 * degree of every neighbour with an atomic fetch-and-subtract, and the one
 * subtraction that takes a neighbour from its threshold to one below it (the
 * unique crossing, so each vertex is queued once) appends that neighbour to
 * the thread's own buffer; the buffers, concatenated, are the next round's
 * frontier.  The survivors are the core (Definition 1), whatever the order.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int cp_max_threads(void) { return omp_get_max_threads(); }

/* member[x] = 1 for core vertices; *rounds (nullable) receives the number of
 * non-empty rounds.  nthreads <= 0: all threads.  Returns 0, -1 on OOM. */
int cp_peel(int32_t nU, int32_t nL, const int64_t *off, const int32_t *cols, int64_t alpha,
            int64_t beta, uint8_t *member, int nthreads, int64_t *rounds) {
  const int64_t n = (int64_t)nU + nL;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  int64_t *deg = malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
  int32_t *front = malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
  int32_t *next = malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
  int64_t *cnt = calloc((size_t)nthreads + 1, sizeof(int64_t));
  int32_t **buf = calloc((size_t)nthreads, sizeof(int32_t *));
  int64_t *cap = calloc((size_t)nthreads, sizeof(int64_t));
  if (!deg || !front || !next || !cnt || !buf || !cap) {
    free(deg); free(front); free(next); free(cnt); free(buf); free(cap);
    return -1;
  }
  int64_t nf = 0;
  int failed = 0;
#pragma omp parallel num_threads(nthreads)
  {
    const int t = omp_get_thread_num();
    const int nt = omp_get_num_threads();
    int64_t mine = 0, mycap = 1024;
    int32_t *my = malloc(sizeof(int32_t) * (size_t)mycap);
    if (!my) {
#pragma omp atomic write
      failed = 1;
    }
    /* scan phase (Algorithm 1's): every vertex below its threshold */
#pragma omp for schedule(static)
    for (int64_t x = 0; x < n; ++x) {
      deg[x] = off[x + 1] - off[x];
      if (my && deg[x] < (x < nU ? alpha : beta)) {
        if (mine == mycap) {
          int32_t *g2 = realloc(my, sizeof(int32_t) * (size_t)(2 * mycap));
          if (!g2) {
#pragma omp atomic write
            failed = 1;
            continue;
          }
          my = g2;
          mycap *= 2;
        }
        my[mine++] = (int32_t)x;
      }
    }
    buf[t] = my;
    cap[t] = mycap;
    cnt[t + 1] = mine;
#pragma omp barrier
#pragma omp single
    {
      for (int i = 0; i < nt; ++i) cnt[i + 1] += cnt[i];
      nf = cnt[nt];
      if (rounds) *rounds = nf > 0 ? 1 : 0;
    }
    if (buf[t]) memcpy(front + cnt[t], buf[t], sizeof(int32_t) * (size_t)(cnt[t + 1] - cnt[t]));
#pragma omp barrier
    while (nf > 0 && !failed) {
      mine = 0;
      my = buf[t];
      mycap = cap[t];
#pragma omp for schedule(dynamic, 64)
      for (int64_t i = 0; i < nf; ++i) {
        const int32_t x = front[i];
        for (int64_t j = off[x]; j < off[x + 1]; ++j) {
          const int32_t w = cols[j];
          const int64_t thr = w < nU ? alpha : beta;
          int64_t old;
#pragma omp atomic capture
          old = deg[w]--;
          if (old == thr) {
            if (mine == mycap) {
              int32_t *g2 = realloc(my, sizeof(int32_t) * (size_t)(2 * mycap));
              if (!g2) {
#pragma omp atomic write
                failed = 1;
                continue;
              }
              my = g2;
              mycap *= 2;
            }
            my[mine++] = w;
          }
        }
      }
      buf[t] = my;
      cap[t] = mycap;
      cnt[t + 1] = mine;
#pragma omp barrier
#pragma omp single
      {
        cnt[0] = 0;
        for (int i = 0; i < nt; ++i) cnt[i + 1] += cnt[i];
        nf = cnt[nt];
        if (rounds && nf > 0) *rounds += 1;
      }
      memcpy(next + cnt[t], buf[t], sizeof(int32_t) * (size_t)(cnt[t + 1] - cnt[t]));
#pragma omp barrier
#pragma omp single
      {
        int32_t *tmp = front;
        front = next;
        next = tmp;
      }
    }
    /* a vertex is removed iff it was queued, i.e. iff its final degree is
     * below its threshold (degrees only fall) */
#pragma omp for schedule(static)
    for (int64_t x = 0; x < n; ++x) member[x] = deg[x] >= (x < nU ? alpha : beta);
    free(buf[t]);
  }
  free(deg); free(front); free(next); free(cnt); free(buf); free(cap);
  return failed ? -1 : 0;
}
