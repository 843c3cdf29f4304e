/*
 * CPU oracle for the BMLP hot path.  TEST INFRASTRUCTURE ONLY: tests, the
 * smoke check and the CPU-baseline leg of the benchmark call it; the product
 * path never does.  It shares no code with the HIP library.
 *
 * Everything here is the plain definition of what the method computes,
 * written as breadth-first search over an adjacency list:
 *
 *   closure   R1+ = sum_{k>=1} R1^k (Section 2, Eq. 1; Section 3.3, the
 *             output of Algorithm 1): (R1+)_ij = 1 iff a directed path of
 *             length >= 1 leads from i to j.
 *   selection v* = v R1+ (Section 3.3, Eq. 5 and Algorithm 2): the nodes
 *             reached by a path of length >= 1 from any set bit of v.
 *   compose   P = Rs* Rb, the least solution of P = Rb + Rs P, i.e. the
 *             least model of  p(X,Y) <- b(X,Y).  p(X,Y) <- s(X,Z), p(Z,Y).
 *             (Section 3.4, Theorem 1; Eq. 1 with a separate base relation).
 *   warshall  R1+ by Warshall's algorithm: a brute-force cross-check on small
 *             matrices, independent of the BFS code path.
 *
 * Bit layout of every matrix argument: row-major, row i starts at word
 * i*ld; column j is bit (j & 63) of word (j >> 6) (least significant bit
 * first).  Bits of columns >= n are zero in every output.
 *
 * Sources are NOT marked as reached before the search: a source is in its own
 * answer only when it lies on a cycle, which is what makes the closure strict
 * (R1+ rather than I + R1+).  The reflexive flag adds the sources afterwards
 * (used by compose, whose step closure includes paths of length zero).
 *
 * Threads: OpenMP over independent rows; the number actually used is
 * returned through *threads_used.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct {
  int64_t n;
  int64_t *rp;   /* n+1 row offsets */
  int32_t *ci;   /* successor lists */
} oracle_graph;

static int graph_build(int64_t n, int64_t m, const int32_t *src,
                       const int32_t *dst, oracle_graph *g) {
  g->n = n;
  g->rp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  g->ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  if (!g->rp || !g->ci) return -1;
  for (int64_t e = 0; e < m; ++e) {
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return -2;
    g->rp[src[e] + 1]++;
  }
  for (int64_t i = 0; i < n; ++i) g->rp[i + 1] += g->rp[i];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!fill) return -1;
  for (int64_t i = 0; i < n; ++i) fill[i] = g->rp[i];
  for (int64_t e = 0; e < m; ++e) g->ci[fill[src[e]]++] = dst[e];
  free(fill);
  return 0;
}

static void graph_free(oracle_graph *g) {
  free(g->rp);
  free(g->ci);
}

static inline int bit_get(const uint64_t *row, int64_t j) {
  return (int)((row[j >> 6] >> (j & 63)) & 1u);
}
static inline void bit_set(uint64_t *row, int64_t j) {
  row[j >> 6] |= (uint64_t)1 << (j & 63);
}

/* Nodes reachable by a path of length >= 1 from any node of S.  out must
 * hold ceil(n/64) zeroed words; queue holds n entries. */
static void reach_from(const oracle_graph *g, const int32_t *S, int64_t ns,
                       int reflexive, uint64_t *out, int32_t *queue) {
  int64_t head = 0, tail = 0;
  for (int64_t s = 0; s < ns; ++s) {
    int32_t u = S[s];
    for (int64_t e = g->rp[u]; e < g->rp[u + 1]; ++e) {
      int32_t w = g->ci[e];
      if (!bit_get(out, w)) {
        bit_set(out, w);
        queue[tail++] = w;
      }
    }
  }
  while (head < tail) {
    int32_t u = queue[head++];
    for (int64_t e = g->rp[u]; e < g->rp[u + 1]; ++e) {
      int32_t w = g->ci[e];
      if (!bit_get(out, w)) {
        bit_set(out, w);
        queue[tail++] = w;
      }
    }
  }
  if (reflexive)
    for (int64_t s = 0; s < ns; ++s) bit_set(out, S[s]);
}

/* threads <= 0: the OpenMP default of the process (taken at the first call), so that an earlier call
   that asked for a fixed count does not leave it in force */
static int default_threads = 0;

static int set_threads(int threads) {
  if (default_threads == 0) default_threads = omp_get_max_threads();
  omp_set_num_threads(threads > 0 ? threads : default_threads);
  int used = 1;
#pragma omp parallel
  {
#pragma omp single
    used = omp_get_num_threads();
  }
  return used;
}

/* Rows `rows[0..nrows)` of R1+ (all rows 0..n-1 when rows == NULL). */
int bmlp_oracle_closure_rows(int64_t n, int64_t m, const int32_t *src,
                             const int32_t *dst, const int64_t *rows,
                             int64_t nrows, uint64_t *out, int64_t ld,
                             int threads, int *threads_used) {
  if (n < 0 || m < 0 || ld < (n + 63) / 64) return -3;
  oracle_graph g;
  int rc = graph_build(n, m, src, dst, &g);
  if (rc) { graph_free(&g); return rc; }
  if (!rows) nrows = n;
  int used = set_threads(threads);
  if (threads_used) *threads_used = used;
  int bad = 0;
#pragma omp parallel
  {
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!queue) {
#pragma omp atomic write
      bad = 1;
    }
#pragma omp for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; ++r) {
      uint64_t *o = out + r * ld;
      memset(o, 0, sizeof(uint64_t) * (size_t)ld);
      int32_t s = (int32_t)(rows ? rows[r] : r);
      if (queue && s >= 0 && s < n) reach_from(&g, &s, 1, 0, o, queue);
    }
    free(queue);
  }
  graph_free(&g);
  return bad ? -1 : 0;
}

/* out[r] = V[r] R1+  (or V[r] R1* = V[r] + V[r] R1+ when reflexive). */
int bmlp_oracle_smp(int64_t n, int64_t m, const int32_t *src,
                    const int32_t *dst, const uint64_t *V, int64_t k,
                    int64_t ldv, uint64_t *out, int reflexive, int threads,
                    int *threads_used) {
  if (n < 0 || m < 0 || k < 0 || ldv < (n + 63) / 64) return -3;
  oracle_graph g;
  int rc = graph_build(n, m, src, dst, &g);
  if (rc) { graph_free(&g); return rc; }
  int used = set_threads(threads);
  if (threads_used) *threads_used = used;
  int bad = 0;
#pragma omp parallel
  {
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *S = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!queue || !S) {
#pragma omp atomic write
      bad = 1;
    }
#pragma omp for schedule(dynamic, 4)
    for (int64_t r = 0; r < k; ++r) {
      uint64_t *o = out + r * ldv;
      memset(o, 0, sizeof(uint64_t) * (size_t)ldv);
      if (!queue || !S) continue;
      int64_t ns = 0;
      for (int64_t j = 0; j < n; ++j)
        if (bit_get(V + r * ldv, j)) S[ns++] = (int32_t)j;
      reach_from(&g, S, ns, reflexive, o, queue);
    }
    free(queue);
    free(S);
  }
  graph_free(&g);
  return bad ? -1 : 0;
}

/* Rows of P = Rs* Rb: P[X,:] = OR of Rb[Z,:] over Z reachable from X by a
 * step path of length >= 0. */
int bmlp_oracle_compose_rows(int64_t n, int64_t mb, const int32_t *bsrc,
                             const int32_t *bdst, int64_t ms,
                             const int32_t *ssrc, const int32_t *sdst,
                             const int64_t *rows, int64_t nrows,
                             uint64_t *out, int64_t ld, int threads,
                             int *threads_used) {
  if (n < 0 || mb < 0 || ms < 0 || ld < (n + 63) / 64) return -3;
  oracle_graph gb, gs;
  int rc = graph_build(n, mb, bsrc, bdst, &gb);
  if (!rc) rc = graph_build(n, ms, ssrc, sdst, &gs);
  else gs.rp = NULL, gs.ci = NULL;
  if (rc) { graph_free(&gb); graph_free(&gs); return rc; }
  if (!rows) nrows = n;
  int used = set_threads(threads);
  if (threads_used) *threads_used = used;
  int64_t nw = (n + 63) / 64;
  int bad = 0;
#pragma omp parallel
  {
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    uint64_t *zs = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nw > 0 ? nw : 1));
    if (!queue || !zs) {
#pragma omp atomic write
      bad = 1;
    }
#pragma omp for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; ++r) {
      uint64_t *o = out + r * ld;
      memset(o, 0, sizeof(uint64_t) * (size_t)ld);
      int32_t x = (int32_t)(rows ? rows[r] : r);
      if (!queue || !zs || x < 0 || x >= n) continue;
      memset(zs, 0, sizeof(uint64_t) * (size_t)nw);
      reach_from(&gs, &x, 1, 1, zs, queue);
      for (int64_t z = 0; z < n; ++z) {
        if (!bit_get(zs, z)) continue;
        for (int64_t e = gb.rp[z]; e < gb.rp[z + 1]; ++e) bit_set(o, gb.ci[e]);
      }
    }
    free(queue);
    free(zs);
  }
  graph_free(&gb);
  graph_free(&gs);
  return bad ? -1 : 0;
}

/* Warshall (1962): for every intermediate node k, every row that reaches k
 * also reaches everything k reaches.  In place on an n x n bit matrix. */
int bmlp_oracle_warshall(int64_t n, uint64_t *R, int64_t ld) {
  if (n < 0 || ld < (n + 63) / 64) return -3;
  for (int64_t k = 0; k < n; ++k)
    for (int64_t i = 0; i < n; ++i)
      if (bit_get(R + i * ld, k))
        for (int64_t w = 0; w < ld; ++w) R[i * ld + w] |= R[k * ld + w];
  return 0;
}
