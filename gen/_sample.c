/* Input sampling helper for the synthetic workload generator.
 *
 * This file holds no part of the estimators: it only turns a stream of
 * uniform random numbers (drawn by numpy's PCG64 on the Python side) into
 * word ids drawn from a truncated Zipf law, keeping for each document the
 * first m distinct ids of its draw sequence.  A vectorised numpy version of
 * the same loop needs a sort per document, which is slow at a million
 * documents; this loop is linear in the number of draws.
 */
#include <stdint.h>

/* Index of the first cdf entry strictly greater than u (numpy searchsorted,
 * side="right"), accelerated by a guide table: guide[g] is the first index i
 * with cdf[i] > g / G, so the answer for u in [g/G, (g+1)/G) is >= guide[g]. */
static int64_t inv_cdf(const double* cdf, int64_t V, const int64_t* guide,
                       int64_t G, double u) {
  int64_t g = (int64_t)(u * (double)G);
  if (g >= G) g = G - 1;
  int64_t i = guide[g];
  while (i < V - 1 && !(cdf[i] > u)) ++i;
  return i;
}

void gen_build_guide(const double* cdf, int64_t V, int64_t G, int64_t* guide) {
  int64_t i = 0;
  for (int64_t g = 0; g < G; ++g) {
    double t = (double)g / (double)G;
    while (i < V - 1 && !(cdf[i] > t)) ++i;
    guide[g] = i;
  }
}

/* Consume uniforms u[pos..n_u) doc by doc, starting at document doc0.
 * Document j needs sizes[j] distinct ids; they are written to
 * out_ids[out_off[j] .. out_off[j] + sizes[j]) in order of first appearance.
 * stamp[V] must hold values different from every doc index + 1 on entry for
 * the documents processed (it is used as a per-document "seen" marker).
 * Returns the index of the first document that could not be completed with
 * the uniforms available (n_docs when all were); *pos_io is advanced past the
 * uniforms used by the completed documents only, so the caller can append
 * more uniforms and resume at the same document with identical results. */
int64_t gen_first_distinct(const double* cdf, int64_t V, const int64_t* guide,
                           int64_t G, const double* u, int64_t n_u,
                           int64_t* pos_io, const int64_t* sizes,
                           const int64_t* out_off, int64_t doc0, int64_t n_docs,
                           uint32_t* out_ids, int64_t* stamp) {
  int64_t pos = *pos_io;
  for (int64_t j = doc0; j < n_docs; ++j) {
    int64_t need = sizes[j], got = 0, p = pos;
    uint32_t* dst = out_ids + out_off[j];
    while (got < need) {
      if (p >= n_u) {
        for (int64_t t = 0; t < got; ++t) stamp[dst[t]] = 0; /* undo doc j */
        *pos_io = pos;
        return j;
      }
      int64_t id = inv_cdf(cdf, V, guide, G, u[p++]);
      if (stamp[id] != j + 1) { stamp[id] = j + 1; dst[got++] = (uint32_t)id; }
    }
    pos = p;
  }
  *pos_io = pos;
  return n_docs;
}

/* k-th smallest (0-based) of a[0..m) by Hoare's selection; a is permuted. */
static uint32_t select_kth(uint32_t* a, int64_t m, int64_t k) {
  int64_t lo = 0, hi = m - 1;
  while (lo < hi) {
    uint32_t piv = a[lo + (hi - lo) / 2];
    int64_t i = lo, j = hi;
    while (i <= j) {
      while (a[i] < piv) ++i;
      while (a[j] > piv) --j;
      if (i <= j) { uint32_t t = a[i]; a[i] = a[j]; a[j] = t; ++i; --j; }
    }
    if (k <= j) hi = j;
    else if (k >= i) lo = i;
    else return a[k];
  }
  return a[k];
}

/* Uniform fixed-point masses: distribution j over m distinct ids gets
 * floor(2^Q / m) per id, plus one unit for the (2^Q mod m) smallest ids.
 * scratch must hold the largest support.  Returns -1 on an empty support. */
int64_t gen_uniform_masses(const int64_t* off, const uint32_t* ids, int64_t n,
                           int32_t Q, uint32_t* mass, uint32_t* scratch) {
  const int64_t total = (int64_t)1 << Q;
  for (int64_t j = 0; j < n; ++j) {
    int64_t a = off[j], m = off[j + 1] - off[j];
    if (m <= 0) return -1;
    int64_t base = total / m, rem = total - base * m;
    uint32_t cut = 0;
    if (rem > 0) {
      for (int64_t t = 0; t < m; ++t) scratch[t] = ids[a + t];
      cut = select_kth(scratch, m, rem - 1);
    }
    for (int64_t t = 0; t < m; ++t)
      mass[a + t] = (uint32_t)(base + (rem > 0 && ids[a + t] <= cut ? 1 : 0));
  }
  return 0;
}
