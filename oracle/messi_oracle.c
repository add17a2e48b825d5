/*
 * CPU oracle for the MESSI hot path.  TEST INFRASTRUCTURE ONLY: loaded by
 * the tests, the smoke check and the benchmark's CPU-baseline leg, never by
 * the library.  Plain loops in the order the definitions state; built with
 * FP contraction off so every FP32 step rounds exactly once.
 *
 * Citations name the paper's sections, algorithms and equations.
 */
#include "messi_oracle.h"

#include <float.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Summarisation: Section 2.1 (z-normalised data), Section 2.2 (PAA, iSAX). */

/* Threads the OpenMP scans use. */
int32_t oracle_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

/* Whether series and queries are z-normalised before anything else (the
 * paper's default) or taken as they are (its non-normalised variant). */
static int g_normalise = 1;
void oracle_set_normalise(int32_t on) { g_normalise = on ? 1 : 0; }

void oracle_znorm(const float* x, int32_t len, float* z) {
  float s = 0.0f;
  for (int32_t t = 0; t < len; ++t) s = s + x[t];
  const float mu = s / (float)len;
  float v = 0.0f;
  for (int32_t t = 0; t < len; ++t) {
    const float d = x[t] - mu;
    v = v + d * d;
  }
  const float sd = sqrtf(v / (float)len);
  if (!(sd > 0.0f)) {
    for (int32_t t = 0; t < len; ++t) z[t] = 0.0f;
    return;
  }
  for (int32_t t = 0; t < len; ++t) z[t] = (x[t] - mu) / sd;
}

void oracle_paa(const float* z, int32_t len, int32_t w, float* paa) {
  const int32_t m = len / w;
  for (int32_t s = 0; s < w; ++s) {
    float a = 0.0f;
    for (int32_t t = s * m; t < s * m + m; ++t) a = a + z[t];
    paa[s] = a / (float)m;
  }
}

static double std_normal_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

void oracle_breakpoints(int32_t card_bits, float* beta) {
  /* N(0,1) is symmetric: beta at k/card is minus beta at (card-k)/card and
   * the middle breakpoint is exactly 0, so only the lower half is solved. */
  const int32_t card = 1 << card_bits;
  for (int32_t k = 1; 2 * k < card; ++k) {
    const double target = (double)k / (double)card;
    double lo = -40.0, hi = 0.0;
    for (int it = 0; it < 2000; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (mid == lo || mid == hi) break;
      if (std_normal_cdf(mid) < target)
        lo = mid;
      else
        hi = mid;
    }
    /* pick whichever end of the final bracket is closer in Phi */
    const double elo = fabs(std_normal_cdf(lo) - target);
    const double ehi = fabs(std_normal_cdf(hi) - target);
    const double b = elo < ehi ? lo : hi;
    beta[k - 1] = (float)b;
    beta[card - k - 1] = (float)(-b);
  }
  beta[card / 2 - 1] = 0.0f;
}

int32_t oracle_symbol(float p, const float* beta, int32_t card_bits) {
  const int32_t card = 1 << card_bits;
  int32_t c = 0;
  for (int32_t k = 1; k < card; ++k)
    if (beta[k - 1] <= p) c = c + 1;
  return c;
}

/* A series as the index sees it: z-normalised, or as given. */
static void prep_row(const float* x, int32_t len, float* z) {
  if (g_normalise) {
    oracle_znorm(x, len, z);
  } else {
    for (int32_t t = 0; t < len; ++t) z[t] = x[t];
  }
}

void oracle_words(const float* raw, int64_t n, int32_t len, int32_t w, int32_t card_bits,
                  uint8_t* words) {
  float beta[255];
  oracle_breakpoints(card_bits, beta);
  float* z = (float*)malloc(sizeof(float) * (size_t)len);
  float paa[ORACLE_MAX_SEGMENTS];
  for (int64_t i = 0; i < n; ++i) {
    prep_row(raw + i * len, len, z);
    oracle_paa(z, len, w, paa);
    for (int32_t s = 0; s < w; ++s) words[i * w + s] = (uint8_t)oracle_symbol(paa[s], beta, card_bits);
  }
  free(z);
}

/* ------------------------------------------------------------------------ */
/* Leaf partition: root subtrees keyed by the first bit of every segment
 * (Section 3.2, "root subtree" of Algorithm 3; at most 2^w children of the
 * root, Section 2.2); a node holding more than leaf_size series splits on
 * the segment whose next bit divides it most evenly (Section 2.2), ties to
 * the lowest segment, 0-bit child first.  Children left empty are dropped;
 * a node with no segment left to refine stays one over-full leaf. */

typedef struct part_ctx {
  const uint8_t* words;
  int32_t w, card_bits, leaf_size;
  int32_t* perm;
  int32_t* tmp;
  oracle_leaf* leaves;
  int64_t max_leaves, n_leaves;
  int overflow;
} part_ctx;

static int next_bit(const part_ctx* c, int32_t id, int32_t seg, int32_t bits) {
  const uint8_t sym = c->words[(int64_t)id * c->w + seg];
  return (sym >> (c->card_bits - 1 - bits)) & 1;
}

static void emit_leaf(part_ctx* c, int64_t b, int64_t e, const uint8_t* sym, const uint8_t* bits) {
  if (c->n_leaves >= c->max_leaves) {
    c->overflow = 1;
    return;
  }
  oracle_leaf* L = &c->leaves[c->n_leaves++];
  memset(L, 0, sizeof(*L));
  L->begin = b;
  L->end = e;
  for (int32_t s = 0; s < c->w; ++s) {
    L->sym[s] = sym[s];
    L->bits[s] = bits[s];
  }
}

static void split_node(part_ctx* c, int64_t b, int64_t e, const uint8_t* sym, const uint8_t* bits) {
  const int64_t count = e - b;
  if (count == 0) return;
  if (count <= c->leaf_size) {
    emit_leaf(c, b, e, sym, bits);
    return;
  }
  int32_t best = -1;
  int64_t best_gap = 0;
  for (int32_t s = 0; s < c->w; ++s) {
    if (bits[s] >= c->card_bits) continue;
    int64_t c1 = 0;
    for (int64_t i = b; i < e; ++i) c1 += next_bit(c, c->perm[i], s, bits[s]);
    const int64_t gap = llabs(2 * c1 - count);
    if (best < 0 || gap < best_gap) {
      best = s;
      best_gap = gap;
    }
  }
  if (best < 0) { /* every segment at full cardinality */
    emit_leaf(c, b, e, sym, bits);
    return;
  }
  /* stable partition: 0-bit entries first, then 1-bit entries */
  int64_t nz = 0;
  for (int64_t i = b; i < e; ++i)
    if (!next_bit(c, c->perm[i], best, bits[best])) c->tmp[b + nz++] = c->perm[i];
  int64_t no = nz;
  for (int64_t i = b; i < e; ++i)
    if (next_bit(c, c->perm[i], best, bits[best])) c->tmp[b + no++] = c->perm[i];
  for (int64_t i = b; i < e; ++i) c->perm[i] = c->tmp[i];

  uint8_t csym[ORACLE_MAX_SEGMENTS], cbits[ORACLE_MAX_SEGMENTS];
  memcpy(csym, sym, ORACLE_MAX_SEGMENTS);
  memcpy(cbits, bits, ORACLE_MAX_SEGMENTS);
  cbits[best] = (uint8_t)(bits[best] + 1);
  csym[best] = (uint8_t)(sym[best] << 1);
  split_node(c, b, b + nz, csym, cbits);
  csym[best] = (uint8_t)((sym[best] << 1) | 1);
  split_node(c, b + nz, e, csym, cbits);
}

int64_t oracle_leaf_partition(const uint8_t* words, int64_t n, int32_t w, int32_t card_bits,
                              int32_t leaf_size, int32_t* perm, oracle_leaf* leaves,
                              int64_t max_leaves) {
  const int64_t nkeys = (int64_t)1 << w;
  int64_t* count = (int64_t*)calloc((size_t)nkeys + 1, sizeof(int64_t));
  /* root key: first bit of every segment, segment 0 the most significant */
  uint32_t* key = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < n; ++i) {
    uint32_t k = 0;
    for (int32_t s = 0; s < w; ++s) k = (k << 1) | (uint32_t)(words[i * w + s] >> (card_bits - 1));
    key[i] = k;
    count[k + 1] += 1;
  }
  for (int64_t k = 0; k < nkeys; ++k) count[k + 1] += count[k];
  int64_t* cursor = (int64_t*)malloc(sizeof(int64_t) * (size_t)nkeys);
  memcpy(cursor, count, sizeof(int64_t) * (size_t)nkeys);
  for (int64_t i = 0; i < n; ++i) perm[cursor[key[i]]++] = (int32_t)i; /* ascending id per key */

  part_ctx c;
  c.words = words;
  c.w = w;
  c.card_bits = card_bits;
  c.leaf_size = leaf_size;
  c.perm = perm;
  c.tmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  c.leaves = leaves;
  c.max_leaves = max_leaves;
  c.n_leaves = 0;
  c.overflow = 0;
  for (int64_t k = 0; k < nkeys; ++k) {
    if (count[k + 1] == count[k]) continue;
    uint8_t sym[ORACLE_MAX_SEGMENTS] = {0}, bits[ORACLE_MAX_SEGMENTS] = {0};
    for (int32_t s = 0; s < w; ++s) {
      sym[s] = (uint8_t)((k >> (w - 1 - s)) & 1);
      bits[s] = 1;
    }
    split_node(&c, count[k], count[k + 1], sym, bits);
  }
  free(c.tmp);
  free(cursor);
  free(key);
  free(count);
  return c.overflow ? -1 : c.n_leaves;
}

/* ------------------------------------------------------------------------ */
/* Distances (Section 2.1; DTW with a Sakoe-Chiba band of radius r,
 * Section 3.4).  Squared, FP64, index order. */

double oracle_ed2(const float* q, const float* x, int32_t len) {
  double s = 0.0;
  for (int32_t t = 0; t < len; ++t) {
    const double d = (double)q[t] - (double)x[t];
    s = s + d * d;
  }
  return s;
}

/* D(i,j) = c(i,j) + min(D(i-1,j-1), D(i-1,j), D(i,j-1)) over |i-j| <= r,
 * D(0,0) = c(0,0), cells outside the band or the matrix = +inf,
 * c(i,j) = (q_i - x_j)^2; returns D(len-1, len-1). */
double oracle_dtw2(const float* q, const float* x, int32_t len, int32_t r) {
  double* prev = (double*)malloc(sizeof(double) * (size_t)len);
  double* cur = (double*)malloc(sizeof(double) * (size_t)len);
  for (int32_t j = 0; j < len; ++j) prev[j] = INFINITY;
  for (int32_t i = 0; i < len; ++i) {
    for (int32_t j = 0; j < len; ++j) cur[j] = INFINITY;
    const int32_t jlo = i - r < 0 ? 0 : i - r;
    const int32_t jhi = i + r > len - 1 ? len - 1 : i + r;
    for (int32_t j = jlo; j <= jhi; ++j) {
      const double d = (double)q[i] - (double)x[j];
      const double c = d * d;
      if (i == 0 && j == 0) {
        cur[j] = c;
        continue;
      }
      double m = INFINITY;
      if (i > 0 && j > 0 && prev[j - 1] < m) m = prev[j - 1];
      if (i > 0 && prev[j] < m) m = prev[j];
      if (j > 0 && cur[j - 1] < m) m = cur[j - 1];
      cur[j] = c + m;
    }
    double* t = prev;
    prev = cur;
    cur = t;
  }
  const double out = prev[len - 1];
  free(prev);
  free(cur);
  return out;
}

void oracle_envelope(const float* q, int32_t len, int32_t r, float* upper, float* lower) {
  for (int32_t i = 0; i < len; ++i) {
    const int32_t lo = i - r < 0 ? 0 : i - r;
    const int32_t hi = i + r > len - 1 ? len - 1 : i + r;
    float u = q[lo], l = q[lo];
    for (int32_t j = lo; j <= hi; ++j) {
      if (q[j] > u) u = q[j];
      if (q[j] < l) l = q[j];
    }
    upper[i] = u;
    lower[i] = l;
  }
}

double oracle_lb_keogh2(const float* upper, const float* lower, const float* x, int32_t len) {
  double s = 0.0;
  for (int32_t i = 0; i < len; ++i) {
    if (x[i] > upper[i]) {
      const double d = (double)x[i] - (double)upper[i];
      s = s + d * d;
    } else if (x[i] < lower[i]) {
      const double d = (double)x[i] - (double)lower[i];
      s = s + d * d;
    }
  }
  return s;
}

/* Box of a symbol prefix `sym` of `bits` bits: [beta_lo, beta_hi) on the
 * full-cardinality breakpoint table, open ends at -inf / +inf. */
static void box_of(uint8_t sym, uint8_t bits, const float* beta, int32_t card_bits, double* lo,
                   double* hi) {
  const int32_t card = 1 << card_bits;
  const int32_t shift = card_bits - bits;
  const int32_t a = (int32_t)sym << shift;
  const int32_t b = ((int32_t)sym + 1) << shift;
  *lo = a == 0 ? -INFINITY : (double)beta[a - 1];
  *hi = b >= card ? INFINITY : (double)beta[b - 1];
}

double oracle_mindist2_ed(const float* qpaa, const uint8_t* sym, const uint8_t* bits,
                          const float* beta, int32_t w, int32_t len, int32_t card_bits) {
  double s = 0.0;
  for (int32_t k = 0; k < w; ++k) {
    double lo, hi;
    box_of(sym[k], bits[k], beta, card_bits, &lo, &hi);
    const double p = (double)qpaa[k];
    double d = 0.0;
    if (p < lo)
      d = lo - p;
    else if (p > hi)
      d = p - hi;
    s = s + d * d;
  }
  return (double)(len / w) * s;
}

double oracle_mindist2_dtw(const float* upaa, const float* lpaa, const uint8_t* sym,
                           const uint8_t* bits, const float* beta, int32_t w, int32_t len,
                           int32_t card_bits) {
  double s = 0.0;
  for (int32_t k = 0; k < w; ++k) {
    double lo, hi;
    box_of(sym[k], bits[k], beta, card_bits, &lo, &hi);
    double d = 0.0;
    if (lo > (double)upaa[k]) /* box above the upper envelope */
      d = lo - (double)upaa[k];
    else if (hi < (double)lpaa[k]) /* box below the lower envelope */
      d = (double)lpaa[k] - hi;
    s = s + d * d;
  }
  return (double)(len / w) * s;
}

/* ------------------------------------------------------------------------ */
/* k-best lists ordered by (d2, id): the BSF array of Section 5.4. */

static int knn_less(double da, int64_t ia, double db, int64_t ib) {
  if (da < db) return 1;
  if (da > db) return 0;
  if (ia < 0) return 0;
  if (ib < 0) return 1;
  return ia < ib;
}

/* Insert (d, id) into the sorted list of length k; returns 1 if it entered. */
static int knn_insert(int64_t* ids, double* d2, int32_t k, double d, int64_t id) {
  if (!knn_less(d, id, d2[k - 1], ids[k - 1])) return 0;
  int32_t p = k - 1;
  while (p > 0 && knn_less(d, id, d2[p - 1], ids[p - 1])) {
    d2[p] = d2[p - 1];
    ids[p] = ids[p - 1];
    p = p - 1;
  }
  d2[p] = d;
  ids[p] = id;
  return 1;
}

static double pair_dist2(const float* q, const float* x, int32_t len, int32_t distance, int32_t r) {
  return distance == ORACLE_DTW ? oracle_dtw2(q, x, len, r) : oracle_ed2(q, x, len);
}

void oracle_knn_scan(const float* raw_chunk, int64_t id0, int64_t count, int32_t len,
                     const float* raw_queries, int32_t nq, int32_t k, int32_t distance,
                     int32_t r, int64_t* ids, double* d2) {
  float* zq = (float*)malloc(sizeof(float) * (size_t)nq * (size_t)len);
  for (int32_t j = 0; j < nq; ++j) prep_row(raw_queries + (int64_t)j * len, len, zq + (int64_t)j * len);
#pragma omp parallel
  {
    int64_t* lid = (int64_t*)malloc(sizeof(int64_t) * (size_t)nq * (size_t)k);
    double* ld = (double*)malloc(sizeof(double) * (size_t)nq * (size_t)k);
    float* z = (float*)malloc(sizeof(float) * (size_t)len);
    for (int64_t t = 0; t < (int64_t)nq * k; ++t) {
      lid[t] = -1;
      ld[t] = INFINITY;
    }
#pragma omp for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
      prep_row(raw_chunk + i * len, len, z);
      for (int32_t j = 0; j < nq; ++j) {
        const double d = pair_dist2(zq + (int64_t)j * len, z, len, distance, r);
        knn_insert(lid + (int64_t)j * k, ld + (int64_t)j * k, k, d, id0 + i);
      }
    }
#pragma omp critical
    {
      for (int32_t j = 0; j < nq; ++j)
        for (int32_t t = 0; t < k; ++t)
          if (lid[(int64_t)j * k + t] >= 0)
            knn_insert(ids + (int64_t)j * k, d2 + (int64_t)j * k, k, ld[(int64_t)j * k + t],
                       lid[(int64_t)j * k + t]);
    }
    free(z);
    free(ld);
    free(lid);
  }
  free(zq);
}

/* LB_Improved (Lemire, Pattern Recognition 42(9), 2009), the tighter DTW
 * bound Section 3.4 names beside LB_Keogh: LB_Keogh of x against the
 * query's envelope, plus LB_Keogh of the query against the envelope (same
 * radius r) of h, where h is x clamped into the query's envelope. */
double oracle_lb_improved2(const float* q, const float* upper, const float* lower, const float* x,
                           int32_t len, int32_t r) {
  float* h = (float*)malloc(sizeof(float) * (size_t)len);
  float* hu = (float*)malloc(sizeof(float) * (size_t)len);
  float* hl = (float*)malloc(sizeof(float) * (size_t)len);
  for (int32_t t = 0; t < len; ++t)
    h[t] = x[t] > upper[t] ? upper[t] : (x[t] < lower[t] ? lower[t] : x[t]);
  oracle_envelope(h, len, r, hu, hl);
  const double v = oracle_lb_keogh2(upper, lower, x, len) + oracle_lb_keogh2(hu, hl, q, len);
  free(h);
  free(hu);
  free(hl);
  return v;
}

static void knn_scan_filtered(const float* raw_chunk, int64_t id0, int64_t count, int32_t len,
                              const float* raw_queries, int32_t nq, int32_t k, int32_t r,
                              int32_t improved, int64_t* ids, double* d2);

/* Brute-force DTW k-NN with the LB_Keogh filter (Section 3.4): a pair is
 * skipped only when its LB_Keogh exceeds the running k-th best by more than
 * FP64 rounding of two length-len sums can explain (relative 1e-12), so the
 * lists equal those of oracle_knn_scan.  Each thread filters against the
 * smaller of its own k-th best and the k-th best before the chunk, both
 * never below the final one. */
void oracle_knn_scan_lbk(const float* raw_chunk, int64_t id0, int64_t count, int32_t len,
                         const float* raw_queries, int32_t nq, int32_t k, int32_t r,
                         int64_t* ids, double* d2) {
  knn_scan_filtered(raw_chunk, id0, count, len, raw_queries, nq, k, r, 0, ids, d2);
}

/* The same scan filtered by LB_Improved instead of LB_Keogh. */
void oracle_knn_scan_lbi(const float* raw_chunk, int64_t id0, int64_t count, int32_t len,
                         const float* raw_queries, int32_t nq, int32_t k, int32_t r,
                         int64_t* ids, double* d2) {
  knn_scan_filtered(raw_chunk, id0, count, len, raw_queries, nq, k, r, 1, ids, d2);
}

static void knn_scan_filtered(const float* raw_chunk, int64_t id0, int64_t count, int32_t len,
                              const float* raw_queries, int32_t nq, int32_t k, int32_t r,
                              int32_t improved, int64_t* ids, double* d2) {
  float* zq = (float*)malloc(sizeof(float) * (size_t)nq * (size_t)len);
  float* up = (float*)malloc(sizeof(float) * (size_t)nq * (size_t)len);
  float* lo = (float*)malloc(sizeof(float) * (size_t)nq * (size_t)len);
  for (int32_t j = 0; j < nq; ++j) {
    prep_row(raw_queries + (int64_t)j * len, len, zq + (int64_t)j * len);
    oracle_envelope(zq + (int64_t)j * len, len, r, up + (int64_t)j * len, lo + (int64_t)j * len);
  }
  double* bound = (double*)malloc(sizeof(double) * (size_t)nq);  /* k-th best before this chunk */
  for (int32_t j = 0; j < nq; ++j) bound[j] = d2[(int64_t)j * k + k - 1];
#pragma omp parallel
  {
    int64_t* lid = (int64_t*)malloc(sizeof(int64_t) * (size_t)nq * (size_t)k);
    double* ld = (double*)malloc(sizeof(double) * (size_t)nq * (size_t)k);
    float* z = (float*)malloc(sizeof(float) * (size_t)len);
    for (int64_t t = 0; t < (int64_t)nq * k; ++t) {
      lid[t] = -1;
      ld[t] = INFINITY;
    }
#pragma omp for schedule(dynamic, 256)
    for (int64_t i = 0; i < count; ++i) {
      prep_row(raw_chunk + i * len, len, z);
      for (int32_t j = 0; j < nq; ++j) {
        const double own = ld[(int64_t)j * k + k - 1];
        const double kth = own < bound[j] ? own : bound[j];
        const float* qj = zq + (int64_t)j * len;
        const double lb = improved
                              ? oracle_lb_improved2(qj, up + (int64_t)j * len, lo + (int64_t)j * len, z, len, r)
                              : oracle_lb_keogh2(up + (int64_t)j * len, lo + (int64_t)j * len, z, len);
        if (lb > kth * (1.0 + 1e-12)) continue;
        const double d = oracle_dtw2(zq + (int64_t)j * len, z, len, r);
        knn_insert(lid + (int64_t)j * k, ld + (int64_t)j * k, k, d, id0 + i);
      }
    }
#pragma omp critical
    {
      for (int32_t j = 0; j < nq; ++j)
        for (int32_t t = 0; t < k; ++t)
          if (lid[(int64_t)j * k + t] >= 0)
            knn_insert(ids + (int64_t)j * k, d2 + (int64_t)j * k, k, ld[(int64_t)j * k + t],
                       lid[(int64_t)j * k + t]);
    }
    free(z);
    free(ld);
    free(lid);
  }
  free(bound);
  free(lo);
  free(up);
  free(zq);
}

/* ------------------------------------------------------------------------ */
/* Serial index search (Algorithms 5-10, one priority order over all
 * leaves; k-best list per Section 5.4).
 *
 * Lower bounds are computed in FP64 from FP32 PAA values; the FP32 PAA of a
 * series differs from the exact mean of its FP32 points by rounding, so a
 * node is pruned only if its bound exceeds the k-th best by more than that
 * rounding can explain: sqrt(LB2) > sqrt(kth) + eta, with
 * eta = 16 u len sqrt(len / w), u = 2^-24. */

typedef struct lb_order {
  double lb;
  int64_t leaf;
} lb_order;

static int lb_order_cmp(const void* a, const void* b) {
  const lb_order* x = (const lb_order*)a;
  const lb_order* y = (const lb_order*)b;
  if (x->lb < y->lb) return -1;
  if (x->lb > y->lb) return 1;
  return x->leaf < y->leaf ? -1 : (x->leaf > y->leaf ? 1 : 0);
}

static int pruned(double lb2, double kth, double eta) {
  if (isinf(kth)) return 0;
  return sqrt(lb2) > sqrt(kth) + eta;
}

static double norm2_of(const float* v, int32_t len) {
  double a = 0.0;
  for (int32_t t = 0; t < len; ++t) a += (double)v[t] * (double)v[t];
  return a;
}

void oracle_index_search(const float* raw, int64_t n, int32_t len, int32_t w, int32_t card_bits,
                         const uint8_t* words, const int32_t* perm, const oracle_leaf* leaves,
                         int64_t n_leaves, const float* raw_query, int32_t k, int32_t distance,
                         int32_t r, int64_t* ids, double* d2, oracle_search_stats* stats) {
  float beta[255];
  oracle_breakpoints(card_bits, beta);
  float* q = (float*)malloc(sizeof(float) * (size_t)len);
  float* z = (float*)malloc(sizeof(float) * (size_t)len);
  float* U = (float*)malloc(sizeof(float) * (size_t)len);
  float* L = (float*)malloc(sizeof(float) * (size_t)len);
  float qpaa[ORACLE_MAX_SEGMENTS], upaa[ORACLE_MAX_SEGMENTS], lpaa[ORACLE_MAX_SEGMENTS];
  prep_row(raw_query, len, q);
  oracle_paa(q, len, w, qpaa);
  if (distance == ORACLE_DTW) { /* PAA of the query's LB_Keogh envelope */
    oracle_envelope(q, len, r, U, L);
    oracle_paa(U, len, w, upaa);
    oracle_paa(L, len, w, lpaa);
  }
  /* The words and PAAs are FP32 segment means: one is off from the exact
   * mean of a row v by at most 2u sqrt(m)|v|, so a bound moves by at most
   * 2u sqrt(len m)(|x| + |q|), with |x| the largest series norm and |q|
   * the largest of the query and envelope norms.  eta takes 4x that. */
  double xmax = 0.0, qmax = norm2_of(q, len);
  for (int64_t i = 0; i < n; ++i) {
    prep_row(raw + i * len, len, z);
    const double v = norm2_of(z, len);
    if (v > xmax) xmax = v;
  }
  if (distance == ORACLE_DTW) {
    const double nu = norm2_of(U, len), nl = norm2_of(L, len);
    if (nu > qmax) qmax = nu;
    if (nl > qmax) qmax = nl;
  }
  const double eta = 8.0 * ldexp(1.0, -24) * sqrt((double)len * (double)(len / w)) * (sqrt(xmax) + sqrt(qmax));
  memset(stats, 0, sizeof(*stats));
  stats->leaves_total = n_leaves;
  stats->bsf_monotone = 1;
  for (int32_t t = 0; t < k; ++t) {
    ids[t] = -1;
    d2[t] = INFINITY;
  }

  lb_order* order = (lb_order*)malloc(sizeof(lb_order) * (size_t)(n_leaves > 0 ? n_leaves : 1));
  for (int64_t l = 0; l < n_leaves; ++l) {
    const double lb = distance == ORACLE_DTW
                          ? oracle_mindist2_dtw(upaa, lpaa, leaves[l].sym, leaves[l].bits, beta, w, len, card_bits)
                          : oracle_mindist2_ed(qpaa, leaves[l].sym, leaves[l].bits, beta, w, len, card_bits);
    order[l].lb = lb;
    order[l].leaf = l;
  }
  qsort(order, (size_t)n_leaves, sizeof(lb_order), lb_order_cmp);

  uint8_t full_bits[ORACLE_MAX_SEGMENTS];
  for (int32_t s = 0; s < ORACLE_MAX_SEGMENTS; ++s) full_bits[s] = (uint8_t)card_bits;
  double kth_prev = INFINITY;

  /* Pass 0 is the approximate search: the leaf with the smallest bound (the
   * leaf holding the query's own word when there is one), every series
   * refined, giving the first k-best list.  Pass 1 takes the other leaves
   * in ascending bound and stops at the first bound past the k-th best
   * (every later bound is larger). */
  for (int32_t pass = 0; pass < 2; ++pass) {
    int64_t o_begin = 0, o_end = n_leaves > 0 ? 1 : 0;
    if (pass == 0 && n_leaves > 0) stats->approx_leaf = order[0].leaf;
    if (pass == 1) {
      o_begin = 1;
      o_end = n_leaves;
      for (int64_t o = 1; o < n_leaves; ++o)
        if (!pruned(order[o].lb, d2[k - 1], eta)) stats->leaves_enqueued += 1;
    }
    for (int64_t o = o_begin; o < o_end; ++o) {
      if (pass == 1 && pruned(order[o].lb, d2[k - 1], eta)) break;
      const oracle_leaf* lf = &leaves[order[o].leaf];
      if (pass == 1) stats->leaves_processed += 1;
      for (int64_t e = lf->begin; e < lf->end; ++e) {
        const int64_t id = perm[e];
        if (pass == 1) {
          const uint8_t* wd = words + id * w;
          const double slb = distance == ORACLE_DTW
                                 ? oracle_mindist2_dtw(upaa, lpaa, wd, full_bits, beta, w, len, card_bits)
                                 : oracle_mindist2_ed(qpaa, wd, full_bits, beta, w, len, card_bits);
          stats->series_lb += 1;
          if (pruned(slb, d2[k - 1], eta)) continue;
        }
        prep_row(raw + id * len, len, z);
        if (distance == ORACLE_DTW && pass == 1) {
          const double lbk = oracle_lb_keogh2(U, L, z, len);
          stats->lb_keogh += 1;
          if (!isinf(d2[k - 1]) && lbk > d2[k - 1] * (1.0 + 1e-12)) continue;
        }
        const double d = pair_dist2(q, z, len, distance, r);
        stats->real_dist += 1;
        if (knn_insert(ids, d2, k, d, id) && d2[k - 1] != kth_prev) {
          if (!(d2[k - 1] < kth_prev)) stats->bsf_monotone = 0; /* Observation 1 */
          kth_prev = d2[k - 1];
          stats->bsf_updates += 1;
        }
      }
    }
  }
  free(order);
  free(L);
  free(U);
  free(z);
  free(q);
}

/* k-NN classifier (Section 5.4): each query takes the class held by most of
 * its k nearest neighbours; entries with id -1 (fewer than k series) and
 * labels outside [0, n_classes) are skipped; a tie goes to the tied class whose first member comes earliest
 * in the (distance, id) order; no neighbour at all gives -1. */
void oracle_knn_vote(const int64_t* ids, int32_t nq, int32_t k, const int32_t* labels,
                     int32_t n_classes, int32_t* out) {
  int32_t* count = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_classes);
  int32_t* first = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_classes);
  for (int32_t q = 0; q < nq; ++q) {
    for (int32_t c = 0; c < n_classes; ++c) {
      count[c] = 0;
      first[c] = k;
    }
    for (int32_t j = 0; j < k; ++j) {
      const int64_t id = ids[(int64_t)q * k + j];
      if (id < 0) continue;
      const int32_t c = labels[id];
      if (c < 0 || c >= n_classes) continue;  /* not a class: not counted */
      count[c] = count[c] + 1;
      if (first[c] == k) first[c] = j;
    }
    int32_t best = -1;
    for (int32_t c = 0; c < n_classes; ++c) {
      if (count[c] == 0) continue;
      if (best < 0 || count[c] > count[best] || (count[c] == count[best] && first[c] < first[best]))
        best = c;
    }
    out[q] = best;
  }
  free(first);
  free(count);
}
