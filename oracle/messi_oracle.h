/*
 * CPU oracle for the MESSI hot path (Peng, Fatourou, Palpanas: "Fast Data
 * Series Indexing for In-Memory Data").
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the plain, slow definition that
 * the GPU library is checked against.  Only the tests, the smoke check and
 * the benchmark's CPU-baseline leg may load it; the library never calls it
 * and shares no code with it.
 *
 * Every float array is row-major; ids are 0-based row numbers of the raw
 * collection.  All distances returned are SQUARED (the method compares
 * squares; callers take the root), computed in FP64 from the FP32
 * z-normalised values.
 *
 * Parity unpinned: the canonical leaf partition (oracle_leaf_partition) is
 * this code's own reading of the split rule of Section 2.2; the paper fixes
 * its invariants (Theorem 1) but not the partition itself.
 */
#ifndef MESSI_ORACLE_H
#define MESSI_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_ED 0
#define ORACLE_DTW 1
#define ORACLE_MAX_SEGMENTS 16

typedef struct oracle_leaf {
  int64_t begin, end;                   /* range in the permutation */
  uint8_t sym[ORACLE_MAX_SEGMENTS];     /* symbol prefix of each segment */
  uint8_t bits[ORACLE_MAX_SEGMENTS];    /* bits of that prefix (1..card_bits) */
} oracle_leaf;

typedef struct oracle_search_stats {
  int64_t leaves_total;       /* leaves in the index */
  int64_t leaves_enqueued;    /* leaves whose LB passed the first BSF */
  int64_t leaves_processed;   /* leaves taken in LB order before the stop */
  int64_t series_lb;          /* series-level lower bounds computed */
  int64_t lb_keogh;           /* LB_Keogh computations (DTW only) */
  int64_t real_dist;          /* real distance computations */
  int64_t bsf_updates;        /* changes of the k-th best distance */
  int64_t approx_leaf;        /* leaf used by the approximate search */
  int32_t bsf_monotone;       /* 1 if every change decreased the k-th best */
} oracle_search_stats;

/* Z-normalisation (Section 2.1): mean 0, population standard deviation 1,
 * FP32, sums taken in index order.  A constant series maps to zeros. */
/* 0: series and queries are used as given (no z-normalisation) by every
 * function below that takes raw data; 1 (default): z-normalised first. */
void oracle_set_normalise(int32_t on);

/* Number of threads the OpenMP scans use. */
int32_t oracle_threads(void);

void oracle_znorm(const float* x, int32_t len, float* z);

/* PAA (Section 2.2): w equal segments, each the FP32 mean of its points,
 * summed in index order. */
void oracle_paa(const float* z, int32_t len, int32_t w, float* paa);

/* Breakpoints of the equiprobable N(0,1) regions (Section 2.2, iSAX):
 * beta[k-1] = Phi^-1(k / 2^card_bits), k = 1 .. 2^card_bits - 1, found by
 * bisection on Phi(x) = erfc(-x / sqrt 2) / 2 in FP64, rounded to FP32. */
void oracle_breakpoints(int32_t card_bits, float* beta);

/* iSAX symbol of one PAA value: the number of breakpoints <= p. */
int32_t oracle_symbol(float p, const float* beta, int32_t card_bits);

/* Words of n raw series: z-normalise, PAA, symbols (card_bits per symbol). */
void oracle_words(const float* raw, int64_t n, int32_t len, int32_t w, int32_t card_bits,
                  uint8_t* words);

/* Canonical leaf partition of the words (Section 2.2 split rule, Algorithm
 * 4 run top-down on the whole set).  Writes perm[n] and up to max_leaves
 * leaves in depth-first order; returns the leaf count, or -1 if max_leaves
 * is too small. */
int64_t oracle_leaf_partition(const uint8_t* words, int64_t n, int32_t w, int32_t card_bits,
                              int32_t leaf_size, int32_t* perm, oracle_leaf* leaves,
                              int64_t max_leaves);

/* Distances, squared, FP64, points taken in index order. */
double oracle_ed2(const float* q, const float* x, int32_t len);
double oracle_dtw2(const float* q, const float* x, int32_t len, int32_t r);

/* LB_Keogh envelope (Section 3.4) with radius r, clipped to the series. */
void oracle_envelope(const float* q, int32_t len, int32_t r, float* upper, float* lower);
double oracle_lb_keogh2(const float* upper, const float* lower, const float* x, int32_t len);
/* LB_Improved (Lemire 2009; named in Section 3.4): LB_Keogh of x plus
 * LB_Keogh of q against the radius-r envelope of x clamped into [lower,
 * upper].  Squared, like the DTW here. */
double oracle_lb_improved2(const float* q, const float* upper, const float* lower, const float* x,
                           int32_t len, int32_t r);

/* mindist_PAA_iSAX, squared: (len / w) * sum over segments of the squared
 * gap between the query PAA and the box of the node's symbol at its bits.
 * The DTW form uses the PAA of the envelope (upper, lower). */
double oracle_mindist2_ed(const float* qpaa, const uint8_t* sym, const uint8_t* bits,
                          const float* beta, int32_t w, int32_t len, int32_t card_bits);
double oracle_mindist2_dtw(const float* upaa, const float* lpaa, const uint8_t* sym,
                           const uint8_t* bits, const float* beta, int32_t w, int32_t len,
                           int32_t card_bits);

/* Brute-force k-NN by definition over a chunk of the raw collection (rows
 * id0 .. id0+count-1), merged into running per-query lists ids/d2 of
 * length k (initialise to -1 / +inf).  Queries are raw; both sides are
 * z-normalised here.  Lists stay sorted by (d2, id). */
void oracle_knn_scan(const float* raw_chunk, int64_t id0, int64_t count, int32_t len,
                     const float* raw_queries, int32_t nq, int32_t k, int32_t distance,
                     int32_t r, int64_t* ids, double* d2);

/* The same lists for DTW, with LB_Keogh (Section 3.4) skipping pairs whose
 * bound exceeds the running k-th best beyond FP64 rounding. */
void oracle_knn_scan_lbk(const float* raw_chunk, int64_t id0, int64_t count, int32_t len,
                         const float* raw_queries, int32_t nq, int32_t k, int32_t r,
                         int64_t* ids, double* d2);
/* The same scan with the LB_Improved filter. */
void oracle_knn_scan_lbi(const float* raw_chunk, int64_t id0, int64_t count, int32_t len,
                         const float* raw_queries, int32_t nq, int32_t k, int32_t r,
                         int64_t* ids, double* d2);

/* k-NN classifier vote (Section 5.4) over k-NN lists ids [nq][k] (-1 =
 * none): the majority class; a tie goes to the tied class whose first
 * member is nearest; -1 if a list is empty. */
void oracle_knn_vote(const int64_t* ids, int32_t nq, int32_t k, const int32_t* labels,
                     int32_t n_classes, int32_t* out);

/* Serial index search with the method's semantics (Algorithms 5-10 with
 * one priority order): approximate search for the first k-best list, leaf
 * lower bounds, leaves in ascending bound until the bound passes the k-th
 * best, series bounds, (LB_Keogh,) real distances.  The index is given as
 * the raw collection, its words, perm and leaves. */
void oracle_index_search(const float* raw, int64_t n, int32_t len, int32_t w, int32_t card_bits,
                         const uint8_t* words, const int32_t* perm, const oracle_leaf* leaves,
                         int64_t n_leaves, const float* raw_query, int32_t k, int32_t distance,
                         int32_t r, int64_t* ids, double* d2, oracle_search_stats* stats);

#ifdef __cplusplus
}
#endif

#endif /* MESSI_ORACLE_H */
