/*
 * libmessi: exact k-NN search over an HBM-resident collection of data series
 * with an iSAX index (Peng, Fatourou, Palpanas, "Fast Data Series Indexing
 * for In-Memory Data"), for one MI355X (gfx950).
 *
 * Problem (Section 2.1): given a collection of same-length series and a
 * query of that length, find the series at the smallest distance, under
 * Euclidean distance or DTW with a Sakoe-Chiba window (Section 3.4); the
 * k-NN form keeps the k best (Section 5.4).  Series and queries are
 * z-normalised by the library (mean 0, standard deviation 1, Section 2.1),
 * unless the index was built with messi_options.raw.
 *
 * Conventions for every call:
 *   - Returns MESSI_OK (0) or a negative MESSI_E* code, and
 *     messi_last_error() describes the cause.  On error the output
 *     buffers' contents are unspecified: a call may fail after its kernels
 *     have written part of them (a rerun that cannot get the memory it
 *     needs, a device error).  Argument errors (MESSI_EINVAL found before
 *     any device work) leave them untouched.
 *   - "device pointer" = memory on the current HIP device (hipMalloc'd or a
 *     torch CUDA tensor); "host pointer" = ordinary process memory.
 *     Passing a host pointer where a device pointer is required is rejected
 *     with MESSI_EINVAL (checked with hipPointerGetAttributes).
 *   - ids are 0-based row numbers of the collection passed to messi_build
 *     (window numbers for messi_build_windows).
 *   - Work is ordered on the index's stream (messi_set_stream; default the
 *     null stream); every call returns after its outputs are complete.
 *   - One index may be queried from one host thread at a time; calls that
 *     overlap on one index return MESSI_EBUSY.
 */
#ifndef MESSI_H
#define MESSI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MESSI_OK = 0,
  MESSI_EINVAL = -1, /* bad argument (sizes, pointer kind, unknown option) */
  MESSI_ENOMEM = -2, /* device memory exhausted or over the option budget */
  MESSI_EDEVICE = -3, /* a HIP call or kernel launch failed */
  MESSI_EBUSY = -4   /* the index is in use by another call */
};

enum { MESSI_ED = 0, MESSI_DTW = 1 };

/* Flags of messi_query_batch, messi_classify and the server
 * (MESSI_GRAPH: messi_query_batch only). */
enum { MESSI_SCREEN_BF16 = 1, MESSI_LB_IMPROVED = 2, MESSI_GRAPH = 4 };

typedef struct messi_index messi_index; /* opaque; owned by the library */

/* Leaf record as exported by messi_get_leaves: the series at leaf-order
 * positions [begin, end) share, in every segment s, the symbol prefix
 * sym[s] of bits[s] bits (Section 2.2, variable cardinality). */
typedef struct messi_leaf {
  int64_t begin, end;
  uint8_t sym[16];
  uint8_t bits[16];
} messi_leaf;

/* Per-call work counters (Table 4 of the paper counts the same things). */
typedef struct messi_stats {
  int64_t queries;
  int64_t leaves_total;     /* leaves in the index, times queries */
  int64_t leaves_kept;      /* 512-series chunks of leaves processed (bound within the k-th best) */
  int64_t series_lb;        /* series-level lower bounds computed */
  int64_t lb_keogh;         /* LB_Keogh bounds computed (DTW) */
  int64_t refined;          /* real distances computed in FP32 */
  int64_t rechecked_fp64;   /* near-tie candidates recomputed in FP64 */
  int64_t log_overflows;    /* reruns forced by a full near-tie log */
  /* device time of each phase in microseconds (HIP events on the index's
   * stream), summed over calls: query preparation; approximate search with
   * the leaf bounds and their order; leaf processing with refinement (for
   * screened batches: the BF16 rows and the screen); FP64 recheck and
   * output */
  double us_prep, us_stage1, us_process, us_finalize;
  int64_t screened;         /* (query, series) pairs through the BF16 screen */
  int64_t lb_improved;      /* LB_Improved second passes (DTW, MESSI_LB_IMPROVED) */
  int64_t bsf_updates;      /* insertions into the k best after the approximate
                               search (the BSF updates of Section 5.4) */
  int64_t dtw_cells;        /* band cells computed by the FP32 register-band DTW
                               (rows computed before the pair ended, within
                               |i - j| <= r and the matrix) */
  /* the work the search needs once its final k-th best is known, counted
   * by a separate pass of messi_query_stats (its time is in no phase
   * above; batches leave these 0): leaves whose bound is within it, the
   * series of those leaves, and those series whose own bound is within it
   * (the series the approximate search refined are left out of the last
   * two) */
  int64_t min_leaves, min_series, min_refined;
} messi_stats;

/* Build an index (Section 3.2: iSAX summaries, then the leaves of the
 * root subtrees).
 *   series      device pointer, float32 [n][len] row-major, read only; the
 *               caller keeps ownership (the library stores its own
 *               z-normalised copy in leaf order).
 *   n           number of series, 1 <= n < 2^31.
 *   len         series length; len % segments == 0, len <= 4096.
 *   segments    PAA segments w, 1..16 (the paper fixes 16, Section 3.1).
 *   cardinality symbols per segment, a power of two in [2, 256] (the paper
 *               uses 256, Section 2.2).
 *   leaf_size   leaf capacity (the paper uses 2000, Section 5.2); a leaf
 *               holds more only when no segment is left to refine.
 *   out         receives the index; free it with messi_free. */
int messi_build(const float* series, int64_t n, int32_t len, int32_t segments,
                int32_t cardinality, int32_t leaf_size, messi_index** out);

/* Build options (zero-initialised = the defaults of messi_build). */
typedef struct messi_options {
  int32_t inplace;     /* 1: z-normalise `series` in place and use it as the
                          store (rows stay in id order, reached through the
                          leaf permutation); the index keeps no copy, so a
                          collection may take most of the device memory.
                          The caller keeps ownership: the buffer must stay
                          allocated and unmodified until messi_free.
                          2: the same, and the index takes the buffer over:
                          messi_free releases it with hipFree, so it must
                          be the start of a hipMalloc allocation (checked
                          with hipMemGetAddressRange; MESSI_EINVAL
                          otherwise) that the caller no longer uses.  If
                          the build fails the caller keeps it.
                          Either way it must be 16-byte aligned. */
  int32_t bf16_screen; /* 1: also make the BF16 copy used by MESSI_SCREEN_BF16 */
  int32_t raw;         /* 1: index the series as given, without z-normalising
                          them (the non-normalised search the paper's
                          Section 1 names); queries on such an index are
                          not normalised either.  Breakpoints, bounds and
                          distances are unchanged; with inplace the rows
                          are left as they are.  Values must be finite with squared
                          row norms below FP32's range. */
  int64_t mem_budget_bytes; /* 0: no limit beyond the device.  Otherwise the
                          device bytes the index may hold - its tables, a
                          store it owns (its copy, or an inplace = 2
                          buffer), the BF16 copy and the buffers of its own
                          calls; a build or call that would exceed it
                          fails with MESSI_ENOMEM.  A server started with
                          mem_budget_bytes 0 takes what is left of it. */
  const char* autotune_cache; /* NULL: none.  Path of a JSON file of tuned
                          knobs (messi_autotune): read here (a missing file
                          is an empty cache; a file this library did not
                          write is MESSI_EINVAL) and written back by every
                          messi_autotune that measures; its entries steer
                          messi_query_batch for the batch shapes they name. */
} messi_options;

/* messi_build with options (NULL = defaults): the same index construction
 * (Section 3.2; Algorithms 1-4).  With inplace, `series` is overwritten
 * with its z-normalised rows and becomes the store, which lets a
 * collection of most of the device's memory be indexed (the paper's
 * in-memory setting, Section 5.1); otherwise it is only read.  Errors as
 * for messi_build, plus MESSI_ENOMEM over mem_budget_bytes and
 * MESSI_EINVAL for an autotune_cache file it cannot read. */
int messi_build_ex(float* series, int64_t n, int32_t len, int32_t segments, int32_t cardinality,
                   int32_t leaf_size, const messi_options* opts, messi_index** out);

/* Subsequence matching (Section 2.1; the sliding-window adaptation noted
 * with the related work in Section 6): index every window of length `len`
 * of one long device series.
 *   series      device float32[total], the long series (only read).
 *   total       its number of points, >= len.
 *   stride      distance between window starts (1 = every window).
 *   segments, cardinality, leaf_size, opts: as for messi_build_ex; opts->raw
 *               selects raw windows (the usual setting of subsequence
 *               search) or z-normalised ones; opts->inplace is ignored.
 * The index materialises the (total - len) / stride + 1 windows in device
 * memory it owns and frees in messi_free; id i of a query answer is the
 * window starting at point i * stride.  Errors: MESSI_EINVAL on bad
 * arguments, MESSI_ENOMEM if the windows or the index do not fit. */
int messi_build_windows(const float* series, int64_t total, int32_t len, int32_t stride,
                        int32_t segments, int32_t cardinality, int32_t leaf_size,
                        const messi_options* opts, messi_index** out);

/* Exact k-NN (Algorithms 5-10; k-NN per Section 5.4).
 *   queries    device pointer, float32 [nq][len] (raw; z-normalised here).
 *   nq         number of queries, >= 0 (0 returns at once).
 *   k          neighbours per query, 1 <= k <= 1024.
 *   distance   MESSI_ED or MESSI_DTW.
 *   window     DTW Sakoe-Chiba radius r in points (0 <= r; r >= len-1 is
 *              unconstrained DTW; ignored for ED).
 *   out_ids    device pointer, int64 [nq][k]; out_dists device pointer,
 *              float32 [nq][k]; each row ascending by (distance, id); the
 *              distance is the square root of the sum of squared
 *              differences (ED) or of the squared-cost DTW; rows past n
 *              neighbours hold id -1, distance +inf.
 * Answers are exact: equal, id for id, to a brute-force scan that computes
 * every distance in FP64 from the z-normalised FP32 values, ties broken by
 * the lower id.
 * Long series: the query kernels keep the query and per-wave rows in LDS,
 * up to what one block may use on the device (160 KB on gfx950).  There,
 * ED and DTW with r <= 31 accept every len up to 4096, DTW with r <= 64
 * up to len 3968, and DTW with a wider window up to len 1670; longer ones
 * fail with MESSI_EINVAL. */
int messi_query(messi_index* index, const float* queries, int32_t nq, int32_t k,
                int32_t distance, int32_t window, int64_t* out_ids, float* out_dists);

/* messi_query for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * same queries, kernels and answers, with the query state in a
 * file-scope device array of 64 MiB instead of memory the library
 * allocates; the call makes no hipMalloc, hipFree or other allocation.
 * Each GPU the library runs on holds its own copy of the array until the
 * process ends.
 *   Arguments and outputs as for messi_query; nq <= 1024.
 *   Limits: the state of the nq queries (about 16 bytes per 512-series
 *   chunk of the index, 4 bytes per leaf and about 330 KB more per query)
 *   must fit the 64 MiB, else MESSI_EINVAL with the sizes in the message;
 *   a query whose near-tie log (32768 entries) overflows returns
 *   MESSI_ENOMEM (messi_query, which grows the log, answers it).
 *   Every call on one GPU shares the array: calls that overlap on one GPU
 *   (on any index) race and must not be made. */
int messi_query_noalloc(messi_index* index, const float* queries, int32_t nq, int32_t k,
                        int32_t distance, int32_t window, int64_t* out_ids, float* out_dists);

/* Same as messi_query, also returning work counters (stats may be NULL). */
int messi_query_stats(messi_index* index, const float* queries, int32_t nq, int32_t k,
                      int32_t distance, int32_t window, int64_t* out_ids, float* out_dists,
                      messi_stats* stats);

/* Batch of exact k-NN queries with per-query k, distance and window
 * (Section 5.4's k-best array per query; Sections 3.3 and 3.4).  Queries
 * that share a distance and an effective window run together, one launch
 * per phase for the whole group.
 *   queries    device pointer, float32 [nq][len] (raw).
 *   k, distance, window   HOST arrays of nq entries (as in messi_query);
 *              1 <= k[i] <= kmax.
 *   kmax       row length of the outputs, 1..1024.
 *   flags      MESSI_SCREEN_BF16: ED queries, in groups of at least 32,
 *              go through a BF16 MFMA screen (q.x with FP32 accumulation
 *              and a rigorous error bound) in front of the FP32 refinement; needs len 64, 128, 256 or 512
 *              (otherwise ignored) and 2 len bytes per series of
 *              device memory for a BF16 copy of the store, made on first
 *              use (or ahead of time by messi_prepare_screen).  Answers are
 *              identical with and without the flag.
 *              MESSI_LB_IMPROVED: DTW candidates that pass LB_Keogh are
 *              also tested with LB_Improved (Lemire 2009, named in Section
 *              3.4 as the tighter, costlier alternative) before DTW.  Same
 *              answers; ignored where its LDS buffers do not fit (long
 *              series with a small window).
 *              MESSI_GRAPH: the batch's launches are captured in a HIP
 *              graph, kept (up to 8 per index) and replayed by later calls
 *              whose launches would be identical, argument for argument
 *              (same queries and output pointers, nq, kmax, k, distance,
 *              window, flags and buffers); ignored when stats is given.
 *              Same answers.
 *   out_ids    device pointer, int64 [nq][kmax]; out_dists device pointer,
 *              float32 [nq][kmax]: row i holds query i's k[i] neighbours
 *              ascending by (distance, id), then (-1, +inf) up to kmax.
 *   stats      may be NULL; counters and phase times summed over groups
 *              (groups may run concurrently, so the times may add up to
 *              more than the call took).
 * Groups of different (distance, window) run concurrently on streams of
 * their own, joined back into the index's stream, unless the tuned knobs
 * for this batch shape say otherwise (messi_autotune). */
int messi_query_batch(messi_index* index, const float* queries, int32_t nq, const int32_t* k,
                      const int32_t* distance, const int32_t* window, int32_t kmax, int32_t flags,
                      int64_t* out_ids, float* out_dists, messi_stats* stats);

/* Knobs of messi_query_batch for one batch shape, as messi_autotune
 * chose them (the defaults are the built-in choices). */
typedef struct messi_tune {
  int32_t screen;      /* 1: ED groups take the BF16 screen when asked for */
  int32_t screen_min;  /* fewest ED queries in a screened group (32) */
  int32_t screen_nt;   /* 16-series column tiles per wave of the screen
                          kernel (0: 4, or 1 for len 512) */
  int32_t screen_occ;  /* screen blocks per CU (0: the occupancy limit) */
  int32_t ed_scale;    /* ED process grid, in resident grids (1) */
  int32_t dtw_scale;   /* DTW process blocks per query, in multiples of an
                          even share of the resident grid (1) */
  int32_t overlap;     /* 1: groups run concurrently (1) */
  int32_t from_cache;  /* 1: found in the cache, nothing measured */
  int32_t candidates;  /* knob settings timed */
  int32_t screen_waves; /* waves per screen block (0: 4, two blocks to a
                          CU; 8: one) */
  double ms;           /* batch time with these knobs (best of up to 2 runs) */
  double ms_default;   /* batch time with the defaults */
} messi_tune;

/* Autotuner of messi_query_batch (not part of the paper's method): times
 * the batch (arguments as for messi_query_batch) with the default knobs
 * and then one knob at a time - screen on / off, the screen kernel's
 * column tiles, waves per block and blocks per CU, the ED grid, DTW
 * blocks per query, concurrent groups - keeping a setting only if it is at least 2% faster,
 * and checks that every setting's answers equal the defaults' bit for bit
 * (MESSI_EDEVICE if not).  The choice is kept in the index for batches of
 * the same shape (device, index shape, nq rounded up to a power of two,
 * (distance, window) mix, flags) and written to messi_options'
 * autotune_cache file if one was given.  A shape already tuned (in this
 * index or the file) returns its entry with from_cache = 1 at once.
 * The runs write to buffers of the library's own (2 nq kmax x 12 bytes). */
int messi_autotune(messi_index* index, const float* queries, int32_t nq, const int32_t* k,
                   const int32_t* distance, const int32_t* window, int32_t kmax, int32_t flags,
                   messi_tune* out);

/* k-NN classifier (Section 5.4): each query takes the class held by most of
 * its k nearest neighbours (as messi_query_batch computes them, flags
 * alike); a tie goes to the tied class whose first member is nearest in
 * the (distance, id) order.
 *   labels     device pointer, int32 [n], the class of each series by id;
 *              values outside [0, n_classes) are not counted.
 *   n_classes  1..4096.
 *   out_class  device pointer, int32 [nq]: the class, or -1 if no series.
 *   out_ids, out_dists   device pointers [nq][k]: the neighbours voted on. */
int messi_classify(messi_index* index, const int32_t* labels, int32_t n_classes,
                   const float* queries, int32_t nq, int32_t k, int32_t distance, int32_t window,
                   int32_t flags, int32_t* out_class, int64_t* out_ids, float* out_dists);

/* Make the BF16 copy of the store and its row norms used by
 * MESSI_SCREEN_BF16 now rather than on the first screened batch.  The
 * copy lives until messi_free. */
int messi_prepare_screen(messi_index* index);

/* Serving loop over a built index.  Requests carry one raw query (HOST
 * memory, len floats, copied at submit) with its k, distance and window.
 * Worker threads, each with its own HIP stream and buffers, repeatedly take
 * the pending requests that fit - at most the batch capacity, and only while
 * the device bytes held by admitted, unfinished requests stay within
 * mem_budget_bytes (a request alone is always admitted) - and run them as
 * one messi_query_batch-style batch; requests arriving meanwhile go to the
 * next free worker, so batches overlap on the GPU.  Answers equal those of
 * messi_query for the same query, k, distance and window.
 * The index must outlive the server and must not be freed while it runs. */
typedef struct messi_server messi_server;

typedef struct messi_server_options { /* zero-initialised = defaults */
  int32_t workers;          /* concurrent batches, 1..8 (0: 2) */
  int32_t max_batch;        /* most requests per batch (0: 1024) */
  int64_t mem_budget_bytes; /* device bytes the workers may hold (0: what the
                               index's budget leaves, or no limit): every
                               worker holds the buffers of its batch
                               capacity from the start, which is cut until
                               all workers fit; a batch whose near-tie log
                               grows charges the growth to the in-flight
                               bytes and returns it when the log is shrunk
                               back after the batch */
  int32_t flags;            /* MESSI_SCREEN_BF16: screen ED requests;
                               MESSI_LB_IMPROVED: LB_Improved for DTW requests */
  int32_t kmax;             /* largest k a request may ask (0: 64) */
} messi_server_options;

typedef struct messi_server_stats {
  int64_t submitted, completed, batches, max_batch_seen;
  int64_t inflight_bytes, peak_inflight_bytes, mem_budget_bytes;
  int64_t request_bytes;    /* device bytes accounted per admitted request */
  int64_t batch_capacity;   /* requests a worker can take at once */
  double busy_us;           /* summed worker time with a batch on the GPU */
  int64_t resident_bytes;   /* device bytes the workers hold now */
  int64_t log_growth_bytes; /* near-tie log growth charged so far (summed);
                               in-flight bytes stay within the budget plus
                               what a growth charges while its batch runs */
} messi_server_stats;

int messi_server_start(messi_index* index, const messi_server_options* opts, messi_server** out);
/* Queue one request; *id receives its number (0, 1, 2, ... in submit order). */
int messi_server_submit(messi_server* server, const float* query, int32_t k, int32_t distance,
                        int32_t window, uint64_t* id);
/* Up to max finished requests into HOST arrays: req_ids[max], status[max]
 * (MESSI_OK or the batch's error), ids[max][kmax], dists[max][kmax] (k
 * entries then -1 / +inf), latency_us[max] (submit to result); any array
 * may be NULL.  Waits up to timeout_ms for the first one (-1: no limit,
 * 0: no wait).  *count receives the number returned. */
int messi_server_poll(messi_server* server, int32_t max, int32_t timeout_ms, uint64_t* req_ids,
                      int32_t* status, int64_t* ids, float* dists, double* latency_us,
                      int32_t* count);
int messi_server_get_stats(messi_server* server, messi_server_stats* stats);
/* Finish every queued request, stop the workers and free the server. */
void messi_server_stop(messi_server* server);

/* Order the index's work after / before the caller's on this HIP stream
 * (e.g. torch.cuda.current_stream().cuda_stream).  NULL = null stream.
 * Library plumbing (no passage of the paper): a batch's further groups
 * and graph captures use streams of the library's own, joined back into
 * this one; the stream must stay valid while the index uses it. */
int messi_set_stream(messi_index* index, void* hip_stream);

/* Shape of a built index (any pointer may be NULL). */
int messi_index_info(const messi_index* index, int64_t* n, int32_t* len, int32_t* segments,
                     int32_t* card_bits, int64_t* n_leaves, int64_t* device_bytes);

/* Host wall time of the build call that made the index, in ms, and the part
 * of it spent in device allocation (hipMalloc), which depends on the device's
 * state: a driver may clear reused memory before handing it out.  Library
 * plumbing (no passage of the paper).  Either pointer may be NULL. */
int messi_build_times(const messi_index* index, double* build_ms, double* alloc_ms);

/* Copies out of a built index into HOST buffers, for inspection and tests:
 *   words   uint8 [n][segments], series in id order (Section 2.2 symbols);
 *   perm    int32 [n], the id at each leaf-order position;
 *   leaves  messi_leaf [cap]; *count receives the number of leaves (if
 *           cap is too small nothing is copied and MESSI_EINVAL returned). */
int messi_get_words(const messi_index* index, uint8_t* words);
int messi_get_perm(const messi_index* index, int32_t* perm);
int messi_get_leaves(const messi_index* index, messi_leaf* leaves, int64_t cap, int64_t* count);

/* The library's breakpoint table (Section 2.2): beta[k-1] = Phi^-1(k/2^b)
 * for k = 1 .. 2^b - 1, as FP32, into a HOST buffer. */
int messi_breakpoints(int32_t card_bits, float* beta);

/* Library plumbing (no passage of the paper): releases every device and
 * pinned host buffer of the index, and an inplace = 2 store; NULL is a
 * no-op.  No call on the index may be running. */
void messi_free(messi_index* index);

/* Description of the last error on this thread; valid until the next call
 * (library plumbing, no passage of the paper). */
const char* messi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MESSI_H */
