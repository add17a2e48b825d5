// Shared device-side definitions of libmessi (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace messi {

constexpr int kMaxSeg = 16;       // PAA segments per word (one byte each)
constexpr int kMaxLen = 4096;     // longest series accepted
constexpr int kWave = 64;         // CDNA wavefront width
constexpr int kLbBuckets = 2048;  // logarithmic bound buckets that order the leaves
constexpr int kShards = 64;       // work counters per query (leaves dealt round robin)
constexpr int kChunkSeries = 512; // series per work item of the process phase
constexpr int kCounterStride = 64;  // ints between two shard counters (own 256-byte line)
constexpr int kCounterInts = kShards * kCounterStride + kCounterStride;
constexpr int kApproxCap = 8192;  // most series refined by the approximate search
constexpr int kTopCap = 2048;     // k best + near-tie candidates rechecked per FP64 pass

// Packed (squared distance, id) key: positive FP32 bit patterns order like
// the values, so one 64-bit integer min gives the lexicographic (d2, id)
// min.  The empty slot is (+inf, 0xffffffff).
constexpr unsigned long long kEmptyKey = (0x7f800000ull << 32) | 0xffffffffull;

__device__ __forceinline__ unsigned long long pack_key(float d2, uint32_t id) {
  return ((unsigned long long)__float_as_uint(d2) << 32) | (unsigned long long)id;
}
__device__ __forceinline__ float key_dist(unsigned long long k) {
  return __uint_as_float((uint32_t)(k >> 32));
}
__device__ __forceinline__ uint32_t key_id(unsigned long long k) { return (uint32_t)k; }

// Per-call query constants.
struct QueryParams {
  int nq, len, w, m, card_bits, k, distance;
  int window;        // DTW radius, clipped to len - 1
  int n_leaves;
  int64_t n;
  float win;         // near-tie window factor (1+rho)/(1-rho), rounded up
  float lb_rel;      // (1+rho)(1+2^-16): relative slack on the k-th best
  float eta_c;       // PAA-bound slack per unit of series norm (k_prep turns it into eta[q])
  float xnorm;       // largest 2-norm of an indexed series, rounded up
  float lb_scale;    // power of two that brings bounds into the bucket range
  int raw;           // 1: the index holds series as given (no z-normalisation)
  int lb_improved;   // 1 (DTW): LB_Improved's second pass after LB_Keogh
  int leaf_in_prep;  // 1: k_prep finds the approximate leaf (batches), 0: stage1 does
  int log_cap;       // near-tie log entries per query
  int fin_waves;     // waves used by the FP64 DTW recheck
  int item_cap;      // leaf chunks per query (all shards)
  int lds_words;     // floats of dynamic LDS of the process kernel
  int out_stride;    // output row stride (k of the call, or kmax of a batch)
  int order_leaves;  // 1: stage1 also writes the chunk order of the process kernel
  int count_work;    // 1: the kernels add up their work counters (statistics asked for)
};

// Per-query device state, one entry per query (all arrays sized by nq).
struct QueryState {
  float* zq;                  // [nq][len]   query as the index sees it (z-normalised unless raw)
  float* eta;                 // [nq] absolute slack (distance units) of the PAA-based bounds
  float* upper;               // [nq][len]   LB_Keogh envelope (DTW)
  float* lower;               // [nq][len]
  float* paa;                 // [nq][3][16] query PAA, envelope PAA upper, lower
  int64_t* approx_range;      // [nq][2] positions refined by the approximate search
  float* approx_d2;           // [nq][kApproxCap] their FP32 distances
  unsigned long long* slots;  // [nq][k] running k best (packed keys)
  unsigned long long* log;    // [nq][log_cap] near-tie candidates (d2, position)
  int* log_count;             // [nq]
  float* leaf_lb;             // [nq][n_leaves] leaf bounds
  unsigned long long* items;  // [nq][item_cap] leaf chunks, shard by shard in bucket order (lb bits, leaf)
  int2* ranges;               // [nq][item_cap] their position ranges
  int* next;                  // [nq][kCounterInts]: kShards counters kCounterStride apart, then a finished-shard mask
  unsigned long long* stats;  // [nq][kStatCount] counters (see kStat*)
  int* status;                // [nq] bit 0: near-tie log overflow
  const int* kq;              // [nq] k of each query (batches), or null: every query uses p.k
  const int* qmap;            // [nq] input / output row of each query (batches), or null: row q
};

// k of query q: its own in a batch, else the call's; slots are always p.k apart.
__device__ __forceinline__ int k_of(const QueryParams& p, const QueryState& s, int q) {
  return s.kq ? s.kq[q] : p.k;
}
__device__ __forceinline__ int row_of(const QueryState& s, int q) { return s.qmap ? s.qmap[q] : q; }

// Per-query work counters.  The kStatMin* ones are the work the search
// needs once the final k-th best is known (counted only for statistics).
enum { kStatLeavesKept = 0, kStatSeriesLb, kStatLbKeogh, kStatRefined, kStatRecheck, kStatLbImproved,
       kStatBsf, kStatCells, kStatMinLeaves, kStatMinSeries, kStatMinRefined, kStatCount = 16 };

// Adds a block's work counters to query q's, one device atomic per counter
// per block: each wave first adds its (wave-reduced, lane 0) counts into
// `part` in LDS, which thread 0 then adds to the query's counters.  Device
// atomics on a few addresses from every wave of the grid would queue at the
// memory channel that holds them, so the kernels count only when asked
// (QueryParams::count_work).  Called by every thread of the block.
template <int N>
__device__ __forceinline__ void add_block_counts(unsigned long long* stq, const int (&which)[N],
                                                 const unsigned long long (&val)[N],
                                                 unsigned long long* part) {
  const int tid = threadIdx.x;
  if (tid < N) part[tid] = 0;
  __syncthreads();
  if ((tid & 63) == 0)
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (val[i]) atomicAdd(&part[i], val[i]);
  __syncthreads();
  if (tid < N && part[tid]) atomicAdd(&stq[which[tid]], part[tid]);
  __syncthreads();
}

// iSAX symbol of a PAA value: the number of breakpoints beta_1..beta_{card-1}
// that are <= p, given bp[j] = beta_j (bp[0] = -inf).
__device__ __forceinline__ int symbol_of(float p, const float* __restrict__ bp, int card) {
  int lo = 0, hi = card - 1;  // answer in [lo, hi]
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bp[mid] <= p)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Wavefront reductions with DPP lane moves (quad permutes, row shifts and
// row broadcasts) instead of LDS permutes; the result is read from the last
// lane, so every lane gets the total.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v, float old) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL,
                                                    0xf, 0xf, false));
}

__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f<0xb1>(v, 0.0f);   // quad_perm [1,0,3,2]
  v += dpp_f<0x4e>(v, 0.0f);   // quad_perm [2,3,0,1]
  v += dpp_f<0x114>(v, 0.0f);  // row_shr:4
  v += dpp_f<0x118>(v, 0.0f);  // row_shr:8
  v += dpp_f<0x142>(v, 0.0f);  // row_bcast:15
  v += dpp_f<0x143>(v, 0.0f);  // row_bcast:31
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ float wave_min(float v) {
  const float inf = __builtin_inff();
  v = fminf(v, dpp_f<0xb1>(v, inf));
  v = fminf(v, dpp_f<0x4e>(v, inf));
  v = fminf(v, dpp_f<0x114>(v, inf));
  v = fminf(v, dpp_f<0x118>(v, inf));
  v = fminf(v, dpp_f<0x142>(v, inf));
  v = fminf(v, dpp_f<0x143>(v, inf));
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    unsigned long long u = __shfl_xor(v, o, kWave);
    v = u < v ? u : v;
  }
  return v;
}

// Relaxed load of a value other blocks update atomically (device scope).
__device__ __forceinline__ unsigned long long load_relaxed(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Lock-free insertion into a sorted array of k packed keys held in global
// memory.  Slot j keeps the minimum of everything offered to it and passes
// the larger value on to slot j+1, so after all insertions slot j holds the
// (j+1)-th smallest key ever offered.  Slots only decrease, which makes any
// read of slot k-1 a safe (never too small) pruning threshold.
__device__ __forceinline__ void topk_insert(unsigned long long* slots, int k,
                                            unsigned long long key) {
  for (int j = 0; j < k; ++j) {
    unsigned long long cur = load_relaxed(&slots[j]);
    if (cur <= key) continue;  // slot j already at or below key: key moves on
    unsigned long long old = atomicMin(&slots[j], key);
    key = old > key ? old : key;
    if (key == kEmptyKey) return;
  }
}

}  // namespace messi
