// Exact k-NN query kernels (Algorithms 5-10 of the paper, k-NN per Section
// 5.4), for ED and for DTW with a Sakoe-Chiba band (Section 3.4).
//
// Phases, each one launch over all queries of a call (grid.y = query):
//   prep     z-normalise the query, PAA (and LB_Keogh envelope + its PAA),
//            the per-segment bound table, and the approximate-search leaf:
//            the leaf reached by descending the tree along the query's word.
//   stage1   two kinds of blocks in one launch: some refine the series of
//            the approximate leaf (the first k-best list, Algorithm 5), the
//            others compute mindist of every leaf; leaves are dealt to 64
//            shards (leaf l to shard l mod 64) and each shard's block
//            writes its leaves' 512-series chunks in ascending order of
//            2048 logarithmic bound buckets: the ascending-bound order the
//            paper's priority queues give, kept per shard.
//   process  chunks are taken in that order (the queues' DeleteMin): for
//            DTW by blocks through the shards' atomic counters, for ED by
//            the waves of a block from the block's share of every shard,
//            through counters in LDS; per chunk: series bounds from the
//            table in LDS, [LB_Keogh,] FP32 refinement, the k best kept by
//            a lock-free atomicMin cascade.  A shard (or a block's share of
//            it) stops at the first chunk whose bucket starts above the
//            current k-th best (every later chunk is at least that far).
//   finalize FP64 recheck of the near ties and the exact (distance, id)
//            order of the answer.
//
// Exactness: every prune compares a bound against the k-th best with slack
// covering the FP32 rounding of both sides; every refined distance within
// the FP32 error window of the running k-th best is logged, and the final
// order is decided on FP64 distances of the logged candidates.
#include <hip/hip_runtime.h>

#include <atomic>
#include <algorithm>
#include <mutex>
#include <stdint.h>

#include "query.h"

namespace messi {

__device__ __forceinline__ unsigned long long load_key(const unsigned long long* p) {
  return load_relaxed(p);
}

__device__ __forceinline__ float kth_dist(const unsigned long long* slots, int k) {
  return key_dist(load_key(&slots[k - 1]));
}

// Bound threshold: a series whose bound exceeds it cannot be among the k
// best.  (sqrt(kth (1+rho)) + eta)^2, with a last relative margin for the
// rounding of this expression itself; eta is the query's own slack.
__device__ __forceinline__ float lb_threshold(float thr, float eta, const QueryParams& p) {
  if (!(thr < INFINITY)) return INFINITY;
  const float r = sqrtf(thr * p.lb_rel) + eta;
  return r * r * 1.0001f;
}

// Logarithmic bound buckets: exponent and top 6 mantissa bits of the FP32
// bound, over [2^-16, 2^16); monotone in the bound.  Callers pass the bound
// times p.lb_scale (a power of two, so the product is exact).
constexpr int kBucketBase = (127 - 16) << 6;
__device__ __forceinline__ int lb_bucket(float lb) {
  const int b = (int)(__float_as_uint(lb) >> 17) - kBucketBase;
  return b < 0 ? 0 : (b >= kLbBuckets ? kLbBuckets - 1 : b);
}
__device__ __forceinline__ float bucket_floor(int b) {
  return b <= 0 ? 0.0f : __uint_as_float((uint32_t)(b + kBucketBase) << 17);
}

__device__ __forceinline__ uint32_t byte_of(const uint4& v, int s) {
  const uint32_t x = s < 4 ? v.x : (s < 8 ? v.y : (s < 12 ? v.z : v.w));
  return (x >> (8 * (s & 3))) & 0xffu;
}

__device__ __forceinline__ unsigned long long umin64(unsigned long long a, unsigned long long b) {
  return a < b ? a : b;
}

// Workgroup-scope atomics on LDS words shared by the waves of a block.
__device__ __forceinline__ int lds_add(int* a, int v) {
  return __hip_atomic_fetch_add(a, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ int lds_load_acq(int* a) {
  return __hip_atomic_load(a, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_store_rel(int* a, int v) {
  __hip_atomic_store(a, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ unsigned lds_load_acq_u(unsigned* a) {
  return __hip_atomic_load(a, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_or_u(unsigned* a, unsigned v) {
  __hip_atomic_fetch_or(a, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Lane 0's 64-bit value, to every lane (lane 0 must be active).
__device__ __forceinline__ unsigned long long first_lane_u64(unsigned long long v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

// Squared ED between an LDS query and a global row, one wave.
__device__ __forceinline__ float ed_wave(const float* __restrict__ zq, const float* __restrict__ x,
                                         int len, int lane) {
  float acc = 0.0f;
  if ((len & 3) == 0) {
    for (int t = 4 * lane; t < len; t += 4 * kWave) {
      const float4 a = *reinterpret_cast<const float4*>(x + t);
      const float4 b = *reinterpret_cast<const float4*>(zq + t);
      const float d0 = a.x - b.x, d1 = a.y - b.y, d2 = a.z - b.z, d3 = a.w - b.w;
      acc = __builtin_fmaf(d0, d0, acc);
      acc = __builtin_fmaf(d1, d1, acc);
      acc = __builtin_fmaf(d2, d2, acc);
      acc = __builtin_fmaf(d3, d3, acc);
    }
  } else {
    for (int t = lane; t < len; t += kWave) {
      const float d = x[t] - zq[t];
      acc = __builtin_fmaf(d, d, acc);
    }
  }
  return wave_sum(acc);
}

// Squared ED (or LB_Keogh) of up to eight rows at once, their loads in
// flight together.  Rows are given by wave-uniform positions and an active
// mask; results for inactive rows are undefined.  Every row is loaded,
// active or not (an inactive row reads the first active one, which the
// caches then serve): a load under a per-row branch would be waited for
// before the next one issues, one memory round trip per row.
constexpr int kGroup = 8;

template <int G>
__device__ __forceinline__ void group_rows(const float* __restrict__ Z, int len, const int (&pos)[G],
                                           unsigned& act, const float* (&row)[G]) {
  act = __builtin_amdgcn_readfirstlane(act);
  const int lead = pos[__builtin_ctz(act | (1u << (G - 1)))];
#pragma unroll
  for (int c = 0; c < G; ++c) {
    const int pc = __builtin_amdgcn_readfirstlane(((act >> c) & 1u) ? pos[c] : lead);
    row[c] = Z + (int64_t)pc * len;
  }
}

template <int G>
__device__ __forceinline__ void ed_rows(const float* __restrict__ zq, const float* __restrict__ Z,
                                        int len, const int (&pos)[G], unsigned act, int lane,
                                        float (&out)[G]) {
  const float* row[G];
  group_rows<G>(Z, len, pos, act, row);
  float acc[G];
#pragma unroll
  for (int c = 0; c < G; ++c) acc[c] = 0.0f;
  if ((len & 3) == 0) {
    for (int t = 4 * lane; t < len; t += 4 * kWave) {
      const float4 b = *reinterpret_cast<const float4*>(zq + t);
      float4 x[G];
#pragma unroll
      for (int c = 0; c < G; ++c) x[c] = *reinterpret_cast<const float4*>(row[c] + t);
#pragma unroll
      for (int c = 0; c < G; ++c) {
        const float e0 = x[c].x - b.x, e1 = x[c].y - b.y, e2 = x[c].z - b.z, e3 = x[c].w - b.w;
        acc[c] = __builtin_fmaf(e0, e0, acc[c]);
        acc[c] = __builtin_fmaf(e1, e1, acc[c]);
        acc[c] = __builtin_fmaf(e2, e2, acc[c]);
        acc[c] = __builtin_fmaf(e3, e3, acc[c]);
      }
    }
  } else {
    for (int t = lane; t < len; t += kWave) {
      const float b = zq[t];
      float x[G];
#pragma unroll
      for (int c = 0; c < G; ++c) x[c] = row[c][t];
#pragma unroll
      for (int c = 0; c < G; ++c) {
        const float e = x[c] - b;
        acc[c] = __builtin_fmaf(e, e, acc[c]);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < G; ++c) out[c] = ((act >> c) & 1u) ? wave_sum(acc[c]) : 0.0f;
}

__device__ __forceinline__ void ed_group(const float* __restrict__ zq, const float* __restrict__ Z,
                                         int len, const int (&pos)[kGroup], unsigned act, int lane,
                                         float (&out)[kGroup]) {
  ed_rows<kGroup>(zq, Z, len, pos, act, lane, out);
}

__device__ __forceinline__ void lbk_group(const float* __restrict__ U, const float* __restrict__ L,
                                          const float* __restrict__ Z, int len, const int (&pos)[kGroup],
                                          unsigned act, int lane, float (&out)[kGroup]) {
  const float* row[kGroup];
  group_rows<kGroup>(Z, len, pos, act, row);
  float acc[kGroup];
#pragma unroll
  for (int c = 0; c < kGroup; ++c) acc[c] = 0.0f;
  for (int t = lane; t < len; t += kWave) {
    const float u = U[t], l = L[t];
    float x[kGroup];
#pragma unroll
    for (int c = 0; c < kGroup; ++c) x[c] = row[c][t];
#pragma unroll
    for (int c = 0; c < kGroup; ++c) {
      const float v = x[c];
      const float e = fmaxf(v - u, 0.0f) + fmaxf(l - v, 0.0f);  // one of the two is zero
      acc[c] = __builtin_fmaf(e, e, acc[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < kGroup; ++c) out[c] = ((act >> c) & 1u) ? wave_sum(acc[c]) : 0.0f;
}

// LB_Improved's second pass (Lemire 2009) for one row, by one wave: the row
// clamped into the query's envelope [L, U] goes to hb (len floats of the
// wave's LDS), and the query is measured against that projection's
// radius-r envelope.  The squared sum is returned to every lane; adding it
// to the row's LB_Keogh gives LB_Improved, still a lower bound of DTW.
__device__ __forceinline__ float lbi_second(const float* __restrict__ q, const float* __restrict__ U,
                                            const float* __restrict__ L, const float* __restrict__ x,
                                            int len, int r, float* __restrict__ hb, int lane) {
  for (int t = lane; t < len; t += kWave) hb[t] = fminf(fmaxf(x[t], L[t]), U[t]);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  float acc = 0.0f;
  for (int t = lane; t < len; t += kWave) {
    const int a = t - r < 0 ? 0 : t - r;
    const int b = t + r > len - 1 ? len - 1 : t + r;
    // eight reads in flight per step, two independent max / min chains
    // (max and min are exact, so the grouping does not change the result)
    float hu = hb[a], hl = hu, hu2 = hu, hl2 = hu;
    int j = a + 1;
    for (; j + 8 <= b + 1; j += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = hb[j + u];
      hu = fmaxf(hu, fmaxf(fmaxf(v[0], v[1]), fmaxf(v[2], v[3])));
      hu2 = fmaxf(hu2, fmaxf(fmaxf(v[4], v[5]), fmaxf(v[6], v[7])));
      hl = fminf(hl, fminf(fminf(v[0], v[1]), fminf(v[2], v[3])));
      hl2 = fminf(hl2, fminf(fminf(v[4], v[5]), fminf(v[6], v[7])));
    }
    for (; j <= b; ++j) {
      const float v = hb[j];
      hu = fmaxf(hu, v);
      hl = fminf(hl, v);
    }
    hu = fmaxf(hu, hu2);
    hl = fminf(hl, hl2);
    const float v = q[t];
    const float e = fmaxf(v - hu, 0.0f) + fmaxf(hl - v, 0.0f);  // one of the two is zero
    acc = __builtin_fmaf(e, e, acc);
  }
  const float tot = wave_sum(acc);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();  // hb is rewritten for the next row
  return tot;
}

// Banded DTW, squared costs, FP32, one pair per thread.  Rows run over the
// candidate x (j), the band over the query (i = j - R + b, b in [0, 2R]); in
// band coordinates D(j,i) needs old D[b] (diagonal), old D[b+1] (up) and new
// D[b-1] (left), so one in-place ascending sweep per row suffices.  qpad is
// the query in LDS with R +inf pads on each side (matrix edges cost +inf).
// A path crosses every row, so a row minimum above `cutoff` ends the pair;
// the result is then minus the number of rows computed (a distance is
// never negative).
// Wide bands run as a call, where pointers arrive untyped; the body gives
// them their address spaces (the query in LDS, the row in global memory).
// With generic pointers every query read is a flat load that also counts
// as a vector-memory access, and waiting for it stalls on the row load
// too; typed, the query reads are LDS reads and the next points of the
// row load while the current ones are processed.
typedef __attribute__((address_space(3))) const float lds_float;
typedef __attribute__((address_space(1))) const float glb_float;
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) f4v glb_f4v;
__device__ __forceinline__ float4 as_float4(f4v v) { return make_float4(v.x, v.y, v.z, v.w); }

template <int R, bool MASK>
__device__ __forceinline__ void dtw_row(float (&D)[2 * R + 1], const lds_float* __restrict__ qpad,
                                        int j, float xj, int r) {
  float left = INFINITY;
#pragma unroll
  for (int b = 0; b <= 2 * R; ++b) {
    const float d = xj - qpad[j + b];
    const float up = (b < 2 * R) ? D[b + 1] : INFINITY;
    float c = __builtin_fmaf(d, d, fminf(fminf(D[b], up), left));
    if (MASK) {
      // outside the band +inf, inside c: the median of (c, pen, +inf),
      // with pen chosen by a scalar select, so no branch per cell
      const float pen = (b - R > r || R - b > r) ? INFINITY : -INFINITY;
      c = __builtin_amdgcn_fmed3f(c, pen, INFINITY);
    }
    D[b] = c;
    left = c;
  }
}

template <int R, bool MASK>
__device__ __forceinline__ float dtw_band_body(const float* __restrict__ qpad_any,
                                               const float* __restrict__ x_any, int len, int r,
                                               float cutoff) {
  const lds_float* qpad = (const lds_float*)qpad_any;
  const glb_float* x = (const glb_float*)x_any;
  if (MASK) r = __builtin_amdgcn_readfirstlane(r);  // the same for every lane
  float D[2 * R + 1];
#pragma unroll
  for (int b = 0; b <= 2 * R; ++b) D[b] = (b == R) ? 0.0f : INFINITY;
  // four rows per step share their query values (r = 25: 205 VGPRs, two
  // waves per SIMD, faster than one row per step at 142); two rows from
  // radius 32, whose four-row form would need more than 256 VGPRs; one
  // row for the widest bands
  if (R < 32 && (len & 3) == 0) {
    float4 xn = as_float4(*(const glb_f4v*)x);
#pragma unroll 1
    for (int j = 0; j < len; j += 4) {
      const float4 xa = xn;
      if (j + 4 < len) xn = as_float4(*(const glb_f4v*)(x + j + 4));
      dtw_row<R, MASK>(D, qpad, j + 0, xa.x, r);
      dtw_row<R, MASK>(D, qpad, j + 1, xa.y, r);
      dtw_row<R, MASK>(D, qpad, j + 2, xa.z, r);
      dtw_row<R, MASK>(D, qpad, j + 3, xa.w, r);
      if ((j & 7) == 4) {
        float mn = D[0];
#pragma unroll
        for (int b = 1; b <= 2 * R; ++b) mn = fminf(mn, D[b]);
        if (mn > cutoff) return -(float)(j + 4);
      }
    }
  } else if (R < 48 && (len & 1) == 0) {
    // two rows per step: the second row's query values are the first's
    // shifted by one, read once; abandonment checked after the same rows as
    // one row per step
    typedef float f2v __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(1))) f2v glb_f2v;
    f2v xn = *(const glb_f2v*)x;
#pragma unroll 1
    for (int j = 0; j < len; j += 2) {
      const f2v xa = xn;
      if (j + 2 < len) xn = *(const glb_f2v*)(x + j + 2);
      dtw_row<R, MASK>(D, qpad, j + 0, xa.x, r);
      dtw_row<R, MASK>(D, qpad, j + 1, xa.y, r);
      if ((j & 7) == 6) {
        float mn = D[0];
#pragma unroll
        for (int b = 1; b <= 2 * R; ++b) mn = fminf(mn, D[b]);
        if (mn > cutoff) return -(float)(j + 2);
      }
    }
  } else {
    // one row per step (wide bands), the next point loading while the
    // current row runs
    float xn = x[0];
#pragma unroll 1
    for (int j = 0; j < len; ++j) {
      const float xj = xn;
      if (j + 1 < len) xn = x[j + 1];
      dtw_row<R, MASK>(D, qpad, j, xj, r);
      if ((j & 7) == 7) {
        float mn = D[0];
#pragma unroll
        for (int b = 1; b <= 2 * R; ++b) mn = fminf(mn, D[b]);
        if (mn > cutoff) return -(float)(j + 1);
      }
    }
  }
  return D[R];
}

// Cells of the band |i - j| <= r inside the len x len matrix in its first
// `rows` rows: the DTW work of a pair abandoned after `rows` rows (all len
// rows when it completes).
__device__ __forceinline__ unsigned long long band_cells(int rows, int len, int r) {
  const long long R1 = rows, L = len, rr = r;
  long long a = L - rr;  // rows whose band reaches j + r <= len - 1
  a = a < 0 ? 0 : (a > R1 ? R1 : a);
  const long long upper = a * (a - 1) / 2 + a * (rr + 1) + (R1 - a) * L;
  const long long lower = R1 > rr ? (R1 - rr - 1) * (R1 - rr) / 2 : 0;
  return (unsigned long long)(upper - lower);
}

// Bands below 48 (up to 32 among the instances) are inlined: the kernel
// allocates the band with its own registers and no call saves registers.
// Wider ones stay a call, which measured faster at 51.
template <int R, bool MASK>
__device__ __attribute__((noinline)) float dtw_band_call(const float* __restrict__ qpad,
                                                        const float* __restrict__ x, int len, int r,
                                                        float cutoff) {
  return dtw_band_body<R, MASK>(qpad, x, len, r, cutoff);
}

template <int R, bool MASK>
__device__ __forceinline__ float dtw_band(const float* __restrict__ qpad, const float* __restrict__ x,
                                          int len, int r, float cutoff) {
  if constexpr (R >= 48)
    return dtw_band_call<R, MASK>(qpad, x, len, r, cutoff);
  else
    return dtw_band_body<R, MASK>(qpad, x, len, r, cutoff);
}

// Wave-cooperative DTW over anti-diagonals d = i + j; cells of one diagonal
// are independent, so lanes share them.  buf holds three diagonals (d, d-1,
// d-2) of len values each, indexed by i.  A diagonal's cells inside the
// band and the matrix lie in one index range [lo, hi]; the lanes cover it
// plus one index on each side, written +inf, so the next two diagonals
// read +inf wherever they step outside the band (older values there are
// never read).  Each cell is computed from the same three neighbours as in
// row order, so the result is bit-identical to the sequential recurrence.
// Used in FP64 for the near-tie recheck and in FP32 for radii beyond the
// register band.
template <typename T>
__device__ T dtw_wave(const float* __restrict__ q, const float* __restrict__ x, int len, int r,
                      T* __restrict__ buf, T cutoff, int lane) {
  const T inf = (T)INFINITY;
  for (int i = lane; i < 3 * len; i += kWave) buf[i] = inf;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const int last = 2 * (len - 1);
  T result = inf, prev_min = inf;
  for (int d = 0; d <= last; ++d) {
    T* cur = buf + (d % 3) * len;
    const T* p1 = buf + ((d + 2) % 3) * len;  // diagonal d-1
    const T* p2 = buf + ((d + 1) % 3) * len;  // diagonal d-2
    // band |i - j| <= r on this diagonal: ceil((d - r) / 2) <= i <= floor((d + r) / 2)
    const int lo = max(max(0, d - len + 1), (d - r + 1) >> 1);
    const int hi = min(min(len - 1, d), (d + r) >> 1);
    const int wlo = max(0, lo - 1), whi = min(len - 1, hi + 1);
    T local_min = inf;
    for (int i = wlo + lane; i <= whi; i += kWave) {
      const int j = d - i;
      T v = inf;
      if (i >= lo && i <= hi) {
        const T diff = (T)q[i] - (T)x[j];
        const T c = diff * diff;
        if (d == 0) {
          v = c;
        } else {
          T m = inf;
          if (i > 0 && j > 0 && p2[i - 1] < m) m = p2[i - 1];
          if (i > 0 && p1[i - 1] < m) m = p1[i - 1];
          if (j > 0 && p1[i] < m) m = p1[i];
          v = c + m;
        }
      }
      local_min = v < local_min ? v : local_min;
      cur[i] = v;
      if (d == last && i == len - 1) result = v;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (cutoff < inf && (d & 7) == 7) {
      // min over diagonals d and d-1: every path visits one of any two
      // consecutive anti-diagonals
      T mn = local_min < prev_min ? local_min : prev_min;
      for (int o = 32; o >= 1; o >>= 1) {
        const T u = __shfl_xor(mn, o, kWave);
        mn = u < mn ? u : mn;
      }
      if (mn > cutoff) return inf;
    }
    prev_min = local_min;
  }
  // the final cell was written by one lane; every other lane holds +inf
  for (int o = 32; o >= 1; o >>= 1) {
    const T u = __shfl_xor(result, o, kWave);
    result = u < result ? u : result;
  }
  return result;
}

// FP64 DTW of one pair by one wave when the band fits the wave
// (2r + 1 <= 64): lane k holds the cells of band offset k = i - j + r, one
// on every other anti-diagonal (d + k - r even), so a cell's neighbours
// (i-1, j-1), (i-1, j) and (i, j-1) are the lane's own previous value and
// the latest values of lanes k-1 and k+1, exchanged by lane shuffles with
// no LDS and no barrier.  The same operations as the row-order recurrence:
// bit-identical to it.
__device__ double dtw_reg64(const float* __restrict__ q, const float* __restrict__ x, int len,
                            int r, int lane) {
  const double inf = (double)INFINITY;
  double own = inf;
  const bool in_band = lane <= 2 * r;
  const int last = 2 * (len - 1);
  for (int d = 0; d <= last; ++d) {
    const double up = __shfl_up(own, 1, kWave);    // lane k-1: cell (i-1, j)
    const double dn = __shfl_down(own, 1, kWave);  // lane k+1: cell (i, j-1)
    if (in_band && !((d + lane - r) & 1)) {
      const int i = (d + lane - r) >> 1, j = d - i;
      if (i < 0 || j < 0 || i >= len || j >= len) {
        own = inf;
      } else {
        const double diff = (double)q[i] - (double)x[j];
        const double c = diff * diff;
        if (d == 0) {
          own = c;
        } else {
          double m = inf;
          if (i > 0 && j > 0 && own < m) m = own;
          if (i > 0 && lane > 0 && up < m) m = up;
          if (j > 0 && lane < kWave - 1 && dn < m) m = dn;
          own = c + m;
        }
      }
    }
  }
  return __shfl(own, r, kWave);  // the last cell (len-1, len-1) has offset r
}

// The approximate search's leaf (Algorithm 5): descend the split tree along
// the query's word (computed again from its PAA, as k_prep does); a word
// whose root key holds no series starts from the root with the smallest
// bound.  Called by every thread of a block; the leaf's position range,
// clamped to kApproxCap series and widened to at least k, is left in rng.
__device__ void approx_leaf_range(const IndexDev& ix, const QueryParams& p, const QueryState& s, int q,
                                  int64_t* rng) {
  __shared__ float bpl[257];
  __shared__ int wsym[kMaxSeg];
  __shared__ unsigned long long best_s;
  const int tid = threadIdx.x, w = p.w, cb = p.card_bits, card = 1 << cb;
  for (int j = tid; j <= card; j += blockDim.x) bpl[j] = ix.bp[j];
  if (tid == 0) best_s = ~0ull;
  __syncthreads();
  const float* pq = s.paa + (int64_t)q * 3 * kMaxSeg;  // PAA, envelope PAA upper, lower
  if (tid < w) wsym[tid] = symbol_of(pq[tid], bpl, card);
  __syncthreads();
  uint8_t word[kMaxSeg];
  uint32_t key = 0;
  for (int sg = 0; sg < w; ++sg) {
    word[sg] = (uint8_t)wsym[sg];
    key = (key << 1) | (word[sg] >> (cb - 1));
  }
  int node = ix.root_node[key];
  if (node < 0) {  // no series under that root: the root with the smallest bound
    unsigned long long best = ~0ull;
    const int nkeys = 1 << w;
    for (int kk = tid; kk < nkeys; kk += blockDim.x) {
      if (ix.root_node[kk] < 0) continue;
      float lb = 0.0f;
      for (int sg = 0; sg < w; ++sg) {
        const int b = (kk >> (w - 1 - sg)) & 1;
        const float lo = bpl[b << (cb - 1)], hi = bpl[(b + 1) << (cb - 1)];
        const float g = fmaxf(lo - pq[kMaxSeg + sg], 0.0f) + fmaxf(pq[2 * kMaxSeg + sg] - hi, 0.0f);
        lb += g * g;
      }
      const unsigned long long c = ((unsigned long long)__float_as_uint(lb) << 32) | (unsigned)kk;
      best = c < best ? c : best;
    }
    best = wave_min_u64(best);
    if ((tid & (kWave - 1)) == 0) atomicMin(&best_s, best);
    __syncthreads();
    node = ix.root_node[(int)(best_s & 0xffffffffu)];
  }
  if (tid == 0) {
    int4 t = ix.tree[node];
    for (int guard = 0; guard < 4096 && t.x >= 0; ++guard) {
      const int bit = (word[t.x & 0xff] >> (t.x >> 8)) & 1;
      int ch = bit ? t.w : t.z;
      if (ch < 0) ch = bit ? t.z : t.w;
      t = ix.tree[ch];
    }
    int64_t b = t.y, e = t.z;
    const int kk = k_of(p, s, q);
    if (e - b > kApproxCap) e = b + kApproxCap;
    if (e - b < kk) {
      e = b + kk < ix.n ? b + kk : ix.n;
      if (e - b < kk) b = e - kk > 0 ? e - kk : 0;
    }
    rng[0] = b;
    rng[1] = e;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// prep: one block per query: z-normalisation (unless raw), envelope (DTW),
// the bound slack eta, PAAs, and the reset of the query's state.

__global__ __launch_bounds__(256) void k_prep(IndexDev ix, const float* __restrict__ queries,
                                              QueryParams p, QueryState s) {
  const int q = blockIdx.x;
  const int tid = threadIdx.x;
  const int len = p.len, w = p.w, m = p.m;
  extern __shared__ float sm[];
  float* x = sm;
  float* z = x + len;
  float* U = z + len;
  float* L = U + len;
  __shared__ float paa[3][kMaxSeg];
  __shared__ float s_mu, s_sd;

  const float* src = queries + (int64_t)row_of(s, q) * len;
  for (int t = tid; t < len; t += blockDim.x) x[t] = src[t];
  __syncthreads();
  if (p.raw) {  // series are indexed as given: z = x exactly below
    if (tid == 0) {
      s_mu = 0.0f;
      s_sd = 1.0f;
    }
  } else if (tid == 0) {  // same order and rounding as the build's summary pass
    // (values read kB at a time, so one LDS wait covers kB adds)
    constexpr int kB = 64;
    float sum = 0.0f;
    int t = 0;
    for (; t + kB <= len; t += kB) {
      float v[kB];
#pragma unroll
      for (int i = 0; i < kB; ++i) v[i] = x[t + i];
#pragma unroll
      for (int i = 0; i < kB; ++i) sum = sum + v[i];
    }
    for (; t < len; ++t) sum = sum + x[t];
    const float mu = __fdiv_rn(sum, (float)len);
    float var = 0.0f;
    for (t = 0; t + kB <= len; t += kB) {
      float v[kB];
#pragma unroll
      for (int i = 0; i < kB; ++i) {
        const float d = x[t + i] - mu;
        v[i] = d * d;
      }
#pragma unroll
      for (int i = 0; i < kB; ++i) var = var + v[i];
    }
    for (; t < len; ++t) {
      const float d = x[t] - mu;
      var = var + d * d;
    }
    s_mu = mu;
    s_sd = sqrtf(__fdiv_rn(var, (float)len));
  }
  __syncthreads();
  const float mu = s_mu, sd = s_sd;
  const bool flat = !(sd > 0.0f);
  float* zq = s.zq + (int64_t)q * len;
  for (int t = tid; t < len; t += blockDim.x) {
    const float v = flat ? 0.0f : __fdiv_rn(x[t] - mu, sd);
    z[t] = v;
    zq[t] = v;
  }
  __syncthreads();
  if (p.distance == 1) {
    const int r = p.window;
    for (int t = tid; t < len; t += blockDim.x) {
      const int a = t - r < 0 ? 0 : t - r;
      const int b = t + r > len - 1 ? len - 1 : t + r;
      float u = z[a], l = z[a];
      for (int j = a; j <= b; ++j) {
        u = fmaxf(u, z[j]);
        l = fminf(l, z[j]);
      }
      U[t] = u;
      L[t] = l;
      s.upper[(int64_t)q * len + t] = u;
      s.lower[(int64_t)q * len + t] = l;
    }
    __syncthreads();
  }
  {
    // Slack of the PAA-based bounds.  A segment mean computed in FP32 is off
    // by at most 2 u sqrt(m) |v| for a row v, so a bound sqrt(m sum gap^2)
    // moves by at most 2 u sqrt(len m) (|x| + |q'|), with q' the largest of
    // the query and its envelope rows; eta_c carries an 8x margin on that.
    __shared__ float red[3][256 / kWave];
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
    for (int t = tid; t < len; t += blockDim.x) {
      a0 += z[t] * z[t];
      if (p.distance == 1) {
        a1 += U[t] * U[t];
        a2 += L[t] * L[t];
      }
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    if ((tid & (kWave - 1)) == 0) {
      red[0][tid / kWave] = a0;
      red[1][tid / kWave] = a1;
      red[2][tid / kWave] = a2;
    }
    __syncthreads();
    if (tid == 0) {
      float n2 = 0.0f;
      for (int j = 0; j < 3; ++j) {
        float t2 = 0.0f;
        for (int v = 0; v < (int)(blockDim.x / kWave); ++v) t2 += red[j][v];
        n2 = fmaxf(n2, t2);
      }
      s.eta[q] = p.eta_c * (p.xnorm + sqrtf(n2) * 1.001f);
    }
  }
  if (tid < w) {
    const float fm = (float)m;
    float a = 0.0f;
    for (int t = tid * m; t < tid * m + m; ++t) a = a + z[t];
    paa[0][tid] = __fdiv_rn(a, fm);
    if (p.distance == 1) {
      float au = 0.0f, al = 0.0f;
      for (int t = tid * m; t < tid * m + m; ++t) {
        au = au + U[t];
        al = al + L[t];
      }
      paa[1][tid] = __fdiv_rn(au, fm);
      paa[2][tid] = __fdiv_rn(al, fm);
    } else {
      paa[1][tid] = paa[0][tid];
      paa[2][tid] = paa[0][tid];
    }
    for (int j = 0; j < 3; ++j) s.paa[((int64_t)q * 3 + j) * kMaxSeg + tid] = paa[j][tid];
  }
  __syncthreads();
  if (tid == 0) {
    s.log_count[q] = 0;
    s.status[q] = 0;
  }
  if (p.leaf_in_prep) {  // batches: here once per query (stage1 has many blocks per query)
    __shared__ int64_t rng[2];
    approx_leaf_range(ix, p, s, q, rng);
    if (tid == 0) {
      s.approx_range[2 * q] = rng[0];
      s.approx_range[2 * q + 1] = rng[1];
    }
  }
  for (int j = tid; j < p.k; j += blockDim.x) s.slots[(int64_t)q * p.k + j] = kEmptyKey;
  for (int j = tid; j < kStatCount; j += blockDim.x) s.stats[(int64_t)q * kStatCount + j] = 0;
  for (int j = tid; j < kCounterInts; j += blockDim.x) s.next[(int64_t)q * kCounterInts + j] = 0;
}

// ---------------------------------------------------------------------------
// Offer of refined distances (one lane per candidate): insert into the k
// best if below the (cached) k-th best; log if within the near-tie window of
// it.  `ckey` is this lane's view of slot k-1, never below the true one.

__device__ __forceinline__ bool offer(const IndexDev& ix, const QueryParams& p, const QueryState& s,
                                      int q, float d2, int64_t pos, unsigned long long ckey,
                                      bool log_it) {
  if (!(d2 <= key_dist(ckey) * p.win)) return false;
  unsigned long long* slots = s.slots + (int64_t)q * p.k;
  const int kk = k_of(p, s, q);
  const unsigned long long key = pack_key(d2, (uint32_t)ix.perm[pos]);
  if (log_it) {
    const int i = atomicAdd(&s.log_count[q], 1);
    if (i < p.log_cap) s.log[(int64_t)q * p.log_cap + i] = pack_key(d2, (uint32_t)pos);
  }
  if (key < ckey) {
    topk_insert(slots, kk, key);
    return true;
  }
  return false;
}

// Insertion of an approximate-search distance into the k best, skipped when
// it is not below `known`, the caller's last view of slot k-1 (slots only
// decrease, so such a key could not enter); returns the new view.  Keeps
// most candidates off the slots' few addresses.
__device__ __forceinline__ unsigned long long approx_insert(unsigned long long* slots, int k,
                                                            unsigned long long key,
                                                            unsigned long long known) {
  if (key >= known) return known;
  topk_insert(slots, k, key);
  return load_key(&slots[k - 1]);
}

// ---------------------------------------------------------------------------
// stage1: blocks [0, A) refine the approximate range, blocks [A, ..) compute
// the bound of every leaf and its bucket histogram.

template <int R, bool MASK>
__global__ __launch_bounds__(256) void k_stage1(IndexDev ix, QueryParams p, QueryState s,
                                                int approx_blocks) {
  const int q = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const int len = p.len;
  extern __shared__ float sm[];
  const float* zq = s.zq + (int64_t)q * len;
  if ((int)blockIdx.x >= approx_blocks) {
    // leaf bounds (Algorithm 7's FindDist for every leaf).  Block `shard`
    // takes leaves shard, shard + kShards, ... and writes their chunks into
    // the shard's fixed item range in ascending bound-bucket order: a
    // counting sort over the logarithmic buckets, in LDS.
    const int shard = (int)blockIdx.x - approx_blocks;
    const int w = p.w, cb = p.card_bits, card = 1 << cb;
    // Per segment, a min-tree over the series table: node (b, y) = the
    // smallest entry among symbols y 2^(cb-b) .. (y+1) 2^(cb-b) - 1, which
    // is the table value of the box of the b-bit prefix y (the gap to a
    // union of adjacent boxes is attained at its first or last box).
    const int tw = 2 * card - 1;
    float* tree = sm;                                          // [16][2 card - 1]
    int* cnt = reinterpret_cast<int*>(tree + kMaxSeg * tw);    // [kLbBuckets] chunks, then cursors
    __shared__ int part[256];
    __shared__ float s_bp[257], s_pu[kMaxSeg], s_pl[kMaxSeg];
    for (int j = tid; j <= card; j += blockDim.x) s_bp[j] = ix.bp[j];
    if (tid < kMaxSeg) {
      s_pu[tid] = s.paa[((int64_t)q * 3 + 1) * kMaxSeg + tid];
      s_pl[tid] = s.paa[((int64_t)q * 3 + 2) * kMaxSeg + tid];
    }
    for (int j = tid; j < kLbBuckets; j += blockDim.x) cnt[j] = 0;
    __syncthreads();
    // the trees' bottom level is the series table, computed here from the
    // query's PAA with the same arithmetic as k_prep (no reload of it)
    const float fm = (float)p.m;
    for (int i = tid; i < kMaxSeg * card; i += blockDim.x) {
      const int sg = i >> cb, j = i & (card - 1);
      float v = 0.0f;
      if (sg < w) {
        const float g = fmaxf(s_bp[j] - s_pu[sg], 0.0f) + fmaxf(s_pl[sg] - s_bp[j + 1], 0.0f);
        v = fm * (g * g);
      }
      tree[sg * tw + card - 1 + j] = v;
    }
    __syncthreads();
    for (int b = cb - 1; b >= 0; --b) {
      for (int i = tid; i < (kMaxSeg << b); i += blockDim.x) {
        const int sg = i >> b, y = i & ((1 << b) - 1);
        const float* c = tree + sg * tw + (2 << b) - 1 + 2 * y;
        tree[sg * tw + (1 << b) - 1 + y] = fminf(c[0], c[1]);
      }
      __syncthreads();
    }
    float* lbq = s.leaf_lb + (int64_t)q * p.n_leaves;
    // with the chunk order, one shard per block; without it (the screen
    // needs the bounds only) a few blocks per query take every shard
    const int nlb = (int)gridDim.x - approx_blocks;
    int j0 = 0, nl = 0;
    // bound of a leaf: sixteen min-tree lookups, summed pairwise
    auto leaf_bound = [&](const uint4& sy, const uint4& bi) {
      float t[kMaxSeg];  // segments past w read level 0 of an all-zero row
#pragma unroll
      for (int sg = 0; sg < kMaxSeg; ++sg)
        t[sg] = tree[sg * tw + (1 << byte_of(bi, sg)) - 1 + (int)byte_of(sy, sg)];
#pragma unroll
      for (int h = kMaxSeg / 2; h >= 1; h >>= 1)
#pragma unroll
        for (int sg = 0; sg < h; ++sg) t[sg] = t[sg] + t[sg + h];
      return t[0];
    };
    constexpr int kLB = 4;  // leaves per thread whose loads are in flight together
    const int bs = (int)blockDim.x;
    for (int sh = shard; sh < kShards; sh += nlb) {
      j0 = ix.leaf_sh_off[sh];
      nl = ix.leaf_sh_off[sh + 1] - j0;
      for (int jb = tid; jb < nl; jb += kLB * bs) {
        uint4 sy[kLB], bi[kLB];
        int2 rg[kLB];
#pragma unroll
        for (int u = 0; u < kLB; ++u)
          if (jb + u * bs < nl) {
            sy[u] = ix.sh_sym[j0 + jb + u * bs];
            bi[u] = ix.sh_bits[j0 + jb + u * bs];
            rg[u] = ix.sh_rng[j0 + jb + u * bs];
          }
#pragma unroll
        for (int u = 0; u < kLB; ++u)
          if (jb + u * bs < nl) {
            const float lb = leaf_bound(sy[u], bi[u]);
            lbq[sh + (jb + u * bs) * kShards] = lb;
            if (p.order_leaves)
              atomicAdd(&cnt[lb_bucket(lb * p.lb_scale)], (rg[u].y - rg[u].x + kChunkSeries - 1) / kChunkSeries);
          }
      }
    }
    __syncthreads();
    if (!p.order_leaves) return;  // the screen reads the bounds only
    // exclusive scan of the bucket counts (8 per thread)
    constexpr int per = kLbBuckets / 256;
    int loc[per], sum = 0;
#pragma unroll
    for (int j = 0; j < per; ++j) {
      loc[j] = cnt[tid * per + j];
      sum += loc[j];
    }
    part[tid] = sum;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      const int v = tid >= o ? part[tid - o] : 0;
      __syncthreads();
      part[tid] += v;
      __syncthreads();
    }
    int run = ix.shard_off[shard] + part[tid] - sum;
#pragma unroll
    for (int j = 0; j < per; ++j) {
      cnt[tid * per + j] = run;
      run += loc[j];
    }
    __syncthreads();
    unsigned long long* items = s.items + (int64_t)q * p.item_cap;
    int2* ranges = s.ranges + (int64_t)q * p.item_cap;
    for (int jb = tid; jb < nl; jb += kLB * bs) {
      uint4 sy[kLB], bi[kLB];
      int2 rg[kLB];
#pragma unroll
      for (int u = 0; u < kLB; ++u)
        if (jb + u * bs < nl) {
          sy[u] = ix.sh_sym[j0 + jb + u * bs];
          bi[u] = ix.sh_bits[j0 + jb + u * bs];
          rg[u] = ix.sh_rng[j0 + jb + u * bs];
        }
#pragma unroll
      for (int u = 0; u < kLB; ++u) {
        if (jb + u * bs >= nl) continue;
        const float lb = leaf_bound(sy[u], bi[u]);  // the same value as in the count pass
        const int nc = (rg[u].y - rg[u].x + kChunkSeries - 1) / kChunkSeries;
        const int at = atomicAdd(&cnt[lb_bucket(lb * p.lb_scale)], nc);
        const unsigned long long it = ((unsigned long long)__float_as_uint(lb) << 32) |
                                      (unsigned)(shard + (jb + u * bs) * kShards);
        for (int c = 0; c < nc; ++c) {
          const int cb0 = rg[u].x + c * kChunkSeries;
          items[at + c] = it;
          ranges[at + c] = make_int2(cb0, cb0 + kChunkSeries < rg[u].y ? cb0 + kChunkSeries : rg[u].y);
        }
      }
    }
    return;
  }
  // approximate search (Algorithm 5, approxSearch): real distances of the
  // series of the query's leaf.  For a few queries the leaf is found here,
  // off the bound blocks' path (block 0 records its range for the later
  // phases); for batches k_prep found it once per query.
  __shared__ int64_t s_rng[2];
  if (p.leaf_in_prep) {
    if (tid == 0) {
      s_rng[0] = s.approx_range[2 * q];
      s_rng[1] = s.approx_range[2 * q + 1];
    }
    __syncthreads();
  } else {
    approx_leaf_range(ix, p, s, q, s_rng);
    if (blockIdx.x == 0 && tid == 0) {
      s.approx_range[2 * q] = s_rng[0];
      s.approx_range[2 * q + 1] = s_rng[1];
    }
  }
  const int64_t P0 = s_rng[0], P1 = s_rng[1];
  const int cnt = (int)(P1 - P0);
  float* approx_d2 = s.approx_d2 + (int64_t)q * kApproxCap;
  unsigned long long* slots = s.slots + (int64_t)q * p.k;
  const int kk = k_of(p, s, q);
  if constexpr (R == -1) {  // ED: one wave per series
    float* zl = sm;
    for (int t = tid; t < len; t += blockDim.x) zl[t] = zq[t];
    __syncthreads();
    // eight consecutive rows per wave at a time, their loads in flight
    // together
    const int gw = blockIdx.x * (blockDim.x / kWave) + wv;
    const int nw = approx_blocks * (blockDim.x / kWave);
    unsigned long long known = kEmptyKey;  // this wave's view of slot k-1 (never below it)
    for (int j0 = gw * kGroup; j0 < cnt; j0 += nw * kGroup) {
      int gr[kGroup];
      unsigned act = 0;
#pragma unroll
      for (int c = 0; c < kGroup; ++c) {
        const bool in = j0 + c < cnt;
        const int64_t pos = P0 + (in ? j0 + c : j0);
        gr[c] = ix.zrow ? ix.zrow[pos] : (int)pos;
        act |= in ? (1u << c) : 0u;
      }
      float dv[kGroup];
      ed_rows<kGroup>(zl, ix.Z, len, gr, act, lane, dv);
      if (lane == 0) {
#pragma unroll
        for (int c = 0; c < kGroup; ++c)
          if ((act >> c) & 1u) {
            approx_d2[j0 + c] = dv[c];
            known = approx_insert(slots, kk, pack_key(dv[c], (uint32_t)ix.perm[P0 + j0 + c]), known);
          }
      }
    }
  } else if constexpr (R == -2) {  // DTW, wide band: one wave per series
    float* ql = sm;
    float* xl = ql + len;          // [4][len]
    float* buf = xl + 4 * len;     // [4][3 len]
    for (int t = tid; t < len; t += blockDim.x) ql[t] = zq[t];
    __syncthreads();
    const int gw = blockIdx.x * 4 + wv, nw = approx_blocks * 4;
    unsigned long long known = kEmptyKey;
    for (int j = gw; j < cnt; j += nw) {
      const int64_t pos = P0 + j;
      const float* xr = zrow_ptr(ix, pos);
      for (int t = lane; t < len; t += kWave) xl[wv * len + t] = xr[t];
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const float d2 = dtw_wave<float>(ql, xl + wv * len, len, p.window, buf + wv * 3 * len,
                                       (float)INFINITY, lane);
      if (lane == 0) {
        approx_d2[j] = d2;
        known = approx_insert(slots, kk, pack_key(d2, (uint32_t)ix.perm[pos]), known);
      }
    }
  } else {  // DTW, register band: one thread per series
    float* qpad = sm;
    for (int t = tid; t < len + 2 * R; t += blockDim.x)
      qpad[t] = (t >= R && t < R + len) ? zq[t - R] : INFINITY;
    __syncthreads();
    unsigned long long known = kEmptyKey;
    for (int j = blockIdx.x * blockDim.x + tid; j < cnt; j += approx_blocks * blockDim.x) {
      const int64_t pos = P0 + j;
      const float d2 = dtw_band<R, MASK>(qpad, zrow_ptr(ix, pos), len, p.window, INFINITY);
      approx_d2[j] = d2;
      known = approx_insert(slots, kk, pack_key(d2, (uint32_t)ix.perm[pos]), known);
    }
  }
}

// Leaf bounds of a batch when only the bounds are needed (the screen's leaf
// lists): block (x, y) takes 256 leaves and kBoundQueries queries, so each
// leaf's box ends are looked up once and serve every query of the tile.
// The box of a b-bit prefix y of segment s is the union of the symbols
// y 2^(cb-b) .. (y+1) 2^(cb-b) - 1, so its ends are bp[y << (cb-b)] and
// bp[(y+1) << (cb-b)], and its gap equals the smallest gap of its symbols'
// boxes (the one at its first or last symbol, or zero), which is the value
// the bound blocks' min-tree holds: the same arithmetic gives the same bits.
constexpr int kBoundQueries = 32;

__global__ __launch_bounds__(256) void k_leaf_bounds(IndexDev ix, QueryParams p, QueryState s) {
  __shared__ float s_bp[257];
  __shared__ float s_pu[kBoundQueries][kMaxSeg], s_pl[kBoundQueries][kMaxSeg];
  const int tid = threadIdx.x, cb = p.card_bits, card = 1 << cb, w = p.w;
  const int q0 = blockIdx.y * kBoundQueries;
  const int nqt = min(kBoundQueries, p.nq - q0);
  for (int j = tid; j <= card; j += blockDim.x) s_bp[j] = ix.bp[j];
  for (int i = tid; i < nqt * kMaxSeg; i += blockDim.x) {
    const int qi = i / kMaxSeg, sg = i % kMaxSeg;
    s_pu[qi][sg] = s.paa[((int64_t)(q0 + qi) * 3 + 1) * kMaxSeg + sg];
    s_pl[qi][sg] = s.paa[((int64_t)(q0 + qi) * 3 + 2) * kMaxSeg + sg];
  }
  __syncthreads();
  const int l = blockIdx.x * blockDim.x + tid;
  if (l >= p.n_leaves) return;
  const uint4 sy = ix.leaf_sym[l], bi = ix.leaf_bits[l];
  float lo[kMaxSeg], hi[kMaxSeg];
#pragma unroll
  for (int sg = 0; sg < kMaxSeg; ++sg) {
    const int b = (int)byte_of(bi, sg), y = (int)byte_of(sy, sg);
    lo[sg] = s_bp[y << (cb - b)];
    hi[sg] = s_bp[(y + 1) << (cb - b)];
  }
  const float fm = (float)p.m;
  float* out = s.leaf_lb + (int64_t)q0 * p.n_leaves + l;
  for (int qi = 0; qi < nqt; ++qi) {
    float t[kMaxSeg];
#pragma unroll
    for (int sg = 0; sg < kMaxSeg; ++sg) {
      const float g = fmaxf(lo[sg] - s_pu[qi][sg], 0.0f) + fmaxf(s_pl[qi][sg] - hi[sg], 0.0f);
      t[sg] = sg < w ? fm * (g * g) : 0.0f;
    }
#pragma unroll
    for (int h = kMaxSeg / 2; h >= 1; h >>= 1)
#pragma unroll
      for (int sg = 0; sg < h; ++sg) t[sg] = t[sg] + t[sg + h];
    out[(int64_t)qi * p.n_leaves] = t[0];
  }
}

// Near-tie log entries of the approximate search: its distances within the
// window of the first k-th best (the k-th best only decreases afterwards,
// so this covers the window of the final one).
__device__ __forceinline__ void log_approx(const QueryParams& p, const QueryState& s, int q,
                                           int tid, int nthreads) {
  const unsigned long long* slots = s.slots + (int64_t)q * p.k;
  const float win = kth_dist(slots, k_of(p, s, q)) * p.win;
  const int64_t P0 = s.approx_range[2 * q], P1 = s.approx_range[2 * q + 1];
  const float* ad = s.approx_d2 + (int64_t)q * kApproxCap;
  for (int j = tid; j < (int)(P1 - P0); j += nthreads) {
    const float d2 = ad[j];
    if (d2 <= win) {
      const int i = atomicAdd(&s.log_count[q], 1);
      if (i < p.log_cap) s.log[(int64_t)q * p.log_cap + i] = pack_key(d2, (uint32_t)(P0 + j));
    }
  }
}

// ---------------------------------------------------------------------------
// process (DTW): persistent blocks over the ordered leaf chunks.
// R >= 0: a register band of radius R; R = -2: wave anti-diagonals (radius
// beyond the register band).
//
// A block takes kDtwWaves consecutive chunks of one shard with one atomic
// (one chunk per wave).  Each wave computes the series bounds of its chunk
// and appends the survivors to the block's list in LDS; then all waves take
// LB_Keogh of the list together, eight rows per wave at a time, and its
// survivors wait in a block list until there is one pair per thread.

constexpr int kUnroll = kChunkSeries / kWave;  // words per lane per chunk

// ED process kernel shape: waves per block, and each wave's survivor list
// (refined once it holds kEdDefer entries, so a whole chunk always fits)
constexpr int kEdWaves = 16;
constexpr int kEdThreads = kEdWaves * kWave;
static_assert(kShards % kEdWaves == 0, "a shard's waves come from whole blocks");
constexpr int kEdRows = 8;               // rows refined together (their loads in flight at once)
constexpr int kEdLoad = 8;  // words per lane loaded together in the bound pass
constexpr unsigned kEdTick = 16;  // wave-steps of a block per read of the global k-th best
constexpr int kEdDefer = 2 * kEdRows;
constexpr int kEdList = kChunkSeries + kEdDefer;

template <int R>
struct ProcShape {
  static constexpr int waves = 4;  // one chunk per wave
  static constexpr int threads = waves * kWave;
  static constexpr int surv_cap = waves * kChunkSeries;
  static constexpr int pend_cap = (R >= 0) ? surv_cap + threads : 0;
};

template <int R, bool MASK, bool LBI>
__device__ __forceinline__ void process_body(const IndexDev& ix, const QueryParams& p,
                                             const QueryState& s) {
  using Sh = ProcShape<R>;
  constexpr int kW = Sh::waves;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const int len = p.len, card = 1 << p.card_bits;
  extern __shared__ float sm[];
  float* table = sm;                          // [16][card]
  float* ql = table + kMaxSeg * card;         // query (ED, wave DTW) / padded query (band DTW)
  const int qlen = (R >= 0) ? len + 2 * R : len;
  float* U = ql + qlen;                       // envelope (DTW)
  float* Lw = U + len;
  int* surv = reinterpret_cast<int*>(Lw + len);                 // survivors of a grab
  float* survlb = reinterpret_cast<float*>(surv + Sh::surv_cap);  // their bounds
  int* pend = reinterpret_cast<int*>(survlb + Sh::surv_cap);    // DTW pairs waiting
  float* wx = reinterpret_cast<float*>(pend + Sh::pend_cap);     // wave DTW rows / LB_Improved [kW][len]
  float* wbuf = wx + (R == -2 ? kW * len : 0);                   // wave DTW [kW][3 len]
  __shared__ int s_batch, s_shard, s_stop, s_nsurv, s_npend, s_skip;
  __shared__ unsigned long long s_ckey;
  __shared__ int s_shard_done;

  // A block starts on query blockIdx.x % nq and, once every shard of that
  // query is finished, moves on to the next query, so the blocks of queries
  // that end early help the ones still running.
  for (int visit = 0; visit < p.nq; ++visit) {
  const int q = (int)((blockIdx.x + (unsigned)visit) % (unsigned)p.nq);
  const int k = k_of(p, s, q);
  // the near-tie log entries of the approximate search, once per query,
  // by block q mod gridDim.x (block q, on its first visit, when the grid
  // has a block per query); it runs even if the query is already done
  if (q % (int)gridDim.x == (int)blockIdx.x) log_approx(p, s, q, tid, blockDim.x);
  {
    int* cq = s.next + (int64_t)q * kCounterInts;
    if (tid == 0)
      s_skip = load_relaxed(reinterpret_cast<unsigned long long*>(cq + kShards * kCounterStride)) == ~0ull;
    __syncthreads();
    const bool skip = s_skip;
    __syncthreads();
    if (skip) continue;
  }

  {
    // the series table from the query's PAA (the same arithmetic as k_prep)
    const float* pu = s.paa + ((int64_t)q * 3 + 1) * kMaxSeg;
    const float* pl = s.paa + ((int64_t)q * 3 + 2) * kMaxSeg;
    const int cb = p.card_bits;
    const float fm = (float)p.m;
    for (int i = tid; i < kMaxSeg * card; i += blockDim.x) {
      const int sg = i >> cb, j = i & (card - 1);
      float v = 0.0f;
      if (sg < p.w) {
        const float g = fmaxf(ix.bp[j] - pu[sg], 0.0f) + fmaxf(pl[sg] - ix.bp[j + 1], 0.0f);
        v = fm * (g * g);
      }
      table[i] = v;
    }
  }
  const float* zq = s.zq + (int64_t)q * len;
  if (R >= 0) {
    for (int t = tid; t < qlen; t += blockDim.x) ql[t] = (t >= R && t < R + len) ? zq[t - R] : INFINITY;
  } else {
    for (int t = tid; t < len; t += blockDim.x) ql[t] = zq[t];
  }
  {
    for (int t = tid; t < len; t += blockDim.x) {
      U[t] = s.upper[(int64_t)q * len + t];
      Lw[t] = s.lower[(int64_t)q * len + t];
    }
  }
  unsigned long long* slots = s.slots + (int64_t)q * p.k;
  if (tid == 0) {
    s_ckey = load_key(&slots[k - 1]);
    s_nsurv = 0;
    s_npend = 0;
    s_shard = (int)((blockIdx.x / (unsigned)p.nq) % kShards);
  }
  __syncthreads();

  const int64_t P0 = s.approx_range[2 * q], P1 = s.approx_range[2 * q + 1];
  const float eta = s.eta[q];
  const unsigned long long* items = s.items + (int64_t)q * p.item_cap;
  const int2* ranges = s.ranges + (int64_t)q * p.item_cap;

  int* counters = s.next + (int64_t)q * kCounterInts;
  unsigned long long* finished =
      reinterpret_cast<unsigned long long*>(counters + kShards * kCounterStride);
  unsigned long long c_lb = 0, c_lbk = 0, c_lbi = 0, c_ref = 0, c_leaf = 0, c_bsf = 0, c_cells = 0;

  // DTW pairs in the pending list, one per thread, first `cnt` entries
  auto run_pairs = [&](int cnt, unsigned long long ck) {
    if constexpr (R >= 0) {
      const float cut = key_dist(ck) * p.win * p.win;
      bool ch = false;
      unsigned long long mine = ck;
      if (tid < cnt) {
        const int pp = pend[tid];
        const float e = dtw_band<(R >= 0 ? R : 0), MASK>(ql, zrow_ptr(ix, pp), len, p.window, cut);
        ++c_ref;
        c_cells += band_cells(e >= 0.0f ? len : (int)-e, len, p.window);
        if (e >= 0.0f) ch = offer(ix, p, s, q, e, pp, ck, true);
        c_bsf += ch ? 1 : 0;
      }
      if (__ballot(ch) && lane == 0) {
        mine = load_key(&slots[k - 1]);
        atomicMin(&s_ckey, mine);
      }
    }
  };

  // refine survivors [0, ns), eight rows per wave; bounds re-checked
  // against the latest k-th best this wave knows
  auto refine = [&](int ns, unsigned long long& ckey) {
    for (int g = wv * kGroup; g < ns; g += kW * kGroup) {
      const float tcur = lb_threshold(key_dist(ckey), eta, p);
      int gp[kGroup];
      unsigned act = 0;
#pragma unroll
      for (int c = 0; c < kGroup; ++c) {
        const bool in = g + c < ns;
        gp[c] = in ? surv[g + c] : 0;
        act |= (in && survlb[g + c] <= tcur) ? (1u << c) : 0u;
      }
      if (!act) continue;
      float dv[kGroup];
      int gr[kGroup];  // rows of Z (the positions themselves unless Z is in id order)
#pragma unroll
      for (int c = 0; c < kGroup; ++c) gr[c] = ix.zrow ? ix.zrow[gp[c]] : gp[c];
      {
        // LB_Keogh on the raw values (Algorithm 10, second test)
        lbk_group(U, Lw, ix.Z, len, gr, act, lane, dv);
        c_lbk += (lane == 0) ? __popc(act) : 0;
        const float tk = key_dist(ckey) * p.win * p.win;
        unsigned pass = 0;
#pragma unroll
        for (int c = 0; c < kGroup; ++c)
          pass |= (((act >> c) & 1u) && dv[c] <= tk) ? (1u << c) : 0u;
        if (LBI && pass) {
          // LB_Improved (the tighter bound Section 3.4 names) on the
          // LB_Keogh survivors, same test against the k-th best.  The
          // group's LB_Keogh values wait in the survivors' LDS slots, so
          // no per-row registers stay live across the pass.
          if (lane == 0) {
#pragma unroll
            for (int c = 0; c < kGroup; ++c)
              if ((pass >> c) & 1u) survlb[g + c] = dv[c];
          }
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
          const float* qv = ql + (R >= 0 ? R : 0);
#pragma unroll 1
          for (int c = 0; c < kGroup; ++c) {
            if (!((pass >> c) & 1u)) continue;
            const int pos = surv[g + c];
            const float* x = zrow_ptr(ix, pos);
            const float e2 = lbi_second(qv, U, Lw, x, len, p.window, wx + wv * len, lane);
            c_lbi += (lane == 0) ? 1 : 0;
            if (!(survlb[g + c] + e2 <= tk)) pass &= ~(1u << c);
          }
        }
        if constexpr (R >= 0) {
          if (pass) {
            int at = 0;
            if (lane == 0) at = atomicAdd(&s_npend, __popc(pass));
            at = __shfl(at, 0, kWave);
#pragma unroll
            for (int c = 0; c < kGroup; ++c)
              if ((pass >> c) & 1u) {
                if (lane == 0) pend[at] = surv[g + c];
                ++at;
              }
          }
        } else {
#pragma unroll 1
          for (int c = 0; c < kGroup; ++c) {
            if (!((pass >> c) & 1u)) continue;
            const int pos = surv[g + c];
            const float* x = zrow_ptr(ix, pos);
            for (int t = lane; t < len; t += kWave) wx[wv * len + t] = x[t];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const float cut = key_dist(ckey) * p.win * p.win;
            const float e = dtw_wave<float>(ql, wx + wv * len, len, p.window, wbuf + wv * 3 * len,
                                            cut, lane);
            bool ch = false;
            if (lane == 0) {
              ++c_ref;
              ch = e < INFINITY && offer(ix, p, s, q, e, pos, ckey, true);
              c_bsf += ch ? 1 : 0;
            }
            if (__ballot(ch)) ckey = umin64(ckey, load_key(&slots[k - 1]));
          }
        }
      }
    }
  };

  // Thread 0 keeps one grab in flight: right after a grab is published to
  // the block it already asks for the next batch of the same shard and for
  // the current k-th best, so both round trips overlap the chunk work.  The
  // finished-shard mask is consulted only when the shard has to change.
  int next_batch = 0;
  bool have_next = false;
  unsigned long long next_key = ~0ull;
  for (;;) {
    if (tid == 0) {
      s_stop = 0;
      s_shard_done = 0;
      if (!have_next) {
        const unsigned long long fin = load_relaxed(finished);
        if (fin == ~0ull) {
          s_stop = 1;
        } else {
          int shard = s_shard;
          if ((fin >> shard) & 1ull) {  // next unfinished shard after this one
            const unsigned long long rot = ~((fin >> shard) | (fin << ((kShards - shard) & 63)));
            shard = (shard + __ffsll((long long)rot) - 1) & (kShards - 1);
          }
          s_shard = shard;
          next_batch = atomicAdd(&counters[shard * kCounterStride], 1);
          next_key = load_key(&slots[k - 1]);
        }
      }
      s_batch = next_batch;
      s_ckey = umin64(s_ckey, next_key);
      have_next = false;
    }
    __syncthreads();
    if (s_stop) break;
    const int shard = s_shard;
    if (tid == 0) {  // prefetch the next grab of this shard
      next_batch = atomicAdd(&counters[shard * kCounterStride], 1);
      next_key = load_key(&slots[k - 1]);
      have_next = true;
    }
    unsigned long long ckey = s_ckey;
    const float tadj = lb_threshold(key_dist(ckey), eta, p);
    // one chunk per wave, consecutive in the shard's bound order
    const int i = ix.shard_off[shard] + s_batch * kW + wv;
    bool take = false;
    int2 rg = make_int2(0, 0);
    if (i < ix.shard_off[shard + 1]) {
      const unsigned long long item = items[i];
      rg = ranges[i];
      const float lb = key_dist(item);
      take = lb <= tadj;
      if (!take && bucket_floor(lb_bucket(lb * p.lb_scale)) > tadj * p.lb_scale && lane == 0) {  // all later chunks above too
        atomicOr(finished, 1ull << shard);
        s_shard_done = 1;
      }
    } else if (lane == 0) {
      atomicOr(finished, 1ull << shard);
      s_shard_done = 1;
    }
    if (take) {
      c_leaf += (lane == 0) ? 1 : 0;
      // series bounds (Algorithm 9 / Algorithm 10, first test)
      uint4 wd[kUnroll];
      bool ok[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int pos = rg.x + lane + u * kWave;
        ok[u] = pos < rg.y && !(pos >= P0 && pos < P1);
        // defined words on skipped lanes keep them from staying live
        // across the refinement (occupancy)
        wd[u] = make_uint4(0u, 0u, 0u, 0u);
        if (ok[u]) wd[u] = ix.words[pos];
      }
      float lbv[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        lbv[u] = 0.0f;
        if (ok[u]) {
          // all sixteen lookups are independent; summed pairwise
          float t[kMaxSeg];
#pragma unroll
          for (int sg = 0; sg < kMaxSeg; ++sg) t[sg] = table[sg * card + (int)byte_of(wd[u], sg)];
#pragma unroll
          for (int h = kMaxSeg / 2; h >= 1; h >>= 1)
#pragma unroll
            for (int sg = 0; sg < h; ++sg) t[sg] = t[sg] + t[sg + h];
          ++c_lb;
          lbv[u] = t[0];
          ok[u] = lbv[u] <= tadj;
        }
      }
      int nmine = 0;
      unsigned long long msk[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        msk[u] = __ballot(ok[u]);
        nmine += __popcll(msk[u]);
      }
      if (nmine) {
        int base = 0;
        if (lane == 0) base = atomicAdd(&s_nsurv, nmine);
        base = __shfl(base, 0, kWave);
        const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          if (ok[u]) {
            const int at = base + __popcll(msk[u] & below);
            surv[at] = rg.x + lane + u * kWave;
            survlb[at] = lbv[u];
          }
          base += __popcll(msk[u]);
        }
      }
    }
    __syncthreads();
    const int ns = s_nsurv;
    refine(ns, ckey);
    if (lane == 0) atomicMin(&s_ckey, ckey);
    __syncthreads();
    if constexpr (R >= 0) {
      // full rounds of one DTW pair per thread; the rest waits for more
      int np = s_npend;
      while (np >= Sh::threads) {
        run_pairs(Sh::threads, s_ckey);
        __syncthreads();
        const int rem = np - Sh::threads;  // move the rest to the front, block-uniform steps
        for (int b0 = 0; b0 < rem; b0 += Sh::threads) {
          const int t = b0 + tid;
          const int v = t < rem ? pend[Sh::threads + t] : 0;
          __syncthreads();
          if (t < rem) pend[t] = v;
          __syncthreads();
        }
        np = rem;
      }
      if (tid == 0) s_npend = np;
    }
    if (tid == 0) {
      s_nsurv = 0;
      if (s_shard_done) have_next = false;  // the prefetched batch lies past the shard's end
    }
    __syncthreads();
  }
  if constexpr (R >= 0) {  // the block's last DTW pairs
    const int np = s_npend;
    if (np > 0) run_pairs(np, s_ckey);
  }
  // statistics
  for (int o = 32; o >= 1; o >>= 1) {
    c_lb += __shfl_xor(c_lb, o, kWave);
    c_lbk += __shfl_xor(c_lbk, o, kWave);
    c_lbi += __shfl_xor(c_lbi, o, kWave);
    c_ref += __shfl_xor(c_ref, o, kWave);
    c_leaf += __shfl_xor(c_leaf, o, kWave);
    c_bsf += __shfl_xor(c_bsf, o, kWave);
    c_cells += __shfl_xor(c_cells, o, kWave);
  }
  if (p.count_work) {
    __shared__ unsigned long long s_part[7];
    const int which[7] = {kStatLeavesKept, kStatSeriesLb, kStatLbKeogh, kStatLbImproved, kStatRefined,
                          kStatBsf, kStatCells};
    const unsigned long long val[7] = {c_leaf, c_lb, c_lbk, c_lbi, c_ref, c_bsf, c_cells};
    add_block_counts<7>(s.stats + (int64_t)q * kStatCount, which, val, s_part);
  }
  __syncthreads();  // LDS is reloaded for the next query
  }
}

// LBI: LB_Improved after LB_Keogh.  Its own instances (masked bands and
// the wave kernel only), so the default kernels keep their registers.
template <int R, bool MASK, bool LBI = false>
__global__ __launch_bounds__(ProcShape<R>::threads) void k_process(IndexDev ix, QueryParams p,
                                                                   QueryState s) {
  process_body<R, MASK, LBI>(ix, p, s);
}

// ---------------------------------------------------------------------------
// ED process kernel.  Every wave runs on its own, with no block barrier
// between chunks: while some waves wait on memory, others compute bounds,
// so the loads of many chunks are in flight on every CU at once.  The
// chunks of a shard are dealt to waves statically: of the grid's G waves,
// G / kShards take each shard, and wave j of a shard takes its chunks
// j, j + G / kShards, ... in the shard's ascending bound order, so the
// waves sweep every shard's order together and later chunks meet a
// tighter k-th best.  A wave stops at its first chunk whose bucket starts
// above the k-th best (all its later chunks are above too).  Per chunk it
// computes the series bounds from the table in LDS, appends the survivors
// to its own list in LDS and refines them eight rows at a time once the
// list holds two groups.  Every block visits every query of the launch
// (starting with query blockIdx.x mod nq), building the query's table once
// per visit.

// CB: the symbols' bits when known at compile time (8, the paper's
// cardinality: the table's segment offsets become immediates), else 0.
template <int CB>
__global__ __launch_bounds__(kEdThreads) void k_process_ed(IndexDev ix, QueryParams p,
                                                         QueryState s) {
  constexpr int kW = kEdWaves;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const int len = p.len, card = CB ? (1 << CB) : (1 << p.card_bits);
  extern __shared__ float sm[];
  // the block's copy of the k-th best: waves read it here, and only one
  // wave-step in kEdTick reads the global slot (every wave of the grid
  // reading that one address would queue at the memory channel holding it)
  __shared__ unsigned long long s_ckey;
  __shared__ unsigned s_tick;
  // work sharing of the refinement: wave w's published list holds s_n[w]
  // entries, handed out from s_h[w] on; s_busy[w] counts other waves
  // copying from it, s_done the waves whose own chunks are all done
  __shared__ int s_n[kW], s_h[kW], s_busy[kW], s_done;
  // the [16][card] table: in static LDS when the cardinality is known at
  // compile time (its place, and so every lookup's offset, is then a
  // constant), else at the head of the dynamic LDS
  __shared__ float s_table[CB ? kMaxSeg << CB : 1];
  float* table = CB ? s_table : sm;
  float* ql = sm + kMaxSeg * card;                             // query row [len]
  int* const lpos_all = reinterpret_cast<int*>(ql + len);       // survivors [kW][kEdList]
  float* const llb_all = reinterpret_cast<float*>(lpos_all + kW * kEdList);  // their bounds
  int* lpos = lpos_all + wv * kEdList;                         // this wave's list
  float* llb = llb_all + wv * kEdList;
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  // The block's kW streams of chunks: stream x is shard
  // (blockIdx.x mod kBpS) kW + x from its chunk `place` on, every stride-th
  // chunk, where stride is the number of blocks that share a shard.  The
  // places of a block's streams lie stride / kW apart, so the front of
  // the shards (the chunks of lowest bound, which hold most survivors)
  // falls on different blocks.  The block's waves take the streams' chunks
  // through counters in LDS, so the block's chunks are shared out evenly.
  constexpr int kBpS = kShards / kW;  // blocks whose streams cover every shard once
  constexpr unsigned kAllStreams = (1u << kW) - 1;
  const int stride = (int)gridDim.x / kBpS;
  __shared__ int s_first[kW], s_end[kW], s_idx[kW];
  __shared__ unsigned s_sdone;
  if (tid < kW) {
    const int shx = ((int)blockIdx.x % kBpS) * kW + tid;
    const int plx = ((int)blockIdx.x / kBpS + tid * (stride / kW > 0 ? stride / kW : 1)) % stride;
    s_first[tid] = ix.shard_off[shx] + plx;
    s_end[tid] = ix.shard_off[shx + 1];
  }

  for (int visit = 0; visit < p.nq; ++visit) {
    const int q = (int)((blockIdx.x + (unsigned)visit) % (unsigned)p.nq);
    const int k = k_of(p, s, q);
    // the near-tie log entries of the approximate search, once per query,
    // by block q mod gridDim.x: with fewer blocks than queries, block b
    // logs every query q = b (mod gridDim.x) when it reaches it (a later
    // k-th best gives a narrower window that still holds the final one's)
    if (q % (int)gridDim.x == (int)blockIdx.x) log_approx(p, s, q, tid, blockDim.x);
    {
      // the series table from the query's PAA (the same arithmetic as k_prep)
      const float* pu = s.paa + ((int64_t)q * 3 + 1) * kMaxSeg;
      const float* pl = s.paa + ((int64_t)q * 3 + 2) * kMaxSeg;
      const int cb = p.card_bits;
      const float fm = (float)p.m;
      for (int i = tid; i < kMaxSeg * card; i += blockDim.x) {
        const int sg = i >> cb, j = i & (card - 1);
        float v = 0.0f;
        if (sg < p.w) {
          const float g = fmaxf(ix.bp[j] - pu[sg], 0.0f) + fmaxf(pl[sg] - ix.bp[j + 1], 0.0f);
          v = fm * (g * g);
        }
        table[i] = v;
      }
      const float* zq = s.zq + (int64_t)q * len;
      for (int t = tid; t < len; t += blockDim.x) ql[t] = zq[t];
      if (tid == 0) {
        s_ckey = load_key(&s.slots[(int64_t)q * p.k + k - 1]);
        s_tick = 0;
        s_done = 0;
      }
      if (tid < kW) {
        s_n[tid] = 0;
        s_h[tid] = 0;
        s_busy[tid] = 0;
        s_idx[tid] = 0;
      }
      if (tid == 0) s_sdone = 0;
    }
    __syncthreads();
    unsigned long long* slots = s.slots + (int64_t)q * p.k;
    const int P0 = (int)s.approx_range[2 * q], P1 = (int)s.approx_range[2 * q + 1];
    const float eta = s.eta[q];
    const unsigned long long* items = s.items + (int64_t)q * p.item_cap;
    const int2* ranges = s.ranges + (int64_t)q * p.item_cap;
    unsigned long long c_lb = 0, c_ref = 0, c_leaf = 0, c_bsf = 0;
    unsigned long long ckey = s_ckey;
    int nl = 0;  // survivors in this wave's list (wave-uniform)

    // refinement of up to kEdRows entries taken from a list, each bound
    // re-checked against the latest k-th best the wave knows
    auto refine_rows = [&](const int (&gp)[kEdRows], const float (&gl)[kEdRows], int cnt) {
      const float tcur = lb_threshold(key_dist(ckey), eta, p);
      unsigned act = 0;
#pragma unroll
      for (int c = 0; c < kEdRows; ++c) act |= (c < cnt && gl[c] <= tcur) ? (1u << c) : 0u;
      if (!act) return;
      int gr[kEdRows];
#pragma unroll
      for (int c = 0; c < kEdRows; ++c) gr[c] = ix.zrow ? ix.zrow[gp[c]] : gp[c];
      float dv[kEdRows];
      ed_rows<kEdRows>(ql, ix.Z, len, gr, act, lane, dv);
      c_ref += (lane == 0) ? __popc(act) : 0;
      // the rare rows within the window of the k-th best, one at a time
      // (one copy of the offer's code)
      unsigned win = 0;
#pragma unroll
      for (int c = 0; c < kEdRows; ++c) win |= (((act >> c) & 1u) && dv[c] <= key_dist(ckey) * p.win) ? (1u << c) : 0u;
      win = __builtin_amdgcn_readfirstlane(win);
      bool ch = false;
      if (win) {
        // lane c holds row c's distance and position
        float dl = 0.0f;
        int gl2 = 0;
#pragma unroll
        for (int c = 0; c < kEdRows; ++c) {
          dl = lane == c ? dv[c] : dl;
          gl2 = lane == c ? gp[c] : gl2;
        }
        while (win) {
          const int c = __builtin_ctz(win);
          win &= win - 1;
          const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dl), c));
          const int gc = __builtin_amdgcn_readlane(gl2, c);
          if (lane == 0) {
            const bool in = offer(ix, p, s, q, d, gc, ckey, true);
            c_bsf += in ? 1 : 0;
            ch |= in;
          }
        }
      }
      if (__ballot(ch)) {
        ckey = umin64(ckey, load_key(&slots[k - 1]));
        if (lane == 0) atomicMin(&s_ckey, ckey);
      }
    };
    // take up to kEdRows entries of wave w's published list; returns how many
    auto take = [&](int w, int (&gp)[kEdRows], float (&gl)[kEdRows]) {
      int n = 0, h = 0;
      if (lane == 0) {
        n = lds_load_acq(&s_n[w]);
        h = n > 0 ? lds_add(&s_h[w], kEdRows) : 0;
      }
      n = __builtin_amdgcn_readfirstlane(n);
      h = __builtin_amdgcn_readfirstlane(h);
      const int cnt = n - h < 0 ? 0 : (n - h > kEdRows ? kEdRows : n - h);
#pragma unroll
      for (int c = 0; c < kEdRows; ++c) {
        gp[c] = c < cnt ? lpos_all[w * kEdList + h + c] : 0;
        gl[c] = c < cnt ? llb_all[w * kEdList + h + c] : INFINITY;
      }
      return cnt;
    };
    // the owner's refinement of its full list: publish it, take groups from
    // it until none is left (other waves may take some), wait until no
    // other wave is still copying from it, then start a new list
    auto refine_own = [&]() {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      if (lane == 0) lds_store_rel(&s_n[wv], nl);
      for (;;) {
        int gp[kEdRows];
        float gl[kEdRows];
        const int cnt = take(wv, gp, gl);
        if (cnt == 0) break;
        refine_rows(gp, gl, cnt);
      }
      if (lane == 0) {
        while (lds_load_acq(&s_busy[wv]) != 0) __builtin_amdgcn_s_sleep(1);
        lds_store_rel(&s_n[wv], 0);
        lds_store_rel(&s_h[wv], 0);
      }
      nl = 0;
    };
    // one group taken from another wave's published list, if any has
    // entries left (the first such wave after this one)
    auto steal = [&]() {
      int rem = 0;
      if (lane < kW && lane != wv) rem = lds_load_acq(&s_n[lane]) - lds_load_acq(&s_h[lane]);
      const unsigned long long any = __ballot(rem > 0);
      if (!any) return false;
      const unsigned long long rot = (any >> (wv + 1)) | (any << (kW - wv - 1));
      const int v = (wv + 1 + __ffsll((long long)(rot & ((1ull << kW) - 1))) - 1) % kW;
      if (lane == 0) lds_add(&s_busy[v], 1);
      int gp[kEdRows];
      float gl[kEdRows];
      const int cnt = take(v, gp, gl);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      if (lane == 0) lds_add(&s_busy[v], -1);
      if (cnt > 0) refine_rows(gp, gl, cnt);
      return true;
    };

    // the next chunk of a stream not yet done, the streams visited from a
    // place that rotates with the wave and the step; false once every
    // stream is done (each failed try marks one, so at most kW + 1 tries)
    unsigned rot = (unsigned)wv;
    auto grab = [&](int& x, int& c) {
      int rx = 0, rc = -1;
      if (lane == 0) {
#pragma unroll 1
        for (int tries = 0; tries <= kW; ++tries) {
          const unsigned dn = lds_load_acq_u(&s_sdone);
          if (dn == kAllStreams) break;
          const int x0 = (int)(rot++ % kW);
          const unsigned free = ~((dn >> x0) | (dn << (kW - x0))) & kAllStreams;
          const int xx = (x0 + __ffs((int)free) - 1) % kW;
          const int cc = s_first[xx] + lds_add(&s_idx[xx], 1) * stride;
          if (cc < s_end[xx]) {
            rx = xx;
            rc = cc;
            break;
          }
          lds_or_u(&s_sdone, 1u << xx);  // stream exhausted
        }
      }
      x = __builtin_amdgcn_readfirstlane(rx);
      c = __builtin_amdgcn_readfirstlane(rc);
      return c >= 0;
    };
    // the first chunk's record; each step loads the next one's (and, now
    // and then, the global k-th best) while the current chunk is worked on
    int x = 0, c = -1;
    grab(x, c);
    unsigned long long item = 0;
    int2 rg = make_int2(0, 0);
    if (c >= 0) {
      item = items[c];
      rg = ranges[c];
    }
    for (;;) {
      // stop: every stream of the block is done
      const bool stop = c < 0;
      int nx = 0, cn = -1;
      unsigned long long n_item = 0, nkey = ~0ull;
      int2 n_rg = make_int2(0, 0);
      if (!stop) {
        if (grab(nx, cn)) {
          n_item = items[cn];
          n_rg = ranges[cn];
        }
        // one wave-step in kEdTick of the block refreshes the block's copy
        unsigned tick = 0;
        if (lane == 0) tick = atomicAdd(&s_tick, 1u);
        if (lane == 0 && tick % kEdTick == 0) nkey = load_key(&slots[k - 1]);
        const float tadj = lb_threshold(key_dist(ckey), eta, p);
        const float lb = key_dist(item);
        if (lb <= tadj) {
          ++c_leaf;
          // series bounds (Algorithm 9): sixteen table lookups, summed
          // pairwise; kEdLoad words per lane in flight at once, each
          // bound's survivor appended to the wave's list once known
#pragma unroll
          for (int h = 0; h < kUnroll; h += kEdLoad) {
            uint4 wd[kEdLoad];
#pragma unroll
            for (int u = 0; u < kEdLoad; ++u) {
              const int pos = rg.x + lane + (h + u) * kWave;
              wd[u] = ix.words[pos < rg.y ? pos : rg.x];
            }
#pragma unroll
            for (int u = 0; u < kEdLoad; ++u) {
              const int pos = rg.x + lane + (h + u) * kWave;
              bool ok = pos < rg.y && !(pos >= P0 && pos < P1);
              float lbv = 0.0f;
              if (ok) {
                float t[kMaxSeg];
#pragma unroll
                for (int sg = 0; sg < kMaxSeg; ++sg) t[sg] = table[sg * card + (int)byte_of(wd[u], sg)];
#pragma unroll
                for (int w2 = kMaxSeg / 2; w2 >= 1; w2 >>= 1)
#pragma unroll
                  for (int sg = 0; sg < w2; ++sg) t[sg] = t[sg] + t[sg + w2];
                lbv = t[0];
                ++c_lb;
                ok = lbv <= tadj;
              }
              const unsigned long long m = __ballot(ok);
              if (ok) {
                const int at = nl + __popcll(m & below);
                lpos[at] = pos;
                llb[at] = lbv;
              }
              nl += __popcll(m);
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
        } else if (bucket_floor(lb_bucket(lb * p.lb_scale)) > tadj * p.lb_scale) {
          // this chunk's bucket starts above the k-th best: so do those of
          // the stream's later chunks
          if (lane == 0) lds_or_u(&s_sdone, 1u << x);
        }
      }
      if (nl >= kEdDefer || (stop && nl > 0)) refine_own();
      if (stop) break;
      nkey = first_lane_u64(nkey);
      if (nkey != ~0ull && lane == 0) atomicMin(&s_ckey, nkey);
      ckey = umin64(ckey, first_lane_u64(s_ckey));
      x = nx;
      c = cn;
      item = n_item;
      rg = n_rg;
    }
    // this wave's chunks are done: help the others until every wave of
    // the block is done and no list has entries left
    if (lane == 0) lds_add(&s_done, 1);
    for (;;) {
      if (steal()) continue;
      int done = 0;
      if (lane == 0) done = lds_load_acq(&s_done);
      if (__builtin_amdgcn_readfirstlane(done) == kW) break;
      __builtin_amdgcn_s_sleep(16);
    }
    // statistics
    for (int o = 32; o >= 1; o >>= 1) {
      c_lb += __shfl_xor(c_lb, o, kWave);
      c_ref += __shfl_xor(c_ref, o, kWave);
    }
    if (p.count_work) {
      __shared__ unsigned long long s_part[4];
      const int which[4] = {kStatLeavesKept, kStatSeriesLb, kStatRefined, kStatBsf};
      const unsigned long long val[4] = {lane == 0 ? c_leaf : 0ull, c_lb, c_ref, c_bsf};
      add_block_counts<4>(s.stats + (int64_t)q * kStatCount, which, val, s_part);
    }
    __syncthreads();  // LDS is reloaded for the next query
  }
}

// ---------------------------------------------------------------------------
// The work the search needs once its final k-th best is known (statistics
// only, run after finalize): the leaves whose bound is within it, their
// series, and those series whose own bound is within it (rows to refine,
// or LB_Keogh to take for DTW).  The approximate search's series are left
// out, as the process kernel leaves them out.  grid.y = query.

__global__ __launch_bounds__(256) void k_min_work(IndexDev ix, QueryParams p, QueryState s) {
  const int q = blockIdx.y;
  const int tid = threadIdx.x;
  const int card = 1 << p.card_bits;
  extern __shared__ float table[];  // [16][card]
  {
    const float* pu = s.paa + ((int64_t)q * 3 + 1) * kMaxSeg;
    const float* pl = s.paa + ((int64_t)q * 3 + 2) * kMaxSeg;
    const float fm = (float)p.m;
    for (int i = tid; i < kMaxSeg * card; i += blockDim.x) {
      const int sg = i >> p.card_bits, j = i & (card - 1);
      float v = 0.0f;
      if (sg < p.w) {
        const float g = fmaxf(ix.bp[j] - pu[sg], 0.0f) + fmaxf(pl[sg] - ix.bp[j + 1], 0.0f);
        v = fm * (g * g);
      }
      table[i] = v;
    }
  }
  __syncthreads();
  const float thr = lb_threshold(kth_dist(s.slots + (int64_t)q * p.k, k_of(p, s, q)), s.eta[q], p);
  const int64_t P0 = s.approx_range[2 * q], P1 = s.approx_range[2 * q + 1];
  const float* lbq = s.leaf_lb + (int64_t)q * p.n_leaves;
  unsigned long long n_leaf = 0, n_series = 0, n_pass = 0;
  for (int l = blockIdx.x; l < p.n_leaves; l += gridDim.x) {
    if (!(lbq[l] <= thr)) continue;
    n_leaf += tid == 0 ? 1 : 0;
    for (int64_t pos = ix.leaf_begin[l] + tid; pos < ix.leaf_end[l]; pos += blockDim.x) {
      if (pos >= P0 && pos < P1) continue;
      const uint4 wd = ix.words[pos];
      float t[kMaxSeg];
#pragma unroll
      for (int sg = 0; sg < kMaxSeg; ++sg) t[sg] = table[sg * card + (int)byte_of(wd, sg)];
#pragma unroll
      for (int h = kMaxSeg / 2; h >= 1; h >>= 1)
#pragma unroll
        for (int sg = 0; sg < h; ++sg) t[sg] = t[sg] + t[sg + h];
      ++n_series;
      n_pass += t[0] <= thr ? 1 : 0;
    }
  }
  for (int o = 32; o >= 1; o >>= 1) {
    n_leaf += __shfl_xor(n_leaf, o, kWave);
    n_series += __shfl_xor(n_series, o, kWave);
    n_pass += __shfl_xor(n_pass, o, kWave);
  }
  if ((tid & (kWave - 1)) == 0) {
    unsigned long long* stq = s.stats + (int64_t)q * kStatCount;
    if (n_leaf) atomicAdd(&stq[kStatMinLeaves], n_leaf);
    if (n_series) atomicAdd(&stq[kStatMinSeries], n_series);
    if (n_pass) atomicAdd(&stq[kStatMinRefined], n_pass);
  }
}

void launch_min_work(const IndexDev& ix, const QueryParams& qp, const QueryState& qs, int blocks,
                     hipStream_t st) {
  const size_t lds = (size_t)kMaxSeg * ((size_t)1 << qp.card_bits) * sizeof(float);
  hipLaunchKernelGGL(k_min_work, dim3((unsigned)blocks, (unsigned)qp.nq), dim3(256), lds, st, ix, qp, qs);
}

// ---------------------------------------------------------------------------
// finalize: one block per query.  FP64 recheck of the near ties, exact
// (distance, id) order, outputs.  The log is taken in chunks; each chunk's
// candidates in the window are recomputed in FP64 and merged with the
// running k best by rank, so any number of ties fits.

constexpr int kFinBatch = 4;  // points per lane per step of the FP64 ED recheck

__global__ __launch_bounds__(kProcThreads) void k_finalize(IndexDev ix, QueryParams p, QueryState s,
                                                           int64_t* __restrict__ out_ids,
                                                           float* __restrict__ out_dists) {
  const int q = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const int len = p.len, k = k_of(p, s, q);
  extern __shared__ float sm[];
  // layout: E[kTopCap] doubles | pos[kTopCap] | id[kTopCap] | q[len] |
  // x rows[fin_waves][len] | (8-byte aligned) DP buffers[fin_waves][3 len] doubles
  double* E = reinterpret_cast<double*>(sm);
  int* pos_l = reinterpret_cast<int*>(E + kTopCap);
  int* id_l = pos_l + kTopCap;
  float* ql = reinterpret_cast<float*>(id_l + kTopCap);
  float* xl = ql + len;
  const size_t dbuf_off = (((size_t)4 * kTopCap + len + (size_t)p.fin_waves * len) + 1) & ~(size_t)1;
  double* dbuf = reinterpret_cast<double*>(sm + dbuf_off);
  __shared__ int s_cnt;
  const unsigned long long* slots = s.slots + (int64_t)q * p.k;
  const float T = kth_dist(slots, k);
  const float win = T * p.win;
  const int lc = s.log_count[q];
  if (lc > p.log_cap) {
    if (tid == 0) s.status[q] |= 1;
    return;
  }
  const float* zq = s.zq + (int64_t)q * len;
  for (int t = tid; t < len; t += blockDim.x) ql[t] = zq[t];
  const unsigned long long* lg = s.log + (int64_t)q * p.log_cap;
  const int chunk = kTopCap - k;
  int topn = 0;
  unsigned long long rechecked = 0;
  for (int base = 0; base < lc; base += chunk) {
    if (tid == 0) s_cnt = topn;
    __syncthreads();
    const int lim = base + chunk < lc ? base + chunk : lc;
    for (int i = base + tid; i < lim; i += blockDim.x) {
      const unsigned long long e = lg[i];
      if (key_dist(e) <= win) pos_l[atomicAdd(&s_cnt, 1)] = (int)key_id(e);
    }
    __syncthreads();
    const int cnt = s_cnt;
    rechecked += (unsigned long long)(cnt - topn);
    // exact distances of the new entries, FP64, index order, unfused
    if (p.distance == 0) {
      // one wave per candidate: the lanes load and square kFinBatch
      // points each, the squares go to the wave's LDS strip in index order,
      // and lane 0 adds them in that order, unfused
      const int nw = blockDim.x / kWave;
      double* sqb = dbuf + wv * (kFinBatch * kWave);
      for (int c0 = topn; c0 < cnt; c0 += nw) {
        const int c = c0 + wv;
        if (c < cnt) {
          const float* x = zrow_ptr(ix, pos_l[c]);
          double acc = 0.0;
          for (int t0 = 0; t0 < len; t0 += kFinBatch * kWave) {
            float xv[kFinBatch];
#pragma unroll
            for (int u = 0; u < kFinBatch; ++u) {
              const int t = t0 + u * kWave + lane;
              xv[u] = t < len ? x[t] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < kFinBatch; ++u) {
              const int t = t0 + u * kWave + lane;
              if (t < len) {
                const double d = (double)ql[t] - (double)xv[u];
                sqb[u * kWave + lane] = __dmul_rn(d, d);
              }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) {  // 16 reads in flight before their 16 adds
              const int nn = len - t0 < kFinBatch * kWave ? len - t0 : kFinBatch * kWave;
              int i = 0;
              for (; i + 16 <= nn; i += 16) {
                double v[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) v[j] = sqb[i + j];
#pragma unroll
                for (int j = 0; j < 16; ++j) acc = __dadd_rn(acc, v[j]);
              }
              for (; i < nn; ++i) acc = __dadd_rn(acc, sqb[i]);
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();  // the strip is rewritten next
          }
          if (lane == 0) {
            E[c] = acc;
            id_l[c] = ix.perm[pos_l[c]];
          }
        }
      }
    } else {
      for (int c0 = topn; c0 < cnt; c0 += p.fin_waves) {
        const int c = c0 + wv;
        if (wv < p.fin_waves && c < cnt) {
          const float* x = zrow_ptr(ix, pos_l[c]);
          for (int t = lane; t < len; t += kWave) xl[wv * len + t] = x[t];
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
          const double v =
              2 * p.window + 1 <= kWave
                  ? dtw_reg64(ql, xl + wv * len, len, p.window, lane)
                  : dtw_wave<double>(ql, xl + wv * len, len, p.window, dbuf + wv * 3 * len,
                                     (double)INFINITY, lane);
          if (lane == 0) {
            E[c] = v;
            id_l[c] = ix.perm[pos_l[c]];
          }
        }
      }
    }
    __syncthreads();
    // keep the k smallest (E, id): rank in registers, then move
    constexpr int kPer = kTopCap / kProcThreads;
    double e_r[kPer];
    int p_r[kPer], i_r[kPer], rk[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int c = tid + j * kProcThreads;
      rk[j] = kTopCap;
      if (c < cnt) {
        const double e = E[c];
        const int id = id_l[c];
        int r = 0;
        for (int o = 0; o < cnt; ++o) {
          const double eo = E[o];
          r += (eo < e || (eo == e && id_l[o] < id)) ? 1 : 0;
        }
        rk[j] = r;
        e_r[j] = e;
        p_r[j] = pos_l[c];
        i_r[j] = id;
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      if (rk[j] < k) {
        E[rk[j]] = e_r[j];
        pos_l[rk[j]] = p_r[j];
        id_l[rk[j]] = i_r[j];
      }
    }
    __syncthreads();
    topn = cnt < k ? cnt : k;
  }
  const int64_t orow = (int64_t)row_of(s, q) * p.out_stride;
  for (int j = tid; j < p.out_stride; j += blockDim.x) {
    if (j < topn) {
      out_ids[orow + j] = (int64_t)id_l[j];
      out_dists[orow + j] = (float)sqrt(E[j]);
    } else {
      out_ids[orow + j] = -1;
      out_dists[orow + j] = INFINITY;
    }
  }
  if (tid == 0) s.stats[(int64_t)q * kStatCount + kStatRecheck] = rechecked;
}

// ---------------------------------------------------------------------------
// BF16 screen of batched ED queries (a lower-bound filter in front of the
// FP32 refinement; not part of the paper's method, the answers stay exact).
//
// The leaves are taken leaf-major: each leaf is read once for every query
// whose leaf bound passed its first k-th best, and q.x of every (query,
// series) pair comes from BF16 MFMA (16x16x32, FP32 accumulation).  With
// s~ that dot product, d~^2 = |q|^2 + |x|^2 - 2 s~ is within
//   E = c_dot |q| |x| + c_abs (|q|^2 + |x|^2 + 2 |s~|)
// of the exact squared distance of the FP32 rows: c_dot covers the BF16
// rounding of both operands, 2 (2 u_b + u_b^2), u_b = 2^-8, and the FP32
// accumulation of len products, 2 gamma_len (1 + u_b)^2 with gamma taken
// at unit 2^-23; c_abs covers the FP32 norms and the FP32 evaluation of
// d~^2.  A pair is dropped only if d~^2 - E, a lower bound of its exact
// squared distance, exceeds the k-th best times the near-tie window.  So
// every pair whose exact squared distance is within that window survives
// and is refined in FP32, among them every true k nearest (an exact
// distance of at most the final k-th best over 1 - rho is inside the
// window).  A pair just outside the window by exact distance may be
// dropped where the unscreened path, whose FP32 distance can round into
// the window, would log it; the answers are the same, as the log only has
// to hold the true k best.  The series the approximate search already
// refined are skipped (their keys are in the k best; they are logged from
// the approximate distances).

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));  // 16 bytes kept in registers
// Global-memory views of generic pointers: loads through them are global
// loads, which the hardware counts in order with the other vector loads
// (a load through a generic pointer also counts as an LDS access, and
// waiting for one waits for every load issued before it).
typedef __attribute__((address_space(1))) const int g_int;
typedef __attribute__((address_space(1))) const float g_float;
typedef __attribute__((address_space(1))) const u32x4 g_u32x4;

__device__ __forceinline__ uint32_t bf16_bits(float f) {  // finite f, round to nearest even
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// One wave per row: BF16 copy and FP64 squared norm (len % 4 == 0).
__global__ __launch_bounds__(256) void k_bf16_rows(const float* __restrict__ src,
                                                   const int32_t* __restrict__ src_row, int64_t rows,
                                                   int len, uint16_t* __restrict__ dst,
                                                   float* __restrict__ norms) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < rows;
       r += waves) {
    const float* x = src + (src_row ? (int64_t)src_row[r] : r) * len;
    uint2* y = reinterpret_cast<uint2*>(dst + r * len);
    double acc = 0.0;
    for (int t = 4 * lane; t < len; t += 4 * kWave) {
      const float4 v = *reinterpret_cast<const float4*>(x + t);
      acc += (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
      y[t >> 2] = make_uint2(bf16_bits(v.x) | (bf16_bits(v.y) << 16),
                             bf16_bits(v.z) | (bf16_bits(v.w) << 16));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, kWave);
    if (lane == 0) norms[r] = (float)acc;
  }
}

// Leaf query lists: a query keeps a leaf whose bound passes its first k-th
// best (from the approximate search).  Thread per leaf, queries in LDS
// chunks; `fill` = false counts, true writes the lists.
__global__ __launch_bounds__(256) void k_leaf_lists(QueryParams p, QueryState s, ScreenDev sc,
                                                    bool fill) {
  __shared__ float thr[256];
  const int l = blockIdx.x * 256 + threadIdx.x;
  int c = 0;
  int64_t at = (fill && l < p.n_leaves) ? sc.off[l] : 0;
  for (int q0 = 0; q0 < p.nq; q0 += 256) {
    __syncthreads();
    const int q = q0 + (int)threadIdx.x;
    if (q < p.nq)
      thr[threadIdx.x] = lb_threshold(kth_dist(s.slots + (int64_t)q * p.k, k_of(p, s, q)), s.eta[q], p);
    __syncthreads();
    const int nn = min(256, p.nq - q0);
    if (l < p.n_leaves) {
      // sixteen queries' bounds of this leaf in flight at a time (the index
      // is clamped, the comparison masked past the chunk)
      const float* __restrict__ col = s.leaf_lb + (int64_t)q0 * p.n_leaves + l;
      int* __restrict__ lists = sc.lists;
      for (int j0 = 0; j0 < nn; j0 += 16) {
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = col[(int64_t)min(j0 + u, nn - 1) * p.n_leaves];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (j0 + u < nn && v[u] <= thr[j0 + u]) {
            if (fill) lists[at++] = q0 + j0 + u;
            ++c;
          }
      }
    }
  }
  if (!fill && l < p.n_leaves) sc.cnt[l] = c;
}

__global__ __launch_bounds__(256) void k_log_approx(QueryParams p, QueryState s) {
  log_approx(p, s, blockIdx.x, threadIdx.x, blockDim.x);
}

// Exclusive scan of the list lengths (one block, tiles of 4,096 lengths:
// four consecutive per thread, a wave scan, a scan of the wave sums, and
// the running total carried between tiles); also resets the work counter
// and the tallies.
__global__ __launch_bounds__(1024) void k_list_scan(QueryParams p, ScreenDev sc) {
  __shared__ int64_t wsum[16];
  __shared__ int64_t s_carry;
  const int L = p.n_leaves;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid >> 6;
  if (tid == 0) s_carry = 0;
  __syncthreads();
  for (int base = 0; base < L; base += 4096) {
    const int i0 = base + 4 * tid;
    int c[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) c[u] = i0 + u < L ? sc.cnt[i0 + u] : 0;
    const int64_t t = (int64_t)c[0] + c[1] + c[2] + c[3];
    int64_t x = t;  // inclusive scan over the wave
    for (int o = 1; o < kWave; o <<= 1) {
      const int64_t y = __shfl_up(x, o, kWave);
      if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wsum[wv] = x;
    __syncthreads();
    if (wv == 0) {  // inclusive scan of the 16 wave sums
      int64_t w = lane < 16 ? wsum[lane] : 0;
      for (int o = 1; o < 16; o <<= 1) {
        const int64_t y = __shfl_up(w, o, kWave);
        if (lane >= o) w += y;
      }
      if (lane < 16) wsum[lane] = w;
    }
    __syncthreads();
    int64_t run = s_carry + (wv ? wsum[wv - 1] : 0) + (x - t);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (i0 + u < L) sc.off[i0 + u] = run;
      run += c[u];
    }
    __syncthreads();  // every thread has read s_carry and wsum
    if (tid == 0) s_carry += wsum[15];
    __syncthreads();
  }
  if (tid == 0) {
    sc.off[L] = s_carry;
    *sc.counter = 0;
    sc.tally[0] = 0;
    sc.tally[1] = 0;
  }
}

// Screen and refinement, leaf-major, as a tiled BF16 GEMM per leaf: the
// block's W waves hold 16 NT series each of a column pass in registers
// (MFMA B operand); the leaf's query list streams through LDS in chunks of
// 8 W queries (A operand), double buffered.  Lane l holds output rows
// 4 (l / 16) .. + 3 of column l % 16 of each 16 x 16 tile.  With W = 4 two
// blocks share a CU, and one block's loads of a new pass's B operands
// overlap the other's MFMA work (a block waits at its own barriers only).
//
// The test of a pair is folded into per-row and per-column terms.  With
// |s~| <= (|q|^2 + |x|^2) / 2 the bound is at most
//   c_dot |q| |x| + c_abs (|q|^2 + |x|^2),   c_abs = 2^-17,
// which also covers the FP32 rounding of the folded expression, so a pair
// is dropped iff
//   R_q + C_x - a_q s_x - 2 s~ > 0,
//   R_q = |q|^2 (1 - c_abs) - thr_q,  C_x = |x|^2 (1 - c_abs),
//   a_q = c_dot |q|,  s_x = |x|.
// The terms are kept halved (exact scalings by 1/2), so T = fl(fl(R_q / 2 +
// C_x / 2) - a_q s_x / 2) is half the folded FP32 value, and the test is one
// exact comparison, s~ < T.
// Rows past the list and columns past the leaf get R_q / C_x = +inf.  Pairs
// kept are refined by the whole wave in FP32 and offered to their query's
// k best, except the query's own approximate-search range (already in its
// k best and logged).
constexpr int kScreenGrab = 4;  // leaves taken per grab of the screen's work counter
constexpr int kScreenListCap = 2048;  // query-list entries of a leaf staged in LDS

// KS: 32-element K steps per row (len / 32); NT: 16-series column tiles
// each wave holds in registers (its B operands: NT x KS x 4 VGPRs); W:
// waves per block, with query chunks of 8 W rows (so a thread stages KS / 2
// 16-byte pieces of A per chunk whatever W is).
template <int KS, int NT, int W>
struct ScreenShape {
  static constexpr int len = 32 * KS;
  static constexpr int waves = W;
  static constexpr int threads = W * kWave;
  static constexpr int chunk = 8 * W;             // query rows per A chunk
  static constexpr int row_bytes = 2 * len + 16;  // padded: rows start 4 banks apart
  static constexpr int a_bytes = chunk * row_bytes;
  static constexpr int per_thread = chunk * (len / 8) / threads;  // uint4 loads
  static constexpr size_t lds = 2 * (size_t)a_bytes;
  static constexpr int tiles = NT;
  static constexpr int pass = 16 * tiles * W;
};

// Column tiles per wave when no tuned value is given.
constexpr int screen_default_nt(int len) { return len >= 512 ? 1 : 4; }

template <int KS, int NT, int W>
__global__ __launch_bounds__(W * kWave) __attribute__((amdgpu_waves_per_eu(2)))
void k_screen(IndexDev ix, QueryParams p, QueryState s, ScreenDev sc) {
  using Sh = ScreenShape<KS, NT, W>;
  constexpr int len = Sh::len;
  constexpr int kThreads = Sh::threads;
  constexpr int kScreenChunk = Sh::chunk;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int col = lane & 15, kb = 8 * (lane >> 4);
  extern __shared__ uint4 smem_v[];
  char* abuf = reinterpret_cast<char*>(smem_v);
  __shared__ float s_R[2][kScreenChunk], s_a[2][kScreenChunk];
  __shared__ int s_q[2][kScreenChunk];
  // the leaf's query list when it fits: each entry's query, its k and |q|^2
  __shared__ int s_list[kScreenListCap], s_lk[kScreenListCap];
  __shared__ float s_ln[kScreenListCap];
  __shared__ int s_leaf;
  const float one_m = 1.0f - sc.c_abs;
  unsigned long long screened = 0, passed = 0;
  // leaves are taken kScreenGrab at a time (one device atomic each: the
  // counter is one address for the whole grid)
  for (int leaf = 0, grab_end = 0;; ++leaf) {
    if (leaf >= grab_end) {
      if (tid == 0) s_leaf = atomicAdd(sc.counter, kScreenGrab);
      __syncthreads();
      leaf = s_leaf;
      __syncthreads();
      grab_end = leaf + kScreenGrab;
    }
    if (leaf >= p.n_leaves) break;
    const int64_t l0 = sc.off[leaf], l1 = sc.off[leaf + 1];
    const int64_t b = ix.leaf_begin[leaf], e = ix.leaf_end[leaf];
    // the list in segments of at most kScreenListCap queries (one, unless
    // the batch is larger), each screened against the whole leaf
    for (int64_t s0 = l0; s0 < l1; s0 += kScreenListCap) {
      const int nlist = (int)min<int64_t>(l1 - s0, kScreenListCap);
      const int nch = (nlist + kScreenChunk - 1) / kScreenChunk;
      // the segment's entries, with each query's k and |q|^2, into LDS, so
      // that fetching a chunk is one round trip to memory (its rows and k-th
      // best distances), which the chunk before it covers
      // (the previous segment's or leaf's last chunk step ended at a barrier)
      g_int* glist = (g_int*)(sc.lists + s0);
      for (int i = tid; i < nlist; i += kThreads) {
        const int q = glist[i];
        s_list[i] = q;
        s_lk[i] = ((g_int*)s.kq)[q];
        s_ln[i] = ((g_float*)sc.qn)[q];
      }
      __syncthreads();
      // chunk c of the list into registers: A rows and the row terms.  Every
      // load is unconditional (rows past the list read the list's last query
      // and are masked by R = +inf), so they are all in flight together
      u32x4 pa[Sh::per_thread];
      int pq = -1;
      float pqn = 0.0f;   // the row's |q|^2
      float pkth = 0.0f;  // its query's k-th best squared distance when fetched
      auto fetch = [&](int c) __attribute__((always_inline)) {
        int qi[Sh::per_thread];
        const int li = c * kScreenChunk + tid;
        const int l1c = min(li, nlist - 1);
#pragma unroll
        for (int u = 0; u < Sh::per_thread; ++u)
          qi[u] = s_list[min(c * kScreenChunk + (tid + u * kThreads) / (len / 8), nlist - 1)];
        const int q0 = s_list[l1c], kq = s_lk[l1c];
        const float qn = s_ln[l1c];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < Sh::per_thread; ++u) {
          const int c16 = (tid + u * kThreads) % (len / 8);
          pa[u] = ((g_u32x4*)(sc.qb + (int64_t)qi[u] * len))[c16];
        }
        __builtin_amdgcn_sched_barrier(0);
        // the row terms are formed when the chunk is stashed, so that nothing
        // here waits for these loads.  A plain load of the upper half (the
        // distance) of the k-th best key: a stale value is larger (slots only
        // decrease), so only looser
        pkth = ((g_float*)s.slots)[2 * ((int64_t)q0 * p.k + kq - 1) + 1];
        pqn = qn;
        pq = li < nlist ? q0 : -1;
      };
      auto stash = [&](int buf) __attribute__((always_inline)) {
        char* dst = abuf + buf * Sh::a_bytes;
#pragma unroll
        for (int u = 0; u < Sh::per_thread; ++u) {
          const int v = tid + u * kThreads;
          const int row = v / (len / 8), c16 = v % (len / 8);
          *reinterpret_cast<u32x4*>(dst + row * Sh::row_bytes + 16 * c16) = pa[u];
        }
        if (tid < kScreenChunk) {
          const bool ok = pq >= 0;
          s_q[buf][tid] = pq;
          s_R[buf][tid] = ok ? 0.5f * (pqn * one_m - pkth * p.win) : INFINITY;
          s_a[buf][tid] = ok ? 0.5f * (sc.c_dot * sqrtf(pqn)) : 0.0f;
        }
      };
      // Column passes over the leaf.  The query list is the same for every
      // pass: chunk c of a pass sits in LDS buffer cur ^ (c & 1), and the last
      // chunk's step stages chunk 0 again for the next pass (a one-chunk list
      // simply stays in buffer cur), so only the leaf's first pass waits for
      // its chunk 0.  Its row terms keep the k-th best of that first fetch,
      // which only makes them looser.  Every fetch is unconditional (a step
      // with nothing to stage fetches its own chunk again and discards it),
      // so no loaded value has to be merged at a branch's end, which would
      // wait for it there.
      int cur = 0;
      fetch(0);
      stash(0);
      __syncthreads();
      for (int64_t base = b; base < e; base += Sh::pass) {
        const int64_t wbase = base + 16 * NT * wv;
        float cx[NT], sx[NT], xnv[NT];
        bf16x8 B[NT][KS];
        // the column norms, then the B operands, all loads unconditional
        // (columns past the leaf read its last row; their column term C_x =
        // +inf masks them).  Loads complete in issue order: the column terms
        // formed next wait for the norms only, and the B operands are issued
        // in the order the products use them, so the pass's first products
        // wait for the first K step only
        const u32x4* src[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int64_t j = wbase + 16 * t + col;
          const int64_t jc = j < e ? j : e - 1;
          xnv[t] = sc.xn[jc];
          src[t] = reinterpret_cast<const u32x4*>(sc.Zb + jc * len + kb);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
          for (int t = 0; t < NT; ++t) B[t][ks] = __builtin_bit_cast(bf16x8, src[t][4 * ks]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const bool v = wbase + 16 * t + col < e;
          cx[t] = v ? 0.5f * (xnv[t] * one_m) : INFINITY;
          sx[t] = sqrtf(xnv[t]);
        }
        const int ncols = (int)((e - wbase) < 16 * NT ? ((e - wbase) > 0 ? (e - wbase) : 0) : 16 * NT);
        const bool more = base + Sh::pass < e;
        for (int c = 0; c < nch; ++c) {
          const int buf = cur ^ (c & 1);
          // the next chunk of this pass, or chunk 0 again for the next pass
          const int nxt = c + 1 < nch ? c + 1 : (more && nch > 1 ? 0 : -1);
          fetch(nxt >= 0 ? nxt : c);
          const char* A = abuf + buf * Sh::a_bytes;
          const int rows_valid = min(kScreenChunk, nlist - c * kScreenChunk);
#pragma unroll 1
          // (a wave whose columns all lie past the leaf, in a leaf's last
          // pass, has nothing to screen: the other block on the CU gets its
          // share of the matrix cores meanwhile)
          for (int qt = 0; ncols > 0 && qt < kScreenChunk / 16 && 16 * qt < rows_valid; ++qt) {
            f32x4 acc[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            const char* arow = A + (16 * qt + col) * Sh::row_bytes + 2 * kb;
            // the tile's A operands all in flight before the first product
            bf16x8 av[KS];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
              av[ks] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(arow + 64 * ks));
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
              for (int t = 0; t < NT; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[ks], B[t][ks], acc[t], 0, 0, 0);
            }
            screened += (unsigned long long)(min(16, rows_valid - 16 * qt) * ncols);
            float Rh[4], ah[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = 16 * qt + 4 * (lane >> 4) + r;
              Rh[r] = s_R[buf][row];
              ah[r] = s_a[buf][row];
            }
            // kept: s~ >= T (or NaN); which pairs, only when some lane has one
            bool any = false;
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
              for (int t = 0; t < NT; ++t) any |= !(acc[t][r] < __builtin_fmaf(-ah[r], sx[t], Rh[r] + cx[t]));
            if (__ballot(any)) {  // rare: refine the kept pairs one at a time
              uint32_t keep = 0;
#pragma unroll
              for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int t = 0; t < NT; ++t)
                  keep |= (acc[t][r] < __builtin_fmaf(-ah[r], sx[t], Rh[r] + cx[t]) ? 0u : 1u) << (r * NT + t);
              unsigned long long m = __ballot(keep != 0);
              while (m) {
                const int src_lane = __ffsll((long long)m) - 1;
                m &= m - 1;
                uint32_t bits = __shfl(keep, src_lane, kWave);
                while (bits) {
                  const int bit = __ffs(bits) - 1;
                  bits &= bits - 1;
                  const int r = bit / NT, t = bit % NT;
                  const int row = 16 * qt + 4 * (src_lane >> 4) + r;
                  const int qsel = s_q[buf][row];
                  const int64_t jsel = wbase + 16 * t + (src_lane & 15);
                  if (qsel < 0 || jsel >= e) continue;
                  if (jsel >= s.approx_range[2 * qsel] && jsel < s.approx_range[2 * qsel + 1]) continue;
                  const float d2 = ed_wave(s.zq + (int64_t)qsel * len, zrow_ptr(ix, jsel), len, lane);
                  if (lane == 0) {
                    const int kk = k_of(p, s, qsel);
                    const unsigned long long ck = load_key(s.slots + (int64_t)qsel * p.k + kk - 1);
                    const bool in = offer(ix, p, s, qsel, d2, jsel, ck, true);
                    if (p.count_work) {
                      if (in) atomicAdd(&s.stats[(int64_t)qsel * kStatCount + kStatBsf], 1ull);
                      atomicAdd(&s.stats[(int64_t)qsel * kStatCount + kStatRefined], 1ull);
                    }
                  }
                  ++passed;
                }
              }
            }
          }
          if (nxt >= 0) {
            stash(buf ^ 1);
          } else {  // the discarded fetch's loads are waited for here, where they have
                    // long arrived, so that no later step waits on them
#pragma unroll
            for (int u = 0; u < Sh::per_thread; ++u) asm volatile("" ::"v"(pa[u]));
            asm volatile("" ::"v"(pkth));
          }
          __syncthreads();
        }
        if (nch > 1) cur ^= nch & 1;  // where the next pass's chunk 0 was staged
      }
    }
  }
  // lanes of a wave counted the same tiles: one add per wave
  if (lane == 0 && p.count_work) {
    atomicAdd(&sc.tally[0], screened);
    atomicAdd(&sc.tally[1], passed);
  }
}

// ---------------------------------------------------------------------------
// k-NN classifier vote (Section 5.4): one block per query; the class held
// by most of its k neighbours, ties to the class met first in the (distance,
// id) order.  The key (count << 32 | (2047 - first rank) << 12 | class) is
// maximised over classes; labels outside [0, n_classes) are not counted.

__global__ __launch_bounds__(256) void k_vote(const int64_t* __restrict__ ids, int64_t stride, int k,
                                              const int* __restrict__ labels, int n_classes,
                                              int* __restrict__ out) {
  extern __shared__ int vsm[];
  int* cnt = vsm;                 // [n_classes]
  int* first = vsm + n_classes;   // [n_classes]
  __shared__ unsigned long long s_best;
  const int q = blockIdx.x;
  for (int c = threadIdx.x; c < n_classes; c += blockDim.x) {
    cnt[c] = 0;
    first[c] = k;
  }
  if (threadIdx.x == 0) s_best = 0;
  __syncthreads();
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    const int64_t id = ids[(int64_t)q * stride + j];
    if (id < 0) continue;
    const int c = labels[id];
    if (c < 0 || c >= n_classes) continue;
    atomicAdd(&cnt[c], 1);
    atomicMin(&first[c], j);
  }
  __syncthreads();
  unsigned long long best = 0;
  for (int c = threadIdx.x; c < n_classes; c += blockDim.x) {
    if (cnt[c] == 0) continue;
    const unsigned long long key = ((unsigned long long)cnt[c] << 32) |
                                   ((unsigned long long)(2047 - first[c]) << 12) | (unsigned)c;
    best = key > best ? key : best;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    const unsigned long long u = __shfl_xor(best, o, kWave);
    best = u > best ? u : best;
  }
  if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(&s_best, best);
  __syncthreads();
  if (threadIdx.x == 0) out[q] = s_best ? (int)(s_best & 4095u) : -1;
}

void launch_vote(const int64_t* ids, int64_t stride, int nq, int k, const int* labels, int n_classes,
                 int* out, hipStream_t st) {
  if (nq <= 0) return;
  hipLaunchKernelGGL(k_vote, dim3(nq), dim3(256), 2 * sizeof(int) * (size_t)n_classes, st, ids,
                     stride, k, labels, n_classes, out);
}

// ---------------------------------------------------------------------------
// Launchers.  The DTW radius picks a register-band instance: exact radii of
// the common windows, else the next larger band with a mask, else the wave
// anti-diagonal kernels.

#define MESSI_BANDS(X) X(0) X(1) X(2) X(3) X(4) X(6) X(8) X(12) X(13) X(16) X(25) X(26) X(32) X(51) X(64)

static int pick_band(int r, bool* mask) {
  static const int exact[] = {0, 1, 2, 3, 4, 6, 8, 12, 13, 16, 25, 26, 32, 51, 64};
  for (int e : exact)
    if (e == r) {
      *mask = false;
      return r;
    }
  static const int masked[] = {8, 16, 32, 64};
  for (int e : masked)
    if (r < e) {
      *mask = true;
      return e;
    }
  *mask = false;
  return -2;
}

// LB_Improved runs on the masked bands (any radius below the band) and on
// the wave kernel only.
static int pick_band_lbi(int r, bool* mask) {
  static const int masked[] = {8, 16, 32, 64};
  for (int e : masked)
    if (r < e) {
      *mask = true;
      return e;
    }
  *mask = false;
  return -2;
}

static int band_of(const QueryParams& p, bool* mask) {
  *mask = false;
  if (p.distance == 0) return -1;
  return p.lb_improved ? pick_band_lbi(p.window, mask) : pick_band(p.window, mask);
}

template <int R>
static size_t process_lds_words(const QueryParams& p) {
  using Sh = ProcShape<R>;
  const int card = 1 << p.card_bits;
  const int qlen = R >= 0 ? p.len + 2 * R : p.len;
  size_t words = (size_t)kMaxSeg * card + qlen + 2 * (size_t)p.len + 2 * (size_t)Sh::surv_cap +
                 Sh::pend_cap;
  if (R == -2) words += (size_t)Sh::waves * 4 * p.len;
  if (R >= 0 && p.lb_improved) words += (size_t)Sh::waves * p.len;  // LB_Improved projections
  return words;
}

size_t process_lds_bytes(const QueryParams& p) {
  bool mask;
  const int R = band_of(p, &mask);
  size_t w = 0;
  if (R == -1)  // the table is static LDS for 8-bit symbols
    w = (p.card_bits == 8 ? 0 : (size_t)kMaxSeg * (1 << p.card_bits)) + p.len + 2 * (size_t)kEdWaves * kEdList;
  else if (R == -2) w = process_lds_words<-2>(p);
  else w = process_lds_words<0>(p) + 2 * (size_t)R;  // the padded query grows with R
  return w * sizeof(float);
}

static int process_threads(int R) {
  return R == -2 ? ProcShape<-2>::threads : (R == -1 ? kEdThreads : ProcShape<0>::threads);
}

size_t finalize_lds_bytes(const QueryParams& p) {
  // DTW: fin_waves rows and FP64 wave buffers (none when the band fits one
  // wave's registers, 2 r + 1 <= 64); ED: a strip of squares per wave
  const size_t dwords = p.distance == 0 ? (size_t)(kProcThreads / kWave) * kFinBatch * kWave
                        : 2 * p.window + 1 <= kWave ? 0
                                                    : (size_t)p.fin_waves * 3 * p.len;
  const size_t words = ((((size_t)4 * kTopCap + p.len + (size_t)p.fin_waves * p.len) + 1) & ~(size_t)1) +
                       dwords * 2;
  return words * sizeof(float);
}

static size_t stage1_lds_bytes(const QueryParams& p, int R);

size_t stage1_lds_bytes(const QueryParams& p) {
  bool mask;
  return stage1_lds_bytes(p, band_of(p, &mask));
}

static size_t stage1_lds_bytes(const QueryParams& p, int R) {
  const size_t lb_words = (size_t)kMaxSeg * (2 * ((size_t)1 << p.card_bits) - 1) + kLbBuckets;
  const size_t ap_words = R == -1 ? (size_t)p.len : (R == -2 ? 17 * (size_t)p.len : (size_t)p.len + 2 * R);
  return (lb_words > ap_words ? lb_words : ap_words) * sizeof(float);
}

void launch_prep(const IndexDev& ix, const float* queries, const QueryParams& qp,
                 const QueryState& qs, hipStream_t st) {
  const size_t lds = 4 * (size_t)qp.len * sizeof(float);
  hipLaunchKernelGGL(k_prep, dim3(qp.nq), dim3(256), lds, st, ix, queries, qp, qs);
}

void launch_stage1(const IndexDev& ix, const QueryParams& qp, const QueryState& qs,
                   hipStream_t st) {
  bool mask;
  const int R = band_of(qp, &mask);
  // ED: a leaf of at most 2,000 rows is eight-row groups for 16 waves (a
  // batch: the grid has many queries) or, for a few queries, 256 waves
  const int approx_blocks = R == -1 ? (qp.leaf_in_prep ? 4 : 64) : (R == -2 ? 64 : (kApproxCap + 255) / 256);
  // one bound block per shard when the chunk order is written; otherwise
  // the bounds alone come from k_leaf_bounds, query tiles sharing each leaf
  const dim3 g(approx_blocks + (qp.order_leaves ? kShards : 0), qp.nq);
  const size_t lds = stage1_lds_bytes(qp, R);
  if (!qp.order_leaves) {
    const dim3 gb((unsigned)((qp.n_leaves + 255) / 256), (unsigned)((qp.nq + kBoundQueries - 1) / kBoundQueries));
    hipLaunchKernelGGL(k_leaf_bounds, gb, dim3(256), 0, st, ix, qp, qs);
  }
  if (R == -1) {
    hipLaunchKernelGGL((k_stage1<-1, false>), g, dim3(256), lds, st, ix, qp, qs, approx_blocks);
    return;
  }
  if (R == -2) {
    hipLaunchKernelGGL((k_stage1<-2, false>), g, dim3(256), lds, st, ix, qp, qs, approx_blocks);
    return;
  }
#define MESSI_S1_CASE(RR)                                                                          \
  if (R == RR) {                                                                                   \
    if (mask)                                                                                      \
      hipLaunchKernelGGL((k_stage1<RR, true>), g, dim3(256), lds, st, ix, qp, qs, approx_blocks);  \
    else                                                                                           \
      hipLaunchKernelGGL((k_stage1<RR, false>), g, dim3(256), lds, st, ix, qp, qs, approx_blocks); \
    return;                                                                                        \
  }
  MESSI_BANDS(MESSI_S1_CASE)
#undef MESSI_S1_CASE
}

void launch_process(const IndexDev& ix, const QueryParams& qp, const QueryState& qs,
                    int blocks_per_query, hipStream_t st) {
  bool mask;
  const int R = band_of(qp, &mask);
  const dim3 g((unsigned)blocks_per_query * (unsigned)qp.nq);  // block b starts on query b % nq
  const dim3 b(process_threads(R));
  const size_t lds = process_lds_bytes(qp);
  if (R == -1) {  // one grid for all queries: blocks_per_query is its size
    if (qp.card_bits == 8)
      hipLaunchKernelGGL(k_process_ed<8>, dim3((unsigned)blocks_per_query), b, lds, st, ix, qp, qs);
    else
      hipLaunchKernelGGL(k_process_ed<0>, dim3((unsigned)blocks_per_query), b, lds, st, ix, qp, qs);
    return;
  }
  if (qp.lb_improved) {
    switch (R) {
      case 8: hipLaunchKernelGGL((k_process<8, true, true>), g, b, lds, st, ix, qp, qs); break;
      case 16: hipLaunchKernelGGL((k_process<16, true, true>), g, b, lds, st, ix, qp, qs); break;
      case 32: hipLaunchKernelGGL((k_process<32, true, true>), g, b, lds, st, ix, qp, qs); break;
      case 64: hipLaunchKernelGGL((k_process<64, true, true>), g, b, lds, st, ix, qp, qs); break;
      default: hipLaunchKernelGGL((k_process<-2, false, true>), g, b, lds, st, ix, qp, qs); break;
    }
    return;
  }
  if (R == -2) {
    hipLaunchKernelGGL((k_process<-2, false>), g, b, lds, st, ix, qp, qs);
    return;
  }
#define MESSI_PROC_CASE(RR)                                                   \
  if (R == RR) {                                                              \
    if (mask)                                                                 \
      hipLaunchKernelGGL((k_process<RR, true>), g, b, lds, st, ix, qp, qs);   \
    else                                                                      \
      hipLaunchKernelGGL((k_process<RR, false>), g, b, lds, st, ix, qp, qs);  \
    return;                                                                   \
  }
  MESSI_BANDS(MESSI_PROC_CASE)
#undef MESSI_PROC_CASE
}

void launch_finalize(const IndexDev& ix, const QueryParams& qp, const QueryState& qs,
                     int64_t* out_ids, float* out_dists, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(qp.nq), dim3(kProcThreads), finalize_lds_bytes(qp), st, ix,
                     qp, qs, out_ids, out_dists);
}

bool screen_supported(int len) { return len == 64 || len == 128 || len == 256 || len == 512; }

// The (K steps, column tiles, waves) variants of the screen kernel built:
// the B operands take NT x KS x 4 VGPRs, so wider tiles suit shorter
// series (16 x 2 would spill).  Every variant keeps to 256 registers, two
// waves per SIMD, so 4-wave blocks run two to a CU.
#define MESSI_SCREEN_VARIANTS(X)                                                                        \
  X(2, 1, 8) X(2, 2, 8) X(2, 4, 8) X(4, 1, 8) X(4, 2, 8) X(4, 4, 8) X(8, 1, 8) X(8, 2, 8) X(8, 4, 8)   \
  X(16, 1, 8) X(2, 4, 4) X(4, 4, 4) X(8, 2, 4) X(8, 4, 4) X(16, 1, 4)

bool screen_variant(int len, int nt, int waves) {
  const int ks = len / 32;
#define MESSI_SV(K, T, WV) \
  if (ks == K && nt == T && waves == WV && len == 32 * K) return true;
  MESSI_SCREEN_VARIANTS(MESSI_SV)
#undef MESSI_SV
  return false;
}

int screen_blocks_per_cu(int len, int nt, int waves) {
  int per = 0;
  hipError_t e = hipErrorInvalidValue;
  const int ks = len / 32;
#define MESSI_SO(K, T, WV)                                                                 \
  if (ks == K && nt == T && waves == WV) {                                                 \
    constexpr size_t lds = ScreenShape<K, T, WV>::lds;                                     \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_screen<K, T, WV>, WV * kWave, lds); \
  }
  MESSI_SCREEN_VARIANTS(MESSI_SO)
#undef MESSI_SO
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return per < 1 ? 1 : per;
}

int screen_nt_default(int len) { return screen_default_nt(len); }
int screen_waves_default() { return 4; }  // two blocks per CU: one's loads overlap the other's MFMA

void launch_bf16_rows(const float* src, const int32_t* src_row, int64_t rows, int len, uint16_t* dst,
                      float* norms, hipStream_t st) {
  if (rows <= 0) return;
  const int64_t blocks = std::min<int64_t>((rows + 3) / 4, 65536);
  hipLaunchKernelGGL(k_bf16_rows, dim3((unsigned)blocks), dim3(256), 0, st, src, src_row, rows, len,
                     dst, norms);
}

void launch_screen(const IndexDev& ix, const QueryParams& qp, const QueryState& qs,
                   const ScreenDev& sc, int blocks, int nt, int waves, hipStream_t st) {
  const unsigned lb = (unsigned)((qp.n_leaves + 255) / 256);
  hipLaunchKernelGGL(k_log_approx, dim3(qp.nq), dim3(256), 0, st, qp, qs);
  hipLaunchKernelGGL(k_leaf_lists, dim3(lb), dim3(256), 0, st, qp, qs, sc, false);
  hipLaunchKernelGGL(k_list_scan, dim3(1), dim3(1024), 0, st, qp, sc);
  hipLaunchKernelGGL(k_leaf_lists, dim3(lb), dim3(256), 0, st, qp, qs, sc, true);
  const int ks = qp.len / 32;
#define MESSI_SL(K, T, WV)                                                                              \
  if (ks == K && nt == T && waves == WV) {                                                              \
    constexpr size_t lds = ScreenShape<K, T, WV>::lds;                                                  \
    hipLaunchKernelGGL((k_screen<K, T, WV>), dim3(blocks), dim3(WV * kWave), lds, st, ix, qp, qs, sc); \
    return;                                                                                             \
  }
  MESSI_SCREEN_VARIANTS(MESSI_SL)
#undef MESSI_SL
}

// Scratch of the allocation-free query entry point: the query state lives
// in this array instead of memory the library allocates.  Each GPU that
// loads the library holds its own copy until the process ends.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

void* noalloc_scratch(size_t* bytes) {
  // the array's device address on each device, found once with that device
  // current (the name itself is only a host-side stand-in)
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* ptr[kMaxDevices] = {};
  *bytes = kScratchBytes;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    ptr[dev] = p;
  }
  return ptr[dev];
}

size_t process_lds_static(const QueryParams& p) {
  bool mask;
  if (band_of(p, &mask) != -1) return 4096;  // a few shared scalars
  // the kernels' static LDS, asked once per instance (it is fixed at build)
  static std::atomic<long long> cached[2] = {{-1}, {-1}};
  const int which = p.card_bits == 8 ? 1 : 0;
  const long long c = cached[which].load(std::memory_order_relaxed);
  if (c >= 0) return (size_t)c;
  hipFuncAttributes a{};
  const hipError_t e = which ? hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_process_ed<8>))
                             : hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_process_ed<0>));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 48 * 1024;  // above the kernel's own (a refusal rather than a failed launch)
  }
  cached[which].store((long long)a.sharedSizeBytes, std::memory_order_relaxed);
  return a.sharedSizeBytes;
}

int ed_process_blocks(int resident) {
  // the ED kernel deals every shard's chunks to gridDim.x * kEdWaves / kShards waves
  constexpr int unit = kShards / kEdWaves;
  return resident < unit ? unit : resident - resident % unit;
}

int process_blocks_per_cu(const QueryParams& qp) {
  bool mask;
  const int R = band_of(qp, &mask);
  const size_t lds = process_lds_bytes(qp);
  const int th = process_threads(R);
  int nb = 0;
  hipError_t e = hipSuccess;
  if (R == -1) {
    e = qp.card_bits == 8 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_process_ed<8>, th, lds)
                          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_process_ed<0>, th, lds);
  } else if (qp.lb_improved) {
    switch (R) {
      case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_process<8, true, true>, th, lds); break;
      case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_process<16, true, true>, th, lds); break;
      case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_process<32, true, true>, th, lds); break;
      case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_process<64, true, true>, th, lds); break;
      default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_process<-2, false, true>, th, lds); break;
    }
  } else if (R == -2) {
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_process<-2, false>, th, lds);
  }
#define MESSI_OCC_CASE(RR)                                                                  \
  else if (R == RR) {                                                                       \
    if (mask)                                                                               \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_process<RR, true>, th, lds);  \
    else                                                                                    \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_process<RR, false>, th, lds); \
  }
  MESSI_BANDS(MESSI_OCC_CASE)
#undef MESSI_OCC_CASE
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return nb > 0 ? nb : 1;
}

}  // namespace messi
