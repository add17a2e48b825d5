// Exact k-NN query kernels (Algorithms 5-10 of the paper, k-NN per Section
// 5.6), for ED and for DTW with a Sakoe-Chiba band (Section 3.4).
//
// Phases, each one launch over all queries of a call (grid.y = query):
//   prep     z-normalise the query, PAA (and LB_Keogh envelope + its PAA),
//            the per-segment bound table, and the approximate-search leaf:
//            the leaf reached by descending the query's own word.
//   approx   real distances to that leaf's series -> the first k-best list.
//   select   mindist of every leaf against the first k-th best; kept leaves
//            are ordered by bound (counting sort over 1024 bound buckets)
//            by the last block to finish -- the paper's priority queues.
//   process  persistent blocks take leaves in bound order (one atomic
//            counter replaces the queues' DeleteMin); per leaf: series
//            bounds from the table in LDS, [LB_Keogh,] FP32 refinement, the
//            k best kept by a lock-free atomicMin cascade.  A block stops
//            when the next leaf's bound exceeds the current k-th best.  The
//            last block to finish rechecks the near ties in FP64 and writes
//            the answer.
//
// Exactness: every prune compares a bound against the k-th best with slack
// covering the FP32 rounding of both sides; every refined distance within
// the FP32 error window of the running k-th best is logged, and the final
// order is decided on FP64 distances of the logged candidates.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "query.h"

namespace messi {

__device__ __forceinline__ float kth_dist(const unsigned long long* slots, int k) {
  return key_dist(__atomic_load_n(&slots[k - 1], __ATOMIC_RELAXED));
}

// Bound threshold: a series whose bound exceeds it cannot be among the k
// best.  (sqrt(kth (1+rho)) + eta)^2, with a last relative margin for the
// rounding of this expression itself.
__device__ __forceinline__ float lb_threshold(float thr, const QueryParams& p) {
  if (!(thr < INFINITY)) return INFINITY;
  const float r = __fsqrt_rn(thr * p.lb_rel) + p.eta;
  return r * r * 1.0001f;
}

__device__ __forceinline__ int bucket_of(float lb, float thr0) {
  if (!(thr0 < INFINITY) || !(thr0 > 0.0f)) return 0;
  const float f = lb / thr0 * (float)kBuckets;
  int b = (int)f;
  b = b < 0 ? 0 : b;
  return b >= kBuckets ? kBuckets - 1 : b;
}

__device__ __forceinline__ uint32_t byte_of(const uint4& v, int s) {
  const uint32_t x = s < 4 ? v.x : (s < 8 ? v.y : (s < 12 ? v.z : v.w));
  return (x >> (8 * (s & 3))) & 0xffu;
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

// Squared LB_Keogh of a global row against an LDS envelope, one wave.
__device__ __forceinline__ float lbk_wave(const float* __restrict__ U, const float* __restrict__ L,
                                          const float* __restrict__ x, int len, int lane) {
  float acc = 0.0f;
  for (int t = lane; t < len; t += kWave) {
    const float v = x[t];
    const float a = fmaxf(v - U[t], 0.0f);
    const float b = fmaxf(L[t] - v, 0.0f);
    const float d = a + b;  // at most one is non-zero
    acc = __builtin_fmaf(d, d, acc);
  }
  return wave_sum(acc);
}

// Banded DTW, squared costs, FP32, one pair per thread.  Rows run over the
// candidate x (j), the band over the query (i = j - R + b, b in [0, 2R]); in
// band coordinates D(j,i) needs old D[b] (diagonal), old D[b+1] (up) and new
// D[b-1] (left), so one in-place ascending sweep per row suffices.  qpad is
// the query in LDS with R +inf pads on each side (matrix edges cost +inf).
// A path crosses every row, so a row minimum above `cutoff` ends the pair.
template <int R, bool MASK>
__device__ float dtw_band(const float* __restrict__ qpad, const float* __restrict__ x, int len,
                          int r, float cutoff) {
  float D[2 * R + 1];
#pragma unroll
  for (int b = 0; b <= 2 * R; ++b) D[b] = (b == R) ? 0.0f : INFINITY;
  for (int j = 0; j < len; ++j) {
    const float xj = x[j];
    float left = INFINITY;
#pragma unroll
    for (int b = 0; b <= 2 * R; ++b) {
      const float d = xj - qpad[j + b];
      const float up = (b < 2 * R) ? D[b + 1] : INFINITY;
      float c = __builtin_fmaf(d, d, fminf(fminf(D[b], up), left));
      if (MASK && (b - R > r || R - b > r)) c = INFINITY;
      D[b] = c;
      left = c;
    }
    if ((j & 7) == 7) {
      float mn = D[0];
#pragma unroll
      for (int b = 1; b <= 2 * R; ++b) mn = fminf(mn, D[b]);
      if (mn > cutoff) return INFINITY;
    }
  }
  return D[R];
}

// Wave-cooperative DTW over anti-diagonals d = i + j; cells of one diagonal
// are independent, so lanes share them.  buf holds three diagonals (d, d-1,
// d-2) of len values each, indexed by i; every index is rewritten each step
// (+inf outside the band and the matrix).  Each cell is computed from the
// same three neighbours as in row order, so the result is bit-identical to
// the sequential recurrence.  Used in FP64 for the near-tie recheck and in
// FP32 for radii beyond the register band.
template <typename T>
__device__ T dtw_wave(const float* __restrict__ q, const float* __restrict__ x, int len, int r,
                      T* __restrict__ buf, T cutoff, int lane) {
  const T inf = (T)INFINITY;
  for (int i = lane; i < 3 * len; i += kWave) buf[i] = inf;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const int last = 2 * (len - 1);
  T result = inf;
  for (int d = 0; d <= last; ++d) {
    T* cur = buf + (d % 3) * len;
    const T* p1 = buf + ((d + 2) % 3) * len;  // diagonal d-1
    const T* p2 = buf + ((d + 1) % 3) * len;  // diagonal d-2
    T local_min = inf;
    for (int i = lane; i < len; i += kWave) {
      const int j = d - i;
      T v = inf;
      if (j >= 0 && j < len && (i - j <= r) && (j - i <= r)) {
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
      T mn = local_min;
      for (int i = lane; i < len; i += kWave) mn = p1[i] < mn ? p1[i] : mn;
      for (int o = 32; o >= 1; o >>= 1) {
        const T u = __shfl_xor(mn, o, kWave);
        mn = u < mn ? u : mn;
      }
      if (mn > cutoff) return inf;
    }
  }
  // the final cell was written by the lane owning index len-1
  const int owner = (len - 1) % kWave;
  return __shfl(result, owner, kWave);
}

// ---------------------------------------------------------------------------
// prep: one block per query.

__global__ __launch_bounds__(256) void k_prep(IndexDev ix, const float* __restrict__ queries,
                                              QueryParams p, QueryState s) {
  const int q = blockIdx.x;
  const int tid = threadIdx.x;
  const int len = p.len, w = p.w, m = p.m, cb = p.card_bits, card = 1 << cb;
  extern __shared__ float sm[];
  float* x = sm;
  float* z = x + len;
  float* U = z + len;
  float* L = U + len;
  float* bp = L + len;
  __shared__ float paa[3][kMaxSeg];
  __shared__ float s_mu, s_sd;
  __shared__ unsigned long long s_best;

  const float* src = queries + (int64_t)q * len;
  for (int t = tid; t < len; t += blockDim.x) x[t] = src[t];
  for (int j = tid; j <= card; j += blockDim.x) bp[j] = ix.bp[j];
  __syncthreads();
  if (tid == 0) {  // same order and rounding as the build's summary pass
    float sum = 0.0f;
    for (int t = 0; t < len; ++t) sum = sum + x[t];
    const float mu = __fdiv_rn(sum, (float)len);
    float v = 0.0f;
    for (int t = 0; t < len; ++t) {
      const float d = x[t] - mu;
      v = v + d * d;
    }
    s_mu = mu;
    s_sd = __fsqrt_rn(__fdiv_rn(v, (float)len));
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
  // bound table: T[s][sym] = m * gap(PAA, box of sym)^2 (mindist, Section
  // 2.2 / Property 1; DTW: the envelope PAA against the box, Section 3.4)
  const float fm = (float)m;
  float* table = s.table + (int64_t)q * w * card;
  for (int idx = tid; idx < w * card; idx += blockDim.x) {
    const int sg = idx / card, j = idx - sg * card;
    const float lo = bp[j], hi = bp[j + 1];
    const float g = fmaxf(lo - paa[1][sg], 0.0f) + fmaxf(paa[2][sg] - hi, 0.0f);
    table[idx] = fm * (g * g);
  }
  // approximate search leaf: descend the tree along the query's word
  uint8_t word[kMaxSeg];
  uint32_t key = 0;
  for (int sg = 0; sg < w; ++sg) {
    word[sg] = (uint8_t)symbol_of(paa[0][sg], bp, card);
    key = (key << 1) | (word[sg] >> (cb - 1));
  }
  int node = ix.root_node[key];
  if (node < 0) {  // no series under that root: the root with the smallest bound
    if (tid == 0) s_best = ~0ull;
    __syncthreads();
    unsigned long long best = ~0ull;
    const int nkeys = 1 << w;
    for (int kk = tid; kk < nkeys; kk += blockDim.x) {
      if (ix.root_node[kk] < 0) continue;
      float lb = 0.0f;
      for (int sg = 0; sg < w; ++sg) {
        const int b = (kk >> (w - 1 - sg)) & 1;
        const float lo = bp[b << (cb - 1)], hi = bp[(b + 1) << (cb - 1)];
        const float g = fmaxf(lo - paa[1][sg], 0.0f) + fmaxf(paa[2][sg] - hi, 0.0f);
        lb += g * g;
      }
      const unsigned long long c = ((unsigned long long)__float_as_uint(lb) << 32) | (unsigned)kk;
      best = c < best ? c : best;
    }
    best = wave_min_u64(best);
    if ((tid & (kWave - 1)) == 0) atomicMin(&s_best, best);
    __syncthreads();
    node = ix.root_node[(int)(s_best & 0xffffffffu)];
  }
  if (tid == 0) {
    for (int guard = 0; guard < 4096 && ix.nodes[node].seg >= 0; ++guard) {
      const NodeDev& nd = ix.nodes[node];
      const int sg = nd.seg;
      const int bit = (word[sg] >> (cb - 1 - nd.bits[sg])) & 1;
      int ch = nd.child[bit];
      if (ch < 0) ch = nd.child[bit ^ 1];
      node = ch;
    }
    int64_t b = ix.nodes[node].begin, e = ix.nodes[node].end;
    if (e - b > kApproxCap) e = b + kApproxCap;
    if (e - b < p.k) {
      e = b + p.k < ix.n ? b + p.k : ix.n;
      if (e - b < p.k) b = e - p.k > 0 ? e - p.k : 0;
    }
    s.approx_range[2 * q] = b;
    s.approx_range[2 * q + 1] = e;
    s.log_count[q] = 0;
    s.cand_count[q] = 0;
    s.next[q] = 0;
    s.done[q] = 0;
    s.sel_done[q] = 0;
    s.status[q] = 0;
  }
  for (int j = tid; j < p.k; j += blockDim.x) s.slots[(int64_t)q * p.k + j] = kEmptyKey;
  for (int j = tid; j < kStatCount; j += blockDim.x) s.stats[(int64_t)q * kStatCount + j] = 0;
}

// ---------------------------------------------------------------------------
// Shared per-candidate step: offer a refined distance to the k best and log
// it if it lies within the near-tie window of the k-th best.

__device__ __forceinline__ void offer(const QueryParams& p, const QueryState& s, int q, float d2,
                                      int64_t pos, uint32_t id, bool log_it) {
  unsigned long long* slots = s.slots + (int64_t)q * p.k;
  const float thr = kth_dist(slots, p.k);
  const unsigned long long key = pack_key(d2, id);
  if (key < __atomic_load_n(&slots[p.k - 1], __ATOMIC_RELAXED)) topk_insert(slots, p.k, key);
  if (log_it && d2 <= thr * p.win) {
    const int i = atomicAdd(&s.log_count[q], 1);
    if (i < p.log_cap) s.log[(int64_t)q * p.log_cap + i] = pack_key(d2, (uint32_t)pos);
  }
}

template <int R, bool MASK>
__device__ float dtw_fp32(const float* __restrict__ qpad, const float* __restrict__ x, int len,
                          int r, float cutoff) {
  return dtw_band<R, MASK>(qpad, x, len, r, cutoff);
}

// ---------------------------------------------------------------------------
// approx: refine the approximate-search range.  ED: one wave per series;
// DTW: one thread per series.  Distances go to approx_d2 (logged later by
// select, once the first k-th best is known).

template <int R, bool MASK>
__global__ __launch_bounds__(256) void k_approx(IndexDev ix, QueryParams p, QueryState s) {
  const int q = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int len = p.len;
  extern __shared__ float sm[];
  const int64_t P0 = s.approx_range[2 * q], P1 = s.approx_range[2 * q + 1];
  const int cnt = (int)(P1 - P0);
  const float* zq = s.zq + (int64_t)q * len;
  float* approx_d2 = s.approx_d2 + (int64_t)q * kApproxCap;
  if constexpr (R < 0) {  // ED
    float* zl = sm;
    for (int t = tid; t < len; t += blockDim.x) zl[t] = zq[t];
    __syncthreads();
    const int gw = blockIdx.x * (blockDim.x / kWave) + tid / kWave;
    const int nw = gridDim.x * (blockDim.x / kWave);
    for (int j = gw; j < cnt; j += nw) {
      const int64_t pos = P0 + j;
      const float d2 = ed_wave(zl, ix.Z + pos * len, len, lane);
      if (lane == 0) {
        approx_d2[j] = d2;
        offer(p, s, q, d2, pos, (uint32_t)ix.perm[pos], false);
      }
    }
  } else {  // DTW, band of radius R
    float* qpad = sm;
    for (int t = tid; t < len + 2 * R; t += blockDim.x)
      qpad[t] = (t >= R && t < R + len) ? zq[t - R] : INFINITY;
    __syncthreads();
    for (int j = blockIdx.x * blockDim.x + tid; j < cnt; j += gridDim.x * blockDim.x) {
      const int64_t pos = P0 + j;
      const float d2 = dtw_fp32<R, MASK>(qpad, ix.Z + pos * len, len, p.window, INFINITY);
      approx_d2[j] = d2;
      offer(p, s, q, d2, pos, (uint32_t)ix.perm[pos], false);
    }
  }
}

// Radii beyond the register band: one wave per series, anti-diagonals.
__global__ __launch_bounds__(256) void k_approx_wave(IndexDev ix, QueryParams p, QueryState s) {
  const int q = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const int len = p.len;
  extern __shared__ float sm[];
  float* ql = sm;
  float* xl = ql + len;              // [4][len]
  float* buf = xl + 4 * len;         // [4][3 len]
  const int64_t P0 = s.approx_range[2 * q], P1 = s.approx_range[2 * q + 1];
  const int cnt = (int)(P1 - P0);
  const float* zq = s.zq + (int64_t)q * len;
  for (int t = tid; t < len; t += blockDim.x) ql[t] = zq[t];
  __syncthreads();
  const int gw = blockIdx.x * 4 + wv, nw = gridDim.x * 4;
  for (int j = gw; j < cnt; j += nw) {
    const int64_t pos = P0 + j;
    for (int t = lane; t < len; t += kWave) xl[wv * len + t] = ix.Z[pos * len + t];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const float d2 = dtw_wave<float>(ql, xl + wv * len, len, p.window, buf + wv * 3 * len,
                                     (float)INFINITY, lane);
    if (lane == 0) {
      s.approx_d2[(int64_t)q * kApproxCap + j] = d2;
      offer(p, s, q, d2, pos, (uint32_t)ix.perm[pos], false);
    }
  }
}

// ---------------------------------------------------------------------------
// select: leaf bounds, kept leaves, and (last block) approx-range logging and
// the bucket order of the kept leaves.

__global__ __launch_bounds__(kSelectThreads) void k_select(IndexDev ix, QueryParams p, QueryState s,
                                                           unsigned long long* __restrict__ cand_sorted) {
  const int q = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int w = p.w, cb = p.card_bits, card = 1 << cb;
  __shared__ float bp[257];
  __shared__ float pa[2][kMaxSeg];
  __shared__ int hist[kBuckets];
  __shared__ int s_last;
  for (int j = tid; j <= card; j += blockDim.x) bp[j] = ix.bp[j];
  if (tid < kMaxSeg) {
    pa[0][tid] = s.paa[((int64_t)q * 3 + 1) * kMaxSeg + tid];
    pa[1][tid] = s.paa[((int64_t)q * 3 + 2) * kMaxSeg + tid];
  }
  __syncthreads();
  unsigned long long* slots = s.slots + (int64_t)q * p.k;
  const float thr = kth_dist(slots, p.k);
  const float thr_adj = lb_threshold(thr, p);
  const int64_t P0 = s.approx_range[2 * q], P1 = s.approx_range[2 * q + 1];
  const int L = p.n_leaves;
  unsigned long long* cand = s.cand + (int64_t)q * L;
  const float fm = (float)p.m;
  for (int l0 = blockIdx.x * blockDim.x; l0 < L; l0 += gridDim.x * blockDim.x) {
    const int l = l0 + tid;
    bool keep = false;
    float lb = 0.0f;
    if (l < L) {
      const uint4 sy = ix.leaf_sym[l], bi = ix.leaf_bits[l];
      for (int sg = 0; sg < w; ++sg) {
        const int b = (int)byte_of(bi, sg), y = (int)byte_of(sy, sg);
        const int sh = cb - b;
        const float lo = bp[y << sh], hi = bp[(y + 1) << sh];
        const float g = fmaxf(lo - pa[0][sg], 0.0f) + fmaxf(pa[1][sg] - hi, 0.0f);
        lb += g * g;
      }
      lb *= fm;
      const bool inside = ix.leaf_begin[l] >= P0 && ix.leaf_end[l] <= P1;
      keep = lb <= thr_adj && !inside;
    }
    const unsigned long long mask = __ballot(keep);
    if (mask) {
      int base = 0;
      const int leader = __ffsll((long long)mask) - 1;
      if (lane == leader) base = atomicAdd(&s.cand_count[q], __popcll(mask));
      base = __shfl(base, leader, kWave);
      if (keep) {
        const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
        cand[base + __popcll(mask & below)] = ((unsigned long long)__float_as_uint(lb) << 32) | (unsigned)l;
      }
    }
  }
  // the last block of this query finishes the phase
  __threadfence();
  __syncthreads();
  if (tid == 0) s_last = atomicAdd(&s.sel_done[q], 1) == (int)gridDim.x - 1;
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  // approx-range distances inside the near-tie window of the first k-th best
  const float win = thr * p.win;
  const float* ad = s.approx_d2 + (int64_t)q * kApproxCap;
  for (int j = tid; j < (int)(P1 - P0); j += blockDim.x) {
    const float d2 = ad[j];
    if (d2 <= win) {
      const int i = atomicAdd(&s.log_count[q], 1);
      if (i < p.log_cap) s.log[(int64_t)q * p.log_cap + i] = pack_key(d2, (uint32_t)(P0 + j));
    }
  }
  // bucket order of the kept leaves
  const int cnt = __atomic_load_n(&s.cand_count[q], __ATOMIC_RELAXED);
  if (tid == 0) {
    s.cand_thr[q] = thr_adj;
    s.stats[(int64_t)q * kStatCount + kStatLeavesKept] = (unsigned long long)cnt;
  }
  for (int b = tid; b < kBuckets; b += blockDim.x) hist[b] = 0;
  __syncthreads();
  for (int i = tid; i < cnt; i += blockDim.x) atomicAdd(&hist[bucket_of(key_dist(cand[i]), thr_adj)], 1);
  __syncthreads();
  // exclusive scan over the buckets (kBuckets == blockDim)
  const int mine = hist[tid];
  for (int o = 1; o < kBuckets; o <<= 1) {
    const int v = tid >= o ? hist[tid - o] : 0;
    __syncthreads();
    hist[tid] += v;
    __syncthreads();
  }
  hist[tid] -= mine;
  __syncthreads();
  unsigned long long* out = cand_sorted + (int64_t)q * L;
  for (int i = tid; i < cnt; i += blockDim.x) {
    const unsigned long long c = cand[i];
    const int at = atomicAdd(&hist[bucket_of(key_dist(c), thr_adj)], 1);
    out[at] = c;
  }
}

// ---------------------------------------------------------------------------
// Finalisation (last block of the process phase for a query): FP64 recheck
// of the near ties, exact (distance, id) order, outputs.  The log is taken
// in chunks; each chunk's candidates in the window are recomputed in FP64
// and merged with the running k best by rank, so any number of ties fits.

__device__ void finalize(const IndexDev& ix, const QueryParams& p, const QueryState& s, int q,
                         float* sm, int64_t* out_ids, float* out_dists) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const int len = p.len, k = p.k;
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
  const unsigned long long* slots = s.slots + (int64_t)q * k;
  const float T = kth_dist(slots, k);
  const float win = T * p.win;
  const int lc = __atomic_load_n(&s.log_count[q], __ATOMIC_RELAXED);
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
      for (int c = topn + tid; c < cnt; c += blockDim.x) {
        const float* x = ix.Z + (int64_t)pos_l[c] * len;
        double acc = 0.0;
        for (int t = 0; t < len; ++t) {
          const double d = (double)ql[t] - (double)x[t];
          acc = __dadd_rn(acc, __dmul_rn(d, d));
        }
        E[c] = acc;
        id_l[c] = ix.perm[pos_l[c]];
      }
    } else {
      for (int c0 = topn; c0 < cnt; c0 += p.fin_waves) {
        const int c = c0 + wv;
        if (wv < p.fin_waves && c < cnt) {
          const float* x = ix.Z + (int64_t)pos_l[c] * len;
          for (int t = lane; t < len; t += kWave) xl[wv * len + t] = x[t];
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
          const double v = dtw_wave<double>(ql, xl + wv * len, len, p.window, dbuf + wv * 3 * len,
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
  for (int j = tid; j < k; j += blockDim.x) {
    if (j < topn) {
      out_ids[(int64_t)q * k + j] = (int64_t)id_l[j];
      out_dists[(int64_t)q * k + j] = (float)sqrt(E[j]);
    } else {
      out_ids[(int64_t)q * k + j] = -1;
      out_dists[(int64_t)q * k + j] = INFINITY;
    }
  }
  if (tid == 0) s.stats[(int64_t)q * kStatCount + kStatRecheck] = rechecked;
}

// ---------------------------------------------------------------------------
// process: persistent blocks over the ordered candidate leaves.
// R = -1: ED; R >= 0: DTW with a register band of radius R; R = -2: DTW by
// wave anti-diagonals (radius beyond the register band).

template <int R, bool MASK>
__global__ __launch_bounds__(kProcThreads) void k_process(IndexDev ix, QueryParams p, QueryState s,
                                                          const unsigned long long* __restrict__ cand_sorted,
                                                          int64_t* __restrict__ out_ids,
                                                          float* __restrict__ out_dists) {
  const int q = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const int len = p.len, w = p.w, card = 1 << p.card_bits, k = p.k;
  const bool dtw = R != -1;
  extern __shared__ float sm[];
  float* table = sm;                          // [w][card]
  float* ql = table + w * card;               // query (ED) / padded query (band DTW)
  const int qlen = (R >= 0) ? len + 2 * R : len;
  float* U = ql + qlen;                       // envelope (DTW)
  float* Lw = U + (dtw ? len : 0);
  int* list = reinterpret_cast<int*>(Lw + (dtw ? len : 0));   // [kTile] series survivors
  int* list2 = list + kTile;                                  // [kTile] LB_Keogh survivors
  float* wx = reinterpret_cast<float*>(list2 + kTile);        // wave DTW: [4][len] rows
  float* wbuf = wx + 4 * len;                                 // wave DTW: [4][3 len]
  __shared__ int s_item_leaf;
  __shared__ int s_stop;
  __shared__ int n1, n2;
  __shared__ unsigned long long st_lb, st_lbk, st_ref;
  __shared__ int s_last;

  const float* tq = s.table + (int64_t)q * w * card;
  for (int i = tid; i < w * card; i += blockDim.x) table[i] = tq[i];
  const float* zq = s.zq + (int64_t)q * len;
  if (R >= 0) {
    for (int t = tid; t < qlen; t += blockDim.x) ql[t] = (t >= R && t < R + len) ? zq[t - R] : INFINITY;
  } else {
    for (int t = tid; t < len; t += blockDim.x) ql[t] = zq[t];
  }
  if (dtw) {
    for (int t = tid; t < len; t += blockDim.x) {
      U[t] = s.upper[(int64_t)q * len + t];
      Lw[t] = s.lower[(int64_t)q * len + t];
    }
  }
  if (tid == 0) {
    st_lb = 0;
    st_lbk = 0;
    st_ref = 0;
  }
  __syncthreads();

  unsigned long long* slots = s.slots + (int64_t)q * k;
  const int cnt = __atomic_load_n(&s.cand_count[q], __ATOMIC_RELAXED);
  const float thr0 = s.cand_thr[q];
  const float bw = thr0 / (float)kBuckets;
  const int64_t P0 = s.approx_range[2 * q], P1 = s.approx_range[2 * q + 1];
  const unsigned long long* items = cand_sorted + (int64_t)q * p.n_leaves;
  unsigned long long c_lb = 0, c_lbk = 0, c_ref = 0;

  for (;;) {
    if (tid == 0) {
      s_stop = 0;
      const int i = atomicAdd(&s.next[q], 1);
      if (i >= cnt) {
        s_stop = 1;
      } else {
        const unsigned long long it = items[i];
        const float lb = key_dist(it);
        const float tadj = lb_threshold(kth_dist(slots, k), p);
        if (lb > tadj) {
          // every later leaf is in a bucket at least this one's floor
          const float floor_b = (float)bucket_of(lb, thr0) * bw;
          s_stop = floor_b > tadj ? 1 : 2;
        }
        s_item_leaf = (int)(it & 0xffffffffu);
      }
    }
    __syncthreads();
    const int stop = s_stop;
    if (stop == 1) break;
    if (stop == 2) {
      __syncthreads();
      continue;
    }
    const int leaf = s_item_leaf;
    const int64_t lb_ = ix.leaf_begin[leaf], le_ = ix.leaf_end[leaf];
    for (int64_t t0 = lb_; t0 < le_; t0 += kTile) {
      const int64_t t1 = t0 + kTile < le_ ? t0 + kTile : le_;
      if (tid == 0) {
        n1 = 0;
        n2 = 0;
      }
      __syncthreads();
      const float tadj = lb_threshold(kth_dist(slots, k), p);
      // series-level bounds (Algorithm 9 / Algorithm 10, first test)
      for (int64_t pos = t0 + tid; pos < t1; pos += blockDim.x) {
        if (pos >= P0 && pos < P1) continue;  // refined by the approximate search
        const uint4 wd = ix.words[pos];
        float lb = 0.0f;
        for (int sg = 0; sg < w; ++sg) lb += table[sg * card + (int)byte_of(wd, sg)];
        ++c_lb;
        if (lb <= tadj) list[atomicAdd(&n1, 1)] = (int)(pos - t0);
      }
      __syncthreads();
      const int m1 = n1;
      if (!dtw) {
        for (int c = wv; c < m1; c += blockDim.x / kWave) {
          const int64_t pos = t0 + list[c];
          const float d2 = ed_wave(ql, ix.Z + pos * len, len, lane);
          if (lane == 0) {
            ++c_ref;
            offer(p, s, q, d2, pos, (uint32_t)ix.perm[pos], true);
          }
        }
      } else {
        // LB_Keogh on the raw values (Algorithm 10, second test)
        const float tk = kth_dist(slots, k) * p.win * p.win;
        for (int c = wv; c < m1; c += blockDim.x / kWave) {
          const int64_t pos = t0 + list[c];
          const float lbk = lbk_wave(U, Lw, ix.Z + pos * len, len, lane);
          if (lane == 0) {
            ++c_lbk;
            if (lbk <= tk) list2[atomicAdd(&n2, 1)] = list[c];
          }
        }
        __syncthreads();
        const int m2 = n2;
        const float cut = kth_dist(slots, k) * p.win * p.win;
        if constexpr (R >= 0) {
          for (int c = tid; c < m2; c += blockDim.x) {
            const int64_t pos = t0 + list2[c];
            const float d2 = dtw_band<R, MASK>(ql, ix.Z + pos * len, len, p.window, cut);
            ++c_ref;
            if (d2 < INFINITY) offer(p, s, q, d2, pos, (uint32_t)ix.perm[pos], true);
          }
        } else {
          for (int c = wv; c < m2; c += blockDim.x / kWave) {
            const int64_t pos = t0 + list2[c];
            const float* x = ix.Z + pos * len;
            for (int t = lane; t < len; t += kWave) wx[wv * len + t] = x[t];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const float d2 = dtw_wave<float>(ql, wx + wv * len, len, p.window, wbuf + wv * 3 * len,
                                             cut, lane);
            if (lane == 0) {
              ++c_ref;
              if (d2 < INFINITY) offer(p, s, q, d2, pos, (uint32_t)ix.perm[pos], true);
            }
          }
        }
      }
      __syncthreads();
    }
  }
  atomicAdd(&st_lb, c_lb);
  atomicAdd(&st_lbk, c_lbk);
  atomicAdd(&st_ref, c_ref);
  __syncthreads();
  if (tid == 0) {
    unsigned long long* stq = s.stats + (int64_t)q * kStatCount;
    atomicAdd(&stq[kStatSeriesLb], st_lb);
    atomicAdd(&stq[kStatLbKeogh], st_lbk);
    atomicAdd(&stq[kStatRefined], st_ref);
  }
  // the last block of this query finalises it
  __threadfence();
  __syncthreads();
  if (tid == 0) s_last = atomicAdd(&s.done[q], 1) == (int)gridDim.x - 1;
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  finalize(ix, p, s, q, sm, out_ids, out_dists);
}

// ---------------------------------------------------------------------------
// Launchers.  The DTW radius picks a register-band instance: exact radii of
// the common windows, else the next larger band with a mask, else the wave
// anti-diagonal kernel.

#define MESSI_BANDS(X) X(0) X(1) X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(25) X(32) X(51) X(64)

static int pick_band(int r, bool* mask) {
  static const int exact[] = {0, 1, 2, 3, 4, 6, 8, 12, 16, 25, 32, 51, 64};
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

static size_t process_lds_bytes(const QueryParams& p, int R) {
  const int card = 1 << p.card_bits;
  const bool dtw = p.distance == 1;
  const int qlen = R >= 0 ? p.len + 2 * R : p.len;
  size_t words = (size_t)p.w * card + qlen + (dtw ? 2 * p.len : 0) + 2 * kTile;
  if (R == -2) words += 4 * (size_t)p.len + 4 * 3 * (size_t)p.len;
  // the finalisation reuses the same space (layout in finalize())
  const size_t fin = ((((size_t)4 * kTopCap + p.len + (size_t)p.fin_waves * p.len) + 1) & ~(size_t)1) +
                     (size_t)p.fin_waves * 3 * p.len * 2;
  return (words > fin ? words : fin) * sizeof(float);
}

void launch_prep(const IndexDev& ix, const float* queries, const QueryParams& qp,
                 const QueryState& qs, hipStream_t st) {
  const size_t lds = (4 * (size_t)qp.len + 257) * sizeof(float);
  hipLaunchKernelGGL(k_prep, dim3(qp.nq), dim3(256), lds, st, ix, queries, qp, qs);
}

void launch_approx(const IndexDev& ix, const QueryParams& qp, const QueryState& qs,
                   hipStream_t st) {
  if (qp.distance == 0) {
    hipLaunchKernelGGL((k_approx<-1, false>), dim3(64, qp.nq), dim3(256), qp.len * sizeof(float),
                       st, ix, qp, qs);
    return;
  }
  bool mask = false;
  const int R = pick_band(qp.window, &mask);
  if (R == -2) {
    const size_t lds = (size_t)(qp.len + 4 * qp.len + 12 * qp.len) * sizeof(float);
    hipLaunchKernelGGL(k_approx_wave, dim3(64, qp.nq), dim3(256), lds, st, ix, qp, qs);
    return;
  }
  const size_t lds = (size_t)(qp.len + 2 * R) * sizeof(float);
  const dim3 g((kApproxCap + 255) / 256, qp.nq);
#define MESSI_APPROX_CASE(RR)                                                                 \
  if (R == RR) {                                                                              \
    if (mask)                                                                                 \
      hipLaunchKernelGGL((k_approx<RR, true>), g, dim3(256), lds, st, ix, qp, qs);            \
    else                                                                                      \
      hipLaunchKernelGGL((k_approx<RR, false>), g, dim3(256), lds, st, ix, qp, qs);           \
    return;                                                                                   \
  }
  MESSI_BANDS(MESSI_APPROX_CASE)
#undef MESSI_APPROX_CASE
}

void launch_select(const IndexDev& ix, const QueryParams& qp, const QueryState& qs,
                   unsigned long long* cand_sorted, hipStream_t st) {
  int blocks = (qp.n_leaves + kSelectThreads - 1) / kSelectThreads;
  if (blocks > 256) blocks = 256;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_select, dim3(blocks, qp.nq), dim3(kSelectThreads), 0, st, ix, qp, qs,
                     cand_sorted);
}

void launch_process(const IndexDev& ix, const QueryParams& qp, const QueryState& qs,
                    const unsigned long long* cand_sorted, int blocks_per_query,
                    int64_t* out_ids, float* out_dists, hipStream_t st) {
  const dim3 g(blocks_per_query, qp.nq);
  if (qp.distance == 0) {
    hipLaunchKernelGGL((k_process<-1, false>), g, dim3(kProcThreads), process_lds_bytes(qp, -1), st,
                       ix, qp, qs, cand_sorted, out_ids, out_dists);
    return;
  }
  bool mask = false;
  const int R = pick_band(qp.window, &mask);
  if (R == -2) {
    hipLaunchKernelGGL((k_process<-2, false>), g, dim3(kProcThreads), process_lds_bytes(qp, -2), st,
                       ix, qp, qs, cand_sorted, out_ids, out_dists);
    return;
  }
  const size_t lds = process_lds_bytes(qp, R);
#define MESSI_PROC_CASE(RR)                                                                      \
  if (R == RR) {                                                                                 \
    if (mask)                                                                                    \
      hipLaunchKernelGGL((k_process<RR, true>), g, dim3(kProcThreads), lds, st, ix, qp, qs,      \
                         cand_sorted, out_ids, out_dists);                                       \
    else                                                                                         \
      hipLaunchKernelGGL((k_process<RR, false>), g, dim3(kProcThreads), lds, st, ix, qp, qs,     \
                         cand_sorted, out_ids, out_dists);                                       \
    return;                                                                                      \
  }
  MESSI_BANDS(MESSI_PROC_CASE)
#undef MESSI_PROC_CASE
}

size_t query_process_lds(const QueryParams& qp) {
  if (qp.distance == 0) return process_lds_bytes(qp, -1);
  bool mask = false;
  return process_lds_bytes(qp, pick_band(qp.window, &mask));
}

size_t query_process_lds_for(const QueryParams& qp, int fin_waves) {
  QueryParams p = qp;
  p.fin_waves = fin_waves;
  return query_process_lds(p);
}

}  // namespace messi
