// Index build kernels (Section 3.2 of the paper: iSAX summaries of every
// series, then the leaves of the root subtrees).
//
// GPU layout instead of the paper's per-thread iSAX buffers and pointer
// tree: (1) one pass summarises every series into a packed 16-byte word and
// counts its root key; (2) a counting scatter groups entries by root key;
// (3) rounds of segmented two-way partitions split every over-full node on
// its most balanced segment; (4) each leaf's ids are sorted so leaves are
// contiguous, ascending-id ranges; (5) the z-normalised store and the words
// are gathered into that leaf order.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <stdint.h>

#include "build.h"
#include "common.h"

namespace messi {

// ---------------------------------------------------------------------------
// (1) Summaries.  One lane per series: z-normalisation, PAA and symbols are
// sequential FP32 sums in index order (the fixed order the words are defined
// by), so the series sits in LDS, staged with one coalesced read of the
// block's contiguous rows.  Element t of row l is stored at column
// (t + l) mod len, so at any t the 64 lanes hit 64 distinct banks.

__global__ __launch_bounds__(kWave) void k_summarize(const float* __restrict__ raw, int64_t n, int len,
                                                      int w, int card_bits, int spw,
                                                      const float* __restrict__ bp_g,
                                                      uint4* __restrict__ words,
                                                      float2* __restrict__ musd,
                                                      uint16_t* __restrict__ keys,
                                                      unsigned int* __restrict__ norm2_max) {
  extern __shared__ float smem[];
  float* bp = smem;               // card + 1 entries (bp[0] = -inf, bp[card] = +inf)
  float* tile = smem + 257;       // spw rows of len floats, rotated
  const int card = 1 << card_bits;
  const int lane = threadIdx.x;
  for (int j = lane; j <= card; j += kWave) bp[j] = bp_g[j];

  const int64_t first = (int64_t)blockIdx.x * spw;
  const int rows = (int)((n - first) < spw ? (n - first) : spw);
  const float* src = raw + first * (int64_t)len;
  for (int r = 0; r < rows; ++r) {  // coalesced row reads, rotated LDS rows
    const float* srow = src + (int64_t)r * len;
    float* trow = tile + r * len;
    const int rr = r < len ? r : r % len;
    for (int t = lane; t < len; t += kWave) {
      int c = t + rr;
      c = c >= len ? c - len : c;
      trow[c] = srow[t];
    }
  }
  __syncthreads();
  if (lane >= rows) return;

  const float* row = tile + lane * len;
  const int rot = lane < len ? lane : lane % len;
  auto at = [&](int t) {
    int c = t + rot;
    c = c >= len ? c - len : c;
    return row[c];
  };
  // as given (norm2_max set): mu = 0 and sd = 1, so z = x exactly, and v is
  // the squared norm of the row
  const bool as_given = norm2_max != nullptr;
  const float flen = (float)len;
  float mu = 0.0f;
  if (!as_given) {
    float s = 0.0f;
    for (int t = 0; t < len; ++t) s = s + at(t);
    mu = __fdiv_rn(s, flen);
  }
  float v = 0.0f;
  for (int t = 0; t < len; ++t) {
    const float d = at(t) - mu;
    v = v + d * d;
  }
  const float sd = as_given ? 1.0f : sqrtf(__fdiv_rn(v, flen));
  if (as_given) atomicMax(norm2_max, __float_as_uint(v));
  const bool flat = !(sd > 0.0f);
  const int m = len / w;
  const float fm = (float)m;
  float pv[kMaxSeg];
#pragma unroll
  for (int sg = 0; sg < kMaxSeg; ++sg) {
    float a = 0.0f;
    if (sg < w && !flat) {
      for (int t = sg * m; t < sg * m + m; ++t) a = a + __fdiv_rn(at(t) - mu, sd);
    }
    pv[sg] = __fdiv_rn(a, fm);
  }
  // symbols: the w binary searches advance together, one level per step
  int lo[kMaxSeg], hi[kMaxSeg];
#pragma unroll
  for (int sg = 0; sg < kMaxSeg; ++sg) {
    lo[sg] = 0;
    hi[sg] = card - 1;
  }
  for (int step = 0; step < card_bits; ++step) {
#pragma unroll
    for (int sg = 0; sg < kMaxSeg; ++sg) {
      const int mid = (lo[sg] + hi[sg] + 1) >> 1;
      if (bp[mid] <= pv[sg])
        lo[sg] = mid;
      else
        hi[sg] = mid - 1;
    }
  }
  uint32_t packed[4] = {0u, 0u, 0u, 0u};
  uint32_t key = 0;
#pragma unroll
  for (int sg = 0; sg < kMaxSeg; ++sg) {
    if (sg < w) {
      const uint32_t sym = (uint32_t)lo[sg];
      packed[sg >> 2] |= sym << (8 * (sg & 3));
      key = (key << 1) | (sym >> (card_bits - 1));
    }
  }
  const int64_t id = first + lane;
  words[id] = make_uint4(packed[0], packed[1], packed[2], packed[3]);
  musd[id] = make_float2(mu, flat ? 0.0f : sd);
  keys[id] = (uint16_t)key;
}

// Summaries for 16 segments and len a multiple of 64 up to 256 (the usual
// shapes): 4 lanes per series, lane j of a quad holding points
// j len/4 .. (j+1) len/4 - 1 (segments 4j .. 4j+3) in registers, sixteen
// series per wave, no LDS staging.  The two sequential sums of the
// z-normalisation keep their index order by passing the running sum from
// lane j to lane j+1 of the quad (a DPP quad permutation) after lane j has
// added its points: each sum takes len wave-instructions for sixteen
// series.  The point-wise work (squares, z, segment sums) runs on all lanes.

template <int Q>
__device__ __forceinline__ float chain_sum4(const float (&v)[Q], int j) {
  float acc = 0.0f;
#pragma unroll
  for (int stage = 0; stage < 4; ++stage) {
    if (j == stage) {
#pragma unroll
      for (int i = 0; i < Q; ++i) acc = acc + v[i];
    }
    if (stage < 3)  // quad_perm [0, 0, 1, 2]: lane j receives lane j-1's sum
      acc = __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(acc), __float_as_int(acc), 0x90,
                                                       0xf, 0xf, false));
  }
  // quad_perm [3, 3, 3, 3]: every lane of the quad takes the total
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(acc), __float_as_int(acc), 0xff, 0xf,
                                                    0xf, false));
}

// Correctly rounded num / den for many numerators over one divisor.  The
// hardware's IEEE division runs in three parts: a scaling step that moves
// operands near the exponent limits, a reciprocal of den refined by one
// Newton step followed by two FMA residual corrections of the quotient, and
// a fix-up step for zeros, infinities and NaNs.  Away from the limits the
// scaling and the fix-up leave the corrected quotient unchanged, and the
// reciprocal part depends on den alone, so it is computed once per series
// (refined_rcp) and each numerator costs a multiply and four FMAs (div_by).
// quick_divisor states when that holds for every numerator x - mu of a
// series: with |mu| >= 2^-60 a nonzero x - mu is at least 2^-84 in
// magnitude (within a factor of two of mu it is a multiple of the smaller
// ulp, else at least |mu| / 2), and |x - mu| <= sd sqrt(len) <= 64 sd, so
// for 2^-40 <= sd <= 2^40 every quotient is normal and no operand is near
// a limit.  A zero numerator gives a zero of either sign, which leaves the
// segment sums (started at +0) unchanged.
__device__ __forceinline__ bool quick_divisor(float mu, float sd) {
  return sd >= 0x1p-40f && sd <= 0x1p40f && fabsf(mu) >= 0x1p-60f;
}

__device__ __forceinline__ float refined_rcp(float den) {
  const float r0 = __builtin_amdgcn_rcpf(den);
  const float e0 = __builtin_fmaf(-den, r0, 1.0f);
  return __builtin_fmaf(e0, r0, r0);
}

__device__ __forceinline__ float div_by(float num, float den, float r) {
  const float m = num * r;
  const float e1 = __builtin_fmaf(-den, m, num);
  const float q1 = __builtin_fmaf(e1, r, m);
  const float e2 = __builtin_fmaf(-den, q1, num);
  return __builtin_fmaf(e2, r, q1);
}

// div_by with the sign of a zero quotient as IEEE division gives it (that
// of the numerator, the divisor being positive): the stored rows equal the
// plain division bit for bit.
__device__ __forceinline__ float div_by_signed(float num, float den, float r) {
  return copysignf(div_by(num, den, r), num);
}

template <int C>
__global__ __launch_bounds__(256) void k_summarize16(const float* __restrict__ raw, int64_t n,
                                                     int card_bits, const float* __restrict__ bp_g,
                                                     uint8_t* __restrict__ words,
                                                     float2* __restrict__ musd,
                                                     uint16_t* __restrict__ keys,
                                                     unsigned int* __restrict__ norm2_max) {
  __shared__ float bp[257];
  const int card = 1 << card_bits;
  for (int j = threadIdx.x; j <= card; j += blockDim.x) bp[j] = bp_g[j];
  __syncthreads();
  constexpr int len = 16 * C;  // C points per segment
  constexpr int Q = 4 * C;     // points per lane: four segments
  const int lane = threadIdx.x & 63;
  const int j = lane & 3;      // quarter of the row
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const float flen = (float)len;
  const float fm = (float)C;
  const bool as_given = norm2_max != nullptr;  // mu = 0, sd = 1: z = x exactly
  float n2 = 0.0f;  // largest squared row norm seen (as-given rows)
  for (int64_t grp = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); grp * 16 < n;
       grp += waves) {
    const int64_t id = grp * 16 + (lane >> 2);
    const bool valid = id < n;
    float v[Q];
    {
      const float4* src = reinterpret_cast<const float4*>(raw + (valid ? id : 0) * len + j * Q);
#pragma unroll
      for (int i = 0; i < Q / 4; ++i) {
        const float4 t = src[i];
        v[4 * i] = t.x;
        v[4 * i + 1] = t.y;
        v[4 * i + 2] = t.z;
        v[4 * i + 3] = t.w;
      }
    }
    const float mu = as_given ? 0.0f : __fdiv_rn(chain_sum4<Q>(v, j), flen);
    float sq[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      v[i] = v[i] - mu;  // v holds x - mu from here on
      sq[i] = v[i] * v[i];
    }
    const float ss = chain_sum4<Q>(sq, j);
    if (valid) n2 = fmaxf(n2, ss);
    const float sd = as_given ? 1.0f : sqrtf(__fdiv_rn(ss, flen));
    const bool flat = !(sd > 0.0f);
    // segment sums of z = (v - mu) / sd, each z correctly rounded
    float a4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (as_given) {  // mu = 0, sd = 1: z = x
#pragma unroll
      for (int sg = 0; sg < 4; ++sg)
#pragma unroll
        for (int i = 0; i < C; ++i) a4[sg] = a4[sg] + v[sg * C + i];
    } else if (!flat && quick_divisor(mu, sd)) {
      const float r = refined_rcp(sd);
#pragma unroll
      for (int sg = 0; sg < 4; ++sg)
#pragma unroll
        for (int i = 0; i < C; ++i) a4[sg] = a4[sg] + div_by(v[sg * C + i], sd, r);
    } else if (!flat) {
#pragma unroll
      for (int sg = 0; sg < 4; ++sg)
#pragma unroll
        for (int i = 0; i < C; ++i) a4[sg] = a4[sg] + __fdiv_rn(v[sg * C + i], sd);
    }
    uint32_t part = 0, nib = 0;
#pragma unroll
    for (int sg = 0; sg < 4; ++sg) {
      const float pv = __fdiv_rn(a4[sg], fm);
      int lo = 0, hi = card - 1;
      for (int step = 0; step < card_bits; ++step) {
        const int mid = (lo + hi + 1) >> 1;
        if (bp[mid] <= pv)
          lo = mid;
        else
          hi = mid - 1;
      }
      part |= (uint32_t)lo << (8 * sg);
      nib = (nib << 1) | ((uint32_t)lo >> (card_bits - 1));  // segment 4j + sg, most significant first
    }
    // root key: segment 0 is the most significant bit, so quarter j's four
    // bits sit at 12 - 4j; the quad's nibbles combined in every lane
    uint32_t key = nib << (12 - 4 * j);
    key |= (uint32_t)__builtin_amdgcn_update_dpp((int)key, (int)key, 0xb1, 0xf, 0xf, false);  // [1,0,3,2]
    key |= (uint32_t)__builtin_amdgcn_update_dpp((int)key, (int)key, 0x4e, 0xf, 0xf, false);  // [2,3,0,1]
    if (valid) {
      reinterpret_cast<uint32_t*>(words + id * 16)[j] = part;
      if (j == 0) {
        musd[id] = make_float2(mu, flat ? 0.0f : sd);
        keys[id] = (uint16_t)key;
      }
    }
  }
  if (as_given) {  // one atomic per wave
    for (int o = 32; o >= 1; o >>= 1) n2 = fmaxf(n2, __shfl_xor(n2, o));
    if (lane == 0) atomicMax(norm2_max, __float_as_uint(n2));
  }
}

// ---------------------------------------------------------------------------
// (2) Root grouping: a histogram of the root keys, its exclusive scan (one
// block), then a scatter of (word, id) into each key's range.
//
// Root keys are far from uniform (z-normalised random walks share a few
// sign patterns of their segment means), so one device atomic per series
// on its key's counter would queue thousands of waves at the few memory
// channels holding the hot keys.  Both passes count in LDS instead: block
// (x, r) covers the keys of range r (kKeyRange of them) over the x-th part
// of the series, and adds each nonzero count to memory once.  The scatter
// reserves a block's run of positions per key with that one atomic and
// places its series inside the run with LDS atomics; order inside a key's
// range is the atomics' order (leaves are sorted by id at the end).

constexpr int kKeyRange = 16384;  // keys per block's LDS counters (64 KB)

__global__ __launch_bounds__(1024) void k_key_hist(const uint16_t* __restrict__ keys, int64_t n,
                                                   int nkeys, unsigned int* __restrict__ hist) {
  __shared__ unsigned int cnt[kKeyRange];
  const int r0 = blockIdx.y * kKeyRange;
  const int rn = min(kKeyRange, nkeys - r0);
  for (int j = threadIdx.x; j < rn; j += blockDim.x) cnt[j] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const unsigned k = (unsigned)keys[i] - (unsigned)r0;
    if (k < (unsigned)rn) atomicAdd(&cnt[k], 1u);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < rn; j += blockDim.x)
    if (cnt[j]) atomicAdd(&hist[r0 + j], cnt[j]);
}

__global__ __launch_bounds__(1024) void k_scan_hist(const unsigned int* __restrict__ hist, int nkeys,
                                                     int64_t* __restrict__ begin,
                                                     unsigned long long* __restrict__ cursor) {
  __shared__ int64_t part[1024];
  const int per = (nkeys + 1023) / 1024;
  const int a = threadIdx.x * per;
  const int b = min(a + per, nkeys);
  int64_t s = 0;
  for (int i = a; i < b; ++i) s += hist[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    int64_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int64_t run = part[threadIdx.x] - s;
  for (int i = a; i < b; ++i) {
    begin[i] = run;
    cursor[i] = (unsigned long long)run;
    run += hist[i];
  }
  if (threadIdx.x == 1023) begin[nkeys] = part[1023];
}

// Block (x, r): the series of part x with a key in range r.  First their
// counts per key in LDS; then one device atomic per nonzero key reserves
// the block's run in that key's range; then each series takes its place in
// the run with an LDS atomic.  Positions fit 32 bits (n < 2^31).
__global__ __launch_bounds__(1024) void k_root_scatter(const uint4* __restrict__ words,
                                                       const uint16_t* __restrict__ keys, int64_t n,
                                                       int nkeys, unsigned long long* __restrict__ cursor,
                                                       uint4* __restrict__ W0, int32_t* __restrict__ I0) {
  __shared__ unsigned int cnt[kKeyRange], base[kKeyRange];
  const int r0 = blockIdx.y * kKeyRange;
  const int rn = min(kKeyRange, nkeys - r0);
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t c0 = (int64_t)blockIdx.x * per;
  const int64_t c1 = min(n, c0 + per);
  for (int j = threadIdx.x; j < rn; j += blockDim.x) cnt[j] = 0;
  __syncthreads();
  for (int64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) {
    const unsigned k = (unsigned)keys[i] - (unsigned)r0;
    if (k < (unsigned)rn) atomicAdd(&cnt[k], 1u);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < rn; j += blockDim.x) {
    const unsigned c = cnt[j];
    if (c) base[j] = (unsigned)atomicAdd(&cursor[r0 + j], (unsigned long long)c);
    cnt[j] = 0;
  }
  __syncthreads();
  for (int64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) {
    const unsigned k = (unsigned)keys[i] - (unsigned)r0;
    if (k < (unsigned)rn) {
      const unsigned pos = base[k] + atomicAdd(&cnt[k], 1u);
      W0[pos] = words[i];
      I0[pos] = (int32_t)i;
    }
  }
}

__device__ __forceinline__ int append(int* counter, int cap, int* overflow) {
  const int i = atomicAdd(counter, 1);
  if (i >= cap) {
    atomicOr(overflow, 1);
    return -1;
  }
  return i;
}

// A node over leaf_size goes to the round list, others become leaves.
__device__ void place_node(int id, int64_t count, int leaf_size, BuildDev d) {
  if (count > leaf_size) {
    const int slot = append(d.next_count, d.round_cap, d.overflow);
    if (slot >= 0) d.next_list[slot] = id;
  } else {
    const int leaf = append(d.leaf_count, d.leaf_cap, d.overflow);
    if (leaf >= 0) {
      d.leaves[leaf] = id;
      d.nodes[id].leaf = leaf;
    }
  }
}

__global__ void k_roots(const int64_t* __restrict__ begin, int nkeys, int w, int leaf_size,
                        BuildDev d) {
  const int key = blockIdx.x * blockDim.x + threadIdx.x;
  if (key >= nkeys) return;
  const int64_t b = begin[key], e = begin[key + 1];
  if (e == b) {
    d.root_node[key] = -1;
    return;
  }
  const int id = append(d.node_count, d.node_cap, d.overflow);
  if (id < 0) return;
  NodeDev nd;
  nd.begin = b;
  nd.end = e;
  for (int s = 0; s < kMaxSeg; ++s) {
    nd.sym[s] = s < w ? (uint8_t)((key >> (w - 1 - s)) & 1) : 0;
    nd.bits[s] = s < w ? 1 : 0;
  }
  nd.buf = 0;
  nd.seg = -1;
  nd.child[0] = nd.child[1] = -1;
  nd.leaf = -1;
  d.nodes[id] = nd;
  d.root_node[key] = id;
  place_node(id, e - b, leaf_size, d);
}

// ---------------------------------------------------------------------------
// (3) Split rounds.  Work is cut into chunks of one node each.

__device__ __forceinline__ uint32_t word_byte(const uint4& wd, int s) {
  const uint32_t v = s < 4 ? wd.x : (s < 8 ? wd.y : (s < 12 ? wd.z : wd.w));
  return (v >> (8 * (s & 3))) & 0xffu;
}

__global__ __launch_bounds__(256) void k_round_count(const Chunk* __restrict__ chunks,
                                                      const int* __restrict__ n_chunks, int cap,
                                                      BuildDev d, int w, int card_bits) {
  const int nch = min(*n_chunks, cap);
  __shared__ int acc[kMaxSeg];
  for (int ci = blockIdx.x; ci < nch; ci += gridDim.x) {
    const Chunk ch = chunks[ci];
    const int id = d.cur_list[ch.slot];
    const NodeDev& nd = d.nodes[id];
    const uint4* __restrict__ W = nd.buf ? d.W1 : d.W0;
    int bits[kMaxSeg];
    for (int s = 0; s < kMaxSeg; ++s) bits[s] = nd.bits[s];
    int c[kMaxSeg];
    for (int s = 0; s < kMaxSeg; ++s) c[s] = 0;
    for (int64_t e = ch.begin + threadIdx.x; e < ch.end; e += 256) {
      const uint4 wd = W[e];
      for (int s = 0; s < kMaxSeg; ++s) {
        if (s < w && bits[s] < card_bits) c[s] += (int)((word_byte(wd, s) >> (card_bits - 1 - bits[s])) & 1u);
      }
    }
    if (threadIdx.x < kMaxSeg) acc[threadIdx.x] = 0;
    __syncthreads();
    for (int s = 0; s < kMaxSeg; ++s) {
      int v = c[s];
      for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
      if ((threadIdx.x & (kWave - 1)) == 0 && v) atomicAdd(&acc[s], v);
    }
    __syncthreads();
    if (threadIdx.x < kMaxSeg && acc[threadIdx.x])
      atomicAdd(&d.c1[(int64_t)ch.slot * kMaxSeg + threadIdx.x], acc[threadIdx.x]);
    __syncthreads();  // acc is cleared for the next chunk
  }
}

// Most balanced split: the segment minimising |2 c1 - count| among those
// with a bit left, lowest segment on ties (Section 2.2).
// It clears the slot's counts after reading them, so c1 is zero for the
// next round.
__global__ void k_round_decide(int w, int card_bits, int leaf_size, BuildDev d) {
  const int n_cur = *d.cur_count;  // clamped by k_make_chunks
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= n_cur) return;
  const int id = d.cur_list[slot];
  NodeDev nd = d.nodes[id];
  const int64_t count = nd.end - nd.begin;
  int ones[kMaxSeg];
  int4* c1v = reinterpret_cast<int4*>(d.c1 + (int64_t)slot * kMaxSeg);
  for (int j = 0; j < kMaxSeg / 4; ++j) {
    const int4 v = c1v[j];
    ones[4 * j + 0] = v.x;
    ones[4 * j + 1] = v.y;
    ones[4 * j + 2] = v.z;
    ones[4 * j + 3] = v.w;
    c1v[j] = make_int4(0, 0, 0, 0);
  }
  int best = -1;
  int64_t gap = 0;
  for (int s = 0; s < w; ++s) {
    if (nd.bits[s] >= card_bits) continue;
    const int64_t c1 = ones[s];
    int64_t g = 2 * c1 - count;
    g = g < 0 ? -g : g;
    if (best < 0 || g < gap) {
      best = s;
      gap = g;
    }
  }
  d.split_seg[slot] = best;
  if (best < 0) {  // nothing left to refine: an over-full leaf
    const int leaf = append(d.leaf_count, d.leaf_cap, d.overflow);
    if (leaf >= 0) {
      d.leaves[leaf] = id;
      d.nodes[id].leaf = leaf;
    }
    return;
  }
  int64_t n1 = 0;
  for (int s = 0; s < kMaxSeg; ++s) n1 = s == best ? ones[s] : n1;
  const int64_t n0 = count - n1;
  d.cursor[2 * slot + 0] = (unsigned long long)nd.begin;
  d.cursor[2 * slot + 1] = (unsigned long long)(nd.begin + n0);
  int kids[2] = {-1, -1};
  for (int b = 0; b < 2; ++b) {
    const int64_t cb = b ? nd.begin + n0 : nd.begin;
    const int64_t ce = b ? nd.end : nd.begin + n0;
    if (ce == cb) continue;
    const int cid = append(d.node_count, d.node_cap, d.overflow);
    if (cid < 0) continue;
    NodeDev ch = nd;
    ch.begin = cb;
    ch.end = ce;
    ch.sym[best] = (uint8_t)((nd.sym[best] << 1) | b);
    ch.bits[best] = (uint8_t)(nd.bits[best] + 1);
    ch.buf = nd.buf ^ 1;
    ch.seg = -1;
    ch.child[0] = ch.child[1] = -1;
    ch.leaf = -1;
    d.nodes[cid] = ch;
    kids[b] = cid;
    place_node(cid, ce - cb, leaf_size, d);
  }
  d.nodes[id].seg = best;
  d.nodes[id].child[0] = kids[0];
  d.nodes[id].child[1] = kids[1];
}

// Two-way scatter of one chunk into the other buffer.  The block (256
// threads) holds the chunk in registers, entry begin + 256 i + t in thread
// t's slot i, ranks each entry inside its side by ballots and one scan over
// the chunk's (slot, wave) cells, and reserves the chunk's run on each side
// with one atomic per side.  Inside a side the chunk keeps entry order.
constexpr int kScatterPer = kChunk / 256;  // entries per thread
static_assert(kScatterPer * 4 == kWave, "one wave scans the (slot, wave) cells");

__device__ void scatter_chunk(const Chunk ch, const BuildDev& d, int card_bits) {
  const int seg = d.split_seg[ch.slot];
  if (seg < 0) return;
  const int id = d.cur_list[ch.slot];
  const NodeDev& nd = d.nodes[id];
  const uint4* __restrict__ Win = nd.buf ? d.W1 : d.W0;
  const int32_t* __restrict__ Iin = nd.buf ? d.I1 : d.I0;
  uint4* __restrict__ Wout = nd.buf ? d.W0 : d.W1;
  int32_t* __restrict__ Iout = nd.buf ? d.I0 : d.I1;
  const int shift = card_bits - 1 - nd.bits[seg];
  __shared__ int s_ones[kScatterPer * 4];  // per (slot, wave): ones, then their exclusive scan
  __shared__ int s_zeros[kScatterPer * 4];
  __shared__ unsigned long long base[2];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x >> 6;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint4 wd[kScatterPer];
  int32_t idv[kScatterPer];
  int rank[kScatterPer];  // rank inside the wave's side; -1: past the chunk
  bool one[kScatterPer];
#pragma unroll
  for (int i = 0; i < kScatterPer; ++i) {
    const int64_t e = ch.begin + (int64_t)i * 256 + threadIdx.x;
    const bool valid = e < ch.end;
    wd[i] = valid ? Win[e] : make_uint4(0, 0, 0, 0);
    idv[i] = valid ? Iin[e] : 0;
  }
#pragma unroll
  for (int i = 0; i < kScatterPer; ++i) {
    const bool valid = ch.begin + (int64_t)i * 256 + threadIdx.x < ch.end;
    one[i] = valid && ((word_byte(wd[i], seg) >> shift) & 1u);
    const unsigned long long ones = __ballot(one[i]);
    const unsigned long long vals = __ballot(valid);
    rank[i] = !valid ? -1 : (one[i] ? __popcll(ones & below) : __popcll(vals & ~ones & below));
    if (lane == 0) {
      s_ones[i * 4 + wv] = __popcll(ones);
      s_zeros[i * 4 + wv] = __popcll(vals & ~ones);
    }
  }
  __syncthreads();
  if (threadIdx.x < kWave) {  // one wave scans the 64 cells in entry order
    const int o = s_ones[threadIdx.x], z = s_zeros[threadIdx.x];
    int so = o, sz = z;
    for (int k = 1; k < kWave; k <<= 1) {
      const int po = __shfl_up(so, k, kWave), pz = __shfl_up(sz, k, kWave);
      if (lane >= k) {
        so += po;
        sz += pz;
      }
    }
    s_ones[threadIdx.x] = so - o;
    s_zeros[threadIdx.x] = sz - z;
    if (lane == kWave - 1) {
      base[0] = sz ? atomicAdd(&d.cursor[2 * ch.slot + 0], (unsigned long long)sz) : 0ull;
      base[1] = so ? atomicAdd(&d.cursor[2 * ch.slot + 1], (unsigned long long)so) : 0ull;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kScatterPer; ++i) {
    if (rank[i] < 0) continue;
    const int64_t dst = one[i] ? (int64_t)base[1] + s_ones[i * 4 + wv] + rank[i]
                               : (int64_t)base[0] + s_zeros[i * 4 + wv] + rank[i];
    Wout[dst] = wd[i];
    Iout[dst] = idv[i];
  }
  __syncthreads();  // the cells are rewritten by the block's next chunk
}

__global__ __launch_bounds__(256) void k_round_scatter(const Chunk* __restrict__ chunks,
                                                        const int* __restrict__ n_chunks, int cap,
                                                        BuildDev d, int card_bits) {
  const int nch = min(*n_chunks, cap);
  for (int ci = blockIdx.x; ci < nch; ci += gridDim.x) scatter_chunk(chunks[ci], d, card_bits);
}

// Chunk list of the round (one block): exclusive scan of chunk counts.  It
// opens the round: the node count becomes 0 after an overflow (so nothing
// runs until the host sees it) and at most round_cap, and the next round's
// list starts empty.
__global__ __launch_bounds__(1024) void k_make_chunks(BuildDev d, int chunk,
                                                       Chunk* __restrict__ out, int cap,
                                                       int* __restrict__ out_count,
                                                       int* __restrict__ out_overflow) {
  __shared__ int part[1024];
  const int n_cur = *d.overflow ? 0 : min(*d.cur_count, d.round_cap);
  __syncthreads();
  if (threadIdx.x == 0) {
    *d.cur_count = n_cur;
    *d.next_count = 0;
  }
  const int per = (n_cur + 1023) / 1024;
  const int a = threadIdx.x * per;
  const int b = min(a + per, n_cur);
  int s = 0;
  for (int i = a; i < b; ++i) {
    const NodeDev& nd = d.nodes[d.cur_list[i]];
    s += (int)((nd.end - nd.begin + chunk - 1) / chunk);
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    int v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int run = part[threadIdx.x] - s;
  for (int i = a; i < b; ++i) {
    const NodeDev& nd = d.nodes[d.cur_list[i]];
    for (int64_t e = nd.begin; e < nd.end; e += chunk) {
      if (run < cap) {
        Chunk c;
        c.slot = i;
        c.pad = 0;
        c.begin = e;
        c.end = e + chunk < nd.end ? e + chunk : nd.end;
        out[run] = c;
      }
      ++run;
    }
  }
  if (threadIdx.x == 1023) {
    *out_count = part[1023];
    if (part[1023] > cap) *out_overflow = 1;
  }
}

// ---------------------------------------------------------------------------
// (4) Leaf records and id order inside each leaf.

__global__ void k_leaf_records(BuildDev d, int n_leaves, int64_t* __restrict__ leaf_begin,
                               int64_t* __restrict__ leaf_end, uint4* __restrict__ leaf_sym,
                               uint4* __restrict__ leaf_bits, int* __restrict__ leaf_buf) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n_leaves) return;
  const NodeDev& nd = d.nodes[d.leaves[l]];
  leaf_begin[l] = nd.begin;
  leaf_end[l] = nd.end;
  uint32_t s[4] = {0, 0, 0, 0}, b[4] = {0, 0, 0, 0};
  for (int j = 0; j < kMaxSeg; ++j) {
    s[j >> 2] |= (uint32_t)nd.sym[j] << (8 * (j & 3));
    b[j >> 2] |= (uint32_t)nd.bits[j] << (8 * (j & 3));
  }
  leaf_sym[l] = make_uint4(s[0], s[1], s[2], s[3]);
  leaf_bits[l] = make_uint4(b[0], b[1], b[2], b[3]);
  leaf_buf[l] = nd.buf;
}

// Bitonic sort of one leaf's ids (size up to kLeafSortMax, padded to a
// power of two of at least 128 with INT_MAX).  A wave owns 128-element
// windows (lane l holds positions l and l + 64): the network's steps with
// stride 64 or less stay inside a window and run in registers (stride 64
// inside the lane, smaller ones by lane exchanges), so only the steps with
// stride 128 or more go through LDS between block barriers.

// One compare-exchange of the pair (p, p ^ s), s < 64, from the lane
// holding p: the lower position keeps the minimum when the run ascends.
__device__ __forceinline__ int32_t bitonic_lanes(int32_t x, int s, bool lower, bool up) {
  const int32_t y = __shfl_xor(x, s, kWave);
  return (lower == up) ? min(x, y) : max(x, y);
}

// The steps of stage `size` with stride 64 and less on the window at base.
__device__ __forceinline__ void bitonic_window(int32_t& a, int32_t& b, int base, int lane, int size) {
  const bool upa = ((base + lane) & size) == 0, upb = ((base + lane + 64) & size) == 0;
  if (size >= 128) {  // stride 64: a and b are the pair (same run direction)
    const int32_t lo = min(a, b), hi = max(a, b);
    a = upa ? lo : hi;
    b = upa ? hi : lo;
  }
  for (int s = min(size >> 1, 32); s >= 1; s >>= 1) {
    const bool lower = (lane & s) == 0;
    a = bitonic_lanes(a, s, lower, upa);
    b = bitonic_lanes(b, s, lower, upb);
  }
}

__global__ __launch_bounds__(1024) void k_leaf_sort(const int64_t* __restrict__ leaf_begin,
                                                     const int64_t* __restrict__ leaf_end,
                                                     const int* __restrict__ leaf_buf,
                                                     const int32_t* __restrict__ I0,
                                                     const int32_t* __restrict__ I1,
                                                     int32_t* __restrict__ perm) {
  __shared__ int32_t v[kLeafSortMax];
  const int l = blockIdx.x;
  const int64_t b = leaf_begin[l], e = leaf_end[l];
  const int cnt = (int)(e - b);
  if (cnt > kLeafSortMax) return;  // sorted by k_leaf_sort_global
  const int32_t* __restrict__ I = leaf_buf[l] ? I1 : I0;
  int p2 = 128;
  while (p2 < cnt) p2 <<= 1;
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int i = threadIdx.x; i < p2; i += blockDim.x) v[i] = i < cnt ? I[b + i] : 0x7fffffff;
  __syncthreads();
  for (int base = wv * 128; base < p2; base += nw * 128) {  // stages 2 .. 128
    int32_t x = v[base + lane], y = v[base + lane + 64];
    for (int size = 2; size <= 128; size <<= 1) bitonic_window(x, y, base, lane, size);
    v[base + lane] = x;
    v[base + lane + 64] = y;
  }
  __syncthreads();
  for (int size = 256; size <= p2; size <<= 1) {
    for (int stride = size >> 1; stride >= 128; stride >>= 1) {
      for (int i = threadIdx.x; i < (p2 >> 1); i += blockDim.x) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const int32_t a = v[lo], c = v[hi];
        if ((a > c) == up) {
          v[lo] = c;
          v[hi] = a;
        }
      }
      __syncthreads();
    }
    for (int base = wv * 128; base < p2; base += nw * 128) {
      int32_t x = v[base + lane], y = v[base + lane + 64];
      bitonic_window(x, y, base, lane, size);
      v[base + lane] = x;
      v[base + lane + 64] = y;
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) perm[b + i] = v[i];
}

// Larger (over-full) leaves: the same network over a global scratch area.
__global__ __launch_bounds__(1024) void k_leaf_sort_global(int64_t b, int cnt, int p2,
                                                            const int32_t* __restrict__ I,
                                                            int32_t* __restrict__ scratch,
                                                            int32_t* __restrict__ perm) {
  for (int i = threadIdx.x; i < p2; i += blockDim.x) scratch[i] = i < cnt ? I[b + i] : 0x7fffffff;
  __syncthreads();
  for (int size = 2; size <= p2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < (p2 >> 1); i += blockDim.x) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const int32_t a = scratch[lo], c = scratch[hi];
        if ((a > c) == up) {
          scratch[lo] = c;
          scratch[hi] = a;
        }
      }
      __threadfence();
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) perm[b + i] = scratch[i];
}

// Leaf sizes: out[0] = the largest, out[1] = how many exceed kLeafSortMax
// (those are sorted by k_leaf_sort_global).  out must be zero on entry.
__global__ __launch_bounds__(1024) void k_leaf_stats(const int64_t* __restrict__ begin,
                                                     const int64_t* __restrict__ end, int L,
                                                     int* __restrict__ out) {
  __shared__ int s_max, s_big;
  if (threadIdx.x == 0) {
    s_max = 0;
    s_big = 0;
  }
  __syncthreads();
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = l < L ? (int)(end[l] - begin[l]) : 0;
  int m = c;
  for (int o = 32; o >= 1; o >>= 1) m = max(m, __shfl_xor(m, o, kWave));
  const int big = __popcll(__ballot(c > kLeafSortMax));
  if ((threadIdx.x & (kWave - 1)) == 0) {
    atomicMax(&s_max, m);
    atomicAdd(&s_big, big);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicMax(&out[0], s_max);
    if (s_big) atomicAdd(&out[1], s_big);
  }
}

// The leaf table in the query's shard-major order.  Leaf l belongs to shard
// l % kShards; shard s holds leaves s, s + kShards, ... contiguously,
// starting at s q + min(s, r) for L = kShards q + r.
__device__ __forceinline__ int shard_leaf_start(int s, int L) {
  const int q = L / kShards, r = L % kShards;
  return s * q + min(s, r);
}

// One block: per shard, its work chunks (kChunkSeries series each, per leaf)
// and their exclusive scan (shard_off, n_chunks = shard_off[kShards]); the
// shard-major leaf offsets (leaf_sh_off).
__global__ __launch_bounds__(1024) void k_shard_offsets(const int64_t* __restrict__ begin,
                                                        const int64_t* __restrict__ end, int L,
                                                        int* __restrict__ shard_off,
                                                        int* __restrict__ leaf_sh_off,
                                                        int* __restrict__ n_chunks) {
  __shared__ int cnt[kShards];
  const int lane = threadIdx.x & (kWave - 1);
  const int nw = blockDim.x >> 6;
  for (int sh = threadIdx.x >> 6; sh < kShards; sh += nw) {
    int c = 0;
    for (int l = sh + kShards * lane; l < L; l += kShards * kWave)
      c += (int)((end[l] - begin[l] + kChunkSeries - 1) / kChunkSeries);
    for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, kWave);
    if (lane == 0) cnt[sh] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int sh = 0; sh < kShards; ++sh) {
      shard_off[sh] = run;
      run += cnt[sh];
    }
    shard_off[kShards] = run;
    *n_chunks = run;
  }
  if (threadIdx.x <= kShards) leaf_sh_off[threadIdx.x] = shard_leaf_start(threadIdx.x, L);
}

__global__ void k_shard_tables(const int64_t* __restrict__ begin, const int64_t* __restrict__ end,
                               const uint4* __restrict__ sym, const uint4* __restrict__ bits,
                               int L, uint4* __restrict__ sh_sym, uint4* __restrict__ sh_bits,
                               int2* __restrict__ sh_rng) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= L) return;
  const int j = shard_leaf_start(l % kShards, L) + l / kShards;
  sh_sym[j] = sym[l];
  sh_bits[j] = bits[l];
  sh_rng[j] = make_int2((int)begin[l], (int)end[l]);
}

// ---------------------------------------------------------------------------
// (5) Leaf-ordered store: z = (x - mu) / sd per point (the same rounding as
// in the summary pass), one wave per row, float4 per lane.

// Leaf-ordered store: position p takes row perm[p], z-normalised.  A wave
// moves kGatherRows rows per step, every load of the step issued before
// any is used (the ids, then their (mu, sd), then the rows), so four rows'
// chains are in flight per wave instead of one.
constexpr int kGatherRows = 4;

// The build reads each raw row once here and writes each stored row once:
// non-temporal accesses keep them from displacing cached lines.
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4 load_nt(const float* p) {
  const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ void store_nt(float* p, const float4 o) {
  const f32x4 v = {o.x, o.y, o.z, o.w};
  __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(p));
}

// Four points of a row z-normalised with its (mu, sd): zero for a flat row,
// else each (x - mu) / sd correctly rounded (div_by_signed where
// quick_divisor allows it, the plain division otherwise).
__device__ __forceinline__ float4 znorm4(const float4 v, const float2 ms) {
  const float mu = ms.x, sd = ms.y;
  float4 o = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (!(sd > 0.0f)) return o;
  if (quick_divisor(mu, sd)) {
    const float r = refined_rcp(sd);
    o.x = div_by_signed(v.x - mu, sd, r);
    o.y = div_by_signed(v.y - mu, sd, r);
    o.z = div_by_signed(v.z - mu, sd, r);
    o.w = div_by_signed(v.w - mu, sd, r);
  } else {
    o.x = __fdiv_rn(v.x - mu, sd);
    o.y = __fdiv_rn(v.y - mu, sd);
    o.z = __fdiv_rn(v.z - mu, sd);
    o.w = __fdiv_rn(v.w - mu, sd);
  }
  return o;
}

__global__ __launch_bounds__(256) void k_gather_store(const float* __restrict__ raw, int64_t n, int len,
                                                       const int32_t* __restrict__ perm,
                                                       const float2* __restrict__ musd,
                                                       const uint4* __restrict__ words,
                                                       float* __restrict__ Z,
                                                       uint4* __restrict__ words_sorted) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t p0 = wave * kGatherRows; p0 < n; p0 += nwaves * kGatherRows) {
    int32_t id[kGatherRows];
    float2 ms[kGatherRows];
#pragma unroll
    for (int r = 0; r < kGatherRows; ++r) id[r] = perm[p0 + r < n ? p0 + r : p0];  // past n: a valid row, not stored
#pragma unroll
    for (int r = 0; r < kGatherRows; ++r) ms[r] = musd[id[r]];
    if ((len & 3) == 0) {
      for (int t = 4 * lane; t < len; t += 4 * kWave) {
        float4 v[kGatherRows];
#pragma unroll
        for (int r = 0; r < kGatherRows; ++r) v[r] = load_nt(raw + (int64_t)id[r] * len + t);
#pragma unroll
        for (int r = 0; r < kGatherRows; ++r) {
          if (p0 + r >= n) continue;
          store_nt(Z + (p0 + r) * (int64_t)len + t, znorm4(v[r], ms[r]));
        }
      }
    } else {
      for (int r = 0; r < kGatherRows; ++r) {
        if (p0 + r >= n) continue;
        const bool flat = !(ms[r].y > 0.0f);
        const float* __restrict__ x = raw + (int64_t)id[r] * len;
        float* __restrict__ z = Z + (p0 + r) * (int64_t)len;
        for (int t = lane; t < len; t += kWave) z[t] = flat ? 0.0f : __fdiv_rn(x[t] - ms[r].x, ms[r].y);
      }
    }
    int32_t mine = id[0];  // lane r < kGatherRows moves row r's word
#pragma unroll
    for (int r = 1; r < kGatherRows; ++r) mine = lane == r ? id[r] : mine;
    if (lane < kGatherRows && p0 + lane < n) words_sorted[p0 + lane] = words[mine];
  }
}

// In-place store: the caller's rows are z-normalised where they are (id
// order, the same arithmetic as the leaf-ordered copy) and only the words
// are gathered into leaf order.
__global__ __launch_bounds__(256) void k_store_inplace(float* __restrict__ raw, int64_t n, int len,
                                                        const int32_t* __restrict__ perm,
                                                        const float2* __restrict__ musd,
                                                        const uint4* __restrict__ words,
                                                        uint4* __restrict__ words_sorted, int as_given) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t p = wave; p < n; p += nwaves) {
    const int32_t id = perm[p];
    if (lane == 0) words_sorted[p] = words[id];
    if (as_given) continue;  // the rows already are what the index holds
    const float2 ms = musd[id];
    float* __restrict__ x = raw + (int64_t)id * len;
    const bool flat = !(ms.y > 0.0f);
    if ((len & 3) == 0) {
      for (int t = 4 * lane; t < len; t += 4 * kWave) {
        const float4 v = *reinterpret_cast<const float4*>(x + t);
        *reinterpret_cast<float4*>(x + t) = znorm4(v, ms);
      }
    } else {
      for (int t = lane; t < len; t += kWave) x[t] = flat ? 0.0f : __fdiv_rn(x[t] - ms.x, ms.y);
    }
  }
}

// Compact tree for the approximate-search descent: one 16-byte record per
// node, so each level of the descent is a single load.
__global__ void k_make_tree(const NodeDev* __restrict__ nodes, int n_nodes, int card_bits,
                            int4* __restrict__ tree) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_nodes) return;
  const NodeDev& nd = nodes[i];
  if (nd.seg >= 0) {
    const int shift = card_bits - 1 - nd.bits[nd.seg];
    tree[i] = make_int4(nd.seg | (shift << 8), 0, nd.child[0], nd.child[1]);
  } else {
    tree[i] = make_int4(-1, (int)nd.begin, (int)nd.end, nd.leaf);
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers.

void launch_summarize(const float* raw, int64_t n, int len, int w, int card_bits, int spw,
                      const float* bp, uint4* words, float2* musd, uint16_t* keys,
                      unsigned int* norm2_max, hipStream_t st, int n_cus) {
  // the register path reads float4s: the rows must start 16-byte aligned
  if (w == 16 && len % 64 == 0 && len <= 256 && (reinterpret_cast<uintptr_t>(raw) & 15) == 0) {
    const int64_t groups = (n + 15) / 16;  // 16 series per wave, 4 waves per block
    const int64_t want = (groups + 3) / 4;
    const unsigned blocks = (unsigned)std::min<int64_t>(want, (int64_t)n_cus * 32);
    uint8_t* wb = reinterpret_cast<uint8_t*>(words);
    switch (len / 16) {
      case 4: hipLaunchKernelGGL(k_summarize16<4>, dim3(blocks), dim3(256), 0, st, raw, n, card_bits, bp, wb, musd, keys, norm2_max); break;
      case 8: hipLaunchKernelGGL(k_summarize16<8>, dim3(blocks), dim3(256), 0, st, raw, n, card_bits, bp, wb, musd, keys, norm2_max); break;
      case 12: hipLaunchKernelGGL(k_summarize16<12>, dim3(blocks), dim3(256), 0, st, raw, n, card_bits, bp, wb, musd, keys, norm2_max); break;
      default: hipLaunchKernelGGL(k_summarize16<16>, dim3(blocks), dim3(256), 0, st, raw, n, card_bits, bp, wb, musd, keys, norm2_max); break;
    }
    return;
  }
  const int64_t blocks = (n + spw - 1) / spw;
  const size_t lds = (257 + (size_t)spw * len) * sizeof(float);
  hipLaunchKernelGGL(k_summarize, dim3((unsigned)blocks), dim3(kWave), lds, st, raw, n, len, w,
                     card_bits, spw, bp, words, musd, keys, norm2_max);
}

void launch_key_hist(const uint16_t* keys, int64_t n, int nkeys, unsigned int* hist, int n_cus,
                     hipStream_t st) {
  const dim3 g((unsigned)std::max(1, n_cus), (unsigned)((nkeys + kKeyRange - 1) / kKeyRange));
  hipLaunchKernelGGL(k_key_hist, g, dim3(1024), 0, st, keys, n, nkeys, hist);
}

void launch_scan_hist(const unsigned int* hist, int nkeys, int64_t* begin,
                      unsigned long long* cursor, hipStream_t st) {
  hipLaunchKernelGGL(k_scan_hist, dim3(1), dim3(1024), 0, st, hist, nkeys, begin, cursor);
}

void launch_root_scatter(const uint4* words, const uint16_t* keys, int64_t n, int nkeys,
                         unsigned long long* cursor, uint4* W0, int32_t* I0, int n_cus, hipStream_t st) {
  const dim3 g((unsigned)std::max(1, n_cus), (unsigned)((nkeys + kKeyRange - 1) / kKeyRange));
  hipLaunchKernelGGL(k_root_scatter, g, dim3(1024), 0, st, words, keys, n, nkeys, cursor, W0, I0);
}

void launch_roots(const int64_t* begin, int nkeys, int w, int leaf_size, const BuildDev& d,
                  hipStream_t st) {
  hipLaunchKernelGGL(k_roots, dim3((nkeys + 255) / 256), dim3(256), 0, st, begin, nkeys, w,
                     leaf_size, d);
}

void launch_make_chunks(const BuildDev& d, int chunk, Chunk* out, int cap, int* out_count,
                        int* out_overflow, hipStream_t st) {
  hipLaunchKernelGGL(k_make_chunks, dim3(1), dim3(1024), 0, st, d, chunk, out, cap, out_count,
                     out_overflow);
}

void launch_round_count(const Chunk* chunks, const int* n_chunks, int cap, const BuildDev& d,
                        int w, int card_bits, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_round_count, dim3(blocks), dim3(256), 0, st, chunks, n_chunks, cap, d, w,
                     card_bits);
}

void launch_round_decide(int w, int card_bits, int leaf_size, const BuildDev& d, hipStream_t st) {
  hipLaunchKernelGGL(k_round_decide, dim3((d.round_cap + 255) / 256), dim3(256), 0, st, w,
                     card_bits, leaf_size, d);
}

void launch_round_scatter(const Chunk* chunks, const int* n_chunks, int cap, const BuildDev& d,
                          int card_bits, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_round_scatter, dim3(blocks), dim3(256), 0, st, chunks, n_chunks, cap, d,
                     card_bits);
}

void launch_leaf_records(const BuildDev& d, int n_leaves, int64_t* leaf_begin, int64_t* leaf_end,
                         uint4* leaf_sym, uint4* leaf_bits, int* leaf_buf, hipStream_t st) {
  hipLaunchKernelGGL(k_leaf_records, dim3((n_leaves + 255) / 256), dim3(256), 0, st, d, n_leaves,
                     leaf_begin, leaf_end, leaf_sym, leaf_bits, leaf_buf);
}

void launch_leaf_sort(int n_leaves, const int64_t* leaf_begin, const int64_t* leaf_end,
                      const int* leaf_buf, const int32_t* I0, const int32_t* I1, int32_t* perm,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_leaf_sort, dim3(n_leaves), dim3(1024), 0, st, leaf_begin, leaf_end,
                     leaf_buf, I0, I1, perm);
}

void launch_leaf_sort_global(int64_t b, int cnt, int p2, const int32_t* I, int32_t* scratch,
                             int32_t* perm, hipStream_t st) {
  hipLaunchKernelGGL(k_leaf_sort_global, dim3(1), dim3(1024), 0, st, b, cnt, p2, I, scratch, perm);
}

void launch_leaf_stats(const int64_t* leaf_begin, const int64_t* leaf_end, int n_leaves, int* out,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_leaf_stats, dim3((unsigned)((n_leaves + 1023) / 1024)), dim3(1024), 0, st,
                     leaf_begin, leaf_end, n_leaves, out);
}

void launch_shard_layout(const int64_t* leaf_begin, const int64_t* leaf_end, const uint4* leaf_sym,
                         const uint4* leaf_bits, int n_leaves, int* shard_off, int* leaf_sh_off,
                         int* n_chunks, uint4* sh_sym, uint4* sh_bits, int2* sh_rng, hipStream_t st) {
  hipLaunchKernelGGL(k_shard_offsets, dim3(1), dim3(1024), 0, st, leaf_begin, leaf_end, n_leaves,
                     shard_off, leaf_sh_off, n_chunks);
  hipLaunchKernelGGL(k_shard_tables, dim3((unsigned)((n_leaves + 255) / 256)), dim3(256), 0, st,
                     leaf_begin, leaf_end, leaf_sym, leaf_bits, n_leaves, sh_sym, sh_bits, sh_rng);
}

void launch_make_tree(const NodeDev* nodes, int n_nodes, int card_bits, int4* tree,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_make_tree, dim3((n_nodes + 255) / 256), dim3(256), 0, st, nodes, n_nodes,
                     card_bits, tree);
}

void launch_gather_store(const float* raw, int64_t n, int len, const int32_t* perm,
                         const float2* musd, const uint4* words, float* Z, uint4* words_sorted,
                         hipStream_t st) {
  int64_t blocks = (n + 4 * kGatherRows - 1) / (4 * kGatherRows);
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_gather_store, dim3((unsigned)blocks), dim3(256), 0, st, raw, n, len, perm,
                     musd, words, Z, words_sorted);
}

// Sliding windows of a long series: row i holds points [i stride, i stride
// + len).  Consecutive threads write consecutive floats of a row and read
// consecutive points of the series.
__global__ __launch_bounds__(256) void k_windows(const float* __restrict__ series, int64_t n, int len,
                                                  int stride, float* __restrict__ rows) {
  const int64_t total = n * (int64_t)len;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / len;
    const int t = (int)(e - i * len);
    rows[e] = series[i * stride + t];
  }
}

void launch_windows(const float* series, int64_t n, int len, int stride, float* rows, hipStream_t st) {
  const int64_t want = (n * (int64_t)len + 255) / 256;
  const unsigned blocks = (unsigned)std::min<int64_t>(want, 65536);
  hipLaunchKernelGGL(k_windows, dim3(blocks), dim3(256), 0, st, series, n, len, stride, rows);
}

void launch_store_inplace(float* raw, int64_t n, int len, const int32_t* perm, const float2* musd,
                          const uint4* words, uint4* words_sorted, int raw_mode, hipStream_t st) {
  const int64_t blocks = std::min<int64_t>((n + 3) / 4, 65536);
  hipLaunchKernelGGL(k_store_inplace, dim3((unsigned)blocks), dim3(256), 0, st, raw, n, len, perm, musd,
                     words, words_sorted, raw_mode);
}

}  // namespace messi
