// Query-side device structures and kernel launchers of libmessi.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "build.h"
#include "common.h"

namespace messi {

constexpr int kSelectThreads = 1024;
constexpr int kProcThreads = 256;
constexpr int kMaxBand = 64;       // largest DTW radius served by the register-band kernel

// Read-only view of a built index.
struct IndexDev {
  int64_t n;
  int len, w, m, card_bits, n_leaves;
  const float* Z;            // [n][len] z-normalised series: in leaf order, or in id order when
                             // zrow is set (the caller's buffer, normalised in place)
  const int32_t* zrow;       // null, or [n]: the row of Z holding leaf-order position p
  const uint4* words;        // [n] words in leaf order
  const int32_t* perm;       // [n] id at each leaf-order position
  const int64_t* leaf_begin; // [L]
  const int64_t* leaf_end;   // [L]
  const uint4* leaf_sym;     // [L]
  const uint4* leaf_bits;    // [L]
  const float* bp;           // [card + 1] breakpoints with -inf / +inf ends
  const int4* tree;          // per node: inner {seg | shift << 8, -, child0, child1},
                             //           leaf  {-1, begin, end, leaf index}
  const int* root_node;      // [2^w]
  const int* shard_off;      // [kShards + 1] first chunk of each shard (leaf l in shard l % kShards)
  const uint4* sh_sym;       // leaf symbols, bits and position ranges in shard-major order:
  const uint4* sh_bits;      //   entry leaf_sh_off[s] + i is leaf s + kShards i
  const int2* sh_rng;
  const int* leaf_sh_off;    // [kShards + 1]
};

// Row of Z holding leaf-order position pos.
__device__ __forceinline__ const float* zrow_ptr(const IndexDev& ix, int64_t pos) {
  return ix.Z + (ix.zrow ? (int64_t)ix.zrow[pos] : pos) * ix.len;
}

// BF16 screen of batched ED queries: a BF16 shadow of the store with the
// squared norm of every row, the queries' BF16 rows and norms, the leaves'
// query lists, and the bound constants.
struct ScreenDev {
  const uint16_t* Zb;     // [n][len] BF16 (round to nearest even) of Z
  const float* xn;        // [n] squared norm of each row of Z (FP64 sum, rounded)
  uint16_t* qb;           // [nq][len] BF16 of the normalised queries
  float* qn;              // [nq] their squared norms
  int* cnt;               // [L] queries that keep each leaf
  int64_t* off;           // [L + 1] start of each leaf's query list
  int* lists;             // [sum of cnt] query indices, leaf by leaf
  int* counter;           // leaf work counter
  unsigned long long* tally;  // [2] pairs screened, pairs passed to refinement
  float c_dot;            // bound: c_dot |q||x| + c_abs (|q|^2 + |x|^2)
  float c_abs;
};

bool screen_supported(int len);
// nt: 16-series column tiles per wave of the screen kernel, waves: waves
// per block; the variants built are those screen_variant accepts (the
// defaults, screen_nt_default(len) with screen_waves_default(), always are)
bool screen_variant(int len, int nt, int waves);
int screen_nt_default(int len);
int screen_waves_default();
int screen_blocks_per_cu(int len, int nt, int waves);
void launch_bf16_rows(const float* src, const int32_t* src_row, int64_t rows, int len, uint16_t* dst,
                      float* norms, hipStream_t st);
void launch_screen(const IndexDev& ix, const QueryParams& qp, const QueryState& qs,
                   const ScreenDev& sc, int blocks, int nt, int waves, hipStream_t st);

void launch_vote(const int64_t* ids, int64_t stride, int nq, int k, const int* labels, int n_classes,
                 int* out, hipStream_t st);
void launch_prep(const IndexDev& ix, const float* queries, const QueryParams& qp,
                 const QueryState& qs, hipStream_t st);
void launch_stage1(const IndexDev& ix, const QueryParams& qp, const QueryState& qs,
                   hipStream_t st);
void launch_process(const IndexDev& ix, const QueryParams& qp, const QueryState& qs,
                    int blocks_per_query, hipStream_t st);
void launch_finalize(const IndexDev& ix, const QueryParams& qp, const QueryState& qs,
                     int64_t* out_ids, float* out_dists, hipStream_t st);
// statistics: the work the search needs once the final k-th best is known
void launch_min_work(const IndexDev& ix, const QueryParams& qp, const QueryState& qs, int blocks,
                     hipStream_t st);
size_t process_lds_bytes(const QueryParams& qp);   // dynamic LDS of the process kernel
size_t process_lds_static(const QueryParams& qp);  // its static LDS (upper bound)
size_t finalize_lds_bytes(const QueryParams& qp);
size_t stage1_lds_bytes(const QueryParams& qp);
int process_blocks_per_cu(const QueryParams& qp);
// grid of the ED process kernel (every block visits every query)
int ed_process_blocks(int resident);
// Device address (on the current device) and size of the allocation-free
// entry point's scratch array; nullptr if it cannot be had.
void* noalloc_scratch(size_t* bytes);

}  // namespace messi
