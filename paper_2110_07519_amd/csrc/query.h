// Query-side device structures and kernel launchers of libmessi.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "build.h"
#include "common.h"

namespace messi {

constexpr int kSelectThreads = 1024;
constexpr int kProcThreads = 256;
constexpr int kTile = 1024;        // series of a leaf examined per pass of a block
constexpr int kMaxBand = 64;       // largest DTW radius served by the register-band kernel

// Read-only view of a built index.
struct IndexDev {
  int64_t n;
  int len, w, m, card_bits, n_leaves;
  const float* Z;            // [n][len] z-normalised series in leaf order
  const uint4* words;        // [n] words in leaf order
  const int32_t* perm;       // [n] id at each leaf-order position
  const int64_t* leaf_begin; // [L]
  const int64_t* leaf_end;   // [L]
  const uint4* leaf_sym;     // [L]
  const uint4* leaf_bits;    // [L]
  const float* bp;           // [card + 1] breakpoints with -inf / +inf ends
  const NodeDev* nodes;
  const int* root_node;      // [2^w]
};

void launch_prep(const IndexDev& ix, const float* queries, const QueryParams& qp,
                 const QueryState& qs, hipStream_t st);
void launch_approx(const IndexDev& ix, const QueryParams& qp, const QueryState& qs,
                   hipStream_t st);
void launch_select(const IndexDev& ix, const QueryParams& qp, const QueryState& qs,
                   unsigned long long* cand_sorted, hipStream_t st);
size_t query_process_lds(const QueryParams& qp);
size_t query_process_lds_for(const QueryParams& qp, int fin_waves);
void launch_process(const IndexDev& ix, const QueryParams& qp, const QueryState& qs,
                    const unsigned long long* cand_sorted, int blocks_per_query,
                    int64_t* out_ids, float* out_dists, hipStream_t st);

}  // namespace messi
