// Build-side device structures and kernel launchers of libmessi.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace messi {

constexpr int kLeafSortMax = 4096;  // leaves up to this size are sorted in LDS
constexpr int kChunk = 4096;        // entries per work chunk of a split round

// A node of the index tree (root subtree node, inner node or leaf).
struct NodeDev {
  int64_t begin, end;       // range of entries (in buffer `buf`)
  uint8_t sym[kMaxSeg];     // symbol prefix per segment
  uint8_t bits[kMaxSeg];    // prefix length per segment
  int32_t buf;              // which ping-pong buffer holds the range
  int32_t seg;              // split segment (-1: not split)
  int32_t child[2];         // children node ids (-1: empty)
  int32_t leaf;             // leaf index (-1: not a leaf)
  int32_t pad;
};

struct Chunk {
  int32_t slot;  // index into the round's node list
  int32_t pad;
  int64_t begin, end;
};

// Device pointers shared by the build kernels.
struct BuildDev {
  NodeDev* nodes;
  int* node_count;
  int node_cap;
  int* leaves;       // leaf index -> node id
  int* leaf_count;
  int leaf_cap;
  int* root_node;    // root key -> node id (-1: empty)
  int* cur_list;     // node ids of this round
  int* next_list;    // node ids of the next round
  int* cur_count;    // entries of cur_list (may exceed round_cap after an overflow)
  int* next_count;
  int round_cap;     // capacity of the round lists
  int* c1;           // [round slot][16] ones per segment; zero between rounds
  int* split_seg;    // [round slot]
  unsigned long long* cursor;  // [round slot][2]
  int* overflow;
  uint4* W0;
  uint4* W1;
  int32_t* I0;
  int32_t* I1;
};

// keys: [n] root key of each series (its w symbols' top bits)
void launch_summarize(const float* raw, int64_t n, int len, int w, int card_bits, int spw,
                      const float* bp, uint4* words, float2* musd, uint16_t* keys,
                      unsigned int* norm2_max, hipStream_t st, int n_cus);
// hist must be zero on entry
void launch_key_hist(const uint16_t* keys, int64_t n, int nkeys, unsigned int* hist, int n_cus,
                     hipStream_t st);
void launch_scan_hist(const unsigned int* hist, int nkeys, int64_t* begin,
                      unsigned long long* cursor, hipStream_t st);
void launch_root_scatter(const uint4* words, const uint16_t* keys, int64_t n, int nkeys,
                         unsigned long long* cursor, uint4* W0, int32_t* I0, int n_cus, hipStream_t st);
void launch_roots(const int64_t* begin, int nkeys, int w, int leaf_size, const BuildDev& d,
                  hipStream_t st);
// A split round reads its sizes on the device (*d.cur_count nodes, the
// chunk count that k_make_chunks writes), so rounds queue back to back with
// no host turnaround; a round with no nodes does nothing.  After an overflow
// (*d.overflow != 0) every later round does nothing.
void launch_make_chunks(const BuildDev& d, int chunk, Chunk* out, int cap, int* out_count,
                        int* out_overflow, hipStream_t st);
void launch_round_count(const Chunk* chunks, const int* n_chunks, int cap, const BuildDev& d,
                        int w, int card_bits, int blocks, hipStream_t st);
void launch_round_decide(int w, int card_bits, int leaf_size, const BuildDev& d, hipStream_t st);
void launch_round_scatter(const Chunk* chunks, const int* n_chunks, int cap, const BuildDev& d,
                          int card_bits, int blocks, hipStream_t st);
void launch_leaf_records(const BuildDev& d, int n_leaves, int64_t* leaf_begin, int64_t* leaf_end,
                         uint4* leaf_sym, uint4* leaf_bits, int* leaf_buf, hipStream_t st);
void launch_leaf_sort(int n_leaves, const int64_t* leaf_begin, const int64_t* leaf_end,
                      const int* leaf_buf, const int32_t* I0, const int32_t* I1, int32_t* perm,
                      hipStream_t st);
void launch_leaf_sort_global(int64_t b, int cnt, int p2, const int32_t* I, int32_t* scratch,
                             int32_t* perm, hipStream_t st);
// out[0] = largest leaf, out[1] = leaves over kLeafSortMax; out zero on entry
void launch_leaf_stats(const int64_t* leaf_begin, const int64_t* leaf_end, int n_leaves, int* out,
                       hipStream_t st);
// The query's shard-major leaf table and work-chunk offsets (kShards shards,
// leaf l in shard l % kShards); *n_chunks = shard_off[kShards].
void launch_shard_layout(const int64_t* leaf_begin, const int64_t* leaf_end, const uint4* leaf_sym,
                         const uint4* leaf_bits, int n_leaves, int* shard_off, int* leaf_sh_off,
                         int* n_chunks, uint4* sh_sym, uint4* sh_bits, int2* sh_rng, hipStream_t st);
void launch_make_tree(const NodeDev* nodes, int n_nodes, int card_bits, int4* tree, hipStream_t st);
void launch_windows(const float* series, int64_t n, int len, int stride, float* rows, hipStream_t st);
void launch_store_inplace(float* raw, int64_t n, int len, const int32_t* perm, const float2* musd,
                          const uint4* words, uint4* words_sorted, int raw_mode, hipStream_t st);
void launch_gather_store(const float* raw, int64_t n, int len, const int32_t* perm,
                         const float2* musd, const uint4* words, float* Z, uint4* words_sorted,
                         hipStream_t st);

}  // namespace messi
