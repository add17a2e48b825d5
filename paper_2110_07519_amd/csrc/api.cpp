// libmessi C ABI: index build and exact k-NN queries on one gfx950 GPU.
// Host side only orchestrates: it sizes buffers, launches the kernels of
// build.hip and query.hip on the index's stream, and reads back the few
// counters that decide how many split rounds or reruns are needed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/messi.h"
#include "build.h"
#include "query.h"

using namespace messi;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

struct HipError {
  hipError_t e;
  const char* what;
};

#define HIP_OR_THROW(x)                         \
  do {                                          \
    hipError_t _e = (x);                        \
    if (_e != hipSuccess) throw HipError{_e, #x}; \
  } while (0)

struct OomError {
  size_t bytes;
};

// Device allocation owned by a vector of frees.
struct DevMem {
  std::vector<void*> ptrs;
  size_t bytes = 0;
  template <typename T>
  T* alloc(size_t count) {
    void* p = nullptr;
    const size_t b = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw OomError{b};
    }
    ptrs.push_back(p);
    bytes += b;
    return static_cast<T*>(p);
  }
  void release(void* p) {
    auto it = std::find(ptrs.begin(), ptrs.end(), p);
    if (it != ptrs.end()) {
      (void)hipFree(p);
      ptrs.erase(it);
    }
  }
  void clear() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
    bytes = 0;
  }
  ~DevMem() { clear(); }
};

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  std::memset(&a, 0, sizeof(a));
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// --- Breakpoints: Phi^-1(k / 2^b).  Acklam's rational approximation of the
// normal quantile, refined by two Halley steps on erfc, rounded to FP32; the
// upper half from the lower by symmetry of N(0,1).
double norm_quantile(double p) {
  static const double a[] = {-3.969683028665376e+01, 2.209460984245205e+02, -2.759285104469687e+02,
                             1.383577518672690e+02,  -3.066479806614716e+01, 2.506628277459239e+00};
  static const double b[] = {-5.447609879822406e+01, 1.615858368580409e+02, -1.556989798598866e+02,
                             6.680131188771972e+01,  -1.328068155288572e+01};
  static const double c[] = {-7.784894002430293e-03, -3.223964580411365e-01, -2.400758277161838e+00,
                             -2.549732539343734e+00, 4.374664141464968e+00,  2.938163982698783e+00};
  static const double d[] = {7.784695709041462e-03, 3.224671290700398e-01, 2.445134137142996e+00,
                             3.754408661907416e+00};
  if (p > 0.5) return -norm_quantile(1.0 - p);
  if (p == 0.5) return 0.0;
  double x;
  if (p < 0.02425) {
    const double q = std::sqrt(-2.0 * std::log(p));
    x = (((((c[0] * q + c[1]) * q + c[2]) * q + c[3]) * q + c[4]) * q + c[5]) /
        ((((d[0] * q + d[1]) * q + d[2]) * q + d[3]) * q + 1.0);
  } else {
    const double q = p - 0.5, r = q * q;
    x = (((((a[0] * r + a[1]) * r + a[2]) * r + a[3]) * r + a[4]) * r + a[5]) * q /
        (((((b[0] * r + b[1]) * r + b[2]) * r + b[3]) * r + b[4]) * r + 1.0);
  }
  for (int it = 0; it < 2; ++it) {
    const double e = 0.5 * std::erfc(-x / std::sqrt(2.0)) - p;
    const double u = e * std::sqrt(2.0 * M_PI) * std::exp(0.5 * x * x);
    x = x - u / (1.0 + 0.5 * x * u);
  }
  return x;
}

void breakpoints(int card_bits, float* beta) {
  const int card = 1 << card_bits;
  for (int k = 1; k < card; ++k) beta[k - 1] = (float)norm_quantile((double)k / (double)card);
}

int log2_exact(int v) {
  int b = 0;
  while ((1 << b) < v) ++b;
  return (1 << b) == v ? b : -1;
}

// Per-call query buffers, grown on demand and reused.
struct Workspace {
  DevMem mem;
  int nq = 0, k = 0, len = 0, w = 0, card = 0, log_cap = 0, L = 0;
  QueryState qs{};
};

// Everything one in-flight call needs besides the index: its stream, the
// query workspace, the batch maps and screen buffers, timing events and the
// near-tie log capacity.  An index owns one for its own calls; a server
// owns one per worker, so batches on different workers run concurrently.
struct QueryCtx {
  hipStream_t stream = nullptr;
  Workspace ws;
  DevMem batch_mem;
  int batch_nq = 0;
  int* bmap = nullptr;
  int* bk = nullptr;
  uint16_t* qb = nullptr;
  float* qn = nullptr;
  int* cnt = nullptr;
  int64_t* off = nullptr;
  int* lists = nullptr;
  int* counter = nullptr;
  unsigned long long* tally = nullptr;
  int log_cap = 4096;
  int proc_blocks_ed = 0;  // cached occupancy of the ED process kernel
  hipEvent_t ev[5] = {};
  bool events_ready = false;
  int* h_status = nullptr;  // per-query status words in pinned, device-mapped host memory
  int* d_status = nullptr;  // their device address
  int h_status_cap = 0;

  QueryCtx() = default;
  QueryCtx(const QueryCtx&) = delete;
  QueryCtx& operator=(const QueryCtx&) = delete;
  ~QueryCtx() {
    if (events_ready)
      for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    if (h_status) (void)hipHostFree(h_status);
  }
};

}  // namespace

struct messi_index {
  int64_t n = 0;
  int len = 0, w = 0, card_bits = 0, leaf_size = 0;
  int n_leaves = 0, n_nodes = 0;
  int64_t max_leaf = 0;
  DevMem mem;
  float* Z = nullptr;
  uint4* words = nullptr;
  int32_t* perm = nullptr;
  int64_t* leaf_begin = nullptr;
  int64_t* leaf_end = nullptr;
  uint4* leaf_sym = nullptr;
  uint4* leaf_bits = nullptr;
  float* bp = nullptr;
  NodeDev* nodes = nullptr;
  int4* tree = nullptr;
  int* root_node = nullptr;
  bool inplace = false;      // Z is the caller's buffer, normalised in place, rows in id order
  bool raw = false;          // series indexed as given, without z-normalisation
  float xnorm = 0.0f;        // largest 2-norm of a stored row, rounded up
  DevMem own;                // rows the index materialised itself (sliding windows)
  int* shard_off = nullptr;  // [kShards + 1] first chunk of each shard
  int64_t n_chunks = 0;
  uint4* sh_sym = nullptr;   // leaf table in shard-major order
  uint4* sh_bits = nullptr;
  int2* sh_rng = nullptr;
  int* leaf_sh_off = nullptr;  // [kShards + 1] first shard-major leaf of each shard
  // BF16 screen: shadow of Z and squared row norms, built on first use
  DevMem screen_mem;
  uint16_t* Zb = nullptr;
  float* xn = nullptr;
  int n_cus = 0;
  size_t lds_max = 64 * 1024;  // LDS a block may use on this device
  std::mutex screen_mu;  // first-use construction of the BF16 copy
  QueryCtx ctx;  // the index's own calls (messi_query, messi_query_batch)
  std::atomic<int> busy{0};

  IndexDev view() const {
    IndexDev v;
    v.n = n;
    v.len = len;
    v.w = w;
    v.m = len / w;
    v.card_bits = card_bits;
    v.n_leaves = n_leaves;
    v.Z = Z;
    v.zrow = inplace ? perm : nullptr;
    v.words = words;
    v.perm = perm;
    v.leaf_begin = leaf_begin;
    v.leaf_end = leaf_end;
    v.leaf_sym = leaf_sym;
    v.leaf_bits = leaf_bits;
    v.bp = bp;
    v.tree = tree;
    v.root_node = root_node;
    v.shard_off = shard_off;
    v.sh_sym = sh_sym;
    v.sh_bits = sh_bits;
    v.sh_rng = sh_rng;
    v.leaf_sh_off = leaf_sh_off;
    return v;
  }
};

namespace {

struct BusyGuard {
  std::atomic<int>& f;
  bool ok;
  explicit BusyGuard(std::atomic<int>& flag) : f(flag) {
    int z = 0;
    ok = f.compare_exchange_strong(z, 1);
  }
  ~BusyGuard() {
    if (ok) f.store(0);
  }
};

template <typename T>
void h2d(T* dst, const T* src, size_t count, hipStream_t st) {
  HIP_OR_THROW(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, st));
}
template <typename T>
void d2h(T* dst, const T* src, size_t count, hipStream_t st) {
  HIP_OR_THROW(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyDeviceToHost, st));
  HIP_OR_THROW(hipStreamSynchronize(st));
}

void launch_check() { HIP_OR_THROW(hipGetLastError()); }

// The build proper; throws HipError / OomError.  Returns false if the node
// or leaf tables were too small (caller retries with larger ones).
bool build_index(messi_index* ix, const float* series, int node_cap, int leaf_cap) {
  const int64_t n = ix->n;
  const int len = ix->len, w = ix->w, cb = ix->card_bits, card = 1 << cb;
  const int nkeys = 1 << w;
  hipStream_t st = ix->ctx.stream;
  DevMem tmp;

  // breakpoints with open ends
  std::vector<float> bph(card + 1);
  bph[0] = -INFINITY;
  breakpoints(cb, bph.data() + 1);
  bph[card] = INFINITY;
  ix->bp = ix->mem.alloc<float>(card + 1);
  h2d(ix->bp, bph.data(), card + 1, st);

  // (1) summaries
  uint4* words_id = tmp.alloc<uint4>(n);
  float2* musd = tmp.alloc<float2>(n);
  unsigned int* hist = tmp.alloc<unsigned int>(nkeys);
  HIP_OR_THROW(hipMemsetAsync(hist, 0, sizeof(unsigned int) * nkeys, st));
  int spw = std::min(64, (16384 - 257) / len);
  if (spw < 1) spw = 1;
  int dev = 0;
  HIP_OR_THROW(hipGetDevice(&dev));
  HIP_OR_THROW(hipDeviceGetAttribute(&ix->n_cus, hipDeviceAttributeMultiprocessorCount, dev));
  {
    int lds = 0;
    HIP_OR_THROW(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    ix->lds_max = (size_t)lds;
  }
  unsigned int* norm2 = nullptr;  // raw: largest squared row norm (FP32 bits)
  if (ix->raw) {
    norm2 = tmp.alloc<unsigned int>(1);
    HIP_OR_THROW(hipMemsetAsync(norm2, 0, sizeof(unsigned int), st));
  }
  launch_summarize(series, n, len, w, cb, spw, ix->bp, words_id, musd, hist, norm2, st, ix->n_cus);
  launch_check();
  {
    // z-normalised rows have |z|^2 = len up to a relative len u; a raw
    // row's squared norm is an FP32 sum of len squares, off by at most the
    // same factor.  2^-10 covers both for len <= 4096.
    float n2 = (float)len;
    if (ix->raw) {
      unsigned int bits = 0;
      d2h(&bits, norm2, 1, st);
      std::memcpy(&n2, &bits, sizeof(n2));
    }
    ix->xnorm = (float)(std::sqrt((double)n2) * (1.0 + std::ldexp(1.0, -10)));
  }

  // (2) root grouping
  int64_t* key_begin = tmp.alloc<int64_t>(nkeys + 1);
  unsigned long long* key_cursor = tmp.alloc<unsigned long long>(nkeys);
  launch_scan_hist(hist, nkeys, key_begin, key_cursor, st);
  BuildDev d{};
  d.W0 = tmp.alloc<uint4>(n);
  d.W1 = tmp.alloc<uint4>(n);
  d.I0 = tmp.alloc<int32_t>(n);
  d.I1 = tmp.alloc<int32_t>(n);
  launch_root_scatter(words_id, n, w, cb, key_cursor, d.W0, d.I0, st);
  launch_check();

  // node and leaf tables
  d.nodes = ix->mem.alloc<NodeDev>(node_cap);
  d.node_cap = node_cap;
  d.leaves = tmp.alloc<int>(leaf_cap);
  d.leaf_cap = leaf_cap;
  d.root_node = ix->mem.alloc<int>(nkeys);
  const int round_cap = (int)std::min<int64_t>(n / (ix->leaf_size + 1) + 1, (int64_t)node_cap);
  d.cur_list = tmp.alloc<int>(round_cap);
  d.next_list = tmp.alloc<int>(round_cap);
  d.round_cap = round_cap;
  int* counters = tmp.alloc<int>(8);  // node_count, leaf_count, next_count, overflow, chunk_count
  HIP_OR_THROW(hipMemsetAsync(counters, 0, sizeof(int) * 8, st));
  d.node_count = counters + 0;
  d.leaf_count = counters + 1;
  d.next_count = counters + 2;
  d.overflow = counters + 3;
  int* chunk_count = counters + 4;
  d.c1 = tmp.alloc<int>((size_t)round_cap * kMaxSeg);
  d.split_seg = tmp.alloc<int>(round_cap);
  d.cursor = tmp.alloc<unsigned long long>((size_t)round_cap * 2);
  const int chunk_cap = (int)std::min<int64_t>(n / kChunk + round_cap + 1, (int64_t)1 << 30);
  Chunk* chunks = tmp.alloc<Chunk>(chunk_cap);

  // the next_list of launch_roots becomes the first round's list
  launch_roots(key_begin, nkeys, w, ix->leaf_size, d, st);
  launch_check();

  int hc[8];
  d2h(hc, counters, 8, st);
  if (hc[3]) return false;
  int n_cur = hc[2];
  // (3) split rounds
  for (int round = 0; n_cur > 0; ++round) {
    if (round > 16 * 8 + 8) throw HipError{hipErrorUnknown, "split rounds did not converge"};
    std::swap(d.cur_list, d.next_list);
    HIP_OR_THROW(hipMemsetAsync(d.next_count, 0, sizeof(int), st));
    HIP_OR_THROW(hipMemsetAsync(d.c1, 0, sizeof(int) * (size_t)n_cur * kMaxSeg, st));
    launch_make_chunks(d, n_cur, kChunk, chunks, chunk_cap, chunk_count, st);
    launch_check();
    int n_chunks = 0;
    d2h(&n_chunks, chunk_count, 1, st);
    if (n_chunks > chunk_cap) throw HipError{hipErrorUnknown, "chunk table overflow"};
    launch_round_count(chunks, n_chunks, d, w, cb, st);
    launch_round_decide(n_cur, w, cb, ix->leaf_size, d, st);
    launch_round_scatter(chunks, n_chunks, d, cb, st);
    launch_check();
    d2h(hc, counters, 8, st);
    if (hc[3]) return false;
    n_cur = hc[2];
  }
  const int n_leaves = hc[1];
  ix->n_nodes = hc[0];
  ix->n_leaves = n_leaves;

  // (4) leaf records, ids sorted inside each leaf
  ix->leaf_begin = ix->mem.alloc<int64_t>(n_leaves);
  ix->leaf_end = ix->mem.alloc<int64_t>(n_leaves);
  ix->leaf_sym = ix->mem.alloc<uint4>(n_leaves);
  ix->leaf_bits = ix->mem.alloc<uint4>(n_leaves);
  int* leaf_buf = tmp.alloc<int>(n_leaves);
  launch_leaf_records(d, n_leaves, ix->leaf_begin, ix->leaf_end, ix->leaf_sym, ix->leaf_bits,
                      leaf_buf, st);
  ix->perm = ix->mem.alloc<int32_t>(n);
  launch_leaf_sort(n_leaves, ix->leaf_begin, ix->leaf_end, leaf_buf, d.I0, d.I1, ix->perm, st);
  launch_check();
  std::vector<int64_t> hb(n_leaves), he(n_leaves);
  std::vector<int> hbuf(n_leaves);
  d2h(hb.data(), ix->leaf_begin, n_leaves, st);
  d2h(he.data(), ix->leaf_end, n_leaves, st);
  d2h(hbuf.data(), leaf_buf, n_leaves, st);
  int64_t maxl = 0;
  int32_t* sort_scratch = nullptr;
  for (int l = 0; l < n_leaves; ++l) {
    const int64_t c = he[l] - hb[l];
    maxl = std::max(maxl, c);
    if (c > kLeafSortMax) {
      int p2 = 1;
      while (p2 < c) p2 <<= 1;
      if (!sort_scratch) {
        int64_t big = 1;
        for (int j = 0; j < n_leaves; ++j) big = std::max<int64_t>(big, he[j] - hb[j]);
        int64_t pb = 1;
        while (pb < big) pb <<= 1;
        sort_scratch = tmp.alloc<int32_t>(pb);
      }
      launch_leaf_sort_global(hb[l], (int)c, p2, hbuf[l] ? d.I1 : d.I0, sort_scratch, ix->perm, st);
      launch_check();
    }
  }
  ix->max_leaf = maxl;
  // keep only what queries need
  tmp.release(d.W0);
  tmp.release(d.W1);

  // (5) leaf-ordered words and z-normalised store (a leaf-ordered copy, or
  // the caller's rows normalised in place)
  ix->words = ix->mem.alloc<uint4>(n);
  if (ix->inplace) {
    ix->Z = const_cast<float*>(series);
    launch_store_inplace(const_cast<float*>(series), n, len, ix->perm, musd, words_id, ix->words,
                         ix->raw ? 1 : 0, st);
  } else {
    ix->Z = ix->mem.alloc<float>((size_t)n * len);
    launch_gather_store(series, n, len, ix->perm, musd, words_id, ix->Z, ix->words, st);
  }
  launch_check();
  ix->nodes = d.nodes;
  ix->root_node = d.root_node;
  ix->tree = ix->mem.alloc<int4>(ix->n_nodes);
  launch_make_tree(d.nodes, ix->n_nodes, cb, ix->tree, st);
  launch_check();
  // chunk layout of the query's leaf order: leaf l in shard l % kShards,
  // each shard's chunks contiguous
  {
    const int L = ix->n_leaves;
    std::vector<int64_t> lb(L), le(L);
    d2h(lb.data(), ix->leaf_begin, L, st);
    d2h(le.data(), ix->leaf_end, L, st);
    std::vector<int> off(kShards + 1, 0);
    for (int l = 0; l < L; ++l)
      off[l % kShards + 1] += (int)((le[l] - lb[l] + kChunkSeries - 1) / kChunkSeries);
    for (int sh = 0; sh < kShards; ++sh) off[sh + 1] += off[sh];
    ix->n_chunks = off[kShards];
    ix->shard_off = ix->mem.alloc<int>(kShards + 1);
    h2d(ix->shard_off, off.data(), kShards + 1, st);
    // the leaf table again in shard-major order (shard s: leaves s, s + 64,
    // ...), read contiguously by the per-shard bound blocks
    std::vector<uint4> sy(L), bi(L), shs(L), shb(L);
    std::vector<int2> shr(L);
    std::vector<int> loff(kShards + 1, 0);
    d2h(sy.data(), ix->leaf_sym, L, st);
    d2h(bi.data(), ix->leaf_bits, L, st);
    for (int sh = 0; sh < kShards; ++sh) loff[sh + 1] = loff[sh] + (sh < L ? (L - sh + kShards - 1) / kShards : 0);
    for (int l = 0; l < L; ++l) {
      const int j = loff[l % kShards] + l / kShards;
      shs[j] = sy[l];
      shb[j] = bi[l];
      shr[j] = make_int2((int)lb[l], (int)le[l]);
    }
    ix->sh_sym = ix->mem.alloc<uint4>(L);
    ix->sh_bits = ix->mem.alloc<uint4>(L);
    ix->sh_rng = ix->mem.alloc<int2>(L);
    ix->leaf_sh_off = ix->mem.alloc<int>(kShards + 1);
    h2d(ix->sh_sym, shs.data(), L, st);
    h2d(ix->sh_bits, shb.data(), L, st);
    h2d(ix->sh_rng, shr.data(), L, st);
    h2d(ix->leaf_sh_off, loff.data(), kShards + 1, st);
    HIP_OR_THROW(hipStreamSynchronize(st));  // the host vectors are pageable memory
  }
  return true;
}

// Grow the query workspace to hold (nq, k) with the current log capacity.
void ensure_workspace(messi_index* ix, QueryCtx& c, int nq, int k) {
  Workspace& ws = c.ws;
  const int card = 1 << ix->card_bits;
  if (ws.nq >= nq && ws.k >= k && ws.log_cap >= c.log_cap && ws.L == ix->n_leaves &&
      ws.len == ix->len)
    return;
  const int NQ = std::max(nq, ws.nq), K = std::max(k, ws.k), LC = c.log_cap;
  ws.mem.clear();
  ws = Workspace{};
  QueryState& s = ws.qs;
  const int len = ix->len, L = ix->n_leaves;
  s.zq = ws.mem.alloc<float>((size_t)NQ * len);
  s.eta = ws.mem.alloc<float>(NQ);
  s.upper = ws.mem.alloc<float>((size_t)NQ * len);
  s.lower = ws.mem.alloc<float>((size_t)NQ * len);
  s.paa = ws.mem.alloc<float>((size_t)NQ * 3 * kMaxSeg);
  s.approx_range = ws.mem.alloc<int64_t>((size_t)NQ * 2);
  s.approx_d2 = ws.mem.alloc<float>((size_t)NQ * kApproxCap);
  s.slots = ws.mem.alloc<unsigned long long>((size_t)NQ * K);
  s.log = ws.mem.alloc<unsigned long long>((size_t)NQ * LC);
  s.log_count = ws.mem.alloc<int>(NQ);
  s.leaf_lb = ws.mem.alloc<float>((size_t)NQ * L);
  const int64_t item_cap = ix->n_chunks;
  s.items = ws.mem.alloc<unsigned long long>((size_t)NQ * item_cap);
  s.ranges = ws.mem.alloc<int2>((size_t)NQ * item_cap);
  s.next = ws.mem.alloc<int>((size_t)NQ * kCounterInts);
  s.stats = ws.mem.alloc<unsigned long long>((size_t)NQ * kStatCount);
  s.status = ws.mem.alloc<int>(NQ);
  ws.nq = NQ;
  ws.k = K;
  ws.len = len;
  ws.w = ix->w;
  ws.card = card;
  ws.log_cap = LC;
  ws.L = L;
}

// BF16 shadow of the store (screen operand) and the squared row norms.
void ensure_screen(messi_index* ix) {
  std::lock_guard<std::mutex> lk(ix->screen_mu);
  if (ix->Zb) return;
  ix->Zb = ix->screen_mem.alloc<uint16_t>((size_t)ix->n * ix->len);
  ix->xn = ix->screen_mem.alloc<float>((size_t)ix->n);
  launch_bf16_rows(ix->Z, ix->inplace ? ix->perm : nullptr, ix->n, ix->len, ix->Zb, ix->xn,
                   ix->ctx.stream);
  launch_check();
  HIP_OR_THROW(hipStreamSynchronize(ix->ctx.stream));
}

// Batch maps (row and k of each query) and screen buffers for nq queries.
void ensure_batch(messi_index* ix, QueryCtx& c, int nq) {
  if (c.batch_nq >= nq) return;
  c.batch_mem.clear();
  const int L = ix->n_leaves;
  c.bmap = c.batch_mem.alloc<int>(nq);
  c.bk = c.batch_mem.alloc<int>(nq);
  c.qb = c.batch_mem.alloc<uint16_t>((size_t)nq * ix->len);
  c.qn = c.batch_mem.alloc<float>(nq);
  c.cnt = c.batch_mem.alloc<int>(L);
  c.off = c.batch_mem.alloc<int64_t>((size_t)L + 1);
  c.lists = c.batch_mem.alloc<int>((size_t)nq * L);
  c.counter = c.batch_mem.alloc<int>(1);
  c.tally = c.batch_mem.alloc<unsigned long long>(2);
  c.batch_nq = nq;
}

// One group of queries sharing a distance and window: nq queries whose rows
// (input and output) are d_qmap[i] and whose k are d_kq[i] (both null for a
// plain call: rows 0..nq-1, every k = kmax).  Slots are kmax apart and
// output rows out_stride = kmax entries long.
// Query state laid out in caller-provided device memory (the allocation-free
// entry point): the state, its near-tie log capacity, and a host buffer of
// nq status words.
struct FixedScratch {
  QueryState qs;
  int log_cap;
  int* h_status;
};

int run_group(messi_index* ix, QueryCtx& c, const float* queries, int nq, int kmax, int distance,
              int window, const int* d_kq, const int* d_qmap, bool screen, bool lb_improved,
              int64_t* out_ids, float* out_dists, messi_stats* stats,
              const FixedScratch* fixed = nullptr, bool min_work = false) {
  hipStream_t st = c.stream;
  const int len = ix->len;
  const double u = std::ldexp(1.0, -24);
  QueryParams p{};
  p.nq = nq;
  p.len = len;
  p.w = ix->w;
  p.m = len / ix->w;
  p.card_bits = ix->card_bits;
  p.k = kmax;
  p.out_stride = kmax;
  p.order_leaves = screen ? 0 : 1;
  p.count_work = stats ? 1 : 0;
  // the approximate leaf: found by stage1's approximate blocks for a few
  // queries (shorter prep), once per query in k_prep for batches
  p.leaf_in_prep = nq > 8 ? 1 : 0;
  p.distance = distance;
  p.window = distance == MESSI_DTW ? std::min(window, len - 1) : 0;
  p.n_leaves = ix->n_leaves;
  p.n = ix->n;
  p.item_cap = (int)ix->n_chunks;
  // FP32 error of a refined squared distance: at most rho relative, with
  // rho = (4 len + 64) u covering ED's pairwise sums and DTW's paths of up
  // to 2 len - 1 terms.
  const double rho = (4.0 * len + 64.0) * u;
  p.win = std::nextafter((float)((1.0 + rho) / (1.0 - rho) * (1.0 + std::ldexp(1.0, -20))), INFINITY);
  p.lb_rel = std::nextafter((float)((1.0 + rho) * (1.0 + std::ldexp(1.0, -16))), INFINITY);
  // PAA rounding: a segment mean of a row v is off by at most
  // 2 u sqrt(m) |v|, so a bound moves by at most 2 u sqrt(len m) (|x| + |q|)
  // (series side plus query side); eta_c carries an 8x margin and k_prep
  // completes eta with the query's own norm.
  p.eta_c = (float)(16.0 * u * std::sqrt((double)len * p.m));
  p.xnorm = ix->xnorm;
  p.raw = ix->raw ? 1 : 0;
  // bucket range [2^-16, 2^16) against bounds up to (2 |x|max)^2: a raw
  // index scales them so that the largest possible bound lands near 2^16
  p.lb_scale = 1.0f;
  if (ix->raw && ix->xnorm > 0.0f) {
    const int e = (int)std::ceil(std::log2(4.0 * (double)ix->xnorm * ix->xnorm));
    p.lb_scale = (float)std::ldexp(1.0, std::max(-100, std::min(100, 16 - e)));
  }
  // LDS: the kernels prefer 64 KB (occupancy); longer series may use up
  // to what a block can have on this device (160 KB on gfx950), less 4 KB
  // for the kernels' static shared variables
  const size_t lds_max = ix->lds_max - 4096;
  int fin_waves = 0;
  if (distance == MESSI_DTW) {
    fin_waves = 1;
    for (int fw = 4; fw >= 1; --fw) {
      p.fin_waves = fw;
      if (finalize_lds_bytes(p) <= 64 * 1024) {
        fin_waves = fw;
        break;
      }
    }
  }
  p.fin_waves = fin_waves;
  // LB_Improved only filters: where its projection buffers do not fit the
  // process kernel's LDS, the queries run with LB_Keogh alone
  p.lb_improved = (lb_improved && distance == MESSI_DTW) ? 1 : 0;
  if (p.lb_improved && process_lds_bytes(p) > lds_max) p.lb_improved = 0;
  const size_t proc_lds = process_lds_bytes(p) + process_lds_static(p);
  if (proc_lds > ix->lds_max || finalize_lds_bytes(p) > lds_max || stage1_lds_bytes(p) > lds_max)
    return fail(MESSI_EINVAL, "series length %d too long for the query kernels (window %d)", len,
                p.window);

  int per_cu = 0;
  if (distance == MESSI_DTW) {
    per_cu = process_blocks_per_cu(p);
  } else {
    if (c.proc_blocks_ed == 0) c.proc_blocks_ed = process_blocks_per_cu(p);
    per_cu = c.proc_blocks_ed;
  }
  const int resident = per_cu * ix->n_cus;
  int blocks = resident / std::max(1, nq);
  blocks = std::max(2, std::min(blocks, resident));
  if (distance == MESSI_ED) blocks = ed_process_blocks(resident);  // the whole grid visits every query
  ScreenDev sc{};
  if (screen) {
    sc.Zb = ix->Zb;
    sc.xn = ix->xn;
    sc.qb = c.qb;
    sc.qn = c.qn;
    sc.cnt = c.cnt;
    sc.off = c.off;
    sc.lists = c.lists;
    sc.counter = c.counter;
    sc.tally = c.tally;
    // bound constants (see the screen kernel): u_b = 2^-8, gamma at 2^-23
    const double ub = std::ldexp(1.0, -8);
    const double g = len * std::ldexp(1.0, -23) / (1.0 - len * std::ldexp(1.0, -23));
    const double cdot = 2.0 * ((2.0 * ub + ub * ub) + g * (1.0 + ub) * (1.0 + ub)) * (1.0 + std::ldexp(1.0, -10));
    sc.c_dot = std::nextafter((float)cdot, INFINITY);
    sc.c_abs = (float)std::ldexp(1.0, -17);
  }
  const int screen_blocks = screen ? screen_blocks_per_cu(len) * ix->n_cus : 0;
  // the status words live in pinned host memory the kernels write through
  // its device mapping, so no copy follows the kernels
  if (!fixed && c.h_status_cap < nq) {
    if (c.h_status) HIP_OR_THROW(hipHostFree(c.h_status));
    c.h_status = nullptr;
    c.d_status = nullptr;
    c.h_status_cap = 0;
    HIP_OR_THROW(hipHostMalloc((void**)&c.h_status, sizeof(int) * (size_t)nq, hipHostMallocMapped));
    HIP_OR_THROW(hipHostGetDevicePointer((void**)&c.d_status, c.h_status, 0));
    c.h_status_cap = nq;
  }
  // phase timing (only when the caller asks for statistics)
  hipEvent_t ev[5] = {};
  if (stats) {
    if (!c.events_ready) {
      for (int i = 0; i < 5; ++i) HIP_OR_THROW(hipEventCreate(&c.ev[i]));
      c.events_ready = true;
    }
    for (int i = 0; i < 5; ++i) ev[i] = c.ev[i];
  }
  for (int attempt = 0; attempt < 8; ++attempt) {
    if (!fixed) ensure_workspace(ix, c, nq, kmax);
    p.log_cap = fixed ? fixed->log_cap : c.log_cap;
    const IndexDev v = ix->view();
    QueryState qs = fixed ? fixed->qs : c.ws.qs;
    int* h_status = fixed ? fixed->h_status : c.h_status;
    if (!fixed) qs.status = c.d_status;
    qs.kq = d_kq;
    qs.qmap = d_qmap;
    if (stats) HIP_OR_THROW(hipEventRecord(ev[0], st));
    launch_prep(v, queries, p, qs, st);
    if (stats) HIP_OR_THROW(hipEventRecord(ev[1], st));
    launch_stage1(v, p, qs, st);
    if (stats) HIP_OR_THROW(hipEventRecord(ev[2], st));
    if (screen) {
      launch_bf16_rows(qs.zq, nullptr, nq, len, sc.qb, sc.qn, st);
      launch_screen(v, p, qs, sc, screen_blocks, st);
    } else {
      launch_process(v, p, qs, blocks, st);
    }
    if (stats) HIP_OR_THROW(hipEventRecord(ev[3], st));
    launch_finalize(v, p, qs, out_ids, out_dists, st);
    if (stats) {
      HIP_OR_THROW(hipEventRecord(ev[4], st));
      // the minimal work, once the final k-th best is known (untimed)
      if (min_work) launch_min_work(v, p, qs, std::max(1, ix->n_cus), st);
    }
    launch_check();
    if (fixed)
      d2h(h_status, qs.status, nq, st);
    else
      HIP_OR_THROW(hipStreamSynchronize(st));
    int worst = 0;
    for (int i = 0; i < nq; ++i) worst |= h_status[i];
    if (!(worst & 1)) {
      if (stats) {
        float ms[4] = {0, 0, 0, 0};
        for (int i = 0; i < 4; ++i) HIP_OR_THROW(hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]));
        stats->us_prep += 1e3 * ms[0];
        stats->us_stage1 += 1e3 * ms[1];
        stats->us_process += 1e3 * ms[2];
        stats->us_finalize += 1e3 * ms[3];
        std::vector<unsigned long long> sv((size_t)nq * kStatCount);
        d2h(sv.data(), qs.stats, sv.size(), st);
        stats->queries += nq;
        stats->leaves_total += (int64_t)nq * ix->n_leaves;
        for (int q = 0; q < nq; ++q) {
          const unsigned long long* r = &sv[(size_t)q * kStatCount];
          stats->leaves_kept += (int64_t)r[kStatLeavesKept];
          stats->series_lb += (int64_t)r[kStatSeriesLb];
          stats->lb_keogh += (int64_t)r[kStatLbKeogh];
          stats->refined += (int64_t)r[kStatRefined];
          stats->rechecked_fp64 += (int64_t)r[kStatRecheck];
          stats->lb_improved += (int64_t)r[kStatLbImproved];
          stats->bsf_updates += (int64_t)r[kStatBsf];
          stats->dtw_cells += (int64_t)r[kStatCells];
          stats->min_leaves += (int64_t)r[kStatMinLeaves];
          stats->min_series += (int64_t)r[kStatMinSeries];
          stats->min_refined += (int64_t)r[kStatMinRefined];
        }
        if (screen) {
          unsigned long long t[2];
          int64_t pairs = 0;
          d2h(t, sc.tally, 2, st);
          d2h(&pairs, sc.off + ix->n_leaves, 1, st);
          stats->screened += (int64_t)t[0];
          stats->leaves_kept += pairs;
        }
      }
      return MESSI_OK;
    }
    if (stats) stats->log_overflows += 1;
    if (fixed)  // no room to grow the log: the caller falls back to messi_query
      return fail(MESSI_ENOMEM, "near-tie log of %d entries per query overflowed in the fixed scratch",
                  fixed->log_cap);
    c.log_cap *= 4;  // near-tie log overflowed: rerun with a larger one
  }
  return fail(MESSI_ENOMEM, "near-tie log kept overflowing");
}

int run_query(messi_index* ix, const float* queries, int nq, int k, int distance, int window,
              int64_t* out_ids, float* out_dists, messi_stats* stats) {
  return run_group(ix, ix->ctx, queries, nq, k, distance, window, nullptr, nullptr, false, false, out_ids,
                   out_dists, stats, nullptr, true);
}

constexpr int kScreenMinGroup = 32;  // fewer ED queries go the unscreened way

// Validated batch on one query context: groups of queries sharing
// (distance, effective window), in first-seen order, one run_group each.
int run_batch(messi_index* index, QueryCtx& ctx, const float* queries, int nq, const int32_t* k,
              const int32_t* distance, const int32_t* window, int kmax, int flags,
              int64_t* out_ids, float* out_dists, messi_stats* stats) {
  const int len = index->len;
  std::vector<std::pair<int, int>> keys;
  std::vector<std::vector<int>> members;
  for (int i = 0; i < nq; ++i) {
    const std::pair<int, int> key(distance[i], distance[i] == MESSI_DTW ? std::min(window[i], len - 1) : 0);
    size_t g = 0;
    while (g < keys.size() && keys[g] != key) ++g;
    if (g == keys.size()) {
      keys.push_back(key);
      members.emplace_back();
    }
    members[g].push_back(i);
  }
  try {
    const bool want_screen = (flags & MESSI_SCREEN_BF16) && screen_supported(len);
    ensure_batch(index, ctx, nq);
    std::vector<int> hmap, hk;
    hmap.reserve(nq);
    hk.reserve(nq);
    for (const auto& m : members)
      for (int i : m) {
        hmap.push_back(i);
        hk.push_back(k[i]);
      }
    h2d(ctx.bmap, hmap.data(), (size_t)nq, ctx.stream);
    h2d(ctx.bk, hk.data(), (size_t)nq, ctx.stream);
    int at = 0;
    for (size_t g = 0; g < keys.size(); ++g) {
      const int cnt = (int)members[g].size();
      // the screen streams every leaf some query of the group keeps, so it
      // pays off only when many queries share that pass
      const bool screen = want_screen && keys[g].first == MESSI_ED && cnt >= kScreenMinGroup;
      if (screen && !index->Zb) return fail(MESSI_EINVAL, "the BF16 screen copy is not prepared");
      const int rc = run_group(index, ctx, queries, cnt, kmax, keys[g].first, keys[g].second,
                               ctx.bk + at, ctx.bmap + at, screen, (flags & MESSI_LB_IMPROVED) != 0,
                               out_ids, out_dists, stats);
      if (rc != MESSI_OK) return rc;
      at += cnt;
    }
  } catch (const OomError& e) {
    return fail(MESSI_ENOMEM, "device allocation of %zu bytes failed", e.bytes);
  } catch (const HipError& e) {
    return fail(MESSI_EDEVICE, "%s: %s", e.what, hipGetErrorString(e.e));
  }
  return MESSI_OK;
}

// ---------------------------------------------------------------------------
// Serving loop.  Requests (one raw query each, its k, distance and window)
// are queued on the host; every worker owns a query context (stream,
// workspace, device I/O buffers, pinned staging) and repeatedly takes the
// pending requests that fit - at most its batch capacity, and only while
// the device bytes held by admitted, unfinished requests stay within the
// budget - runs them as one batch, and posts the results.  Requests that
// arrive while a batch is on the GPU are taken by the next free worker, so
// batches overlap on the device and a batch is formed from whatever has
// arrived (continuous batching).

using Clock = std::chrono::steady_clock;

struct SrvRequest {
  uint64_t id;
  int k, distance, window;
  std::vector<float> q;
  Clock::time_point t_submit;
  int64_t bytes;
};

struct SrvResult {
  uint64_t id;
  int status;
  std::vector<int64_t> ids;
  std::vector<float> dists;
  double latency_us;
};

struct SrvWorker {
  QueryCtx ctx;
  int cap = 0;
  float* d_q = nullptr;
  int64_t* d_ids = nullptr;
  float* d_d = nullptr;
  float* h_q = nullptr;
  int64_t* h_ids = nullptr;
  float* h_d = nullptr;
  DevMem io;
  std::thread th;
  ~SrvWorker() {
    if (h_q) (void)hipHostFree(h_q);
    if (h_ids) (void)hipHostFree(h_ids);
    if (h_d) (void)hipHostFree(h_d);
    if (ctx.stream) (void)hipStreamDestroy(ctx.stream);
  }
};

// Device bytes one query holds while in flight: its share of the query
// workspace (normalised query, envelope, bound table, approximate-search
// distances, k best, near-tie log, leaf bounds and order, work counters),
// of the batch buffers (maps, BF16 row, leaf lists) and of the I/O buffers.
int64_t request_bytes(const messi_index* ix, int kmax, int log_cap) {
  const int64_t len = ix->len, L = ix->n_leaves, card = (int64_t)1 << ix->card_bits;
  const int64_t item_cap = ix->n_chunks;
  int64_t b = 0;
  b += 3 * len * 4 + 3 * kMaxSeg * 4 + kMaxSeg * card * 4 + 16 + (int64_t)kApproxCap * 4;
  b += (int64_t)kmax * 8 + (int64_t)log_cap * 8 + 4 + L * 4;
  b += item_cap * 16 + (int64_t)kCounterInts * 4 + kStatCount * 8 + 4;
  b += 8 + len * 2 + 4 + L * 4;
  b += len * 4 + (int64_t)kmax * 12;
  return b;
}

}  // namespace

struct messi_server {
  messi_index* ix = nullptr;
  int device = 0;
  int kmax = 64, flags = 0, workers_n = 2, max_batch = 1024;
  int64_t budget = 0, req_bytes = 0;
  std::mutex mu;
  std::condition_variable cv_work;   // new requests, freed memory, stop
  std::condition_variable cv_done;   // new results
  std::deque<SrvRequest> pending;
  std::deque<SrvResult> done;
  int64_t inflight = 0, peak_inflight = 0;
  int64_t submitted = 0, completed = 0, batches = 0, max_batch_seen = 0;
  double busy_us = 0.0;
  uint64_t next_id = 0;
  bool stopping = false;
  std::vector<std::unique_ptr<SrvWorker>> workers;

  void run(SrvWorker* w);
};

namespace {

void server_worker_main(messi_server* S, SrvWorker* w) { S->run(w); }

}  // namespace

void messi_server::run(SrvWorker* w) {
  (void)hipSetDevice(device);
  const int len = ix->len;
  std::vector<SrvRequest> batch;
  std::vector<int32_t> ks, ds, ws;
  for (;;) {
    batch.clear();
    int64_t taken = 0;
    {
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        if (stopping && pending.empty()) return;
        while (!pending.empty() && (int)batch.size() < w->cap &&
               (budget <= 0 || inflight + taken + pending.front().bytes <= budget ||
                (inflight + taken == 0))) {
          taken += pending.front().bytes;
          batch.push_back(std::move(pending.front()));
          pending.pop_front();
        }
        if (!batch.empty()) break;
        cv_work.wait(lk);
      }
      inflight += taken;
      peak_inflight = std::max(peak_inflight, inflight);
      max_batch_seen = std::max<int64_t>(max_batch_seen, (int64_t)batch.size());
      ++batches;
    }
    const int nb = (int)batch.size();
    ks.resize(nb);
    ds.resize(nb);
    ws.resize(nb);
    for (int i = 0; i < nb; ++i) {
      std::memcpy(w->h_q + (size_t)i * len, batch[i].q.data(), sizeof(float) * len);
      ks[i] = batch[i].k;
      ds[i] = batch[i].distance;
      ws[i] = batch[i].window;
    }
    const auto t0 = Clock::now();
    int rc = MESSI_OK;
    std::string err;
    try {
      HIP_OR_THROW(hipMemcpyAsync(w->d_q, w->h_q, sizeof(float) * len * nb, hipMemcpyHostToDevice,
                                  w->ctx.stream));
      rc = run_batch(ix, w->ctx, w->d_q, nb, ks.data(), ds.data(), ws.data(), kmax, flags,
                     w->d_ids, w->d_d, nullptr);
      if (rc == MESSI_OK) {
        HIP_OR_THROW(hipMemcpyAsync(w->h_ids, w->d_ids, sizeof(int64_t) * kmax * nb,
                                    hipMemcpyDeviceToHost, w->ctx.stream));
        HIP_OR_THROW(hipMemcpyAsync(w->h_d, w->d_d, sizeof(float) * kmax * nb,
                                    hipMemcpyDeviceToHost, w->ctx.stream));
        HIP_OR_THROW(hipStreamSynchronize(w->ctx.stream));
      } else {
        err = g_err;
      }
    } catch (const HipError& e) {
      rc = MESSI_EDEVICE;
    } catch (const OomError& e) {
      rc = MESSI_ENOMEM;
    }
    const auto t1 = Clock::now();
    {
      std::lock_guard<std::mutex> lk(mu);
      for (int i = 0; i < nb; ++i) {
        SrvResult r;
        r.id = batch[i].id;
        r.status = rc;
        if (rc == MESSI_OK) {
          r.ids.assign(w->h_ids + (size_t)i * kmax, w->h_ids + (size_t)i * kmax + batch[i].k);
          r.dists.assign(w->h_d + (size_t)i * kmax, w->h_d + (size_t)i * kmax + batch[i].k);
        }
        r.latency_us = std::chrono::duration<double, std::micro>(t1 - batch[i].t_submit).count();
        done.push_back(std::move(r));
      }
      completed += nb;
      inflight -= taken;
      busy_us += std::chrono::duration<double, std::micro>(t1 - t0).count();
    }
    cv_done.notify_all();
    cv_work.notify_all();
  }
}

namespace {
}  // namespace

extern "C" {

const char* messi_last_error(void) { return g_err.c_str(); }

int messi_breakpoints(int32_t card_bits, float* beta) {
  if (card_bits < 1 || card_bits > 8 || !beta) return fail(MESSI_EINVAL, "card_bits must be 1..8");
  breakpoints(card_bits, beta);
  return MESSI_OK;
}

int messi_build(const float* series, int64_t n, int32_t len, int32_t segments,
                int32_t cardinality, int32_t leaf_size, messi_index** out) {
  return messi_build_ex(const_cast<float*>(series), n, len, segments, cardinality, leaf_size, nullptr,
                        out);
}

int messi_build_ex(float* series, int64_t n, int32_t len, int32_t segments, int32_t cardinality,
                   int32_t leaf_size, const messi_options* opts, messi_index** out) {
  g_err.clear();
  messi_options o{};
  if (opts) o = *opts;
  if (!out) return fail(MESSI_EINVAL, "out is NULL");
  if (n < 1 || n >= ((int64_t)1 << 31) - 1) return fail(MESSI_EINVAL, "n must be in [1, 2^31-2]");
  if (segments < 1 || segments > kMaxSeg) return fail(MESSI_EINVAL, "segments must be in [1, 16]");
  if (len < 1 || len > kMaxLen || len % segments)
    return fail(MESSI_EINVAL, "len must be in [1, %d] and a multiple of segments", kMaxLen);
  const int cb = log2_exact(cardinality);
  if (cb < 1 || cb > 8) return fail(MESSI_EINVAL, "cardinality must be a power of two in [2, 256]");
  if (leaf_size < 1) return fail(MESSI_EINVAL, "leaf_size must be >= 1");
  if (!is_device_ptr(series)) return fail(MESSI_EINVAL, "series is not a device pointer");

  if (o.inplace && (reinterpret_cast<uintptr_t>(series) & 15))
    return fail(MESSI_EINVAL, "an in-place series buffer must be 16-byte aligned");
  messi_index* ix = new messi_index();
  ix->inplace = o.inplace != 0;
  ix->raw = o.raw != 0;
  ix->n = n;
  ix->len = len;
  ix->w = segments;
  ix->card_bits = cb;
  ix->leaf_size = leaf_size;
  size_t free_b = 0, total_b = 0;
  (void)hipMemGetInfo(&free_b, &total_b);
  const size_t need = (ix->inplace ? 0 : (size_t)n * len * 4) + (size_t)n * (16 * 4 + 8 * 2 + 8 + 4 * 3);
  if (need > free_b) {
    delete ix;
    return fail(MESSI_ENOMEM, "index needs about %zu bytes, %zu free", need, free_b);
  }
  int node_cap = (int)std::min<int64_t>(8 * (n / leaf_size) + 2 * ((int64_t)1 << segments) + 4096,
                                        (int64_t)1 << 30);
  int leaf_cap = (int)std::min<int64_t>(4 * (n / leaf_size) + ((int64_t)1 << segments) + 4096,
                                        (int64_t)1 << 30);
  try {
    for (int attempt = 0;; ++attempt) {
      if (build_index(ix, series, node_cap, leaf_cap)) break;
      ix->mem.clear();
      if (attempt >= 6) {
        delete ix;
        return fail(MESSI_ENOMEM, "node table kept overflowing");
      }
      node_cap = (int)std::min<int64_t>((int64_t)node_cap * 4, (int64_t)1 << 30);
      leaf_cap = (int)std::min<int64_t>((int64_t)leaf_cap * 4, (int64_t)1 << 30);
    }
  } catch (const OomError& e) {
    delete ix;
    return fail(MESSI_ENOMEM, "device allocation of %zu bytes failed", e.bytes);
  } catch (const HipError& e) {
    delete ix;
    return fail(MESSI_EDEVICE, "%s: %s", e.what, hipGetErrorString(e.e));
  }
  if (o.bf16_screen && screen_supported(len)) {
    try {
      ensure_screen(ix);
    } catch (const OomError& e) {
      delete ix;
      return fail(MESSI_ENOMEM, "device allocation of %zu bytes failed", e.bytes);
    } catch (const HipError& e) {
      delete ix;
      return fail(MESSI_EDEVICE, "%s: %s", e.what, hipGetErrorString(e.e));
    }
  }
  *out = ix;
  return MESSI_OK;
}

int messi_build_windows(const float* series, int64_t total, int32_t len, int32_t stride,
                        int32_t segments, int32_t cardinality, int32_t leaf_size,
                        const messi_options* opts, messi_index** out) {
  g_err.clear();
  if (!out) return fail(MESSI_EINVAL, "out is NULL");
  if (len < 1 || stride < 1 || total < len)
    return fail(MESSI_EINVAL, "need len >= 1, stride >= 1 and total >= len");
  if (!is_device_ptr(series)) return fail(MESSI_EINVAL, "series is not a device pointer");
  const int64_t n = (total - len) / stride + 1;
  if (n >= ((int64_t)1 << 31) - 1) return fail(MESSI_EINVAL, "more than 2^31-2 windows");
  if (len > kMaxLen || segments < 1 || len % segments)
    return fail(MESSI_EINVAL, "len must be in [1, %d] and a multiple of segments", kMaxLen);
  messi_options o{};
  if (opts) o = *opts;
  o.inplace = 1;  // the window rows are the index's own store
  DevMem rows_mem;
  float* rows = nullptr;
  try {
    rows = rows_mem.alloc<float>((size_t)n * len);
    launch_windows(series, n, len, stride, rows, nullptr);
    launch_check();
    HIP_OR_THROW(hipStreamSynchronize(nullptr));
  } catch (const OomError& e) {
    return fail(MESSI_ENOMEM, "device allocation of %zu bytes failed", e.bytes);
  } catch (const HipError& e) {
    return fail(MESSI_EDEVICE, "%s: %s", e.what, hipGetErrorString(e.e));
  }
  const int rc = messi_build_ex(rows, n, len, segments, cardinality, leaf_size, &o, out);
  if (rc != MESSI_OK) return rc;  // rows_mem frees the windows
  std::swap((*out)->own.ptrs, rows_mem.ptrs);
  (*out)->own.bytes = rows_mem.bytes;
  rows_mem.bytes = 0;
  return MESSI_OK;
}

int messi_query_stats(messi_index* index, const float* queries, int32_t nq, int32_t k,
                      int32_t distance, int32_t window, int64_t* out_ids, float* out_dists,
                      messi_stats* stats) {
  g_err.clear();
  if (!index) return fail(MESSI_EINVAL, "index is NULL");
  if (nq < 0) return fail(MESSI_EINVAL, "nq must be >= 0");
  if (nq == 0) return MESSI_OK;
  if (k < 1 || k > 1024) return fail(MESSI_EINVAL, "k must be in [1, 1024]");
  if (distance != MESSI_ED && distance != MESSI_DTW) return fail(MESSI_EINVAL, "unknown distance");
  if (window < 0) return fail(MESSI_EINVAL, "window must be >= 0");
  if (!is_device_ptr(queries) || !is_device_ptr(out_ids) || !is_device_ptr(out_dists))
    return fail(MESSI_EINVAL, "queries and outputs must be device pointers");
  BusyGuard g(index->busy);
  if (!g.ok) return fail(MESSI_EBUSY, "index is in use by another call");
  try {
    return run_query(index, queries, nq, k, distance, window, out_ids, out_dists, stats);
  } catch (const OomError& e) {
    return fail(MESSI_ENOMEM, "device allocation of %zu bytes failed", e.bytes);
  } catch (const HipError& e) {
    return fail(MESSI_EDEVICE, "%s: %s", e.what, hipGetErrorString(e.e));
  }
}

int messi_query(messi_index* index, const float* queries, int32_t nq, int32_t k, int32_t distance,
                int32_t window, int64_t* out_ids, float* out_dists) {
  return messi_query_stats(index, queries, nq, k, distance, window, out_ids, out_dists, nullptr);
}

namespace {

// The query state of nq queries with k slots and log_cap log entries each,
// carved from `base` (256-byte aligned pieces); returns the bytes it takes.
// With base == nullptr only the size is computed.
size_t carve_state(const messi_index* ix, int nq, int k, int log_cap, char* base, QueryState* qs) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* ptr = base ? base + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return ptr;
  };
  const size_t len = (size_t)ix->len, L = (size_t)ix->n_leaves, C = (size_t)ix->n_chunks, Q = (size_t)nq;
  QueryState s{};
  s.zq = reinterpret_cast<float*>(take(Q * len * sizeof(float)));
  s.eta = reinterpret_cast<float*>(take(Q * sizeof(float)));
  s.upper = reinterpret_cast<float*>(take(Q * len * sizeof(float)));
  s.lower = reinterpret_cast<float*>(take(Q * len * sizeof(float)));
  s.paa = reinterpret_cast<float*>(take(Q * 3 * kMaxSeg * sizeof(float)));
  s.approx_range = reinterpret_cast<int64_t*>(take(Q * 2 * sizeof(int64_t)));
  s.approx_d2 = reinterpret_cast<float*>(take(Q * kApproxCap * sizeof(float)));
  s.slots = reinterpret_cast<unsigned long long*>(take(Q * (size_t)k * 8));
  s.log = reinterpret_cast<unsigned long long*>(take(Q * (size_t)log_cap * 8));
  s.log_count = reinterpret_cast<int*>(take(Q * sizeof(int)));
  s.leaf_lb = reinterpret_cast<float*>(take(Q * L * sizeof(float)));
  s.items = reinterpret_cast<unsigned long long*>(take(Q * C * 8));
  s.ranges = reinterpret_cast<int2*>(take(Q * C * sizeof(int2)));
  s.next = reinterpret_cast<int*>(take(Q * kCounterInts * sizeof(int)));
  s.stats = reinterpret_cast<unsigned long long*>(take(Q * kStatCount * 8));
  s.status = reinterpret_cast<int*>(take(Q * sizeof(int)));
  if (qs) *qs = s;
  return off;
}

constexpr int kNoAllocMaxQueries = 1024;  // status words kept on the host stack
constexpr int kNoAllocLog = 32768;        // near-tie log entries per query

}  // namespace

int messi_query_noalloc(messi_index* index, const float* queries, int32_t nq, int32_t k,
                        int32_t distance, int32_t window, int64_t* out_ids, float* out_dists) {
  g_err.clear();
  if (!index) return fail(MESSI_EINVAL, "index is NULL");
  if (nq < 0) return fail(MESSI_EINVAL, "nq must be >= 0");
  if (nq == 0) return MESSI_OK;
  if (nq > kNoAllocMaxQueries)
    return fail(MESSI_EINVAL, "messi_query_noalloc takes at most %d queries per call", kNoAllocMaxQueries);
  if (k < 1 || k > 1024) return fail(MESSI_EINVAL, "k must be in [1, 1024]");
  if (distance != MESSI_ED && distance != MESSI_DTW) return fail(MESSI_EINVAL, "unknown distance");
  if (window < 0) return fail(MESSI_EINVAL, "window must be >= 0");
  if (!is_device_ptr(queries) || !is_device_ptr(out_ids) || !is_device_ptr(out_dists))
    return fail(MESSI_EINVAL, "queries and outputs must be device pointers");
  BusyGuard g(index->busy);
  if (!g.ok) return fail(MESSI_EBUSY, "index is in use by another call");
  try {
    size_t cap = 0;
    char* base = static_cast<char*>(noalloc_scratch(&cap));
    if (!base) return fail(MESSI_EDEVICE, "the scratch array's device address is not available");
    const size_t need = carve_state(index, nq, k, kNoAllocLog, nullptr, nullptr);
    if (need > cap)
      return fail(MESSI_EINVAL, "%d queries need %zu bytes of scratch, more than the %zu bytes it holds",
                  nq, need, cap);
    int h_status[kNoAllocMaxQueries];
    FixedScratch fx{};
    carve_state(index, nq, k, kNoAllocLog, base, &fx.qs);
    fx.log_cap = kNoAllocLog;
    fx.h_status = h_status;
    return run_group(index, index->ctx, queries, nq, k, distance, window, nullptr, nullptr, false, false,
                     out_ids, out_dists, nullptr, &fx);
  } catch (const OomError& e) {
    return fail(MESSI_ENOMEM, "device allocation of %zu bytes failed", e.bytes);
  } catch (const HipError& e) {
    return fail(MESSI_EDEVICE, "%s: %s", e.what, hipGetErrorString(e.e));
  }
}

int messi_prepare_screen(messi_index* index) {
  g_err.clear();
  if (!index) return fail(MESSI_EINVAL, "index is NULL");
  if (!screen_supported(index->len))
    return fail(MESSI_EINVAL, "the BF16 screen needs len 64, 128, 256 or 512");
  BusyGuard g(index->busy);
  if (!g.ok) return fail(MESSI_EBUSY, "index is in use by another call");
  try {
    ensure_screen(index);
  } catch (const OomError& e) {
    return fail(MESSI_ENOMEM, "device allocation of %zu bytes failed", e.bytes);
  } catch (const HipError& e) {
    return fail(MESSI_EDEVICE, "%s: %s", e.what, hipGetErrorString(e.e));
  }
  return MESSI_OK;
}

int messi_query_batch(messi_index* index, const float* queries, int32_t nq, const int32_t* k,
                      const int32_t* distance, const int32_t* window, int32_t kmax, int32_t flags,
                      int64_t* out_ids, float* out_dists, messi_stats* stats) {
  g_err.clear();
  if (!index) return fail(MESSI_EINVAL, "index is NULL");
  if (nq < 0) return fail(MESSI_EINVAL, "nq must be >= 0");
  if (nq == 0) return MESSI_OK;
  if (kmax < 1 || kmax > 1024) return fail(MESSI_EINVAL, "kmax must be in [1, 1024]");
  if (!k || !distance || !window) return fail(MESSI_EINVAL, "k, distance and window are required");
  if (is_device_ptr(k) || is_device_ptr(distance) || is_device_ptr(window))
    return fail(MESSI_EINVAL, "k, distance and window must be host arrays");
  if (flags & ~(MESSI_SCREEN_BF16 | MESSI_LB_IMPROVED)) return fail(MESSI_EINVAL, "unknown flags");
  if (!is_device_ptr(queries) || !is_device_ptr(out_ids) || !is_device_ptr(out_dists))
    return fail(MESSI_EINVAL, "queries and outputs must be device pointers");
  for (int i = 0; i < nq; ++i) {
    if (k[i] < 1 || k[i] > kmax) return fail(MESSI_EINVAL, "k[%d] must be in [1, kmax]", i);
    if (distance[i] != MESSI_ED && distance[i] != MESSI_DTW)
      return fail(MESSI_EINVAL, "unknown distance[%d]", i);
    if (window[i] < 0) return fail(MESSI_EINVAL, "window[%d] must be >= 0", i);
  }
  BusyGuard guard(index->busy);
  if (!guard.ok) return fail(MESSI_EBUSY, "index is in use by another call");
  if ((flags & MESSI_SCREEN_BF16) && screen_supported(index->len)) {
    try {
      ensure_screen(index);
    } catch (const OomError& e) {
      return fail(MESSI_ENOMEM, "device allocation of %zu bytes failed", e.bytes);
    } catch (const HipError& e) {
      return fail(MESSI_EDEVICE, "%s: %s", e.what, hipGetErrorString(e.e));
    }
  }
  return run_batch(index, index->ctx, queries, nq, k, distance, window, kmax, flags, out_ids,
                   out_dists, stats);
}

int messi_classify(messi_index* index, const int32_t* labels, int32_t n_classes,
                   const float* queries, int32_t nq, int32_t k, int32_t distance, int32_t window,
                   int32_t flags, int32_t* out_class, int64_t* out_ids, float* out_dists) {
  g_err.clear();
  if (!index) return fail(MESSI_EINVAL, "index is NULL");
  if (nq < 0) return fail(MESSI_EINVAL, "nq must be >= 0");
  if (nq == 0) return MESSI_OK;
  if (n_classes < 1 || n_classes > 4096) return fail(MESSI_EINVAL, "n_classes must be in [1, 4096]");
  if (k < 1 || k > 1024) return fail(MESSI_EINVAL, "k must be in [1, 1024]");
  if (distance != MESSI_ED && distance != MESSI_DTW) return fail(MESSI_EINVAL, "unknown distance");
  if (window < 0) return fail(MESSI_EINVAL, "window must be >= 0");
  if (flags & ~(MESSI_SCREEN_BF16 | MESSI_LB_IMPROVED)) return fail(MESSI_EINVAL, "unknown flags");
  if (!is_device_ptr(labels) || !is_device_ptr(queries) || !is_device_ptr(out_class) ||
      !is_device_ptr(out_ids) || !is_device_ptr(out_dists))
    return fail(MESSI_EINVAL, "labels, queries and outputs must be device pointers");
  BusyGuard guard(index->busy);
  if (!guard.ok) return fail(MESSI_EBUSY, "index is in use by another call");
  try {
    if ((flags & MESSI_SCREEN_BF16) && screen_supported(index->len)) ensure_screen(index);
    const std::vector<int32_t> ks(nq, k), ds(nq, distance), ws(nq, window);
    const int rc = run_batch(index, index->ctx, queries, nq, ks.data(), ds.data(), ws.data(), k,
                             flags, out_ids, out_dists, nullptr);
    if (rc != MESSI_OK) return rc;
    launch_vote(out_ids, k, nq, k, labels, n_classes, out_class, index->ctx.stream);
    launch_check();
    HIP_OR_THROW(hipStreamSynchronize(index->ctx.stream));
  } catch (const OomError& e) {
    return fail(MESSI_ENOMEM, "device allocation of %zu bytes failed", e.bytes);
  } catch (const HipError& e) {
    return fail(MESSI_EDEVICE, "%s: %s", e.what, hipGetErrorString(e.e));
  }
  return MESSI_OK;
}

int messi_set_stream(messi_index* index, void* hip_stream) {
  if (!index) return fail(MESSI_EINVAL, "index is NULL");
  index->ctx.stream = (hipStream_t)hip_stream;
  return MESSI_OK;
}

int messi_index_info(const messi_index* index, int64_t* n, int32_t* len, int32_t* segments,
                     int32_t* card_bits, int64_t* n_leaves, int64_t* device_bytes) {
  if (!index) return fail(MESSI_EINVAL, "index is NULL");
  if (n) *n = index->n;
  if (len) *len = index->len;
  if (segments) *segments = index->w;
  if (card_bits) *card_bits = index->card_bits;
  if (n_leaves) *n_leaves = index->n_leaves;
  if (device_bytes)
    *device_bytes = (int64_t)(index->mem.bytes + index->own.bytes + index->ctx.ws.mem.bytes +
                              index->screen_mem.bytes + index->ctx.batch_mem.bytes);
  return MESSI_OK;
}

int messi_get_perm(const messi_index* index, int32_t* perm) {
  if (!index || !perm) return fail(MESSI_EINVAL, "NULL argument");
  try {
    d2h(perm, index->perm, (size_t)index->n, index->ctx.stream);
  } catch (const HipError& e) {
    return fail(MESSI_EDEVICE, "%s: %s", e.what, hipGetErrorString(e.e));
  }
  return MESSI_OK;
}

int messi_get_words(const messi_index* index, uint8_t* words) {
  if (!index || !words) return fail(MESSI_EINVAL, "NULL argument");
  try {
    std::vector<uint4> ws((size_t)index->n);
    std::vector<int32_t> pm((size_t)index->n);
    d2h(ws.data(), index->words, (size_t)index->n, index->ctx.stream);
    d2h(pm.data(), index->perm, (size_t)index->n, index->ctx.stream);
    for (int64_t p = 0; p < index->n; ++p) {
      const uint8_t* b = reinterpret_cast<const uint8_t*>(&ws[(size_t)p]);
      std::memcpy(words + (int64_t)pm[(size_t)p] * index->w, b, (size_t)index->w);
    }
  } catch (const HipError& e) {
    return fail(MESSI_EDEVICE, "%s: %s", e.what, hipGetErrorString(e.e));
  }
  return MESSI_OK;
}

int messi_get_leaves(const messi_index* index, messi_leaf* leaves, int64_t cap, int64_t* count) {
  if (!index || !count) return fail(MESSI_EINVAL, "NULL argument");
  *count = index->n_leaves;
  if (cap < index->n_leaves || !leaves) return fail(MESSI_EINVAL, "leaf buffer too small");
  try {
    const int L = index->n_leaves;
    std::vector<int64_t> b(L), e(L);
    std::vector<uint4> sy(L), bi(L);
    d2h(b.data(), index->leaf_begin, L, index->ctx.stream);
    d2h(e.data(), index->leaf_end, L, index->ctx.stream);
    d2h(sy.data(), index->leaf_sym, L, index->ctx.stream);
    d2h(bi.data(), index->leaf_bits, L, index->ctx.stream);
    std::vector<int> order(L);
    for (int l = 0; l < L; ++l) order[l] = l;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return b[x] < b[y]; });
    for (int i = 0; i < L; ++i) {
      const int l = order[i];
      messi_leaf& o = leaves[i];
      o.begin = b[l];
      o.end = e[l];
      std::memcpy(o.sym, &sy[l], 16);
      std::memcpy(o.bits, &bi[l], 16);
    }
  } catch (const HipError& e) {
    return fail(MESSI_EDEVICE, "%s: %s", e.what, hipGetErrorString(e.e));
  }
  return MESSI_OK;
}


int messi_server_start(messi_index* index, const messi_server_options* opts, messi_server** out) {
  g_err.clear();
  if (!index || !out) return fail(MESSI_EINVAL, "NULL argument");
  messi_server_options o{};
  if (opts) o = *opts;
  const int workers = o.workers == 0 ? 2 : o.workers;
  const int max_batch = o.max_batch == 0 ? 1024 : o.max_batch;
  const int kmax = o.kmax == 0 ? 64 : o.kmax;
  if (workers < 1 || workers > 8) return fail(MESSI_EINVAL, "workers must be in [1, 8]");
  if (max_batch < 1 || max_batch > 65536) return fail(MESSI_EINVAL, "max_batch must be in [1, 65536]");
  if (kmax < 1 || kmax > 1024) return fail(MESSI_EINVAL, "kmax must be in [1, 1024]");
  if (o.mem_budget_bytes < 0) return fail(MESSI_EINVAL, "mem_budget_bytes must be >= 0");
  if (o.flags & ~(MESSI_SCREEN_BF16 | MESSI_LB_IMPROVED)) return fail(MESSI_EINVAL, "unknown flags");
  std::unique_ptr<messi_server> S(new messi_server());
  S->ix = index;
  S->kmax = kmax;
  S->flags = o.flags;
  S->workers_n = workers;
  S->max_batch = max_batch;
  S->budget = o.mem_budget_bytes;
  S->req_bytes = request_bytes(index, kmax, 4096);
  if (hipGetDevice(&S->device) != hipSuccess) return fail(MESSI_EDEVICE, "no current HIP device");
  int cap = max_batch;
  if (S->budget > 0) cap = (int)std::max<int64_t>(1, std::min<int64_t>(cap, S->budget / S->req_bytes));
  try {
    if ((o.flags & MESSI_SCREEN_BF16) && screen_supported(index->len)) ensure_screen(index);
    for (int i = 0; i < workers; ++i) {
      std::unique_ptr<SrvWorker> w(new SrvWorker());
      HIP_OR_THROW(hipStreamCreateWithFlags(&w->ctx.stream, hipStreamNonBlocking));
      w->cap = cap;
      w->d_q = w->io.alloc<float>((size_t)cap * index->len);
      w->d_ids = w->io.alloc<int64_t>((size_t)cap * kmax);
      w->d_d = w->io.alloc<float>((size_t)cap * kmax);
      HIP_OR_THROW(hipHostMalloc((void**)&w->h_q, sizeof(float) * cap * index->len, hipHostMallocDefault));
      HIP_OR_THROW(hipHostMalloc((void**)&w->h_ids, sizeof(int64_t) * cap * kmax, hipHostMallocDefault));
      HIP_OR_THROW(hipHostMalloc((void**)&w->h_d, sizeof(float) * cap * kmax, hipHostMallocDefault));
      S->workers.push_back(std::move(w));
    }
  } catch (const OomError& e) {
    return fail(MESSI_ENOMEM, "device allocation of %zu bytes failed", e.bytes);
  } catch (const HipError& e) {
    return fail(MESSI_EDEVICE, "%s: %s", e.what, hipGetErrorString(e.e));
  }
  for (auto& w : S->workers) w->th = std::thread(server_worker_main, S.get(), w.get());
  *out = S.release();
  return MESSI_OK;
}

int messi_server_submit(messi_server* server, const float* query, int32_t k, int32_t distance,
                        int32_t window, uint64_t* id) {
  g_err.clear();
  if (!server || !query || !id) return fail(MESSI_EINVAL, "NULL argument");
  if (is_device_ptr(query)) return fail(MESSI_EINVAL, "query must be a host pointer");
  if (k < 1 || k > server->kmax) return fail(MESSI_EINVAL, "k must be in [1, kmax]");
  if (distance != MESSI_ED && distance != MESSI_DTW) return fail(MESSI_EINVAL, "unknown distance");
  if (window < 0) return fail(MESSI_EINVAL, "window must be >= 0");
  SrvRequest r;
  r.k = k;
  r.distance = distance;
  r.window = window;
  r.q.assign(query, query + server->ix->len);
  r.bytes = server->req_bytes;
  {
    std::lock_guard<std::mutex> lk(server->mu);
    if (server->stopping) return fail(MESSI_EBUSY, "server is stopping");
    r.id = server->next_id++;
    r.t_submit = Clock::now();
    *id = r.id;
    server->pending.push_back(std::move(r));
    ++server->submitted;
  }
  server->cv_work.notify_one();
  return MESSI_OK;
}

int messi_server_poll(messi_server* server, int32_t max, int32_t timeout_ms, uint64_t* req_ids,
                      int32_t* status, int64_t* ids, float* dists, double* latency_us,
                      int32_t* count) {
  g_err.clear();
  if (!server || !count || max < 0) return fail(MESSI_EINVAL, "bad argument");
  *count = 0;
  std::unique_lock<std::mutex> lk(server->mu);
  if (server->done.empty() && timeout_ms != 0) {
    if (timeout_ms < 0)
      server->cv_done.wait(lk, [&] { return !server->done.empty(); });
    else
      server->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                               [&] { return !server->done.empty(); });
  }
  const int kmax = server->kmax;
  int n = 0;
  while (n < max && !server->done.empty()) {
    SrvResult& r = server->done.front();
    if (req_ids) req_ids[n] = r.id;
    if (status) status[n] = r.status;
    if (latency_us) latency_us[n] = r.latency_us;
    for (int j = 0; j < kmax; ++j) {
      const bool have = j < (int)r.ids.size();
      if (ids) ids[(size_t)n * kmax + j] = have ? r.ids[j] : -1;
      if (dists) dists[(size_t)n * kmax + j] = have ? r.dists[j] : INFINITY;
    }
    server->done.pop_front();
    ++n;
  }
  *count = n;
  return MESSI_OK;
}

int messi_server_get_stats(messi_server* server, messi_server_stats* st) {
  if (!server || !st) return fail(MESSI_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(server->mu);
  st->submitted = server->submitted;
  st->completed = server->completed;
  st->batches = server->batches;
  st->max_batch_seen = server->max_batch_seen;
  st->inflight_bytes = server->inflight;
  st->peak_inflight_bytes = server->peak_inflight;
  st->mem_budget_bytes = server->budget;
  st->request_bytes = server->req_bytes;
  st->batch_capacity = server->workers.empty() ? 0 : server->workers[0]->cap;
  st->busy_us = server->busy_us;
  return MESSI_OK;
}

void messi_server_stop(messi_server* server) {
  if (!server) return;
  {
    std::lock_guard<std::mutex> lk(server->mu);
    server->stopping = true;
  }
  server->cv_work.notify_all();
  for (auto& w : server->workers)
    if (w->th.joinable()) w->th.join();
  delete server;
}

void messi_free(messi_index* index) { delete index; }

}  // extern "C"
