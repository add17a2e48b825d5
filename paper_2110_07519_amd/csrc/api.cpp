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
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <unistd.h>
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

// An allocation that would take the index past its memory budget.
struct BudgetError {
  size_t need, budget;
};

// Host time this thread has spent in hipMalloc (the build reports its part).
thread_local double g_alloc_ms = 0.0;

// Device allocation owned by a vector of frees.
struct DevMem {
  std::vector<void*> ptrs;
  size_t bytes = 0;
  template <typename T>
  T* alloc(size_t count) {
    void* p = nullptr;
    const size_t b = std::max<size_t>(count, 1) * sizeof(T);
    const auto t0 = std::chrono::steady_clock::now();
    hipError_t e = hipMalloc(&p, b);
    g_alloc_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
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

// Temporaries carved from one allocation: one hipMalloc and one hipFree for
// all of them.  A request past the reserved end gets an allocation of its
// own.
struct Slab {
  DevMem mem;
  char* base = nullptr;
  size_t cap = 0, used = 0;
  template <typename T>
  static size_t bytes_for(size_t count) {
    return (std::max<size_t>(count, 1) * sizeof(T) + 255) & ~(size_t)255;
  }
  void reserve(size_t b) {
    base = mem.alloc<char>(b);
    cap = b;
  }
  template <typename T>
  T* alloc(size_t count) {
    const size_t b = bytes_for<T>(count);
    if (base && used + b <= cap) {
      T* p = reinterpret_cast<T*>(base + used);
      used += b;
      return p;
    }
    return mem.alloc<T>(count);
  }
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

// Knobs of the batched path, chosen per batch shape by the autotuner
// (messi_autotune); the defaults are the built-in choices.
struct Tune {
  int screen = 1;       // 1: ED groups take the BF16 screen when MESSI_SCREEN_BF16 asks for it
  int screen_min = 32;  // fewest ED queries in a screened group
  int screen_nt = 0;    // 16-series column tiles per wave of the screen kernel (0: its default)
  int screen_occ = 0;   // screen blocks per CU (0: the occupancy limit)
  int screen_waves = 0; // waves per screen block (0: its default, 4)
  int ed_scale = 1;     // ED process grid, in resident grids
  int dtw_scale = 1;    // DTW process blocks per query, in multiples of the even share
  int overlap = 1;      // 1: a batch's groups run concurrently, each on its own stream
};

struct TuneEntry {
  Tune t;
  double ms = 0.0, ms_default = 0.0;  // batch time with these knobs and with the defaults
};

// A batch's launches captured once and replayed.
struct GraphEntry {
  std::string key;  // every argument of every launch (see launch_key)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  GraphEntry() = default;
  GraphEntry(const GraphEntry&) = delete;
  GraphEntry& operator=(const GraphEntry&) = delete;
  ~GraphEntry() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

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
  hipStream_t own_stream = nullptr;  // a stream this context created (destroyed with it)
  hipEvent_t fork = nullptr;         // overlapped batch: the point the groups start from
  hipEvent_t join = nullptr;         // overlapped batch: the end of this context's group
  hipStream_t cap_stream = nullptr;  // stream the batch graphs are captured on
  std::vector<std::unique_ptr<QueryCtx>> aux;          // contexts of a batch's groups 1, 2, ...
  std::vector<std::unique_ptr<GraphEntry>> graphs;     // captured batches, oldest first
  bool budgeted = false;  // workspace counts against the index's memory budget
  std::function<void(int64_t)> on_grow;  // told of each change of the workspace's bytes

  QueryCtx() = default;
  QueryCtx(const QueryCtx&) = delete;
  QueryCtx& operator=(const QueryCtx&) = delete;
  ~QueryCtx() {
    graphs.clear();
    aux.clear();
    if (events_ready)
      for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (own_stream) (void)hipStreamDestroy(own_stream);
    if (h_status) (void)hipHostFree(h_status);
  }
};

}  // namespace

struct messi_index {
  int64_t n = 0;
  int len = 0, w = 0, card_bits = 0, leaf_size = 0;
  int n_leaves = 0, n_nodes = 0;
  int64_t max_leaf = 0;
  double build_ms = 0.0, build_alloc_ms = 0.0;  // host time of the build call, and in hipMalloc
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
  int64_t budget = 0;           // device bytes the index may hold (0: no limit)
  float* owned_store = nullptr;  // in-place store the index took over (freed with it)
  size_t store_bytes = 0;
  std::string device;           // device tag of the autotune keys (arch and CU count)
  std::string tune_path;        // autotune cache file ("" = none)
  mutable std::mutex tune_mu;
  std::map<std::string, TuneEntry> tunes;  // tuned knobs by batch shape
  QueryCtx ctx;  // the index's own calls (messi_query, messi_query_batch)
  std::atomic<int> busy{0};

  messi_index() { ctx.budgeted = true; }
  ~messi_index() {
    ctx.graphs.clear();
    if (owned_store) (void)hipFree(owned_store);
  }

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

// Device bytes a query context holds: its workspace, batch buffers and the
// contexts of further batch groups.
size_t ctx_bytes(const QueryCtx& c) {
  size_t b = c.ws.mem.bytes + c.batch_mem.bytes;
  for (const auto& a : c.aux) b += ctx_bytes(*a);
  return b;
}

// Device bytes the index holds: tables, store (its own or taken over), BF16
// copy and its own query contexts.
size_t held_bytes(const messi_index* ix) {
  return ix->mem.bytes + ix->own.bytes + ix->screen_mem.bytes + ix->store_bytes + ctx_bytes(ix->ctx);
}

// Throws BudgetError if the index would hold more than its budget after
// releasing `drop` bytes and allocating `add` more (contexts that do not
// count against the budget - a server's workers - are not checked).
void check_budget(const messi_index* ix, const QueryCtx& c, size_t drop, size_t add) {
  if (!c.budgeted || ix->budget <= 0) return;
  const size_t held = held_bytes(ix);
  const size_t after = held - std::min(drop, held) + add;
  if (after > (size_t)ix->budget) throw BudgetError{after, (size_t)ix->budget};
}

// Runs f, turning the library's exceptions into error codes.
template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const OomError& e) {
    return fail(MESSI_ENOMEM, "device allocation of %zu bytes failed", e.bytes);
  } catch (const BudgetError& e) {
    return fail(MESSI_ENOMEM, "the index would hold %zu bytes, over its memory budget of %zu", e.need,
                e.budget);
  } catch (const HipError& e) {
    return fail(MESSI_EDEVICE, "%s: %s", e.what, hipGetErrorString(e.e));
  }
}

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


// The build proper; throws HipError / OomError.  Returns false if the node
// or leaf tables were too small (caller retries with larger ones).
bool build_index(messi_index* ix, const float* series, int node_cap, int leaf_cap) {
  const int64_t n = ix->n;
  const int len = ix->len, w = ix->w, cb = ix->card_bits, card = 1 << cb;
  const int nkeys = 1 << w;
  hipStream_t st = ix->ctx.stream;
  const int round_cap = (int)std::min<int64_t>(n / (ix->leaf_size + 1) + 1, (int64_t)node_cap);
  const int chunk_cap = (int)std::min<int64_t>(n / kChunk + round_cap + 1, (int64_t)1 << 30);
  Slab tmp;
  {
    size_t b = 0;
    b += 3 * Slab::bytes_for<uint4>(n);  // words_id, W0, W1
    b += Slab::bytes_for<float2>(n) + Slab::bytes_for<uint16_t>(n) + 2 * Slab::bytes_for<int32_t>(n);
    b += Slab::bytes_for<unsigned int>(nkeys) + Slab::bytes_for<unsigned int>(1);
    b += Slab::bytes_for<int64_t>(nkeys + 1) + Slab::bytes_for<unsigned long long>(nkeys);
    b += 2 * Slab::bytes_for<int>(leaf_cap) + 3 * Slab::bytes_for<int>(round_cap);
    b += Slab::bytes_for<int>(8) + Slab::bytes_for<int>(4);
    b += Slab::bytes_for<int>((size_t)round_cap * kMaxSeg);
    b += Slab::bytes_for<unsigned long long>((size_t)round_cap * 2);
    b += Slab::bytes_for<Chunk>(chunk_cap);
    tmp.reserve(b);
  }

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
  uint16_t* keys = tmp.alloc<uint16_t>(n);
  launch_summarize(series, n, len, w, cb, spw, ix->bp, words_id, musd, keys, norm2, st, ix->n_cus);
  launch_check();
  launch_key_hist(keys, n, nkeys, hist, ix->n_cus, st);
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
  launch_root_scatter(words_id, keys, n, nkeys, key_cursor, d.W0, d.I0, ix->n_cus, st);
  launch_check();

  // node and leaf tables
  d.nodes = ix->mem.alloc<NodeDev>(node_cap);
  d.node_cap = node_cap;
  d.leaves = tmp.alloc<int>(leaf_cap);
  d.leaf_cap = leaf_cap;
  d.root_node = ix->mem.alloc<int>(nkeys);
  d.cur_list = tmp.alloc<int>(round_cap);
  d.next_list = tmp.alloc<int>(round_cap);
  d.round_cap = round_cap;
  // node_count, leaf_count, round list counts (two, swapped each round),
  // overflow, chunk_count, chunk table overflow
  int* counters = tmp.alloc<int>(8);
  HIP_OR_THROW(hipMemsetAsync(counters, 0, sizeof(int) * 8, st));
  d.node_count = counters + 0;
  d.leaf_count = counters + 1;
  int* list_count[2] = {counters + 2, counters + 5};
  d.next_count = list_count[0];
  d.cur_count = list_count[1];
  d.overflow = counters + 3;
  int* chunk_count = counters + 4;
  int* chunk_overflow = counters + 6;
  d.c1 = tmp.alloc<int>((size_t)round_cap * kMaxSeg);
  HIP_OR_THROW(hipMemsetAsync(d.c1, 0, sizeof(int) * (size_t)round_cap * kMaxSeg, st));
  d.split_seg = tmp.alloc<int>(round_cap);
  d.cursor = tmp.alloc<unsigned long long>((size_t)round_cap * 2);
  Chunk* chunks = tmp.alloc<Chunk>(chunk_cap);

  // the next_list of launch_roots becomes the first round's list
  launch_roots(key_begin, nkeys, w, ix->leaf_size, d, st);
  launch_check();

  // (3) split rounds, queued kRoundsPerSync at a time: each round takes its
  // sizes from the device, so the host only looks at the counters between
  // groups (a round after the last one with nodes, or after an overflow of
  // the roots, does nothing)
  constexpr int kRoundsPerSync = 4;
  const int round_blocks = std::max(1, ix->n_cus) * 8;
  int hc[8];
  for (int round = 0, n_cur = 1; n_cur > 0;) {
    for (int j = 0; j < kRoundsPerSync; ++j, ++round) {
      if (round > 16 * 8 + 8) throw HipError{hipErrorUnknown, "split rounds did not converge"};
      std::swap(d.cur_list, d.next_list);
      std::swap(d.cur_count, d.next_count);
      launch_make_chunks(d, kChunk, chunks, chunk_cap, chunk_count, chunk_overflow, st);
      launch_round_count(chunks, chunk_count, chunk_cap, d, w, cb, round_blocks, st);
      launch_round_decide(w, cb, ix->leaf_size, d, st);
      launch_round_scatter(chunks, chunk_count, chunk_cap, d, cb, round_blocks, st);
      launch_check();
    }
    d2h(hc, counters, 8, st);
    if (hc[3]) return false;
    if (hc[6]) throw HipError{hipErrorUnknown, "chunk table overflow"};
    n_cur = d.next_count == list_count[0] ? hc[2] : hc[5];
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
  // the query's shard-major leaf table, and the leaf sizes the host needs:
  // one readback for the largest leaf, the over-full leaves and the work
  // chunks
  int* small = tmp.alloc<int>(4);  // largest leaf, leaves over kLeafSortMax, chunks
  HIP_OR_THROW(hipMemsetAsync(small, 0, sizeof(int) * 4, st));
  launch_leaf_stats(ix->leaf_begin, ix->leaf_end, n_leaves, small, st);
  ix->shard_off = ix->mem.alloc<int>(kShards + 1);
  ix->leaf_sh_off = ix->mem.alloc<int>(kShards + 1);
  ix->sh_sym = ix->mem.alloc<uint4>(n_leaves);
  ix->sh_bits = ix->mem.alloc<uint4>(n_leaves);
  ix->sh_rng = ix->mem.alloc<int2>(n_leaves);
  launch_shard_layout(ix->leaf_begin, ix->leaf_end, ix->leaf_sym, ix->leaf_bits, n_leaves,
                      ix->shard_off, ix->leaf_sh_off, small + 2, ix->sh_sym, ix->sh_bits, ix->sh_rng,
                      st);
  launch_check();
  int hs[4];
  d2h(hs, small, 4, st);
  const int64_t maxl = hs[0];
  ix->n_chunks = hs[2];
  if (hs[1] > 0) {  // leaves over kLeafSortMax: sorted one at a time through global memory
    std::vector<int64_t> hb(n_leaves), he(n_leaves);
    std::vector<int> hbuf(n_leaves);
    d2h(hb.data(), ix->leaf_begin, n_leaves, st);
    d2h(he.data(), ix->leaf_end, n_leaves, st);
    d2h(hbuf.data(), leaf_buf, n_leaves, st);
    int64_t pb = 1;
    while (pb < maxl) pb <<= 1;
    int32_t* sort_scratch = tmp.alloc<int32_t>(pb);
    for (int l = 0; l < n_leaves; ++l) {
      const int64_t c = he[l] - hb[l];
      if (c > kLeafSortMax) {
        int p2 = 1;
        while (p2 < c) p2 <<= 1;
        launch_leaf_sort_global(hb[l], (int)c, p2, hbuf[l] ? d.I1 : d.I0, sort_scratch, ix->perm, st);
        launch_check();
      }
    }
  }
  ix->max_leaf = maxl;

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
  HIP_OR_THROW(hipStreamSynchronize(st));  // the index is complete when the build returns
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
  const size_t old = ws.mem.bytes;
  check_budget(ix, c, old, carve_state(ix, NQ, K, LC, nullptr, nullptr));
  ws.mem.clear();
  ws = Workspace{};
  QueryState& s = ws.qs;
  const int len = ix->len, L = ix->n_leaves;
  try {
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
  } catch (...) {
    ws.mem.clear();
    ws = Workspace{};
    if (c.on_grow && old) c.on_grow(-(int64_t)old);
    throw;
  }
  ws.nq = NQ;
  ws.k = K;
  ws.len = len;
  ws.w = ix->w;
  ws.card = card;
  ws.log_cap = LC;
  ws.L = L;
  if (c.on_grow) c.on_grow((int64_t)ws.mem.bytes - (int64_t)old);
}

// Back to the starting near-tie log after a batch that grew it: the
// workspace is made again for nq queries with k slots.
constexpr int kLogCap0 = 4096;  // near-tie log entries per query a context starts with

void shrink_log(messi_index* ix, QueryCtx& c, int nq, int k) {
  if (c.log_cap <= kLogCap0 && c.ws.log_cap <= kLogCap0) return;
  c.log_cap = kLogCap0;
  const int64_t old = (int64_t)c.ws.mem.bytes;
  c.ws.mem.clear();
  c.ws = Workspace{};
  std::function<void(int64_t)> report;
  std::swap(report, c.on_grow);  // one report below, of the net change
  try {
    ensure_workspace(ix, c, nq, k);
  } catch (...) {
    std::swap(report, c.on_grow);
    if (c.on_grow) c.on_grow(-old);
    throw;
  }
  std::swap(report, c.on_grow);
  if (c.on_grow) c.on_grow((int64_t)c.ws.mem.bytes - old);
}

// BF16 shadow of the store (screen operand) and the squared row norms.
void ensure_screen(messi_index* ix) {
  std::lock_guard<std::mutex> lk(ix->screen_mu);
  if (ix->Zb) return;
  check_budget(ix, ix->ctx, 0, (size_t)ix->n * ix->len * sizeof(uint16_t) + (size_t)ix->n * sizeof(float));
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
  const int L = ix->n_leaves;
  const size_t need = (size_t)nq * (12 + 2 * (size_t)ix->len + 4 * (size_t)L) + (size_t)L * 12 + 64;
  check_budget(ix, c, c.batch_mem.bytes, need);
  c.batch_mem.clear();
  c.batch_nq = 0;
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

// Everything the launches of one group of queries take (queries sharing a
// distance and window): parameters, state, screen buffers, grids and
// inputs / outputs.  Two groups with bytewise equal records launch the
// same work, which is what a batch graph is matched on.
struct GroupLaunch {
  QueryParams p;
  QueryState qs;
  ScreenDev sc;
  const float* queries;
  int64_t* out_ids;
  float* out_dists;
  int screen, blocks, screen_blocks, screen_nt, screen_waves;
};

// Parameters and grids of a group of nq queries; `main` holds the batch's
// screen buffers.  Fails with MESSI_EINVAL if the kernels' LDS cannot
// hold series of this length with this window.
int plan_group(messi_index* ix, QueryCtx& main, int nq, int kmax, int distance, int window,
               bool screen, bool lb_improved, bool count_work, const Tune& t, GroupLaunch& g) {
  std::memset(&g, 0, sizeof(g));
  const int len = ix->len;
  const double u = std::ldexp(1.0, -24);
  QueryParams& p = g.p;
  p.nq = nq;
  p.len = len;
  p.w = ix->w;
  p.m = len / ix->w;
  p.card_bits = ix->card_bits;
  p.k = kmax;
  p.out_stride = kmax;
  p.order_leaves = screen ? 0 : 1;
  p.count_work = count_work ? 1 : 0;
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
    if (main.proc_blocks_ed == 0) main.proc_blocks_ed = process_blocks_per_cu(p);
    per_cu = main.proc_blocks_ed;
  }
  const int resident = per_cu * ix->n_cus;
  if (distance == MESSI_ED)  // the whole grid visits every query
    g.blocks = ed_process_blocks(resident * std::max(1, t.ed_scale));
  else
    g.blocks = std::max(2, std::min(resident / std::max(1, nq) * std::max(1, t.dtw_scale),
                                    resident * std::max(1, t.dtw_scale)));
  g.screen = screen ? 1 : 0;
  if (screen) {
    ScreenDev& sc = g.sc;
    sc.Zb = ix->Zb;
    sc.xn = ix->xn;
    sc.qb = main.qb;
    sc.qn = main.qn;
    sc.cnt = main.cnt;
    sc.off = main.off;
    sc.lists = main.lists;
    sc.counter = main.counter;
    sc.tally = main.tally;
    // bound constants (see the screen kernel): u_b = 2^-8, gamma at 2^-23
    const double ub = std::ldexp(1.0, -8);
    const double gm = len * std::ldexp(1.0, -23) / (1.0 - len * std::ldexp(1.0, -23));
    const double cdot = 2.0 * ((2.0 * ub + ub * ub) + gm * (1.0 + ub) * (1.0 + ub)) * (1.0 + std::ldexp(1.0, -10));
    sc.c_dot = std::nextafter((float)cdot, INFINITY);
    sc.c_abs = (float)std::ldexp(1.0, -17);
    g.screen_nt = t.screen_nt > 0 ? t.screen_nt : screen_nt_default(len);
    g.screen_waves = t.screen_waves > 0 ? t.screen_waves : screen_waves_default();
    if (!screen_variant(len, g.screen_nt, g.screen_waves)) {  // a shape not built: the defaults
      g.screen_nt = screen_nt_default(len);
      g.screen_waves = screen_waves_default();
    }
    int occ = screen_blocks_per_cu(len, g.screen_nt, g.screen_waves);
    if (t.screen_occ > 0) occ = std::min(occ, t.screen_occ);
    g.screen_blocks = occ * ix->n_cus;
  }
  return MESSI_OK;
}

// Per-query status words in pinned, device-mapped host memory the kernels
// write through its device address, so no copy follows the kernels.
void ensure_status(QueryCtx& c, int nq) {
  if (c.h_status_cap >= nq) return;
  if (c.h_status) HIP_OR_THROW(hipHostFree(c.h_status));
  c.h_status = nullptr;
  c.d_status = nullptr;
  c.h_status_cap = 0;
  HIP_OR_THROW(hipHostMalloc((void**)&c.h_status, sizeof(int) * (size_t)nq, hipHostMallocMapped));
  HIP_OR_THROW(hipHostGetDevicePointer((void**)&c.d_status, c.h_status, 0));
  c.h_status_cap = nq;
}

void ensure_events(QueryCtx& c) {
  if (c.events_ready) return;
  for (int i = 0; i < 5; ++i) HIP_OR_THROW(hipEventCreate(&c.ev[i]));
  c.events_ready = true;
}

// Points a planned group at context c's state (or the fixed scratch) and at
// its inputs and outputs; status words start at c's word `status_at`.
void bind_group(QueryCtx& c, GroupLaunch& g, const float* queries, const int* d_kq, const int* d_qmap,
                int64_t* out_ids, float* out_dists, const FixedScratch* fixed, int status_at = 0) {
  g.p.log_cap = fixed ? fixed->log_cap : c.log_cap;
  g.qs = fixed ? fixed->qs : c.ws.qs;
  if (!fixed) g.qs.status = c.d_status + status_at;
  g.qs.kq = d_kq;
  g.qs.qmap = d_qmap;
  g.queries = queries;
  g.out_ids = out_ids;
  g.out_dists = out_dists;
}

// Launches a bound group's kernels on st (not synchronised).  timed: c's
// events bracket the phases; min_work: the minimal-work count follows.
void enqueue_group(messi_index* ix, QueryCtx& c, const GroupLaunch& g, hipStream_t st, bool timed,
                   bool min_work) {
  const IndexDev v = ix->view();
  if (timed) HIP_OR_THROW(hipEventRecord(c.ev[0], st));
  launch_prep(v, g.queries, g.p, g.qs, st);
  if (timed) HIP_OR_THROW(hipEventRecord(c.ev[1], st));
  launch_stage1(v, g.p, g.qs, st);
  if (timed) HIP_OR_THROW(hipEventRecord(c.ev[2], st));
  if (g.screen) {
    launch_bf16_rows(g.qs.zq, nullptr, g.p.nq, g.p.len, g.sc.qb, g.sc.qn, st);
    launch_screen(v, g.p, g.qs, g.sc, g.screen_blocks, g.screen_nt, g.screen_waves, st);
  } else {
    launch_process(v, g.p, g.qs, g.blocks, st);
  }
  if (timed) HIP_OR_THROW(hipEventRecord(c.ev[3], st));
  launch_finalize(v, g.p, g.qs, g.out_ids, g.out_dists, st);
  if (timed) {
    HIP_OR_THROW(hipEventRecord(c.ev[4], st));
    // the minimal work, once the final k-th best is known (untimed)
    if (min_work) launch_min_work(v, g.p, g.qs, std::max(1, ix->n_cus), st);
  }
  launch_check();
}

// OR of the status words of a finished group (bit 0: near-tie log overflow).
int group_status(const int* h_status, int nq) {
  int worst = 0;
  for (int i = 0; i < nq; ++i) worst |= h_status[i];
  return worst;
}

// Adds a finished group's phase times and work counters to stats.
void add_group_stats(messi_index* ix, QueryCtx& c, const GroupLaunch& g, messi_stats* stats,
                     hipStream_t st) {
  const int nq = g.p.nq;
  float ms[4] = {0, 0, 0, 0};
  for (int i = 0; i < 4; ++i) HIP_OR_THROW(hipEventElapsedTime(&ms[i], c.ev[i], c.ev[i + 1]));
  stats->us_prep += 1e3 * ms[0];
  stats->us_stage1 += 1e3 * ms[1];
  stats->us_process += 1e3 * ms[2];
  stats->us_finalize += 1e3 * ms[3];
  std::vector<unsigned long long> sv((size_t)nq * kStatCount);
  d2h(sv.data(), g.qs.stats, sv.size(), st);
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
  if (g.screen) {
    unsigned long long tl[2];
    int64_t pairs = 0;
    d2h(tl, g.sc.tally, 2, st);
    d2h(&pairs, g.sc.off + ix->n_leaves, 1, st);
    stats->screened += (int64_t)tl[0];
    stats->leaves_kept += pairs;
  }
}

// One group of queries sharing a distance and window, run to completion on
// context c: nq queries whose rows (input and output) are d_qmap[i] and
// whose k are d_kq[i] (both null for a plain call: rows 0..nq-1, every
// k = kmax).  Slots are kmax apart and output rows kmax entries long.  A
// near-tie log overflow reruns the group with a log four times larger.
int run_group(messi_index* ix, QueryCtx& c, QueryCtx& main, const float* queries, int nq, int kmax,
              int distance, int window, const int* d_kq, const int* d_qmap, bool screen,
              bool lb_improved, int64_t* out_ids, float* out_dists, messi_stats* stats,
              const Tune& t, const FixedScratch* fixed = nullptr, bool min_work = false) {
  GroupLaunch g;
  const int rc = plan_group(ix, main, nq, kmax, distance, window, screen, lb_improved, stats != nullptr,
                            t, g);
  if (rc != MESSI_OK) return rc;
  if (!fixed) ensure_status(c, nq);
  if (stats) ensure_events(c);
  const hipStream_t st = c.stream;
  for (int attempt = 0; attempt < 8; ++attempt) {
    if (!fixed) ensure_workspace(ix, c, nq, kmax);
    bind_group(c, g, queries, d_kq, d_qmap, out_ids, out_dists, fixed);
    enqueue_group(ix, c, g, st, stats != nullptr, min_work);
    if (fixed)
      d2h(fixed->h_status, g.qs.status, nq, st);
    else
      HIP_OR_THROW(hipStreamSynchronize(st));
    if (!(group_status(fixed ? fixed->h_status : c.h_status, nq) & 1)) {
      if (stats) add_group_stats(ix, c, g, stats, st);
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
  return run_group(ix, ix->ctx, ix->ctx, queries, nq, k, distance, window, nullptr, nullptr, false, false,
                   out_ids, out_dists, stats, Tune{}, nullptr, true);
}

// Context of a batch's group g >= 1 when groups overlap: its own stream
// (default priority), workspace, status words and events.
QueryCtx& group_ctx(QueryCtx& ctx, int g) {
  if (g == 0) return ctx;
  while ((int)ctx.aux.size() < g) {
    std::unique_ptr<QueryCtx> a(new QueryCtx());
    HIP_OR_THROW(hipStreamCreateWithFlags(&a->own_stream, hipStreamNonBlocking));
    a->stream = a->own_stream;
    a->budgeted = ctx.budgeted;
    a->on_grow = ctx.on_grow;
    ctx.aux.push_back(std::move(a));
  }
  QueryCtx& a = *ctx.aux[g - 1];
  if (!a.join) HIP_OR_THROW(hipEventCreateWithFlags(&a.join, hipEventDisableTiming));
  return a;
}

// Bytes that identify a batch's launches: every argument of every launch
// and the context (so the streams) each group runs on.
std::string launch_key(const std::vector<GroupLaunch>& gl, const std::vector<QueryCtx*>& gc, bool overlap) {
  std::string key(1, overlap ? 'o' : 's');
  for (size_t g = 0; g < gl.size(); ++g) {
    key.append(reinterpret_cast<const char*>(&gl[g]), sizeof(GroupLaunch));
    key.append(reinterpret_cast<const char*>(&gc[g]), sizeof(QueryCtx*));
  }
  return key;
}

// Enqueues every group of a batch: overlapped, group g on its context's
// stream, forked from and joined into `st` with events; otherwise one
// after another on `st`.
void enqueue_batch(messi_index* ix, QueryCtx& ctx, const std::vector<GroupLaunch>& gl,
                   const std::vector<QueryCtx*>& gc, bool overlap, hipStream_t st, bool timed) {
  if (!overlap) {
    for (size_t g = 0; g < gl.size(); ++g) enqueue_group(ix, *gc[g], gl[g], st, timed, false);
    return;
  }
  HIP_OR_THROW(hipEventRecord(ctx.fork, st));
  for (size_t g = 0; g < gl.size(); ++g) {
    const hipStream_t sg = g == 0 ? st : gc[g]->stream;
    if (g > 0) HIP_OR_THROW(hipStreamWaitEvent(sg, ctx.fork, 0));
    enqueue_group(ix, *gc[g], gl[g], sg, timed, false);
    if (g > 0) {
      HIP_OR_THROW(hipEventRecord(gc[g]->join, sg));
      HIP_OR_THROW(hipStreamWaitEvent(st, gc[g]->join, 0));
    }
  }
}

// The graph of a batch's launches: found by its launch key, else captured
// (on the context's capture stream) and kept, the oldest dropped past
// kGraphCache entries.  Capture launches nothing.
constexpr size_t kGraphCache = 8;

hipGraphExec_t batch_graph(messi_index* ix, QueryCtx& ctx, const std::vector<GroupLaunch>& gl,
                           const std::vector<QueryCtx*>& gc, bool overlap, bool* captured) {
  const std::string key = launch_key(gl, gc, overlap);
  for (auto& e : ctx.graphs)
    if (e->key == key) {
      *captured = false;
      return e->exec;
    }
  if (!ctx.cap_stream) HIP_OR_THROW(hipStreamCreateWithFlags(&ctx.cap_stream, hipStreamNonBlocking));
  std::unique_ptr<GraphEntry> e(new GraphEntry());
  e->key = key;
  HIP_OR_THROW(hipStreamBeginCapture(ctx.cap_stream, hipStreamCaptureModeRelaxed));
  try {
    enqueue_batch(ix, ctx, gl, gc, overlap, ctx.cap_stream, false);
  } catch (...) {
    hipGraph_t partial = nullptr;
    (void)hipStreamEndCapture(ctx.cap_stream, &partial);
    if (partial) (void)hipGraphDestroy(partial);
    (void)hipGetLastError();
    throw;
  }
  HIP_OR_THROW(hipStreamEndCapture(ctx.cap_stream, &e->graph));
  HIP_OR_THROW(hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0));
  if (ctx.graphs.size() >= kGraphCache) ctx.graphs.erase(ctx.graphs.begin());
  ctx.graphs.push_back(std::move(e));
  *captured = true;
  return ctx.graphs.back()->exec;
}

constexpr int kScreenMinGroup = 32;  // fewer ED queries go the unscreened way (default)

// A batch's groups: queries sharing (distance, effective window), in
// first-seen order.
struct BatchGroups {
  std::vector<std::pair<int, int>> keys;
  std::vector<std::vector<int>> members;
};

BatchGroups group_batch(const messi_index* ix, int nq, const int32_t* distance, const int32_t* window) {
  BatchGroups b;
  for (int i = 0; i < nq; ++i) {
    const std::pair<int, int> key(distance[i],
                                  distance[i] == MESSI_DTW ? std::min(window[i], ix->len - 1) : 0);
    size_t g = 0;
    while (g < b.keys.size() && b.keys[g] != key) ++g;
    if (g == b.keys.size()) {
      b.keys.push_back(key);
      b.members.emplace_back();
    }
    b.members[g].push_back(i);
  }
  return b;
}

std::string tune_key(const messi_index* ix, int nq, const BatchGroups& b, int flags);
Tune tune_for(const messi_index* ix, const std::string& key);

// How a batch runs: its knobs, and whether its launches go through a
// graph and its groups may overlap.
struct BatchMode {
  const Tune* tune = nullptr;  // null: the tuned knobs of the batch's shape, else the defaults
  bool graph = false;
  bool allow_overlap = true;
  bool* captured = nullptr;    // graph runs: set if the graph was captured by this call
};

// Validated batch on one query context.  Sequential groups (stats, one
// group or no overlap) run one run_group each; otherwise every group is
// bound first and the whole batch is enqueued at once - overlapped on the
// groups' own streams, and / or replayed from a graph - with one
// synchronisation, after which a group whose near-tie log overflowed is
// rerun alone.
int run_batch(messi_index* index, QueryCtx& ctx, const float* queries, int nq, const int32_t* k,
              const int32_t* distance, const int32_t* window, int kmax, int flags,
              int64_t* out_ids, float* out_dists, messi_stats* stats, const BatchMode& mode = BatchMode{}) {
  const int len = index->len;
  const BatchGroups bg = group_batch(index, nq, distance, window);
  const int G = (int)bg.keys.size();
  try {
    const Tune t = mode.tune ? *mode.tune : tune_for(index, tune_key(index, nq, bg, flags));
    const bool want_screen = (flags & MESSI_SCREEN_BF16) && screen_supported(len) && t.screen;
    const bool lbi = (flags & MESSI_LB_IMPROVED) != 0;
    ensure_batch(index, ctx, nq);
    std::vector<int> hmap, hk;
    hmap.reserve(nq);
    hk.reserve(nq);
    for (const auto& m : bg.members)
      for (int i : m) {
        hmap.push_back(i);
        hk.push_back(k[i]);
      }
    h2d(ctx.bmap, hmap.data(), (size_t)nq, ctx.stream);
    h2d(ctx.bk, hk.data(), (size_t)nq, ctx.stream);
    std::vector<int> at(G + 1, 0), cnt(G);
    std::vector<bool> scr(G);
    for (int g = 0; g < G; ++g) {
      cnt[g] = (int)bg.members[g].size();
      at[g + 1] = at[g] + cnt[g];
      // the screen streams every leaf some query of the group keeps, so it
      // pays off only when many queries share that pass
      scr[g] = want_screen && bg.keys[g].first == MESSI_ED && cnt[g] >= std::max(1, t.screen_min);
      if (scr[g] && !index->Zb) return fail(MESSI_EINVAL, "the BF16 screen copy is not prepared");
    }
    // every group's kernels must fit this length and window before any
    // group runs (argument errors leave the outputs untouched)
    for (int g = 0; g < G; ++g) {
      GroupLaunch probe;
      const int rc = plan_group(index, ctx, cnt[g], kmax, bg.keys[g].first, bg.keys[g].second, scr[g], lbi,
                                false, t, probe);
      if (rc != MESSI_OK) return rc;
    }
    const bool overlap = mode.allow_overlap && t.overlap && G > 1;
    if (!mode.graph && !overlap) {
      for (int g = 0; g < G; ++g) {
        const int rc = run_group(index, ctx, ctx, queries, cnt[g], kmax, bg.keys[g].first, bg.keys[g].second,
                                 ctx.bk + at[g], ctx.bmap + at[g], scr[g], lbi, out_ids, out_dists, stats, t);
        if (rc != MESSI_OK) return rc;
      }
      return MESSI_OK;
    }
    const bool timed = stats != nullptr && !mode.graph;
    std::vector<GroupLaunch> gl(G);
    std::vector<QueryCtx*> gc(G);
    int max_cnt = 0;
    for (int g = 0; g < G; ++g) max_cnt = std::max(max_cnt, cnt[g]);
    if (overlap && !ctx.fork) HIP_OR_THROW(hipEventCreateWithFlags(&ctx.fork, hipEventDisableTiming));
    for (int g = 0; g < G; ++g) {
      gc[g] = overlap ? &group_ctx(ctx, g) : &ctx;
      const int rc = plan_group(index, ctx, cnt[g], kmax, bg.keys[g].first, bg.keys[g].second, scr[g], lbi,
                                timed, t, gl[g]);
      if (rc != MESSI_OK) return rc;
    }
    // all allocation before any launch (and before a capture)
    for (int g = 0; g < G; ++g) {
      QueryCtx& c = *gc[g];
      ensure_status(c, overlap ? cnt[g] : nq);
      ensure_workspace(index, c, overlap ? cnt[g] : max_cnt, kmax);
      if (timed) ensure_events(c);
    }
    for (int g = 0; g < G; ++g)
      bind_group(*gc[g], gl[g], queries, ctx.bk + at[g], ctx.bmap + at[g], out_ids, out_dists, nullptr,
                 overlap ? 0 : at[g]);
    if (mode.graph) {
      bool captured = false;
      const hipGraphExec_t exec = batch_graph(index, ctx, gl, gc, overlap, &captured);
      if (mode.captured) *mode.captured = captured;
      HIP_OR_THROW(hipGraphLaunch(exec, ctx.stream));
    } else {
      enqueue_batch(index, ctx, gl, gc, overlap, ctx.stream, timed);
    }
    HIP_OR_THROW(hipStreamSynchronize(ctx.stream));
    for (int g = 0; g < G; ++g) {
      const int* hs = overlap ? gc[g]->h_status : ctx.h_status + at[g];
      if (!(group_status(hs, cnt[g]) & 1)) {
        if (timed) add_group_stats(index, *gc[g], gl[g], stats, gc[g]->stream);
        continue;
      }
      // near-tie log overflow: this group again, alone, with a larger log
      if (stats) stats->log_overflows += 1;
      gc[g]->log_cap *= 4;
      const int rc = run_group(index, *gc[g], ctx, queries, cnt[g], kmax, bg.keys[g].first, bg.keys[g].second,
                               ctx.bk + at[g], ctx.bmap + at[g], scr[g], lbi, out_ids, out_dists, stats, t);
      if (rc != MESSI_OK) return rc;
    }
  } catch (const OomError& e) {
    return fail(MESSI_ENOMEM, "device allocation of %zu bytes failed", e.bytes);
  } catch (const BudgetError& e) {
    return fail(MESSI_ENOMEM, "the index would hold %zu bytes, over its memory budget of %zu", e.need,
                e.budget);
  } catch (const HipError& e) {
    return fail(MESSI_EDEVICE, "%s: %s", e.what, hipGetErrorString(e.e));
  }
  return MESSI_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: the batched path's knobs (Tune) chosen per batch shape by
// timing candidates on a real batch, kept per index and in a JSON file
// (messi_options.autotune_cache) keyed by device, index shape, batch size
// bucket and the batch's (distance, window) mix.

std::string device_tag() {
  int dev = 0;
  hipDeviceProp_t pr{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&pr, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  std::string arch(pr.gcnArchName);
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch.resize(colon);
  return arch + "x" + std::to_string(pr.multiProcessorCount);
}

std::string tune_key(const messi_index* ix, int nq, const BatchGroups& b, int flags) {
  int bucket = 1;
  while (bucket < nq) bucket <<= 1;
  std::vector<std::string> mix;
  for (const auto& key : b.keys)
    mix.push_back(key.first == MESSI_ED ? std::string("ed") : "dtw" + std::to_string(key.second));
  std::sort(mix.begin(), mix.end());
  std::string m;
  for (const auto& s : mix) m += (m.empty() ? "" : "+") + s;
  char buf[256];
  snprintf(buf, sizeof(buf), "%s/n%lld/len%d/w%d/c%d/leaf%d/%s/nq%d/", ix->device.c_str(), (long long)ix->n,
           ix->len, ix->w, ix->card_bits, ix->leaf_size, ix->raw ? "raw" : "z", bucket);
  std::string key = buf + m;
  if ((flags & MESSI_SCREEN_BF16) && screen_supported(ix->len)) key += "/screen";
  if (flags & MESSI_LB_IMPROVED) key += "/lbi";
  return key;
}

Tune tune_for(const messi_index* ix, const std::string& key) {
  std::lock_guard<std::mutex> lk(ix->tune_mu);
  auto it = ix->tunes.find(key);
  return it == ix->tunes.end() ? Tune{} : it->second.t;
}

// The knobs in the cache file's order: name, member.
const std::pair<const char*, int Tune::*> kTuneFields[] = {
    {"screen", &Tune::screen},     {"screen_min", &Tune::screen_min}, {"screen_nt", &Tune::screen_nt},
    {"screen_occ", &Tune::screen_occ}, {"screen_waves", &Tune::screen_waves}, {"ed_scale", &Tune::ed_scale},
    {"dtw_scale", &Tune::dtw_scale}, {"overlap", &Tune::overlap}};

// Minimal reader of the cache file: an object whose members are objects of
// numbers, {"key": {"name": number, ...}, ...}.  Returns false on any
// other text.
struct JsonReader {
  const std::string& s;
  size_t i = 0;
  explicit JsonReader(const std::string& text) : s(text) {}
  void ws() {
    while (i < s.size() && (s[i] == ' ' || s[i] == '\n' || s[i] == '\r' || s[i] == '\t')) ++i;
  }
  bool lit(char c) {
    ws();
    if (i < s.size() && s[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  bool str(std::string* out) {
    ws();
    if (i >= s.size() || s[i] != '"') return false;
    ++i;
    out->clear();
    while (i < s.size() && s[i] != '"') {
      if (s[i] == '\\') return false;  // keys the library writes never need escapes
      out->push_back(s[i++]);
    }
    if (i >= s.size()) return false;
    ++i;
    return true;
  }
  bool num(double* v) {
    ws();
    const char* b = s.c_str() + i;
    char* e = nullptr;
    *v = std::strtod(b, &e);
    if (e == b) return false;
    i += (size_t)(e - b);
    return true;
  }
};

bool parse_tunes(const std::string& text, std::map<std::string, TuneEntry>* out) {
  JsonReader r(text);
  if (!r.lit('{')) return false;
  if (r.lit('}')) return true;
  for (;;) {
    std::string key;
    if (!r.str(&key) || !r.lit(':') || !r.lit('{')) return false;
    TuneEntry e;
    if (!r.lit('}')) {
      for (;;) {
        std::string name;
        double v = 0.0;
        if (!r.str(&name) || !r.lit(':') || !r.num(&v)) return false;
        for (const auto& f : kTuneFields)
          if (name == f.first) e.t.*(f.second) = (int)v;
        if (name == "ms") e.ms = v;
        if (name == "ms_default") e.ms_default = v;
        if (r.lit('}')) break;
        if (!r.lit(',')) return false;
      }
    }
    (*out)[key] = e;
    if (r.lit('}')) break;
    if (!r.lit(',')) return false;
  }
  r.ws();
  return r.i == text.size();
}

std::string format_tunes(const std::map<std::string, TuneEntry>& m) {
  std::string o = "{\n";
  bool first = true;
  for (const auto& kv : m) {
    if (!first) o += ",\n";
    first = false;
    o += "  \"" + kv.first + "\": {";
    for (const auto& f : kTuneFields) o += "\"" + std::string(f.first) + "\": " + std::to_string(kv.second.t.*(f.second)) + ", ";
    char buf[96];
    snprintf(buf, sizeof(buf), "\"ms\": %.4f, \"ms_default\": %.4f}", kv.second.ms, kv.second.ms_default);
    o += buf;
  }
  o += "\n}\n";
  return o;
}

// Reads a cache file; a missing file is an empty cache.
bool read_tune_file(const std::string& path, std::map<std::string, TuneEntry>* out, std::string* err) {
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return true;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
  std::fclose(f);
  if (!parse_tunes(text, out)) {
    *err = "autotune cache " + path + " is not a file this library wrote";
    return false;
  }
  return true;
}

// Merges this index's entries into the file (re-read first, so entries
// other indexes wrote are kept) through a temporary file and a rename.
bool write_tune_file(const std::string& path, const std::map<std::string, TuneEntry>& mine, std::string* err) {
  std::map<std::string, TuneEntry> all;
  if (!read_tune_file(path, &all, err)) return false;
  for (const auto& kv : mine) all[kv.first] = kv.second;
  const std::string tmp = path + ".tmp" + std::to_string((long long)getpid());
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) {
    *err = "cannot write " + tmp;
    return false;
  }
  const std::string text = format_tunes(all);
  const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
  if (std::fclose(f) != 0 || !ok || std::rename(tmp.c_str(), path.c_str()) != 0) {
    std::remove(tmp.c_str());
    *err = "cannot write " + path;
    return false;
  }
  return true;
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
  std::atomic<int64_t> resident{0};  // device bytes this worker holds
  ~SrvWorker() {
    if (h_q) (void)hipHostFree(h_q);
    if (h_ids) (void)hipHostFree(h_ids);
    if (h_d) (void)hipHostFree(h_d);
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
  int64_t log_growth = 0;  // bytes charged for near-tie log growth, summed
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
      BatchMode mode;
      mode.allow_overlap = false;  // one workspace per worker: its size is what the budget counts
      rc = run_batch(ix, w->ctx, w->d_q, nb, ks.data(), ds.data(), ws.data(), kmax, flags,
                     w->d_ids, w->d_d, nullptr, mode);
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
    // a near-tie log grown by this batch (charged to the ledger as it grew)
    // goes back to the starting size, and its bytes back off the ledger
    try {
      shrink_log(ix, w->ctx, w->cap, kmax);
    } catch (const HipError& e) {
      if (rc == MESSI_OK) rc = MESSI_EDEVICE;
    } catch (const OomError& e) {
      if (rc == MESSI_OK) rc = MESSI_ENOMEM;
    }
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
  const auto t_start = std::chrono::steady_clock::now();
  const double alloc0 = g_alloc_ms;
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
  if (o.inplace < 0 || o.inplace > 2) return fail(MESSI_EINVAL, "inplace must be 0, 1 or 2");
  if (o.mem_budget_bytes < 0) return fail(MESSI_EINVAL, "mem_budget_bytes must be >= 0");
  if (o.inplace && (reinterpret_cast<uintptr_t>(series) & 15))
    return fail(MESSI_EINVAL, "an in-place series buffer must be 16-byte aligned");
  const size_t store_b = (size_t)n * len * sizeof(float);
  if (o.inplace == 2) {  // the library takes the buffer over: it must be one whole allocation
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)series) != hipSuccess ||
        (void*)base != (void*)series || size < store_b) {
      (void)hipGetLastError();
      return fail(MESSI_EINVAL, "inplace = 2 takes over only the start of a hipMalloc allocation "
                                "holding the series");
    }
  }
  std::map<std::string, TuneEntry> cached;
  if (o.autotune_cache) {
    std::string err;
    if (!read_tune_file(o.autotune_cache, &cached, &err)) return fail(MESSI_EINVAL, "%s", err.c_str());
  }
  messi_index* ix = new messi_index();
  ix->budget = o.mem_budget_bytes;
  ix->device = device_tag();
  if (o.autotune_cache) ix->tune_path = o.autotune_cache;
  ix->tunes = std::move(cached);
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
  if (ix->budget > 0 && need + (o.inplace == 2 ? store_b : 0) > (size_t)ix->budget) {
    delete ix;
    return fail(MESSI_ENOMEM, "index needs about %zu bytes, over its memory budget of %lld",
                need + (o.inplace == 2 ? store_b : 0), (long long)ix->budget);
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
  // the tables' working buffers are gone: what the index holds now
  if (o.inplace == 2) ix->store_bytes = store_b;
  if (ix->budget > 0 && held_bytes(ix) > (size_t)ix->budget) {
    const size_t held = held_bytes(ix);
    delete ix;
    return fail(MESSI_ENOMEM, "the index holds %zu bytes, over its memory budget of %lld", held,
                (long long)o.mem_budget_bytes);
  }
  if (o.bf16_screen && screen_supported(len)) {
    const int rc = guarded([&]() -> int {
      ensure_screen(ix);
      return MESSI_OK;
    });
    if (rc != MESSI_OK) {
      delete ix;  // the caller keeps an in-place buffer
      return rc;
    }
  }
  if (o.inplace == 2) ix->owned_store = series;  // freed by messi_free from here on
  ix->build_alloc_ms = g_alloc_ms - alloc0;
  ix->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
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
  return guarded([&]() -> int {
    return run_query(index, queries, nq, k, distance, window, out_ids, out_dists, stats);
  });
}

int messi_query(messi_index* index, const float* queries, int32_t nq, int32_t k, int32_t distance,
                int32_t window, int64_t* out_ids, float* out_dists) {
  return messi_query_stats(index, queries, nq, k, distance, window, out_ids, out_dists, nullptr);
}

namespace {

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
    return run_group(index, index->ctx, index->ctx, queries, nq, k, distance, window, nullptr, nullptr, false,
                     false, out_ids, out_dists, nullptr, Tune{}, &fx);
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
  return guarded([&]() -> int {
    ensure_screen(index);
    return MESSI_OK;
  });
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
  if (flags & ~(MESSI_SCREEN_BF16 | MESSI_LB_IMPROVED | MESSI_GRAPH)) return fail(MESSI_EINVAL, "unknown flags");
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
    const int rc = guarded([&]() -> int {
      ensure_screen(index);
      return MESSI_OK;
    });
    if (rc != MESSI_OK) return rc;
  }
  BatchMode mode;
  mode.graph = (flags & MESSI_GRAPH) && !stats;  // statistics time each phase: no graph
  return run_batch(index, index->ctx, queries, nq, k, distance, window, kmax, flags & ~MESSI_GRAPH,
                   out_ids, out_dists, stats, mode);
}

int messi_autotune(messi_index* index, const float* queries, int32_t nq, const int32_t* k,
                   const int32_t* distance, const int32_t* window, int32_t kmax, int32_t flags,
                   messi_tune* out) {
  g_err.clear();
  if (!index) return fail(MESSI_EINVAL, "index is NULL");
  if (nq < 1) return fail(MESSI_EINVAL, "nq must be >= 1");
  if (kmax < 1 || kmax > 1024) return fail(MESSI_EINVAL, "kmax must be in [1, 1024]");
  if (!k || !distance || !window) return fail(MESSI_EINVAL, "k, distance and window are required");
  if (is_device_ptr(k) || is_device_ptr(distance) || is_device_ptr(window))
    return fail(MESSI_EINVAL, "k, distance and window must be host arrays");
  if (flags & ~(MESSI_SCREEN_BF16 | MESSI_LB_IMPROVED)) return fail(MESSI_EINVAL, "unknown flags");
  if (!is_device_ptr(queries)) return fail(MESSI_EINVAL, "queries must be a device pointer");
  for (int i = 0; i < nq; ++i) {
    if (k[i] < 1 || k[i] > kmax) return fail(MESSI_EINVAL, "k[%d] must be in [1, kmax]", i);
    if (distance[i] != MESSI_ED && distance[i] != MESSI_DTW)
      return fail(MESSI_EINVAL, "unknown distance[%d]", i);
    if (window[i] < 0) return fail(MESSI_EINVAL, "window[%d] must be >= 0", i);
  }
  BusyGuard guard(index->busy);
  if (!guard.ok) return fail(MESSI_EBUSY, "index is in use by another call");
  return guarded([&]() -> int {
    const bool screen_flag = (flags & MESSI_SCREEN_BF16) && screen_supported(index->len);
    if (screen_flag) ensure_screen(index);
    const BatchGroups bg = group_batch(index, nq, distance, window);
    const std::string key = tune_key(index, nq, bg, flags);
    auto report = [&](const TuneEntry& e, int from_cache, int candidates) {
      if (!out) return;
      std::memset(out, 0, sizeof(*out));
      out->screen = e.t.screen;
      out->screen_min = e.t.screen_min;
      out->screen_nt = e.t.screen_nt;
      out->screen_occ = e.t.screen_occ;
      out->screen_waves = e.t.screen_waves;
      out->ed_scale = e.t.ed_scale;
      out->dtw_scale = e.t.dtw_scale;
      out->overlap = e.t.overlap;
      out->from_cache = from_cache;
      out->candidates = candidates;
      out->ms = e.ms;
      out->ms_default = e.ms_default;
    };
    {
      std::lock_guard<std::mutex> lk(index->tune_mu);
      auto it = index->tunes.find(key);
      if (it != index->tunes.end()) {
        report(it->second, 1, 0);
        return MESSI_OK;
      }
    }
    // answers of the defaults (slot 0) and of each candidate (slot 1)
    const size_t cells = (size_t)nq * kmax;
    check_budget(index, index->ctx, 0, 2 * cells * (sizeof(int64_t) + sizeof(float)));
    DevMem tmp;
    int64_t* ids[2] = {tmp.alloc<int64_t>(cells), tmp.alloc<int64_t>(cells)};
    float* dd[2] = {tmp.alloc<float>(cells), tmp.alloc<float>(cells)};
    int rc = MESSI_OK;
    auto run = [&](const Tune& t, int slot) -> double {
      BatchMode m;
      m.tune = &t;
      const auto t0 = Clock::now();
      const int r = run_batch(index, index->ctx, queries, nq, k, distance, window, kmax, flags, ids[slot],
                              dd[slot], nullptr, m);
      if (r != MESSI_OK) rc = r;
      return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
    };
    // rows whose answers differ from the defaults' (first one in *first)
    auto rows_differing = [&](int* first) {
      std::vector<int64_t> a(cells), b(cells);
      std::vector<float> x(cells), y(cells);
      d2h(a.data(), ids[0], cells, index->ctx.stream);
      d2h(b.data(), ids[1], cells, index->ctx.stream);
      d2h(x.data(), dd[0], cells, index->ctx.stream);
      d2h(y.data(), dd[1], cells, index->ctx.stream);
      int rows = 0;
      *first = -1;
      for (int i = 0; i < nq; ++i) {
        const size_t o = (size_t)i * kmax;
        if (std::memcmp(&a[o], &b[o], kmax * sizeof(int64_t)) != 0 ||
            std::memcmp(&x[o], &y[o], kmax * sizeof(float)) != 0) {
          if (*first < 0) *first = i;
          ++rows;
        }
      }
      return rows;
    };
    Tune best;
    run(best, 0);  // first use of the kernels and buffers, untimed
    double best_ms = std::min(run(best, 0), run(best, 0));
    if (rc != MESSI_OK) return rc;
    const double default_ms = best_ms;
    bool has_ed = false, has_dtw = false, screenable = false;
    for (size_t g = 0; g < bg.keys.size(); ++g) {
      has_ed |= bg.keys[g].first == MESSI_ED;
      has_dtw |= bg.keys[g].first == MESSI_DTW;
      screenable |= screen_flag && bg.keys[g].first == MESSI_ED && (int)bg.members[g].size() >= kScreenMinGroup;
    }
    int candidates = 1;
    // coordinate descent: each knob in turn, keeping a setting only if it
    // beats the best so far by 2%
    auto try_setting = [&](const char* name, const Tune& c) -> int {
      double ms = run(c, 1);
      if (rc != MESSI_OK) return rc;
      if (ms < 1.15 * best_ms) ms = std::min(ms, run(c, 1));  // a second run only for contenders
      if (rc != MESSI_OK) return rc;
      ++candidates;
      int first = -1;
      const int bad = rows_differing(&first);
      if (bad)
        return fail(MESSI_EDEVICE, "autotune: with %s, %d rows (first: row %d) differ from the defaults' "
                    "answers", name, bad, first);
      if (ms < 0.98 * best_ms) {
        best = c;
        best_ms = ms;
      }
      return MESSI_OK;
    };
    auto try_knob = [&](const char* name, int Tune::*knob, std::initializer_list<int> values) -> int {
      for (int v : values) {
        Tune c = best;
        c.*knob = v;
        if (c.*knob == best.*knob) continue;
        char what[64];
        snprintf(what, sizeof(what), "%s = %d", name, v);
        const int r2 = try_setting(what, c);
        if (r2 != MESSI_OK) return r2;
      }
      return MESSI_OK;
    };
    int r = MESSI_OK;
    if (screenable) r = try_knob("screen", &Tune::screen, {0});
    if (r == MESSI_OK && screenable && best.screen) {
      const int len = index->len, w0 = screen_waves_default();
      for (int nt : {1, 2, 4})
        if (r == MESSI_OK && nt != screen_nt_default(len) && screen_variant(len, nt, w0))
          r = try_knob("screen_nt", &Tune::screen_nt, {nt});
      // the other block size, with each column tile count it is built for
      const int w1 = w0 == 4 ? 8 : 4;
      for (int nt : {1, 2, 4}) {
        if (r != MESSI_OK || !screen_variant(len, nt, w1)) continue;
        Tune c = best;
        c.screen_nt = nt;
        c.screen_waves = w1;
        char what[64];
        snprintf(what, sizeof(what), "screen_nt = %d, screen_waves = %d", nt, w1);
        r = try_setting(what, c);
      }
      if (r == MESSI_OK) r = try_knob("screen_occ", &Tune::screen_occ, {1, 2});
    }
    if (r == MESSI_OK && has_ed && !(screenable && best.screen)) r = try_knob("ed_scale", &Tune::ed_scale, {2});
    if (r == MESSI_OK && has_dtw) r = try_knob("dtw_scale", &Tune::dtw_scale, {2, 4});
    if (r == MESSI_OK && bg.keys.size() > 1) r = try_knob("overlap", &Tune::overlap, {0});
    if (r != MESSI_OK) return r;
    TuneEntry e;
    e.t = best;
    e.ms = best_ms;
    e.ms_default = default_ms;
    std::map<std::string, TuneEntry> snapshot;
    {
      std::lock_guard<std::mutex> lk(index->tune_mu);
      index->tunes[key] = e;
      snapshot = index->tunes;
    }
    report(e, 0, candidates);
    if (!index->tune_path.empty()) {
      std::string err;
      if (!write_tune_file(index->tune_path, snapshot, &err)) return fail(MESSI_EINVAL, "%s", err.c_str());
    }
    return MESSI_OK;
  });
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
  return guarded([&]() -> int {
    if ((flags & MESSI_SCREEN_BF16) && screen_supported(index->len)) ensure_screen(index);
    const std::vector<int32_t> ks(nq, k), ds(nq, distance), ws(nq, window);
    const int rc = run_batch(index, index->ctx, queries, nq, ks.data(), ds.data(), ws.data(), k,
                             flags, out_ids, out_dists, nullptr);
    if (rc != MESSI_OK) return rc;
    launch_vote(out_ids, k, nq, k, labels, n_classes, out_class, index->ctx.stream);
    launch_check();
    HIP_OR_THROW(hipStreamSynchronize(index->ctx.stream));
    return MESSI_OK;
  });
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
  if (device_bytes) *device_bytes = (int64_t)held_bytes(index);
  return MESSI_OK;
}

int messi_build_times(const messi_index* index, double* build_ms, double* alloc_ms) {
  if (!index) return fail(MESSI_EINVAL, "index is NULL");
  if (build_ms) *build_ms = index->build_ms;
  if (alloc_ms) *alloc_ms = index->build_alloc_ms;
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
  if (S->budget == 0 && index->budget > 0)  // the index's budget, less what the index holds
    S->budget = std::max<int64_t>(1, index->budget - (int64_t)held_bytes(index));
  S->req_bytes = request_bytes(index, kmax, kLogCap0);
  if (hipGetDevice(&S->device) != hipSuccess) return fail(MESSI_EDEVICE, "no current HIP device");
  // batch capacity: every worker holds the buffers of `cap` requests from
  // the start, and all of them together stay within the budget
  int cap = max_batch;
  if (S->budget > 0)
    cap = (int)std::max<int64_t>(1, std::min<int64_t>(cap, S->budget / ((int64_t)workers * S->req_bytes)));
  const int rc = guarded([&]() -> int {
    if ((o.flags & MESSI_SCREEN_BF16) && screen_supported(index->len)) ensure_screen(index);
    for (;;) {
      int64_t total = 0;
      for (int i = 0; i < workers; ++i) {
        std::unique_ptr<SrvWorker> w(new SrvWorker());
        HIP_OR_THROW(hipStreamCreateWithFlags(&w->ctx.own_stream, hipStreamNonBlocking));
        w->ctx.stream = w->ctx.own_stream;
        w->cap = cap;
        w->d_q = w->io.alloc<float>((size_t)cap * index->len);
        w->d_ids = w->io.alloc<int64_t>((size_t)cap * kmax);
        w->d_d = w->io.alloc<float>((size_t)cap * kmax);
        HIP_OR_THROW(hipHostMalloc((void**)&w->h_q, sizeof(float) * cap * index->len, hipHostMallocDefault));
        HIP_OR_THROW(hipHostMalloc((void**)&w->h_ids, sizeof(int64_t) * cap * kmax, hipHostMallocDefault));
        HIP_OR_THROW(hipHostMalloc((void**)&w->h_d, sizeof(float) * cap * kmax, hipHostMallocDefault));
        ensure_workspace(index, w->ctx, cap, kmax);
        ensure_batch(index, w->ctx, cap);
        ensure_status(w->ctx, cap);
        w->resident = (int64_t)(ctx_bytes(w->ctx) + w->io.bytes);
        total += w->resident;
        S->workers.push_back(std::move(w));
      }
      if (S->budget <= 0 || total <= S->budget || cap == 1) break;
      // per-worker buffers the request estimate leaves out: fewer requests
      cap = std::max(1, std::min(cap - 1, (int)((double)cap * (double)S->budget / (double)total)));
      S->workers.clear();
    }
    for (auto& wp : S->workers) {
      SrvWorker* w = wp.get();
      messi_server* srv = S.get();
      w->ctx.on_grow = [srv, w](int64_t d) {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->inflight += d;
        srv->peak_inflight = std::max(srv->peak_inflight, srv->inflight);
        if (d > 0) srv->log_growth += d;
        w->resident += d;
      };
    }
    return MESSI_OK;
  });
  if (rc != MESSI_OK) return rc;
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
  st->resident_bytes = 0;
  for (const auto& w : server->workers) st->resident_bytes += w->resident.load();
  st->log_growth_bytes = server->log_growth;
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
