// C-ABI of the hjpd library (declarations and contracts in include/hjpd.h).
//
// A solve is a short, graph-capturable stream sequence:
//   1. k_queue_zero     clear the bucket counters;
//   2. k_queue_count    validate each point (bad inputs get HJPD_PT_BADINPUT
//                       and are not queued), count points per bucket: N
//                       major, a quantised work hint minor;
//   3. k_queue_scan     one block: bucket offsets in descending N and, within
//                       one N, descending hint; begin/end of each tile
//                       class's segment; zero the pop counters;
//   4. k_queue_scatter  write point ids into their bucket;
//   5. one persistent kernel per tile class (or one plain kernel).
// No host synchronisation and no allocation happen inside the sequence, so
// it can be captured into a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hjpd.h"
#include "hjpd_launch.hpp"
#include "hjpd_lintanh.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

bool has_recipe(const hjpd_desc& d) { return d.starts > 1 || d.restarts > 0 || d.value_tol > 0.0; }
bool has_mix(const hjpd_desc& d) { return (d.flags & (HJPD_FORWARD_EULER | HJPD_TRAPEZOID)) != 0; }
// Persistent kernel variant of a descriptor (validated: recipes and weighted
// discretisations exclude each other).
int kernel_variant(const hjpd_desc& d) {
  if (has_recipe(d)) return hjpd::kVarRecipe;
  if (has_mix(d)) return hjpd::kVarMix;
  // Algorithms 1 and 2 for the eikonal family run in the shifted layout (node 0 is an ordinary slot)
  if (d.H == HJPD_H_CNORM && d.d_y == 0) return (d.flags & HJPD_HOPF) ? hjpd::kVarShiftHopf : hjpd::kVarShift;
  if (d.H == HJPD_H_ISAACS && !(d.flags & HJPD_HOPF)) return hjpd::kVarGameLax;
  return hjpd::kVarPlain;
}

#define HIP_OK(expr, what)                                                                 \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(HJPD_EDEVICE, std::string(what) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// Queue builder kernels
// ---------------------------------------------------------------------------

__global__ void k_queue_zero(int32_t* a, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

// Work hint: a point that starts far from the minimiser of g tends to need
// more iterations (its optimal path travels farther), so within one N the
// queue hands out far points first and the slow ones do not start last
// (longest-expected-first scheduling; order only, results are unchanged).
// The hint is the distance to the minimiser of g (QUAD_SHIFT: ||x - a||;
// NORM: ||x||; PAIR_DIST: ||r_P - r_E||; SADDLE_QUAD: ||(x, y)||, the
// distance to its saddle point), quantised on a log scale into kHintBuckets
// buckets.
constexpr int kHintBuckets = 16;
enum : int { kHintNone = 0, kHintShift = 1, kHintNorm = 2, kHintPair = 3 };

template <typename T>
__device__ int hint_bucket(int kind, int64_t i, int d, int d_y, const T* x, const T* gp) {
  if (kind == kHintNone) return 0;
  double ss = 0.0;
  if (kind == kHintPair) {
    const int dx = d - d_y;
    for (int k = 0; k < 3; k++) {
      const double r = double(x[i * d + k]) - double(x[i * d + dx + k]);
      ss += r * r;
    }
  } else {
    for (int k = 0; k < d; k++) {
      const double r = double(x[i * d + k]) - (kind == kHintShift ? double(gp[1 + k]) : 0.0);
      ss += r * r;
    }
  }
  const int b = int(4.0 * log2(1.0 + sqrt(ss)));
  const int q = b < 0 ? 0 : (b >= kHintBuckets ? kHintBuckets - 1 : b);
  return kHintBuckets - 1 - q;  // bucket 0 = largest hint
}

// Per-point validation shared by the counting and scattering passes.
template <typename T>
__device__ bool point_ok(int64_t i, int d, int N_max, const T* x, const T* t, const int32_t* N) {
  const int Ni = N[i];
  const T ti = t[i];
  bool bad = !(ti > T(0)) || !__builtin_isfinite(ti) || Ni < 1 || Ni > N_max;
  for (int k = 0; k < d && !bad; k++) bad = !__builtin_isfinite(x[i * d + k]);
  return !bad;
}

// Bucket keys of every context that uses the queue: N <= kMaxCapacity, so a
// block's histogram over all keys fits in 16.4 KB of LDS.
constexpr int kMaxKeys = (hjpd::kMaxCapacity + 1) * kHintBuckets;
constexpr int kQueueBlock = 256;
constexpr int kQueuePerThread = 1;  // points per thread: 256 per block, enough blocks to cover the chip
constexpr int kScanBlock = 1024;

// Counting and scattering share one shape: each block takes kQueueBlock *
// kQueuePerThread consecutive points, builds its histogram over keys with LDS atomics, and then issues
// one global atomic per key it holds.  All blocks hit the same few dozen
// counters (points share a few N values), so aggregating per block rather
// than per wave keeps those global atomics from serialising.  The position of
// a point inside its block's share of a bucket is the value its LDS atomic
// returned, so the order within a bucket varies from run to run; every point
// is solved on its own and its results do not depend on that order.
template <typename T>
__global__ __launch_bounds__(kQueueBlock) void k_queue_count(int64_t n, int d, int d_y, int N_max, const T* x,
                                                             const T* t, const int32_t* N, int hint, const T* gp,
                                                             int nkeys, int32_t* counts, T* phi, int32_t* iters,
                                                             int32_t* status) {
  __shared__ int32_t hist[kMaxKeys];
  for (int k = threadIdx.x; k < nkeys; k += kQueueBlock) hist[k] = 0;
  __syncthreads();
  const int64_t base = int64_t(blockIdx.x) * (kQueueBlock * kQueuePerThread) + threadIdx.x;
  for (int r = 0; r < kQueuePerThread; r++) {
    const int64_t i = base + int64_t(r) * kQueueBlock;
    if (i >= n) break;
    if (point_ok(i, d, N_max, x, t, N)) {
      atomicAdd(&hist[N[i] * kHintBuckets + hint_bucket(hint, i, d, d_y, x, gp)], 1);
    } else {
      phi[i] = T(NAN);
      iters[i] = 0;
      status[i] = hjpd::kBadInput;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nkeys; k += kQueueBlock)
    if (hist[k]) atomicAdd(&counts[k], hist[k]);
}

template <typename T>
__global__ __launch_bounds__(kQueueBlock) void k_queue_scatter(int64_t n, int d, int d_y, int N_max, const T* x,
                                                               const T* t, const int32_t* N, int hint, const T* gp,
                                                               int nkeys, int32_t* cursor, int32_t* queue) {
  __shared__ int32_t hist[kMaxKeys];
  for (int k = threadIdx.x; k < nkeys; k += kQueueBlock) hist[k] = 0;
  __syncthreads();
  const int64_t base = int64_t(blockIdx.x) * (kQueueBlock * kQueuePerThread) + threadIdx.x;
  int key[kQueuePerThread], rank[kQueuePerThread];
  for (int r = 0; r < kQueuePerThread; r++) {
    const int64_t i = base + int64_t(r) * kQueueBlock;
    key[r] = -1;
    if (i < n && point_ok(i, d, N_max, x, t, N)) {
      key[r] = N[i] * kHintBuckets + hint_bucket(hint, i, d, d_y, x, gp);
      rank[r] = atomicAdd(&hist[key[r]], 1);
    }
  }
  __syncthreads();
  // reserve this block's share of each bucket; the histogram now holds its start
  for (int k = threadIdx.x; k < nkeys; k += kQueueBlock)
    if (hist[k]) hist[k] = atomicAdd(&cursor[k], hist[k]);
  __syncthreads();
  for (int r = 0; r < kQueuePerThread; r++)
    if (key[r] >= 0) queue[hist[key[r]] + rank[r]] = int32_t(base + int64_t(r) * kQueueBlock);
}

// Bucket offsets: buckets are laid out in descending N and, within one N,
// ascending hint bucket (bucket 0 holds the largest hint).  Position o of
// that order holds key (N_max - o / kHintBuckets) * kHintBuckets +
// o % kHintBuckets.  One block: each thread sums a run of consecutive
// positions, a block-wide scan in LDS gives the run's start, and the thread
// writes its offsets.  A class [lo, hi] spans the positions from (hi, 0) up
// to but not including the one after (lo, kHintBuckets - 1).
// cls_bounds: [2*ncls] (lo, hi) N-range of each class, classes disjoint.
// cls_range:  [2*(ncls+1)] begin/end of each class; the extra last entry is
//             the whole queue (used by the plain kernel).
__global__ __launch_bounds__(kScanBlock) void k_queue_scan(int N_max, int ncls, const int32_t* cls_bounds,
                                                           const int32_t* counts, int32_t* cursor, int32_t* cls_range,
                                                           int32_t* heads) {
  __shared__ int32_t part[kScanBlock];
  const int tid = threadIdx.x;
  const int nord = N_max * kHintBuckets;
  const int run = (nord + kScanBlock - 1) / kScanBlock;
  const int o0 = tid * run, o1 = min(o0 + run, nord);
  auto key_of = [&](int o) { return (N_max - o / kHintBuckets) * kHintBuckets + o % kHintBuckets; };
  int mine = 0;
  for (int o = o0; o < o1; o++) mine += counts[key_of(o)];
  part[tid] = mine;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {  // inclusive scan of the run sums
    const int v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int off = part[tid] - mine;
  for (int o = o0; o < o1; o++) {
    for (int c = 0; c < ncls; c++) {
      if (o == (N_max - cls_bounds[2 * c + 1]) * kHintBuckets) cls_range[2 * c] = off;
      if (o == (N_max - cls_bounds[2 * c] + 1) * kHintBuckets) cls_range[2 * c + 1] = off;
    }
    const int k = key_of(o);
    cursor[k] = off;
    off += counts[k];
  }
  if (tid == 0) {
    const int total = part[kScanBlock - 1];
    for (int c = 0; c < ncls; c++) {
      if (cls_bounds[2 * c] == 1) cls_range[2 * c + 1] = total;  // the class that ends the order
      heads[c] = 0;
    }
    cls_range[2 * ncls] = 0;
    cls_range[2 * ncls + 1] = total;
    heads[ncls] = 0;
  }
}

struct Cls {
  int lo, hi, L, K;
  const void* kern;
  int grid;  // persistent grid (blocks of 256)
};

// Device scratch of one solve: the bucket counters and cursors, the class
// segments, the per-class pop counters and the work queue.  hjpd_solve_batch
// takes it from the context (grown on demand); the allocation-free entry
// point takes it from the library's static per-GPU array.
struct Workspace {
  int32_t* counts;     // [(N_max+1) * kHintBuckets]
  int32_t* cursor;     // [(N_max+1) * kHintBuckets]
  int32_t* cls_range;  // [2*(ncls+1)]
  int32_t* heads;      // [ncls+1]
  int32_t* queue;      // [n]
};

// Allocation-free entry point: its scratch is a file-scope device array of
// fixed size (one copy per GPU, resident until the process ends), addressed
// from the host only through the per-device address hipGetSymbolAddress
// returns.  Layout in int32 words: queue [kStaticMaxPoints], counts
// [kMaxKeys], cursor [kMaxKeys], class segments [2*(kStaticMaxCls+1)], pop
// counters [kStaticMaxCls+1].
constexpr int64_t kStaticMaxPoints = int64_t(1) << 20;
constexpr int kStaticMaxCls = 16;
constexpr int64_t kStaticWords = kStaticMaxPoints + 2 * int64_t(kMaxKeys) + 2 * (kStaticMaxCls + 1) + (kStaticMaxCls + 1);
static __device__ __align__(256) int32_t scratch[kStaticWords];

}  // namespace

struct hjpd_ctx {
  hjpd_desc desc;
  int device = 0;
  int n_cu = 0;
  std::vector<Cls> plan;
  const void* plain_kern = nullptr;
  // device workspace
  int32_t* d_cls_bounds = nullptr;  // [2*ncls]
  int32_t* d_counts = nullptr;      // [(N_max+1) * kHintBuckets]
  int32_t* d_cursor = nullptr;      // [(N_max+1) * kHintBuckets]
  int32_t* d_cls_range = nullptr;   // [2*(ncls+1)]
  int32_t* d_heads = nullptr;       // [ncls+1]
  int ncls_alloc = 0;
  int32_t* d_queue = nullptr;
  int64_t queue_cap = 0;
  void* d_work = nullptr;
  size_t work_bytes = 0;
  // graph replay (captured on an internal stream, launched on the caller's)
  hipStream_t cap_stream = nullptr;
  // capacity classes after the first run on side streams, forked from and
  // joined back to the solve's stream (parallel branches of a captured graph)
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev_join;
  hipEvent_t ev_fork = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  std::vector<uintptr_t> gkey;
  // timing
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timing_valid = false;
  int timing_launches = 0;
  // per persistent launch (one per capacity class), recorded on the launch's own stream
  std::vector<hipEvent_t> ev_cls0, ev_cls1;
  std::vector<int> timed_cls;  // class index of each timed launch, in launch order
  // linear-tanh (differentiation) state
  hjpd::LtState* lt = nullptr;
  bool plan_from_cache = false;  // the plan came from the on-disk tuning cache
  int32_t* d_pops = nullptr;     // caller's pop counter (hjpd_set_pop_counter), not owned
};

namespace {

typedef const void* (*Lookup)(int, int, int, int);

Lookup lookup_for(const hjpd_desc& d) {
  const bool f64 = d.dtype == HJPD_F64;
  if (d.H == HJPD_H_CNORM && d.d_y == 0) {
    switch (d.d) {
      case 2: return f64 ? hjpd_lookup_cnorm2_f64 : hjpd_lookup_cnorm2_f32;
      case 3: return f64 ? hjpd_lookup_cnorm3_f64 : hjpd_lookup_cnorm3_f32;
      case 4: return f64 ? hjpd_lookup_cnorm4_f64 : hjpd_lookup_cnorm4_f32;
      case 10: return f64 ? hjpd_lookup_cnorm10_f64 : hjpd_lookup_cnorm10_f32;
    }
    return nullptr;
  }
  if (d.H == HJPD_H_QUADROTOR && d.d == 12 && d.d_y == 0) return f64 ? hjpd_lookup_quad_f64 : hjpd_lookup_quad_f32;
  if (d.H == HJPD_H_PURSUIT_EVASION && d.d == 12 && d.d_y == 6)
    return f64 ? hjpd_lookup_pursuit_f64 : hjpd_lookup_pursuit_f32;
  if (d.H == HJPD_H_ISAACS && d.d == 2 && d.d_y == 1) return f64 ? hjpd_lookup_isaacs_f64 : hjpd_lookup_isaacs_f32;
  return nullptr;
}

// A capacity class of the persistent path: the points with N in (previous
// class's hi, hi] run one launch of the tile (L lanes per point, K nodes per
// lane, L*K >= hi).
struct ClassSpec {
  int hi, L, K;
};

// Capacities a class boundary may sit at (the capacities L*K of the compiled tiles).
const int kCaps[] = {8, 16, 24, 32, 48, 64, 96, 128, 192, 256};
constexpr int kNumCaps = sizeof(kCaps) / sizeof(kCaps[0]);
constexpr int kMaxClasses = 16;
// Parallel branches of a solve: HIP's default number of hardware queues per process.
constexpr int kMaxBranches = 4;

// Default partition: classes at the power-of-two capacities and 96, 192,
// with the tile measured best for each capacity.
std::vector<ClassSpec> default_spec(int N_max) {
  static const ClassSpec kDefault[] = {{8, 8, 1},   {16, 16, 1}, {32, 16, 2}, {64, 32, 2},
                                       {96, 32, 3}, {128, 32, 4}, {192, 64, 3}, {256, 64, 4}};
  std::vector<ClassSpec> v;
  for (const ClassSpec& cs : kDefault) {
    v.push_back(cs);
    if (cs.hi >= N_max) break;
  }
  return v;
}

// Persistent grid at full occupancy: resident blocks per CU times CUs.
int persistent_grid(hjpd_ctx* c, const void* kern) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, 256, 0) != hipSuccess || nb < 1) nb = 1;
  return nb * c->n_cu;
}

// Grid of one class launch.  A persistent launch ends when its slowest points
// have run all their iterations, one after another; every extra wave on their
// SIMD takes issue slots from them (a wave alone issues about twice as fast as
// one of three).  Unless the batch is many times what the grid holds at once,
// when the bulk of points sets the launch time and a third wave per SIMD hides
// more latency, the grid keeps at most kTailBlocksPerCU blocks per CU.  It
// never has more blocks than the batch fills: with a small batch the waves
// that would find the queue empty are not launched, so the busy waves spread
// over the SIMDs instead of sharing some of them.
constexpr int kTailBlocksPerCU = 2;
constexpr int64_t kBulkFactor = 8;

int launch_grid(const hjpd_ctx* c, const Cls& cl, int64_t n) {
  const int per_block = 256 / cl.L;                          // points one block holds at once
  // without refill every group takes one point: enough groups for the whole
  // batch (an upper bound on the class), each block leaving when its groups finish
  if (c->desc.flags & HJPD_NO_REFILL) return int(std::max<int64_t>(1, (n + per_block - 1) / per_block));
  const int64_t resident = int64_t(cl.grid) * per_block;     // points held at once, full occupancy
  int64_t grid = cl.grid;
  if (n <= kBulkFactor * resident) {
    const int nb = cl.grid / c->n_cu;
    grid = int64_t(nb < kTailBlocksPerCU ? nb : kTailBlocksPerCU) * c->n_cu;
  }
  const int64_t fill = (n + per_block - 1) / per_block;
  if (grid > fill) grid = fill > 0 ? fill : 1;
  return int(grid);
}

void drop_graph(hjpd_ctx* c);
int ensure_class_events(hjpd_ctx* c);

// Install a class partition: validate it, look up the kernels, upload the
// class bounds, and make sure there are side streams for the parallel
// branches and (with HJPD_TIMING) per-launch events.  The last class's hi is
// clamped to N_max; classes past N_max are dropped.
int apply_spec(hjpd_ctx* c, const std::vector<ClassSpec>& spec) {
  const hjpd_desc& D = c->desc;
  Lookup lk = lookup_for(D);
  if (!lk) return fail(HJPD_EUNSUPPORTED, "no persistent kernels for this family");
  std::vector<Cls> plan;
  int prev = 0;
  for (const ClassSpec& cs : spec) {
    if (cs.hi <= prev) return fail(HJPD_EINVAL, "plan: class bounds must ascend");
    if (cs.L * cs.K < std::min(cs.hi, D.N_max)) return fail(HJPD_EINVAL, "plan: a tile's capacity L*K is below its class's N");
    Cls cl;
    cl.lo = prev + 1;
    cl.hi = std::min(cs.hi, D.N_max);
    cl.L = cs.L;
    cl.K = cs.K;
    cl.kern = lk(0, cs.L, cs.K, kernel_variant(D));
    if (!cl.kern) return fail(HJPD_EUNSUPPORTED, "plan: tile not built");
    cl.grid = persistent_grid(c, cl.kern);
    plan.push_back(cl);
    prev = cl.hi;
    if (prev >= D.N_max) break;
  }
  if (plan.empty() || prev < D.N_max) return fail(HJPD_EINVAL, "plan: the classes must cover N = 1..N_max");
  if (int(plan.size()) > kMaxClasses) return fail(HJPD_EINVAL, "plan: at most 16 classes");
  const int ncls = int(plan.size());
  if (ncls > c->ncls_alloc) {
    if (c->d_cls_bounds) (void)hipFree(c->d_cls_bounds);
    if (c->d_cls_range) (void)hipFree(c->d_cls_range);
    if (c->d_heads) (void)hipFree(c->d_heads);
    c->d_cls_bounds = c->d_cls_range = c->d_heads = nullptr;
    c->ncls_alloc = 0;
    HIP_OK(hipMalloc(&c->d_cls_bounds, sizeof(int32_t) * 2 * ncls), "hipMalloc");
    HIP_OK(hipMalloc(&c->d_cls_range, sizeof(int32_t) * 2 * (ncls + 1)), "hipMalloc");
    HIP_OK(hipMalloc(&c->d_heads, sizeof(int32_t) * (ncls + 1)), "hipMalloc");
    c->ncls_alloc = ncls;
  }
  std::vector<int32_t> bnd(2 * ncls);
  for (int i = 0; i < ncls; i++) {
    bnd[2 * i] = plan[i].lo;
    bnd[2 * i + 1] = plan[i].hi;
  }
  HIP_OK(hipMemcpy(c->d_cls_bounds, bnd.data(), sizeof(int32_t) * 2 * ncls, hipMemcpyHostToDevice), "hipMemcpy");
  if (ncls > 1 && !c->ev_fork)
    HIP_OK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming), "hipEventCreate");
  while (int(c->side.size()) < std::min(ncls - 1, kMaxBranches - 1)) {
    hipStream_t st = nullptr;
    HIP_OK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
    c->side.push_back(st);
    hipEvent_t ev = nullptr;
    HIP_OK(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
    c->ev_join.push_back(ev);
  }
  drop_graph(c);
  c->plan = plan;
  if (D.flags & HJPD_TIMING) return ensure_class_events(c);
  return HJPD_OK;
}

std::vector<ClassSpec> current_spec(const hjpd_ctx* c) {
  std::vector<ClassSpec> v;
  for (const Cls& cl : c->plan) v.push_back({cl.hi, cl.L, cl.K});
  return v;
}

// On-disk tuning cache ($HJPD_TUNE_CACHE): one line per tuned plan,
//   <key> plan=<hi>:<L>x<K>,<hi>:<L>x<K>,...
// where the key names everything the choice depends on.  hjpd_autotune
// appends; hjpd_create takes the last line whose key matches.
std::string tune_key(const hjpd_desc& d) {
  char buf[192];
  std::snprintf(buf, sizeof(buf), "hjpd-tune v2 arch=gfx950 H=%d g=%d d=%d d_y=%d dtype=%d N_max=%d variant=%d",
                d.H, d.g, d.d, d.d_y, d.dtype, d.N_max, kernel_variant(d));
  return buf;
}

bool read_cached_spec(const hjpd_desc& d, std::vector<ClassSpec>* out) {
  const char* path = std::getenv("HJPD_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  const std::string key = tune_key(d) + " plan=";
  char line[1024];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    if (std::strncmp(line, key.c_str(), key.size()) != 0) continue;
    std::vector<ClassSpec> v;
    const char* q = line + key.size();
    int hi, L, K, used = 0;
    bool ok = true;
    while (std::sscanf(q, "%d:%dx%d%n", &hi, &L, &K, &used) == 3) {
      v.push_back({hi, L, K});
      q += used;
      if (*q == ',') q++;
      else break;
      if (v.size() > size_t(kMaxClasses)) { ok = false; break; }
    }
    if (ok && !v.empty()) {
      *out = v;
      found = true;  // later lines win
    }
  }
  std::fclose(f);
  return found;
}

void append_cached_spec(const hjpd_desc& d, const std::vector<ClassSpec>& v) {
  const char* path = std::getenv("HJPD_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s plan=", tune_key(d).c_str());
  for (size_t i = 0; i < v.size(); i++) std::fprintf(f, "%s%d:%dx%d", i ? "," : "", v[i].hi, v[i].L, v[i].K);
  std::fprintf(f, "\n");
  std::fclose(f);
}

// The plan a new context starts with: the descriptor's tile override (one
// class), else the tuning cache's entry for this problem, else the default.
int build_plan(hjpd_ctx* c, bool* from_cache) {
  if (from_cache) *from_cache = false;
  if (c->desc.lanes_per_point > 0) {
    const int L = c->desc.lanes_per_point, K = c->desc.nodes_per_lane > 0 ? c->desc.nodes_per_lane : 1;
    if (L * K < c->desc.N_max) return fail(HJPD_EINVAL, "tile override capacity below N_max");
    int rc = apply_spec(c, {{c->desc.N_max, L, K}});
    c->plain_kern = lookup_for(c->desc)(1, 0, 0, 0);
    return rc;
  }
  std::vector<ClassSpec> v;
  if (read_cached_spec(c->desc, &v)) {
    if (apply_spec(c, v) == HJPD_OK) {
      if (from_cache) *from_cache = true;
      c->plain_kern = lookup_for(c->desc)(1, 0, 0, 0);
      return HJPD_OK;
    }
    g_err.clear();  // an unusable cache entry falls back to the default
  }
  int rc = apply_spec(c, default_spec(c->desc.N_max));
  c->plain_kern = lookup_for(c->desc)(1, 0, 0, 0);
  return rc;
}

size_t elem_size(const hjpd_desc& d) { return d.dtype == HJPD_F64 ? 8 : 4; }

int validate_desc(const hjpd_desc* d) {
  if (!d) return fail(HJPD_EINVAL, "desc is NULL");
  if (d->d < 1) return fail(HJPD_EINVAL, "d < 1");
  if (d->d_y < 0 || d->d_y >= d->d) return fail(HJPD_EINVAL, "d_y must satisfy 0 <= d_y < d");
  if (!(d->sigma > 0) || !std::isfinite(d->sigma)) return fail(HJPD_EINVAL, "sigma must be > 0");
  if (!(d->tau > 0) || !std::isfinite(d->tau)) return fail(HJPD_EINVAL, "tau must be > 0");
  if (d->sigma * d->tau > 0.25 * (1 + 1e-12))
    return fail(HJPD_EINVAL, "sigma*tau must be <= 1/4 (||D||_2 < 2)");
  if (!(d->theta >= 0 && d->theta <= 1)) return fail(HJPD_EINVAL, "theta must be in [0,1]");
  if (!(d->tol > 0) || !std::isfinite(d->tol)) return fail(HJPD_EINVAL, "tol must be > 0");
  if (d->max_iter < 1) return fail(HJPD_EINVAL, "max_iter must be >= 1");
  if (d->N_max < 1) return fail(HJPD_EINVAL, "N_max must be >= 1");
  if (d->N_max > 1023) return fail(HJPD_EINVAL, "N_max must be <= 1023");
  if (d->H < 0 || d->H > 4) return fail(HJPD_EINVAL, "unknown Hamiltonian family");
  if (d->g < 0 || d->g > 4) return fail(HJPD_EINVAL, "unknown initial-cost family");
  if (d->dtype != HJPD_F32 && d->dtype != HJPD_F64) return fail(HJPD_EINVAL, "unknown dtype");
  if (d->flags & ~unsigned(HJPD_PLAIN | HJPD_FIXED_ITERS | HJPD_GRAPH | HJPD_TIMING | HJPD_NO_ORDER_HINT | HJPD_HOPF |
                          HJPD_FORWARD_EULER | HJPD_TRAPEZOID | HJPD_NO_REFILL))
    return fail(HJPD_EINVAL, "unknown flag bits");
  if ((d->flags & HJPD_NO_REFILL) && (d->flags & HJPD_PLAIN))
    return fail(HJPD_EINVAL, "HJPD_NO_REFILL applies to the persistent kernels");
  if ((d->flags & HJPD_FORWARD_EULER) && (d->flags & HJPD_TRAPEZOID))
    return fail(HJPD_EINVAL, "HJPD_FORWARD_EULER and HJPD_TRAPEZOID exclude each other");
  if (d->lanes_per_point != 0) {
    const int L = d->lanes_per_point, K = d->nodes_per_lane;
    if (!(L == 8 || L == 16 || L == 32 || L == 64) || K < 1 || K > 4)
      return fail(HJPD_EINVAL, "tile override: lanes_per_point in {8,16,32,64}, nodes_per_lane in 1..4");
  } else if (d->nodes_per_lane != 0) {
    return fail(HJPD_EINVAL, "nodes_per_lane given without lanes_per_point");
  }
  if (d->d > 1023) return fail(HJPD_EINVAL, "d must be <= 1023");
  if (d->starts < 0 || d->starts > 1024 || d->restarts < 0 || !(d->sigma_inc >= 0.0) || !std::isfinite(d->sigma_inc) ||
      !(d->value_tol >= 0.0) || !std::isfinite(d->value_tol))
    return fail(HJPD_EINVAL, "recipes: starts in 0..1024, restarts >= 0, sigma_inc >= 0, value_tol >= 0");
  // supported pairs
  const bool game = d->d_y > 0;
  if (has_recipe(*d) && (d->H == HJPD_H_LINEAR_TANH || d->H == HJPD_H_ISAACS ||
                         (d->flags & (HJPD_PLAIN | HJPD_FIXED_ITERS | HJPD_HOPF))))
    return fail(HJPD_EUNSUPPORTED, "recipes are built for the persistent Lax path in tolerance mode "
                                   "(control families and the pursuit-evasion game)");
  if (game && d->starts > 1) return fail(HJPD_EUNSUPPORTED, "several starts are built for the control path only");
  if ((d->flags & HJPD_HOPF) && !(d->H == HJPD_H_CNORM && !game && (d->g == HJPD_G_NORM || d->g == HJPD_G_QUAD_SHIFT)) &&
      !(d->H == HJPD_H_QUADROTOR && !game && d->g == HJPD_G_QUAD_SHIFT && !(d->flags & HJPD_PLAIN)) &&
      d->H != HJPD_H_ISAACS)
    return fail(HJPD_EUNSUPPORTED, "the Hopf formulation is built for CNORM with NORM or QUAD_SHIFT, for QUADROTOR "
                                   "with QUAD_SHIFT (persistent kernel), and for ISAACS");
  if (has_mix(*d) && (game ||
                      !((d->H == HJPD_H_CNORM && (d->g == HJPD_G_NORM || d->g == HJPD_G_QUAD_SHIFT)) ||
                        (d->H == HJPD_H_QUADROTOR && d->g == HJPD_G_QUAD_SHIFT)) ||
                      (d->flags & (HJPD_PLAIN | HJPD_HOPF)) || has_recipe(*d)))
    return fail(HJPD_EUNSUPPORTED, "forward Euler and trapezoid are built for CNORM with NORM or QUAD_SHIFT and for "
                                   "QUADROTOR with QUAD_SHIFT, on the persistent Lax path");
  if (d->H == HJPD_H_PURSUIT_EVASION) {
    if (!(game && d->g == HJPD_G_PAIR_DIST && d->d == 12 && d->d_y == 6))
      return fail(HJPD_EUNSUPPORTED, "pursuit-evasion needs d = 12, d_y = 6, g = PAIR_DIST");
  } else if (d->H == HJPD_H_ISAACS) {
    if (!(game && d->g == HJPD_G_SADDLE_QUAD && d->d == 2 && d->d_y == 1))
      return fail(HJPD_EUNSUPPORTED, "ISAACS needs d = 2, d_y = 1, g = SADDLE_QUAD");
    if (d->flags & HJPD_PLAIN) return fail(HJPD_EUNSUPPORTED, "ISAACS is built for the persistent kernel");
  } else if (game || d->g == HJPD_G_SADDLE_QUAD) {
    return fail(HJPD_EUNSUPPORTED, "the game path is built for the pursuit-evasion and Isaacs families only");
  } else if (d->H == HJPD_H_CNORM) {
    if (!(d->g == HJPD_G_NORM || d->g == HJPD_G_QUAD_SHIFT))
      return fail(HJPD_EUNSUPPORTED, "CNORM pairs with NORM or QUAD_SHIFT");
    if (!(d->d == 2 || d->d == 3 || d->d == 4 || d->d == 10))
      return fail(HJPD_EUNSUPPORTED, "CNORM is built for d in {2,3,4,10}");
  } else if (d->H == HJPD_H_QUADROTOR) {
    if (!(d->g == HJPD_G_QUAD_SHIFT && d->d == 12)) return fail(HJPD_EUNSUPPORTED, "QUADROTOR needs d = 12, QUAD_SHIFT");
  } else if (d->H == HJPD_H_LINEAR_TANH) {
    if (!(d->g == HJPD_G_QUAD_FORM)) return fail(HJPD_EUNSUPPORTED, "LINEAR_TANH pairs with QUAD_FORM");
    if (d->dtype != HJPD_F32) return fail(HJPD_EUNSUPPORTED, "LINEAR_TANH is built for float32");
    if (!(d->d == 16 || d->d == 32 || d->d == 100 || d->d == 128))
      return fail(HJPD_EUNSUPPORTED, "LINEAR_TANH is built for d in {16, 32, 100, 128}");
    if (d->N_max > hjpd::kLtMaxN) return fail(HJPD_EUNSUPPORTED, "LINEAR_TANH is built for N_max <= 64");
    if (d->flags & (HJPD_PLAIN | HJPD_GRAPH)) return fail(HJPD_EUNSUPPORTED, "LINEAR_TANH has one kernel path");
    return HJPD_OK;
  }
  if (d->N_max > hjpd::kMaxCapacity) return fail(HJPD_EUNSUPPORTED, "N_max > 256 is not built");
  return HJPD_OK;
}

void drop_graph(hjpd_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
  c->gkey.clear();
}

template <typename T>
int enqueue_solve(hjpd_ctx* c, const Workspace& ws, int64_t n, const void* x, const void* t, const int32_t* N,
                  const void* hp, const void* gp, void* phi, void* xtraj, void* ptraj, int32_t* iters,
                  int32_t* status, hipStream_t s, bool timed) {
  const hjpd_desc& D = c->desc;
  const int ncls = int(c->plan.size());
  const int nb = int((n + 255) / 256);
  const int nkeys = (D.N_max + 1) * kHintBuckets;
  int hint = kHintNone;
  if (!(D.flags & HJPD_NO_ORDER_HINT))
    hint = D.g == HJPD_G_QUAD_SHIFT ? kHintShift
                                    : ((D.g == HJPD_G_NORM || D.g == HJPD_G_SADDLE_QUAD) ? kHintNorm : kHintPair);
  if (nkeys > kMaxKeys) return fail(HJPD_EUNSUPPORTED, "N_max above the queue's bucket range");
  const int nqb = int((n + kQueueBlock * kQueuePerThread - 1) / (kQueueBlock * kQueuePerThread));
  hipLaunchKernelGGL(k_queue_zero, dim3((nkeys + 255) / 256), dim3(256), 0, s, ws.counts, nkeys);
  hipLaunchKernelGGL(k_queue_count<T>, dim3(nqb), dim3(kQueueBlock), 0, s, n, D.d, D.d_y, D.N_max, (const T*)x,
                     (const T*)t, N, hint, (const T*)gp, nkeys, ws.counts, (T*)phi, iters, status);
  hipLaunchKernelGGL(k_queue_scan, dim3(1), dim3(kScanBlock), 0, s, D.N_max, ncls, c->d_cls_bounds, ws.counts,
                     ws.cursor, ws.cls_range, ws.heads);
  hipLaunchKernelGGL(k_queue_scatter<T>, dim3(nqb), dim3(kQueueBlock), 0, s, n, D.d, D.d_y, D.N_max, (const T*)x,
                     (const T*)t, N, hint, (const T*)gp, nkeys, ws.cursor, ws.queue);
  HIP_OK(hipGetLastError(), "queue kernels");

  hjpd::KArgs<T> a;
  a.x = (const T*)x;
  a.t = (const T*)t;
  a.N = N;
  a.hp = (const T*)hp;
  a.gp = (const T*)gp;
  a.phi = (T*)phi;
  a.xtraj = (T*)xtraj;
  a.ptraj = (T*)ptraj;
  a.iters = iters;
  a.status = status;
  a.queue = ws.queue;
  a.cls_range = ws.cls_range;
  a.heads = ws.heads;
  a.work = (T*)c->d_work;
  a.work_stride = int64_t(nb) * 256;
  a.sigma = T(D.sigma);
  a.tau = T(D.tau);
  a.theta = T(D.theta);
  a.tol = T(D.tol);
  a.max_iter = D.max_iter;
  a.fixed = (D.flags & HJPD_FIXED_ITERS) ? 1 : 0;
  a.N_max = D.N_max;
  a.d = D.d;
  a.gkind = D.g;
  a.hopf = (D.flags & HJPD_HOPF) ? 1 : 0;
  a.wl = (D.flags & HJPD_FORWARD_EULER) ? T(1) : ((D.flags & HJPD_TRAPEZOID) ? T(0.5) : T(0));
  a.wr = (D.flags & HJPD_FORWARD_EULER) ? T(0) : ((D.flags & HJPD_TRAPEZOID) ? T(0.5) : T(1));
  a.starts = D.starts > 1 ? D.starts : 1;
  a.restarts = D.restarts;
  a.sigma_inc = T(D.sigma_inc);
  a.value_tol = T(D.value_tol);
  a.seed = D.seed;
  a.refill = (D.flags & HJPD_NO_REFILL) ? 0 : 1;
  a.pops = c->d_pops;
  void* args[] = {&a};
  if (timed) HIP_OK(hipEventRecord(c->ev0, s), "hipEventRecord");
  int launches = 0;
  if (D.flags & HJPD_PLAIN) {
    a.cls = ncls;
    HIP_OK(hipLaunchKernel(c->plain_kern, dim3(nb), dim3(256), args, 0, s), "plain kernel launch");
    launches = 1;
  } else {
    // One persistent launch per capacity class.  Each launch ends with its own
    // slowest points; the classes run on parallel branches (class 0 on the
    // solve's stream, the others on side streams forked from it and joined
    // back), so one class's tail overlaps the others' bulk.  The classes read
    // disjoint queue segments and write disjoint points.
    // The classes of largest N (the most work) each get a branch of their own;
    // the rest run one after another on the solve's stream.  A process has
    // kMaxBranches hardware queues, so more streams would only share them.
    const int nside = std::min(ncls - 1, kMaxBranches - 1);
    const bool fork = nside > 0 && int(c->side.size()) >= nside;
    const bool per_launch = timed && int(c->ev_cls0.size()) >= ncls;
    if (per_launch) c->timed_cls.clear();
    if (fork) HIP_OK(hipEventRecord(c->ev_fork, s), "hipEventRecord");
    for (int ci = ncls - 1; ci >= 0; ci--) {
      const int rank = ncls - 1 - ci;  // 0: the class of largest N
      hipStream_t st = (fork && rank < nside) ? c->side[rank] : s;
      if (st != s) HIP_OK(hipStreamWaitEvent(st, c->ev_fork, 0), "hipStreamWaitEvent");
      a.cls = ci;
      if (per_launch) HIP_OK(hipEventRecord(c->ev_cls0[ci], st), "hipEventRecord");
      HIP_OK(hipLaunchKernel(c->plan[ci].kern, dim3(launch_grid(c, c->plan[ci], n)), dim3(256), args, 0, st),
             "persistent kernel launch");
      if (per_launch) {
        HIP_OK(hipEventRecord(c->ev_cls1[ci], st), "hipEventRecord");
        c->timed_cls.push_back(ci);
      }
      if (st != s) HIP_OK(hipEventRecord(c->ev_join[rank], st), "hipEventRecord");
      launches++;
    }
    if (fork)
      for (int r = 0; r < nside; r++) HIP_OK(hipStreamWaitEvent(s, c->ev_join[r], 0), "hipStreamWaitEvent");
  }
  if (timed) HIP_OK(hipEventRecord(c->ev1, s), "hipEventRecord");
  c->timing_launches = launches;
  return HJPD_OK;
}

// Start/end events of each class launch, for HJPD_TIMING (created outside any solve).
int ensure_class_events(hjpd_ctx* c) {
  while (c->ev_cls0.size() < c->plan.size()) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_OK(hipEventCreate(&e0), "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      return fail(HJPD_EDEVICE, "hipEventCreate failed");
    }
    c->ev_cls0.push_back(e0);
    c->ev_cls1.push_back(e1);
  }
  return HJPD_OK;
}

Workspace ctx_workspace(const hjpd_ctx* c) {
  return Workspace{c->d_counts, c->d_cursor, c->d_cls_range, c->d_heads, c->d_queue};
}

// Device address of `scratch` on each GPU, resolved once per device (with that
// device current) by hjpd_create.  The array's name in host code is only a
// host-side handle; kernels and copies get these addresses.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch_ptr[kMaxDevices] = {};

int resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(HJPD_EDEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return HJPD_OK;
  void* p = nullptr;
  HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
  g_scratch_ptr[device] = static_cast<int32_t*>(p);
  return HJPD_OK;
}

Workspace static_workspace(int device) {
  int32_t* b = g_scratch_ptr[device];
  Workspace w;
  w.queue = b;
  w.counts = b + kStaticMaxPoints;
  w.cursor = w.counts + kMaxKeys;
  w.cls_range = w.cursor + kMaxKeys;
  w.heads = w.cls_range + 2 * (kStaticMaxCls + 1);
  return w;
}

int ensure_capacity(hjpd_ctx* c, int64_t n) {
  if (n > c->queue_cap) {
    drop_graph(c);
    if (c->d_queue) (void)hipFree(c->d_queue);
    c->d_queue = nullptr;
    c->queue_cap = 0;
    if (hipMalloc(&c->d_queue, sizeof(int32_t) * n) != hipSuccess) return fail(HJPD_ENOMEM, "queue allocation");
    c->queue_cap = n;
  }
  if (c->desc.flags & HJPD_PLAIN) {
    const int64_t stride = ((n + 255) / 256) * 256;
    const size_t need = size_t(3) * (c->desc.N_max + 1) * c->desc.d * stride * elem_size(c->desc);
    if (need > c->work_bytes) {
      drop_graph(c);
      if (c->d_work) (void)hipFree(c->d_work);
      c->d_work = nullptr;
      c->work_bytes = 0;
      if (hipMalloc(&c->d_work, need) != hipSuccess) return fail(HJPD_ENOMEM, "plain workspace allocation");
      c->work_bytes = need;
    }
  }
  return HJPD_OK;
}

}  // namespace

extern "C" {

const char* hjpd_last_error(void) { return g_err.c_str(); }

int hjpd_create(const hjpd_desc* desc, hjpd_ctx** out) {
  g_err.clear();
  if (!out) return fail(HJPD_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate_desc(desc);
  if (rc) return rc;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(HJPD_EDEVICE, "no HIP device");
  hjpd_ctx* c = new hjpd_ctx();
  c->desc = *desc;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(HJPD_EDEVICE, "hipGetDevice failed");
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) {
    delete c;
    return fail(HJPD_EDEVICE, "hipGetDeviceProperties failed");
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    delete c;
    return fail(HJPD_EDEVICE, std::string("kernels are built for gfx950, device is ") + prop.gcnArchName);
  }
  c->n_cu = prop.multiProcessorCount;
  if (desc->H == HJPD_H_LINEAR_TANH) {
    rc = hjpd::lt_create(&c->lt, c->desc);
    if (rc) {
      delete c;
      return rc;
    }
  } else {
    rc = resolve_scratch(c->device);
    if (!rc) rc = build_plan(c, &c->plan_from_cache);
    if (!rc && (hipMalloc(&c->d_counts, sizeof(int32_t) * (desc->N_max + 1) * kHintBuckets) != hipSuccess ||
                hipMalloc(&c->d_cursor, sizeof(int32_t) * (desc->N_max + 1) * kHintBuckets) != hipSuccess))
      rc = fail(HJPD_ENOMEM, "counter allocation");
    if (rc) {
      hjpd_destroy(c);
      return rc;
    }
  }
  if (desc->flags & HJPD_TIMING) {
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
      hjpd_destroy(c);
      return fail(HJPD_EDEVICE, "hipEventCreate failed");
    }
    rc = ensure_class_events(c);
    if (rc) {
      hjpd_destroy(c);
      return rc;
    }
  }
  *out = c;
  return HJPD_OK;
}

int hjpd_destroy(hjpd_ctx* c) {
  if (!c) return HJPD_OK;
  drop_graph(c);
  if (c->d_cls_bounds) (void)hipFree(c->d_cls_bounds);
  if (c->d_counts) (void)hipFree(c->d_counts);
  if (c->d_cursor) (void)hipFree(c->d_cursor);
  if (c->d_cls_range) (void)hipFree(c->d_cls_range);
  if (c->d_heads) (void)hipFree(c->d_heads);
  if (c->d_queue) (void)hipFree(c->d_queue);
  if (c->d_work) (void)hipFree(c->d_work);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  for (hipEvent_t ev : c->ev_cls0) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : c->ev_cls1) (void)hipEventDestroy(ev);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (hipStream_t st : c->side) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : c->ev_join) (void)hipEventDestroy(ev);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->lt) hjpd::lt_destroy(c->lt);
  delete c;
  return HJPD_OK;
}

int hjpd_solve_batch(hjpd_ctx* c, int64_t n, const void* x, const void* t, const int32_t* N, const void* hp,
                     const void* gp, void* phi, void* xtraj, void* ptraj, int32_t* iters, int32_t* status,
                     void* stream) {
  g_err.clear();
  if (!c) return fail(HJPD_EINVAL, "ctx is NULL");
  if (n < 0) return fail(HJPD_EINVAL, "n < 0");
  if (n > INT32_MAX) return fail(HJPD_EINVAL, "n must fit in int32");
  if (n == 0) return HJPD_OK;
  if (!x || !t || !N || !hp || !gp || !phi || !iters || !status) return fail(HJPD_EINVAL, "required pointer is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (c->lt) {
    return hjpd::lt_solve(c->lt, c->desc, n, x, t, N, hp, gp, phi, xtraj, ptraj, iters, status, s,
                          (c->desc.flags & HJPD_TIMING) ? c->ev0 : nullptr, (c->desc.flags & HJPD_TIMING) ? c->ev1 : nullptr,
                          &c->timing_launches, &c->timing_valid);
  }
  int rc = ensure_capacity(c, n);
  if (rc) return rc;
  const bool timed = (c->desc.flags & HJPD_TIMING) != 0;
  c->timing_valid = false;
  auto enqueue_on = [&](hipStream_t st) -> int {
    const bool inner_timed = timed && st == s;
    if (c->desc.dtype == HJPD_F64)
      return enqueue_solve<double>(c, ctx_workspace(c), n, x, t, N, hp, gp, phi, xtraj, ptraj, iters, status, st,
                                    inner_timed);
    return enqueue_solve<float>(c, ctx_workspace(c), n, x, t, N, hp, gp, phi, xtraj, ptraj, iters, status, st,
                                 inner_timed);
  };
  if (c->desc.flags & HJPD_GRAPH) {
    std::vector<uintptr_t> key = {uintptr_t(n),     uintptr_t(x),     uintptr_t(t),     uintptr_t(N),
                                  uintptr_t(hp),    uintptr_t(gp),    uintptr_t(phi),   uintptr_t(xtraj),
                                  uintptr_t(ptraj), uintptr_t(iters), uintptr_t(status), uintptr_t(s)};
    if (!c->gexec || key != c->gkey) {
      drop_graph(c);
      if (!c->cap_stream) HIP_OK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
      // make sure earlier work on the caller's stream is not reordered: the
      // graph itself is launched on the caller's stream below
      HIP_OK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
      rc = enqueue_on(c->cap_stream);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess) return fail(HJPD_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      c->graph = g;
      HIP_OK(hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0), "hipGraphInstantiate");
      c->gkey = key;
    }
    if (timed) HIP_OK(hipEventRecord(c->ev0, s), "hipEventRecord");
    HIP_OK(hipGraphLaunch(c->gexec, s), "hipGraphLaunch");
    if (timed) HIP_OK(hipEventRecord(c->ev1, s), "hipEventRecord");
    c->timing_valid = timed;
    return HJPD_OK;
  }
  rc = enqueue_on(s);
  if (rc) return rc;
  c->timing_valid = timed;
  return HJPD_OK;
}

int hjpd_solve_batch_noalloc(hjpd_ctx* c, int64_t n, const void* x, const void* t, const int32_t* N,
                             const void* hp, const void* gp, void* phi, void* xtraj, void* ptraj, int32_t* iters,
                             int32_t* status, void* stream) {
  g_err.clear();
  if (!c) return fail(HJPD_EINVAL, "ctx is NULL");
  if (c->lt || (c->desc.flags & HJPD_PLAIN))
    return fail(HJPD_EUNSUPPORTED, "the allocation-free solve is built for the persistent kernels");
  if (n < 0) return fail(HJPD_EINVAL, "n < 0");
  if (n > kStaticMaxPoints)
    return fail(HJPD_EINVAL, "n exceeds the allocation-free solve's limit of 1048576 points");
  if (n == 0) return HJPD_OK;
  if (!x || !t || !N || !hp || !gp || !phi || !iters || !status) return fail(HJPD_EINVAL, "required pointer is NULL");
  if (int(c->plan.size()) > kStaticMaxCls) return fail(HJPD_EUNSUPPORTED, "more capacity classes than the scratch holds");
  int dev = -1;
  HIP_OK(hipGetDevice(&dev), "hipGetDevice");
  if (dev != c->device) return fail(HJPD_EINVAL, "the context's device is not the current device");
  if (dev < 0 || dev >= kMaxDevices || !g_scratch_ptr[dev]) return fail(HJPD_EDEVICE, "scratch address not resolved");
  const Workspace ws = static_workspace(dev);
  hipStream_t s = (hipStream_t)stream;
  const bool timed = (c->desc.flags & HJPD_TIMING) != 0;
  c->timing_valid = false;
  int rc;
  if (c->desc.dtype == HJPD_F64)
    rc = enqueue_solve<double>(c, ws, n, x, t, N, hp, gp, phi, xtraj, ptraj, iters, status, s, timed);
  else
    rc = enqueue_solve<float>(c, ws, n, x, t, N, hp, gp, phi, xtraj, ptraj, iters, status, s, timed);
  if (rc) return rc;
  c->timing_valid = timed;
  return HJPD_OK;
}

int hjpd_get_timing(hjpd_ctx* c, double* ms, int* launches) {
  g_err.clear();
  if (!c || !ms) return fail(HJPD_EINVAL, "NULL argument");
  if (!(c->desc.flags & HJPD_TIMING) || !c->timing_valid) return fail(HJPD_EINVAL, "no timed solve recorded");
  HIP_OK(hipEventSynchronize(c->ev1), "hipEventSynchronize");
  float f = 0;
  HIP_OK(hipEventElapsedTime(&f, c->ev0, c->ev1), "hipEventElapsedTime");
  *ms = f;
  if (launches) *launches = c->timing_launches;
  return HJPD_OK;
}

int hjpd_get_launch_timing(hjpd_ctx* c, int i, double* ms, int* N_lo, int* N_hi, int* lanes_per_point,
                           int* nodes_per_lane) {
  g_err.clear();
  if (!c || !ms) return fail(HJPD_EINVAL, "NULL argument");
  if (!(c->desc.flags & HJPD_TIMING) || !c->timing_valid) return fail(HJPD_EINVAL, "no timed solve recorded");
  if (c->lt || (c->desc.flags & (HJPD_PLAIN | HJPD_GRAPH)))
    return fail(HJPD_EINVAL, "per-launch timing is recorded for eager persistent solves only");
  if (i < 0 || i >= int(c->timed_cls.size())) return fail(HJPD_EINVAL, "launch index out of range");
  const int ci = c->timed_cls[i];
  HIP_OK(hipEventSynchronize(c->ev_cls1[ci]), "hipEventSynchronize");
  float f = 0;
  HIP_OK(hipEventElapsedTime(&f, c->ev_cls0[ci], c->ev_cls1[ci]), "hipEventElapsedTime");
  *ms = f;
  if (N_lo) *N_lo = c->plan[ci].lo;
  if (N_hi) *N_hi = c->plan[ci].hi;
  if (lanes_per_point) *lanes_per_point = c->plan[ci].L;
  if (nodes_per_lane) *nodes_per_lane = c->plan[ci].K;
  return HJPD_OK;
}

int hjpd_set_pop_counter(hjpd_ctx* c, int32_t* counts) {
  g_err.clear();
  if (!c) return fail(HJPD_EINVAL, "ctx is NULL");
  if (c->lt || (c->desc.flags & HJPD_PLAIN)) return fail(HJPD_EUNSUPPORTED, "pop counting is for the persistent kernels");
  drop_graph(c);  // a captured graph holds the old kernel arguments
  c->d_pops = counts;
  return HJPD_OK;
}

int hjpd_set_plan(hjpd_ctx* c, int n_classes, const int32_t* hi, const int32_t* L, const int32_t* K) {
  g_err.clear();
  if (!c) return fail(HJPD_EINVAL, "ctx is NULL");
  if (c->lt || (c->desc.flags & HJPD_PLAIN)) return fail(HJPD_EUNSUPPORTED, "no persistent plan for this context");
  if (n_classes < 1 || n_classes > kMaxClasses || !hi || !L || !K) return fail(HJPD_EINVAL, "1..16 classes, non-NULL arrays");
  std::vector<ClassSpec> v;
  for (int i = 0; i < n_classes; i++) v.push_back({hi[i], L[i], K[i]});
  const std::vector<ClassSpec> old = current_spec(c);
  int rc = apply_spec(c, v);
  if (rc) {
    const std::string msg = g_err;
    (void)apply_spec(c, old);
    return fail(rc, msg);
  }
  c->plan_from_cache = false;
  return HJPD_OK;
}

int hjpd_get_plan(hjpd_ctx* c, int max_classes, int32_t* hi, int32_t* L, int32_t* K, int* n_classes,
                  int* from_cache) {
  g_err.clear();
  if (!c || !n_classes) return fail(HJPD_EINVAL, "NULL argument");
  if (c->lt || (c->desc.flags & HJPD_PLAIN)) return fail(HJPD_EUNSUPPORTED, "no persistent plan for this context");
  const int nc = int(c->plan.size());
  *n_classes = nc;
  if (from_cache) *from_cache = c->plan_from_cache ? 1 : 0;
  for (int i = 0; i < nc && i < max_classes; i++) {
    if (hi) hi[i] = c->plan[i].hi;
    if (L) L[i] = c->plan[i].L;
    if (K) K[i] = c->plan[i].K;
  }
  return HJPD_OK;
}

int hjpd_autotune(hjpd_ctx* c, int64_t n, const void* x, const void* t, const int32_t* N, const void* hp,
                  const void* gp, void* phi, int32_t* iters, int32_t* status, int probe_iters, void* stream) {
  g_err.clear();
  if (!c) return fail(HJPD_EINVAL, "ctx is NULL");
  if (c->lt) return fail(HJPD_EUNSUPPORTED, "LINEAR_TANH has a single tile");
  if (c->desc.flags & HJPD_PLAIN) return fail(HJPD_EUNSUPPORTED, "the plain kernel has no tile");
  if (n <= 0) return fail(HJPD_EINVAL, "n must be > 0");
  if (!x || !t || !N || !hp || !gp || !phi || !iters || !status) return fail(HJPD_EINVAL, "required pointer is NULL");
  if (c->desc.lanes_per_point > 0) return fail(HJPD_EINVAL, "tile fixed by the descriptor");
  hipStream_t s = (hipStream_t)stream;
  if (probe_iters <= 0) probe_iters = 200;
  int rc = ensure_capacity(c, n);
  if (rc) return rc;
  const hjpd_desc saved = c->desc;
  const std::vector<ClassSpec> start_spec = current_spec(c);
  // probes: exactly probe_iters iterations at every point, timed from the
  // first class launch to the last one's end on the caller's stream
  c->desc.flags = (saved.flags | HJPD_FIXED_ITERS | HJPD_TIMING) & ~unsigned(HJPD_GRAPH | HJPD_PLAIN);
  c->desc.max_iter = probe_iters;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_OK(hipEventCreate(&e0), "hipEventCreate");
  HIP_OK(hipEventCreate(&e1), "hipEventCreate");
  hipEvent_t sv0 = c->ev0, sv1 = c->ev1;
  c->ev0 = e0;
  c->ev1 = e1;
  Lookup lk = lookup_for(c->desc);
  const int Nmax = c->desc.N_max;

  auto measure = [&](const std::vector<ClassSpec>& spec, double* ms) -> int {
    int r = apply_spec(c, spec);
    if (r) return r;
    double best = 1e300;
    for (int rep = 0; rep < 2; rep++) {
      r = c->desc.dtype == HJPD_F64
              ? enqueue_solve<double>(c, ctx_workspace(c), n, x, t, N, hp, gp, phi, nullptr, nullptr, iters, status, s, true)
              : enqueue_solve<float>(c, ctx_workspace(c), n, x, t, N, hp, gp, phi, nullptr, nullptr, iters, status, s, true);
      if (r) return r;
      if (hipEventSynchronize(e1) != hipSuccess) return fail(HJPD_EDEVICE, "autotune sync");
      float f = 0;
      (void)hipEventElapsedTime(&f, e0, e1);
      best = std::min(best, double(f));
    }
    *ms = best;
    return HJPD_OK;
  };
  // tiles that can hold a class whose top is hi: capacity from hi up to twice hi
  auto candidates = [&](int hi) {
    std::vector<hjpd::Tile> v;
    for (int ti = 0; ti < hjpd::kNumTiles; ti++) {
      const hjpd::Tile tl = hjpd::kTiles[ti];
      const int cap = tl.L * tl.K;
      if (cap >= hi && cap <= std::max(2 * hi, 8) && lk(0, tl.L, tl.K, kernel_variant(c->desc))) v.push_back(tl);
    }
    return v;
  };

  // 1. finest partition: a class boundary at every tile capacity below N_max
  std::vector<ClassSpec> spec;
  for (int ci = 0; ci < kNumCaps && (spec.empty() || spec.back().hi < Nmax); ci++) {
    const int hi = std::min(kCaps[ci], Nmax);
    const std::vector<hjpd::Tile> cand = candidates(hi);
    if (cand.empty()) continue;
    spec.push_back({hi, cand[0].L, cand[0].K});
  }
  double best_ms = 0;
  rc = measure(spec, &best_ms);
  // 2. each class's tile (lanes per point L: 64/L points per wavefront; nodes
  //    per lane K: the unroll of each lane's node loop), whole solve timed
  for (size_t ci = 0; ci < spec.size() && !rc; ci++) {
    for (const hjpd::Tile& tl : candidates(spec[ci].hi)) {
      if (tl.L == spec[ci].L && tl.K == spec[ci].K) continue;
      std::vector<ClassSpec> trial = spec;
      trial[ci].L = tl.L;
      trial[ci].K = tl.K;
      double ms = 0;
      rc = measure(trial, &ms);
      if (rc) break;
      if (ms < best_ms) {
        best_ms = ms;
        spec = trial;
      }
    }
  }
  // 3. class boundaries: merge neighbouring classes while that is faster
  //    (one launch and one tail fewer against more masked nodes)
  for (bool improved = true; improved && !rc && spec.size() > 1;) {
    improved = false;
    std::vector<ClassSpec> best_trial;
    double best_trial_ms = best_ms * 0.99;
    for (size_t ci = 0; ci + 1 < spec.size() && !rc; ci++) {
      for (const hjpd::Tile& tl : candidates(spec[ci + 1].hi)) {
        std::vector<ClassSpec> trial = spec;
        trial[ci + 1].L = tl.L;
        trial[ci + 1].K = tl.K;
        trial.erase(trial.begin() + ci);
        double ms = 0;
        rc = measure(trial, &ms);
        if (rc) break;
        if (ms < best_trial_ms) {
          best_trial_ms = ms;
          best_trial = trial;
        }
      }
    }
    if (!rc && !best_trial.empty()) {
      spec = best_trial;
      best_ms = best_trial_ms;
      improved = true;
    }
  }
  c->ev0 = sv0;
  c->ev1 = sv1;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->desc = saved;
  if (rc) {
    const std::string msg = g_err;
    (void)apply_spec(c, start_spec);
    return fail(rc, msg);
  }
  rc = apply_spec(c, spec);
  if (!rc) {
    append_cached_spec(saved, spec);
    c->plan_from_cache = false;
  }
  return rc;
}

int hjpd_value_grad(hjpd_ctx* c, int64_t n, const void* x, const void* t, const int32_t* N, const void* hp,
                    const void* gp, const void* grad_phi, int K_iters, int ckpt_every, void* phi, void* dphi_dx,
                    void* dh, void* dg, void* stream) {
  g_err.clear();
  if (!c) return fail(HJPD_EINVAL, "ctx is NULL");
  if (!c->lt) return fail(HJPD_EUNSUPPORTED, "value_grad is built for LINEAR_TANH with QUAD_FORM");
  if (n < 0 || K_iters < 1 || ckpt_every < 1) return fail(HJPD_EINVAL, "n < 0, K_iters < 1 or ckpt_every < 1");
  if (n == 0) return HJPD_OK;
  if (!x || !t || !N || !hp || !gp || !grad_phi || !phi || !dphi_dx || !dh || !dg)
    return fail(HJPD_EINVAL, "required pointer is NULL");
  const bool timed = (c->desc.flags & HJPD_TIMING) != 0;
  return hjpd::lt_value_grad(c->lt, c->desc, n, x, t, N, hp, gp, grad_phi, K_iters, ckpt_every, phi, dphi_dx, dh, dg,
                             (hipStream_t)stream, timed ? c->ev0 : nullptr, timed ? c->ev1 : nullptr,
                             &c->timing_launches, &c->timing_valid);
}

}  // extern "C"

// error helper for the linear-tanh unit
int hjpd_fail(int code, const char* msg) { return fail(code, msg); }
