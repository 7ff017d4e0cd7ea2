// C ABI of libsemd (declared in include/semd.h): argument validation, work
// descriptors, stream-ordered workspaces and kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "semd.h"
#include "semd_internal.h"
#include "semd_stream.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(SEMD_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define SEMD_HIP(call, what)                      \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// (M, N) from column-major dims: M = dims[0], N = product of the rest.
int parse_dims(const int64_t* dims, int ndim, int64_t* M, int64_t* N) {
  if (!dims) return fail(SEMD_EINVAL, "dims is NULL");
  if (ndim < 1 || ndim > 4) return fail(SEMD_EINVAL, "ndim must be in [1, 4], got %d", ndim);
  int64_t n = 1;
  for (int d = 0; d < ndim; ++d) {
    if (dims[d] < 1) return fail(SEMD_EINVAL, "dims[%d] = %lld < 1", d, (long long)dims[d]);
    if (d > 0) {
      if (n > (int64_t(1) << 40) / dims[d]) return fail(SEMD_EINVAL, "signal too large");
      n *= dims[d];
    }
  }
  *M = dims[0];
  *N = n;
  return SEMD_OK;
}

int check_params(const semd_params* p, bool ensemble) {
  if (!p) return fail(SEMD_EINVAL, "params is NULL");
  if (p->max_imfs < 1) return fail(SEMD_EINVAL, "max_imfs must be >= 1");
  if (p->max_imfs > 64) return fail(SEMD_EINVAL, "max_imfs must be <= 64");
  if (p->sift_iters < 1) return fail(SEMD_EINVAL, "sift_iters must be >= 1");
  if (p->boundary_rule != SEMD_BOUNDARY_MIRROR)
    return fail(SEMD_EINVAL, "unknown boundary_rule %d", p->boundary_rule);
  if (p->transition_len < 0) return fail(SEMD_EINVAL, "transition_len must be >= 0");
  if (p->path < SEMD_PATH_AUTO || p->path > SEMD_PATH_STREAM)
    return fail(SEMD_EINVAL, "unknown path %d", p->path);
  if (ensemble && p->ensemble < 1) return fail(SEMD_EINVAL, "ensemble must be >= 1");
  if (p->stop_rule != SEMD_STOP_FIXED && p->stop_rule != SEMD_STOP_SD)
    return fail(SEMD_EINVAL, "unknown stop_rule %d", p->stop_rule);
  if (p->stop_rule == SEMD_STOP_SD && !(p->sd_threshold > 0.0 && std::isfinite(p->sd_threshold)))
    return fail(SEMD_EINVAL, "sd_threshold must be positive and finite");
  if (p->reserved != 0) return fail(SEMD_EINVAL, "params.reserved must be 0");
  return SEMD_OK;
}

// The SD threshold a validated params set asks for (0: fixed sift count).
double sd_of(const semd_params* p) {
  return p->stop_rule == SEMD_STOP_SD ? p->sd_threshold : 0.0;
}

// ---------------------------------------------------------------------------
// Graph replay of the streaming step
// ---------------------------------------------------------------------------

// A stream that can be captured: the caller's, or, for the null stream, a
// stream of this thread's own (default priority) joined to the caller's by
// events before and after the work.
struct CaptureStream {
  hipStream_t caller = nullptr, s = nullptr;
  hipEvent_t in = nullptr, out = nullptr;
  bool side = false;

  hipError_t open(hipStream_t c) {
    caller = c;
    if (c != nullptr) {
      s = c;
      return hipSuccess;
    }
    thread_local hipStream_t own = nullptr;
    thread_local hipEvent_t ev_in = nullptr, ev_out = nullptr;
    if (!own) {
      hipError_t e = hipStreamCreateWithFlags(&own, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_in, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_out, hipEventDisableTiming);
      if (e != hipSuccess) return e;
    }
    s = own;
    in = ev_in;
    out = ev_out;
    side = true;
    hipError_t e = hipEventRecord(in, caller);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, in, 0);
    return e;
  }
  // the caller's stream waits for everything enqueued on s so far
  hipError_t join() {
    if (!side) return hipSuccess;
    hipError_t e = hipEventRecord(out, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(caller, out, 0);
    return e;
  }
};

// Executable graphs whose launches may still be in flight, each with an
// event recorded after its last launch; destroyed once the event completes.
struct RetiredGraph {
  hipGraphExec_t exec;
  hipGraph_t graph;
  hipEvent_t ev;
};
std::mutex g_retire_mu;
std::vector<RetiredGraph> g_retired;

void sweep_retired_graphs() {
  std::lock_guard<std::mutex> lock(g_retire_mu);
  for (size_t i = 0; i < g_retired.size();) {
    RetiredGraph& r = g_retired[i];
    if (hipEventQuery(r.ev) == hipSuccess) {
      (void)hipGraphExecDestroy(r.exec);
      (void)hipGraphDestroy(r.graph);
      (void)hipEventDestroy(r.ev);
      g_retired[i] = g_retired.back();
      g_retired.pop_back();
    } else {
      ++i;
    }
  }
}

// The kernels one streaming step launches, captured once as a graph and
// replayed once per step.  retire() hands the graph over for destruction
// after the work already enqueued on a stream.
struct StepGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  StepGraph() = default;
  StepGraph(const StepGraph&) = delete;
  StepGraph& operator=(const StepGraph&) = delete;
  ~StepGraph() { retire(nullptr); }

  // s: the stream its launches went to (nullptr: none are pending)
  void retire(hipStream_t s) {
    if (!exec && !graph) return;
    hipEvent_t ev = nullptr;
    if (s != nullptr || exec) {
      if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
          hipEventRecord(ev, s) != hipSuccess) {
        if (ev) (void)hipEventDestroy(ev);
        ev = nullptr;
        (void)hipDeviceSynchronize();
      }
    }
    if (ev) {
      std::lock_guard<std::mutex> lock(g_retire_mu);
      g_retired.push_back({exec, graph, ev});
    } else {
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
    }
    exec = nullptr;
    graph = nullptr;
  }
  template <typename F>
  hipError_t capture(hipStream_t s, F&& launches) {
    retire(s);
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t le = launches(s);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (le != hipSuccess || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return le != hipSuccess ? le : e;
    }
    graph = g;
    return hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  }
  hipError_t launch(hipStream_t s) const { return hipGraphLaunch(exec, s); }
};

// ---------------------------------------------------------------------------
// Kernel timing (semd_profile_*): HIP events on the launch stream around
// each kernel, read back once they have completed
// ---------------------------------------------------------------------------

enum ProfKind {
  kPLoad, kPScan, kPCompact, kPSolve, kPEval, kPResident,
  // host time (wall clock of the calling thread) in phases of the batch calls
  kHAlloc, kHTables, kHUpload, kHLaunch, kHBatch, kPKinds
};
const char* const kProfNames[kPKinds] = {
    "st_load_kernel",  "st_scan_kernel", "st_compact_kernel", "st_solve_kernel",
    "st_eval_kernel",  "resident_emd_kernel", "host_alloc",    "host_tables",
    "host_upload",     "host_launch",    "host_batch_call"};

struct ProfSpan {
  int kind;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfSpan> g_prof_spans;      // recorded, not yet read
std::vector<hipEvent_t> g_prof_events;   // owned by the profiler
std::vector<hipEvent_t> g_prof_free;     // of those, free for reuse
double g_prof_ms[kPKinds] = {};
int64_t g_prof_n[kPKinds] = {};

bool profiling() {
  std::lock_guard<std::mutex> lock(g_prof_mu);
  return g_prof_on;
}

// n events for one launch sequence (nullptr on failure: timing skipped).
bool prof_events(hipEvent_t* out, int n) {
  std::lock_guard<std::mutex> lock(g_prof_mu);
  for (int i = 0; i < n; ++i) {
    if (g_prof_free.empty()) {
      hipEvent_t ev = nullptr;
      if (hipEventCreate(&ev) != hipSuccess) return false;
      g_prof_events.push_back(ev);
      g_prof_free.push_back(ev);
    }
    out[i] = g_prof_free.back();
    g_prof_free.pop_back();
  }
  return true;
}

// Adds the host time of its scope to a phase while profiling is on.
struct HostPhase {
  int kind;
  bool on;
  std::chrono::steady_clock::time_point t0;
  explicit HostPhase(int k);
  ~HostPhase();
};

void prof_span(int kind, hipEvent_t a, hipEvent_t b) {
  std::lock_guard<std::mutex> lock(g_prof_mu);
  g_prof_spans.push_back({kind, a, b});
}

HostPhase::HostPhase(int k) : kind(k), on(profiling()), t0(std::chrono::steady_clock::now()) {}
HostPhase::~HostPhase() {
  if (!on) return;
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  std::lock_guard<std::mutex> lock(g_prof_mu);
  g_prof_ms[kind] += ms;
  g_prof_n[kind] += 1;
}

// Waits for every recorded span and adds it to the totals; frees the events.
void prof_collect() {
  std::lock_guard<std::mutex> lock(g_prof_mu);
  for (const ProfSpan& sp : g_prof_spans) {
    float ms = 0.f;
    if (hipEventSynchronize(sp.b) == hipSuccess &&
        hipEventElapsedTime(&ms, sp.a, sp.b) == hipSuccess) {
      g_prof_ms[sp.kind] += ms;
      g_prof_n[sp.kind] += 1;
    }
  }
  g_prof_spans.clear();
  g_prof_free = g_prof_events;
}

// ---------------------------------------------------------------------------
// Workspace memory: stream-ordered allocations from a pool of the library's
// own per device, which keeps freed memory for reuse (mapping fresh device
// memory for every call would cost more than the work on large batches)
// ---------------------------------------------------------------------------

constexpr int kPoolDevices = 64;
std::mutex g_pool_dev_mu;
hipMemPool_t g_mem_pool[kPoolDevices] = {};
// The largest block each device's pool has handed out for a large
// workspace (cleared when the pool is trimmed).
size_t g_pool_big[kPoolDevices] = {};
constexpr size_t kStickyMin = size_t(256) << 20;

// The current device's pool, created on first use (nullptr: use the
// device's default pool).
hipMemPool_t lib_pool() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kPoolDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_pool_dev_mu);
  if (!g_mem_pool[dev]) {
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    if (hipMemPoolCreate(&pool, &props) != hipSuccess) return nullptr;
    uint64_t keep = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    g_mem_pool[dev] = pool;
  }
  return g_mem_pool[dev];
}

// Device bytes available to new workspaces: free device memory plus what
// the library's pool holds without using.
size_t available_device_bytes() {
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = size_t(8) << 30;
  hipMemPool_t pool = lib_pool();
  uint64_t reserved = 0, used = 0;
  if (pool && hipMemPoolGetAttribute(pool, hipMemPoolAttrReservedMemCurrent, &reserved) ==
                  hipSuccess &&
      hipMemPoolGetAttribute(pool, hipMemPoolAttrUsedMemCurrent, &used) == hipSuccess &&
      reserved > used)
    free_b += (size_t)(reserved - used);
  return free_b;
}

// A large workspace takes the size of the largest block the pool has handed
// out when that is at most twice its own: consecutive calls of varying size
// (the waves of a batch) then reuse one block in stream order, where each
// larger size would have the pool map new memory, and the call wait for it.
hipError_t dev_alloc(void** p, size_t bytes, hipStream_t s) {
  HostPhase hp(kHAlloc);
  hipMemPool_t pool = lib_pool();
  if (!pool) return hipMallocAsync(p, bytes, s);
  int dev = 0;
  size_t take = bytes;
  if (bytes >= kStickyMin && hipGetDevice(&dev) == hipSuccess && dev >= 0 &&
      dev < kPoolDevices) {
    std::lock_guard<std::mutex> lock(g_pool_dev_mu);
    size_t& big = g_pool_big[dev];
    if (bytes <= big && big / 2 <= bytes) take = big;
    else if (bytes > big) big = bytes;
  }
  hipError_t e = hipMallocFromPoolAsync(p, take, pool, s);
  if (e != hipSuccess && take > bytes) {
    (void)hipGetLastError();  // the rounded size did not fit; the exact one may
    e = hipMallocFromPoolAsync(p, bytes, pool, s);
  }
  return e;
}

// Pinned staging blocks for host -> device descriptor uploads; a block is
// reused once the copy recorded on it has completed.
struct PinnedBlock {
  void* host = nullptr;
  size_t bytes = 0;
  hipEvent_t ev = nullptr;
};
std::mutex g_pool_mu;
std::vector<std::unique_ptr<PinnedBlock>> g_pool;

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

// Consecutive 256-byte-aligned regions handed out from one device buffer
// (the workspace of a whole call, so that its parts need no allocation of
// their own).
struct Carve {
  unsigned char* p = nullptr;
  size_t left = 0;
  unsigned char* take(size_t b) {
    b = al256(std::max<size_t>(b, 1));
    if (b > left) return nullptr;
    unsigned char* q = p;
    p += b;
    left -= b;
    return q;
  }
};

// Copies bytes from src to device memory through a pinned staging block:
// into a region of `into` when given, else into a new stream-ordered
// allocation (*d_out).
int upload(const void* src, size_t bytes, hipStream_t s, void** d_out, Carve* into = nullptr) {
  HostPhase hp(kHUpload);
  PinnedBlock* blk = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_pool_mu);
    for (auto& b : g_pool)
      if (b->bytes >= bytes && hipEventQuery(b->ev) == hipSuccess) { blk = b.get(); break; }
    if (!blk) {
      auto nb = std::make_unique<PinnedBlock>();
      nb->bytes = std::max<size_t>(bytes, 64 * 1024);
      if (hipHostMalloc(&nb->host, nb->bytes, hipHostMallocDefault) != hipSuccess)
        return fail(SEMD_ENOMEM, "pinned staging allocation of %zu bytes failed", nb->bytes);
      if (hipEventCreateWithFlags(&nb->ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipHostFree(nb->host);
        return fail(SEMD_EDEVICE, "event creation failed");
      }
      blk = nb.get();
      g_pool.push_back(std::move(nb));
    }
    std::memcpy(blk->host, src, bytes);
    hipError_t e = hipSuccess;
    if (into) {
      *d_out = into->take(bytes);
      if (!*d_out) return fail(SEMD_ENOMEM, "call workspace too small for %zu bytes", bytes);
    } else {
      e = dev_alloc(d_out, bytes, s);
      if (e != hipSuccess)
        return fail(SEMD_ENOMEM, "device allocation of %zu bytes failed", bytes);
    }
    e = hipMemcpyAsync(*d_out, blk->host, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "descriptor upload");
    e = hipEventRecord(blk->ev, s);
    if (e != hipSuccess) return hip_fail(e, "event record");
  }
  return SEMD_OK;
}

struct Shape {
  int64_t M, N, L;
};

int shape_of(const int64_t* dims, int ndim, int D, Shape* sh) {
  int rc = parse_dims(dims, ndim, &sh->M, &sh->N);
  if (rc) return rc;
  if (D > sh->M)
    return fail(SEMD_EINVAL, "transition_len %d exceeds the fibre length %lld", D,
                (long long)sh->M);
  sh->L = sh->M * sh->N + (int64_t)D * sh->N - D;
  return SEMD_OK;
}

// Longest serialized signal: sample keys (4 * index + kind) are int32.
constexpr int64_t kMaxL = int64_t(1) << 28;

// ---------------------------------------------------------------------------
// Launch shapes of the resident kernel: defaults and the tuned table
// ---------------------------------------------------------------------------

// Length buckets (upper bounds) of the table, and its two regimes: launches
// with fewer items than the device has compute units (latency: a workgroup
// has a CU to itself) and launches with at least as many (throughput).
constexpr int kBuckets[] = {1024, 2048, 3072, 4096, 6144, 8192, 12288, 16384};
constexpr int kNBuckets = (int)(sizeof(kBuckets) / sizeof(kBuckets[0]));
static_assert(kBuckets[kNBuckets - 1] == semd::kResidentMaxL, "buckets cover the resident path");

struct TuneTable {
  semd::ResidentClass cls[2][kNBuckets];
  bool set[2][kNBuckets];
  // streaming batches: unfolded solve blocks per workgroup slot (0: the
  // built-in value)
  int solve_target;
};
// candidates the tuner times for it
constexpr int kSolveTargets[] = {1024, 2048, 4096, 8192, 16384};
constexpr int kMaxSolveTarget = 1 << 20;
std::mutex g_tune_mu;
TuneTable g_tune{};

int device_compute_units() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v < 1)
    return 256;
  return v;
}

int bucket_of(int L) {
  for (int b = 0; b < kNBuckets; ++b)
    if (L <= kBuckets[b]) return b;
  return kNBuckets - 1;
}

semd::ResidentClass class_for(int L, int regime) {
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const int b = bucket_of(L);
    if (g_tune.set[regime][b]) return g_tune.cls[regime][b];
  }
  return semd::resident_class(L, regime);
}

bool class_compiled(semd::ResidentClass c) {
  semd::ResidentClass all[32];
  const int n = semd::resident_classes(all, 32);
  for (int i = 0; i < n; ++i)
    if (all[i].nt == c.nt && all[i].c == c.c) return true;
  return false;
}

// Decompose `work` on the resident path: one workgroup per item, a workspace
// of resident_ws_doubles(L) per item (residue, parked envelope or knot
// store).  force: a launch shape for every item (else the table's choice).
int run_resident(std::vector<semd::WorkItem>& work, int K, int S, hipStream_t stream,
                 const semd::ResidentClass* force = nullptr, Carve* into = nullptr) {
  if (work.empty()) return SEMD_OK;
  // longest first, so the tail of each launch holds the short items
  std::stable_sort(work.begin(), work.end(),
                   [](const semd::WorkItem& a, const semd::WorkItem& b) { return a.L > b.L; });
  int64_t ws_doubles = 0;
  for (const auto& w : work) ws_doubles += semd::resident_ws_doubles(w.L);
  double* ws = nullptr;
  const size_t ws_bytes = sizeof(double) * (size_t)std::max<int64_t>(ws_doubles, 1);
  hipError_t e = hipSuccess;
  if (into) {
    ws = reinterpret_cast<double*>(into->take(ws_bytes));
    if (!ws) return fail(SEMD_ENOMEM, "call workspace too small for the on-chip items");
  } else {
    e = dev_alloc(reinterpret_cast<void**>(&ws), ws_bytes, stream);
  }
  if (e != hipSuccess)
    return fail(SEMD_ENOMEM, "workspace of %lld doubles", (long long)ws_doubles);
  int64_t off = 0;
  for (auto& w : work) {
    w.r = ws + off;
    w.u = w.r + w.L;
    off += semd::resident_ws_doubles(w.L);
  }
  void* d_items = nullptr;
  int rc = upload(work.data(), work.size() * sizeof(semd::WorkItem), stream, &d_items, into);
  if (rc) {
    if (!into) (void)hipFreeAsync(ws, stream);
    return rc;
  }
  // one launch per launch-shape class, each with the LDS its longest item needs
  auto same = [](const semd::ResidentClass& a, const semd::ResidentClass& b) {
    return a.nt == b.nt && a.c == b.c;
  };
  const int regime = (int)work.size() >= device_compute_units() ? 1 : 0;
  auto shape = [&](int L) { return force ? *force : class_for(L, regime); };
  size_t i0 = 0;
  while (i0 < work.size() && rc == SEMD_OK) {
    const semd::ResidentClass cls = shape(work[i0].L);
    size_t i1 = i0;
    while (i1 < work.size() && same(shape(work[i1].L), cls)) ++i1;
    const auto* d = static_cast<const semd::WorkItem*>(d_items) + i0;
    hipEvent_t ev[2];
    const bool timed = profiling() && prof_events(ev, 2);
    if (timed) (void)hipEventRecord(ev[0], stream);
    e = semd::launch_resident(d, (int)(i1 - i0), work[i0].L, cls, K, S, stream);
    if (timed) {
      (void)hipEventRecord(ev[1], stream);
      prof_span(kPResident, ev[0], ev[1]);
    }
    if (e != hipSuccess) rc = hip_fail(e, "resident kernel launch");
    i0 = i1;
  }
  if (!into) {
    (void)hipFreeAsync(d_items, stream);
    (void)hipFreeAsync(ws, stream);
  }
  return rc;
}

// Device bytes the streaming path needs for one signal of L samples, and
// the carving of such a region into the signal's buffers.
size_t stream_bytes(int64_t L) {
  const size_t cap = (size_t)((L - 1) / 2 + 12);
  const size_t ntiles = (size_t)((L + semd::kTile - 1) / semd::kTile);
  return 2 * al256(sizeof(double) * (size_t)L) +
         2 * (al256(sizeof(int32_t) * cap) + 2 * al256(sizeof(double) * cap)) +
         al256(sizeof(semd::TileInfo) * ntiles) + al256(sizeof(double) * 4 * ntiles) +
         al256(sizeof(int32_t) * semd::kTileThreads * ntiles) +
         2 * (al256(sizeof(int32_t) * semd::kTileKnots * ntiles) +
              al256(sizeof(double) * semd::kTileKnots * ntiles)) +
         al256(sizeof(semd::SigStatus));
}

semd::StreamSig stream_sig(const semd::WorkItem& w, int K, int S, unsigned char* region) {
  semd::StreamSig g{};
  g.X = w.X;
  g.out = w.out;
  g.n_imfs = w.n_imfs;
  g.stats = w.stats;
  g.M = w.M;
  g.N = w.N;
  g.D = w.D;
  g.L = w.L;
  g.beta = w.beta;
  g.key = w.key;
  g.flags = w.flags;
  g.addend = w.addend;
  g.scale = w.scale;
  g.slot_stride = w.slot_stride;
  g.sd = w.sd;
  g.ntiles = (w.L + semd::kTile - 1) / semd::kTile;
  g.K = K;
  g.S = S;
  g.cap = (w.L - 1) / 2 + 12;
  size_t o = 0;
  auto take = [&](size_t b) {
    unsigned char* p = region + o;
    o += al256(b);
    return p;
  };
  g.h = reinterpret_cast<double*>(take(sizeof(double) * (size_t)w.L));
  g.r = reinterpret_cast<double*>(take(sizeof(double) * (size_t)w.L));
  for (int e = 0; e < 2; ++e) {
    g.kt[e] = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)g.cap));
    g.ky[e] = reinterpret_cast<double*>(take(sizeof(double) * (size_t)g.cap));
    g.km[e] = reinterpret_cast<double*>(take(sizeof(double) * (size_t)g.cap));
  }
  g.tinfo = reinterpret_cast<semd::TileInfo*>(take(sizeof(semd::TileInfo) * (size_t)g.ntiles));
  g.edge = reinterpret_cast<double*>(take(sizeof(double) * 4 * (size_t)g.ntiles));
  g.trank = reinterpret_cast<int32_t*>(
      take(sizeof(int32_t) * semd::kTileThreads * (size_t)g.ntiles));
  for (int e = 0; e < 2; ++e) {
    g.lpos[e] = reinterpret_cast<int32_t*>(
        take(sizeof(int32_t) * semd::kTileKnots * (size_t)g.ntiles));
    g.lval[e] = reinterpret_cast<double*>(
        take(sizeof(double) * semd::kTileKnots * (size_t)g.ntiles));
  }
  g.st = reinterpret_cast<semd::SigStatus*>(take(sizeof(semd::SigStatus)));
  g.trace = w.trace;
  g.trace_cap = w.trace_cap;
  return g;
}

// Tile and solve-block tables of a list of streaming signals.
// solve_target: unfolded solve blocks per workgroup slot, or < 0 for the
// tuned table's value.
void stream_tables(const std::vector<semd::StreamSig>& sigs, std::vector<int2>& tiles,
                   std::vector<int4>& blocks, int solve_target = -1) {
  tiles.clear();
  blocks.clear();
  if (solve_target < 0) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    solve_target = g_tune.solve_target;
  }
  int64_t total = 0;
  for (const auto& g : sigs) total += 2 * (int64_t)semd::stream_solve_blocks(g.cap);
  const int fold = semd::stream_solve_fold(total, solve_target);
  for (int i = 0; i < (int)sigs.size(); ++i) {
    for (int t = 0; t < sigs[i].ntiles; ++t) tiles.push_back(make_int2(i, t));
    const int G = semd::stream_solve_groups(sigs[i].cap, fold);
    for (int e = 0; e < 2; ++e)
      for (int z = 0; z < G; ++z) blocks.push_back(make_int4(i, e, z, G));
  }
}

// Signals, tiles and blocks packed for one upload; returns byte offsets.
std::vector<unsigned char> pack_tables(const std::vector<semd::StreamSig>& sigs,
                                       const std::vector<int2>& tiles,
                                       const std::vector<int4>& blocks, size_t* o_til,
                                       size_t* o_blk) {
  const size_t b_sig = sizeof(semd::StreamSig) * sigs.size();
  const size_t b_til = sizeof(int2) * tiles.size();
  const size_t b_blk = sizeof(int4) * blocks.size();
  std::vector<unsigned char> pack(std::max<size_t>(b_sig + b_til + b_blk, 16));
  std::memcpy(pack.data(), sigs.data(), b_sig);
  std::memcpy(pack.data() + b_sig, tiles.data(), b_til);
  std::memcpy(pack.data() + b_sig + b_til, blocks.data(), b_blk);
  *o_til = b_sig;
  *o_blk = b_sig + b_til;
  return pack;
}

// Decompose `work` on the streaming path: K*S steps of every signal.
int run_stream(const std::vector<semd::WorkItem>& work, int K, int S, hipStream_t stream,
               Carve* into = nullptr, int solve_target = -1) {
  const int n = (int)work.size();
  if (n == 0) return SEMD_OK;
  size_t bytes = 0;
  std::vector<size_t> offs(n);
  for (int i = 0; i < n; ++i) {
    offs[i] = bytes;
    bytes += al256(stream_bytes(work[i].L));
  }
  unsigned char* arena = nullptr;
  if (into) {
    arena = into->take(bytes);
    if (!arena) return fail(SEMD_ENOMEM, "call workspace too small for the streaming items");
  } else if (dev_alloc(reinterpret_cast<void**>(&arena), std::max<size_t>(bytes, 1), stream) !=
             hipSuccess) {
    return fail(SEMD_ENOMEM, "streaming workspace of %zu bytes", bytes);
  }
  std::vector<semd::StreamSig> sigs(n);
  std::vector<int2> tiles;
  std::vector<int4> blocks;
  size_t o_til, o_blk;
  std::vector<unsigned char> pack;
  {
    HostPhase hp(kHTables);
    for (int i = 0; i < n; ++i) sigs[i] = stream_sig(work[i], K, S, arena + offs[i]);
    stream_tables(sigs, tiles, blocks, solve_target);
    pack = pack_tables(sigs, tiles, blocks, &o_til, &o_blk);
  }
  void* d_pack = nullptr;
  int rc = upload(pack.data(), pack.size(), stream, &d_pack, into);
  if (rc) {
    if (!into) (void)hipFreeAsync(arena, stream);
    return rc;
  }
  unsigned char* dp = static_cast<unsigned char*>(d_pack);
  const auto* d_sigs = reinterpret_cast<const semd::StreamSig*>(dp);
  const auto* d_tiles = reinterpret_cast<const int2*>(dp + o_til);
  const auto* d_blocks = reinterpret_cast<const int4*>(dp + o_blk);
  const int nt = (int)tiles.size(), nb = (int)blocks.size();
  bool any_sd = false;
  for (const auto& w : work) any_sd |= w.sd > 0.0;
  // every signal finishes within K*S steps (each step sifts it or ends an
  // IMF): the step is captured once and replayed K*S times
  sweep_retired_graphs();
  CaptureStream cs;
  hipError_t e = cs.open(stream);
  if (e == hipSuccess && profiling()) {
    // timed: the same launches, issued directly with events between them
    HostPhase hp(kHLaunch);
    hipEvent_t ev[5];
    bool timed = prof_events(ev, 2);
    if (timed) (void)hipEventRecord(ev[0], cs.s);
    e = semd::st_load(d_sigs, d_tiles, nt, cs.s);
    if (timed) {
      (void)hipEventRecord(ev[1], cs.s);
      prof_span(kPLoad, ev[0], ev[1]);
    }
    for (int step = 0; step < K * S && e == hipSuccess; ++step) {
      timed = prof_events(ev, 5);
      e = semd::st_step(d_sigs, n, d_tiles, nt, d_blocks, nb, cs.s, any_sd, false,
                        timed ? ev : nullptr);
      if (timed)
        for (int k = 0; k < 4; ++k) prof_span(kPScan + k, ev[k], ev[k + 1]);
    }
    if (e == hipSuccess) e = cs.join();
    if (e != hipSuccess) rc = hip_fail(e, "streaming kernel launch");
    if (!into) {
      (void)hipFreeAsync(d_pack, stream);
      (void)hipFreeAsync(arena, stream);
    }
    return rc;
  }
  if (e == hipSuccess) e = semd::st_load(d_sigs, d_tiles, nt, cs.s);
  {
    StepGraph g;
    if (e == hipSuccess)
      e = g.capture(cs.s, [&](hipStream_t s) {
        return semd::st_step(d_sigs, n, d_tiles, nt, d_blocks, nb, s, any_sd);
      });
    for (int step = 0; step < K * S && e == hipSuccess; ++step) e = g.launch(cs.s);
    g.retire(cs.s);
    if (e == hipSuccess) e = cs.join();
  }
  if (e != hipSuccess) rc = hip_fail(e, "streaming kernel launch");
  if (!into) {
    (void)hipFreeAsync(d_pack, stream);
    (void)hipFreeAsync(arena, stream);
  }
  return rc;
}

// Route every item to the on-chip path (one workgroup per signal) or the
// streaming path, by `path` and length.
bool routed_onchip(int64_t L, int path) {
  return path == SEMD_PATH_ONCHIP || (path == SEMD_PATH_AUTO && L <= semd::kResidentMaxL);
}

int run_work(std::vector<semd::WorkItem>& work, int K, int S, int path, hipStream_t stream,
             Carve* into = nullptr) {
  std::vector<semd::WorkItem> onchip, streamed;
  for (const auto& w : work) {
    if (routed_onchip(w.L, path)) onchip.push_back(w);
    else streamed.push_back(w);
  }
  int rc = run_resident(onchip, K, S, stream, nullptr, into);
  if (rc == SEMD_OK) rc = run_stream(streamed, K, S, stream, into);
  return rc;
}

// Bytes of device workspace run_work takes from a Carve for these items
// (the regions it carves, each rounded to 256 bytes).
size_t work_scratch_bytes(const std::vector<semd::WorkItem>& work, int path) {
  int64_t ws_doubles = 0;
  size_t n_on = 0, arena = 0, n_st = 0, tiles = 0, blocks = 0;
  for (const auto& w : work) {
    if (routed_onchip(w.L, path)) {
      ws_doubles += semd::resident_ws_doubles(w.L);
      ++n_on;
    } else {
      arena += al256(stream_bytes(w.L));
      ++n_st;
      tiles += (size_t)((w.L + semd::kTile - 1) / semd::kTile);
      blocks += 2 * (size_t)semd::stream_solve_blocks((int)((w.L - 1) / 2 + 12));
    }
  }
  size_t b = 0;
  if (n_on) {
    b += al256(sizeof(double) * (size_t)std::max<int64_t>(ws_doubles, 1));
    b += al256(sizeof(semd::WorkItem) * n_on);
  }
  if (n_st) {
    b += al256(arena);
    b += al256(std::max<size_t>(sizeof(semd::StreamSig) * n_st + sizeof(int2) * tiles +
                                    sizeof(int4) * blocks, 16));
  }
  return b;
}

// Workspace of one signal decomposed on its own (semd_decompose_ex): its
// descriptor, on the streaming path its tile and solve-block tables, and the
// path's buffers, carved from one region that starts 256-byte aligned.
struct SingleLayout {
  bool onchip;
  int ntiles, nblocks;
  size_t o_tiles, o_blocks, o_data, bytes;
};

SingleLayout single_layout(int64_t L, int path) {
  SingleLayout s{};
  s.onchip = path == SEMD_PATH_ONCHIP || (path == SEMD_PATH_AUTO && L <= semd::kResidentMaxL);
  if (s.onchip) {
    s.o_data = al256(sizeof(semd::WorkItem));
    s.bytes = s.o_data + al256(sizeof(double) * (size_t)semd::resident_ws_doubles(L));
  } else {
    const int cap = (int)((L - 1) / 2 + 12);
    s.ntiles = (int)((L + semd::kTile - 1) / semd::kTile);
    s.nblocks = 2 * semd::stream_solve_groups(
                        cap, semd::stream_solve_fold(2 * semd::stream_solve_blocks(cap)));
    s.o_tiles = al256(sizeof(semd::StreamSig));
    s.o_blocks = s.o_tiles + al256(sizeof(int2) * (size_t)s.ntiles);
    s.o_data = s.o_blocks + al256(sizeof(int4) * (size_t)s.nblocks);
    s.bytes = s.o_data + al256(stream_bytes(L));
  }
  return s;
}

// Decompose one signal inside the workspace ws (single_layout's bytes, 256-byte
// aligned): descriptors written by kernels from their arguments, then the
// path's kernels launched directly on `stream` (one resident launch, or the
// load and K*S streaming steps).  Enqueues nothing but kernels.
int run_single(semd::WorkItem w, int K, int S, int path, unsigned char* ws, hipStream_t stream) {
  const SingleLayout lay = single_layout(w.L, path);
  hipError_t e;
  if (lay.onchip) {
    w.r = reinterpret_cast<double*>(ws + lay.o_data);
    w.u = w.r + w.L;
    auto* d = reinterpret_cast<semd::WorkItem*>(ws);
    e = semd::launch_put_work(w, d, stream);
    if (e == hipSuccess)
      e = w.trace ? semd::launch_resident_trace(d, 1, w.L, K, S, stream)
                  : semd::launch_resident(d, 1, w.L, class_for(w.L, 0), K, S, stream);
    return e == hipSuccess ? SEMD_OK : hip_fail(e, "resident kernel launch");
  }
  const semd::StreamSig g = stream_sig(w, K, S, ws + lay.o_data);
  auto* d_sig = reinterpret_cast<semd::StreamSig*>(ws);
  auto* d_tiles = reinterpret_cast<int2*>(ws + lay.o_tiles);
  auto* d_blocks = reinterpret_cast<int4*>(ws + lay.o_blocks);
  e = semd::st_put_single(g, d_sig, d_tiles, d_blocks, stream);
  if (e == hipSuccess) e = semd::st_load(d_sig, d_tiles, lay.ntiles, stream);
  // every signal finishes within K*S steps (each step sifts it or ends an IMF)
  for (int step = 0; step < K * S && e == hipSuccess; ++step)
    e = semd::st_step(d_sig, 1, d_tiles, lay.ntiles, d_blocks, lay.nblocks, stream, w.sd > 0.0,
                      w.trace != nullptr);
  return e == hipSuccess ? SEMD_OK : hip_fail(e, "streaming kernel launch");
}

semd::WorkItem make_work(const double* X, double* out, int32_t* n_imfs, const Shape& sh, int D,
                         double sd, int64_t* stats = nullptr) {
  semd::WorkItem w{};
  w.X = X;
  w.out = out;
  w.n_imfs = n_imfs;
  w.stats = stats;
  w.M = sh.M;
  w.N = sh.N;
  w.D = D;
  w.L = (int32_t)sh.L;
  w.slot_stride = sh.M * sh.N;
  w.sd = sd;
  return w;
}

int check_length(int64_t L, int path, int i) {
  if (L > kMaxL)
    return fail(SEMD_EUNSUPPORTED, "item %d: serialized length %lld exceeds %lld", i,
                (long long)L, (long long)kMaxL);
  if (path == SEMD_PATH_ONCHIP && L > semd::kResidentMaxL)
    return fail(SEMD_EUNSUPPORTED,
                "item %d: serialized length %lld exceeds the on-chip path limit %d", i,
                (long long)L, semd::kResidentMaxL);
  return SEMD_OK;
}

int check_items(const semd_item* items, int n, int D, int path, std::vector<Shape>& shapes) {
  if (n < 0) return fail(SEMD_EINVAL, "n must be >= 0");
  if (n > 0 && !items) return fail(SEMD_EINVAL, "items is NULL");
  shapes.resize(n);
  for (int i = 0; i < n; ++i) {
    const semd_item& it = items[i];
    if (!it.signal || !it.imfs_out) return fail(SEMD_EINVAL, "item %d: NULL signal or output", i);
    if (it.reserved != 0) return fail(SEMD_EINVAL, "item %d: reserved must be 0", i);
    int rc = shape_of(it.dims, it.ndim, D, &shapes[i]);
    if (rc) {
      char msg[sizeof(g_err)];
      std::snprintf(msg, sizeof(msg), "%s", g_err);
      return fail(rc, "item %d: %s", i, msg);
    }
    rc = check_length(shapes[i].L, path, i);
    if (rc) return rc;
  }
  return SEMD_OK;
}

// Workspace of semd_decompose_ex_noalloc: one array per GPU, alive until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in for the symbol); it uses the device address
// hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array, looked up on the
// first call on each device and kept.
int scratch_for_current_device(unsigned char** out) {
  int dev = 0;
  SEMD_HIP(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(SEMD_EUNSUPPORTED, "device %d beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr || reinterpret_cast<uintptr_t>(ptr) % 256 != 0)
      return fail(SEMD_EDEVICE, "scratch array at an unaligned address");
    g_scratch_ptr[dev] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return SEMD_OK;
}

// Validated shape of one signal of semd_decompose_ex (and its workspace).
int check_single(const int64_t* dims, int ndim, const semd_params* p, Shape* sh) {
  int rc = check_params(p, false);
  if (rc) return rc;
  rc = shape_of(dims, ndim, p->transition_len, sh);
  if (rc) return rc;
  return check_length(sh->L, p->path, 0);
}

}  // namespace

extern "C" {

int semd_abi_version(void) { return SEMD_ABI_VERSION; }

const char* semd_last_error(void) { return g_err; }

int64_t semd_serial_length(int64_t M, int64_t N, int64_t D) {
  if (M < 1 || N < 1 || D < 0 || D > M) return -1;
  return M * N + D * N - D;
}

int64_t semd_resident_max_length(void) { return semd::kResidentMaxL; }

int semd_autotune(int64_t max_length, int batch, hipStream_t stream) {
  g_err[0] = 0;
  if (max_length < 3 || max_length > semd::kResidentMaxL)
    return fail(SEMD_EINVAL, "max_length must be in [3, %d]", semd::kResidentMaxL);
  if (batch < 1 || batch > 65536) return fail(SEMD_EINVAL, "batch must be in [1, 65536]");
  const int K = 6, S = 10;
  const int cus = device_compute_units();
  semd::ResidentClass all[32];
  const int nall = semd::resident_classes(all, 32);
  TuneTable t;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    t = g_tune;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(SEMD_EDEVICE, "event creation failed");
  }
  int rc = SEMD_OK;
  for (int regime = 0; regime < 2 && rc == SEMD_OK; ++regime) {
    const int n = regime == 0 ? 1 : std::max(batch, cus);
    for (int b = 0; b < kNBuckets && rc == SEMD_OK; ++b) {
      const int lo = b == 0 ? 3 : kBuckets[b - 1] + 1;
      if (lo > max_length) break;
      const int64_t L = kBuckets[b];  // the bucket's longest signal
      double *X = nullptr, *out = nullptr;
      if (hipMalloc(reinterpret_cast<void**>(&X), sizeof(double) * L * n) != hipSuccess ||
          hipMalloc(reinterpret_cast<void**>(&out), sizeof(double) * L * (K + 1) * n) !=
              hipSuccess) {
        if (X) (void)hipFree(X);
        rc = fail(SEMD_ENOMEM, "tuning buffers for %d signals of %lld samples", n, (long long)L);
        break;
      }
      std::vector<semd::WorkItem> work;
      Shape sh{L, 1, L};
      for (int i = 0; i < n; ++i)
        work.push_back(make_work(X + i * L, out + i * L * (K + 1), nullptr, sh, 0, 0.0));
      hipError_t he = semd::launch_synth(X, L, n, 2106, stream);
      float best_ms = 0.0f;
      semd::ResidentClass best{0, 0};
      for (int ci = 0; ci < nall && he == hipSuccess && rc == SEMD_OK; ++ci) {
        const semd::ResidentClass c = all[ci];
        if (c.nt * c.c < L || c.nt * c.c > 4 * L) continue;
        std::vector<semd::WorkItem> w = work;
        rc = run_resident(w, K, S, stream, &c);  // warm-up
        if (rc == SEMD_OK) he = hipEventRecord(e0, stream);
        for (int r = 0; r < 2 && rc == SEMD_OK && he == hipSuccess; ++r) {
          w = work;
          rc = run_resident(w, K, S, stream, &c);
        }
        if (rc == SEMD_OK && he == hipSuccess) he = hipEventRecord(e1, stream);
        if (rc == SEMD_OK && he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (rc == SEMD_OK && he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (rc == SEMD_OK && he == hipSuccess && (best.nt == 0 || ms < best_ms)) {
          best = c;
          best_ms = ms;
        }
      }
      if (he != hipSuccess && rc == SEMD_OK) rc = hip_fail(he, "tuning run");
      (void)hipStreamSynchronize(stream);
      (void)hipFree(X);
      (void)hipFree(out);
      if (rc == SEMD_OK && best.nt > 0) {
        t.cls[regime][b] = best;
        t.set[regime][b] = true;
      }
    }
  }
  // Streaming batches: the solve launch's fold, timed on a batch of 2 x CUs
  // synthetic signals of 65,536 samples (three sifts of two IMFs), one
  // candidate target after another.  The fold maps blocks to workgroups
  // and leaves the arithmetic as it is.
  if (rc == SEMD_OK) {
    const int64_t L = 65536;
    const int n = 2 * cus, Ks = 2, Ss = 3;
    double *X = nullptr, *out = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(&X), sizeof(double) * L * n) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&out), sizeof(double) * L * (Ks + 1) * n) !=
            hipSuccess) {
      if (X) (void)hipFree(X);
      rc = fail(SEMD_ENOMEM, "tuning buffers for %d signals of %lld samples", n, (long long)L);
    } else {
      std::vector<semd::WorkItem> work;
      Shape sh{L, 1, L};
      for (int i = 0; i < n; ++i)
        work.push_back(make_work(X + i * L, out + i * L * (Ks + 1), nullptr, sh, 0, 0.0));
      hipError_t he = semd::launch_synth(X, L, n, 2106, stream);
      float best_ms = 0.0f;
      int best = 0;
      for (int target : kSolveTargets) {
        if (he != hipSuccess || rc != SEMD_OK) break;
        rc = run_stream(work, Ks, Ss, stream, nullptr, target);  // warm-up
        if (rc == SEMD_OK) he = hipEventRecord(e0, stream);
        for (int r = 0; r < 2 && rc == SEMD_OK && he == hipSuccess; ++r)
          rc = run_stream(work, Ks, Ss, stream, nullptr, target);
        if (rc == SEMD_OK && he == hipSuccess) he = hipEventRecord(e1, stream);
        if (rc == SEMD_OK && he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (rc == SEMD_OK && he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (rc == SEMD_OK && he == hipSuccess && (best == 0 || ms < best_ms)) {
          best = target;
          best_ms = ms;
        }
      }
      if (he != hipSuccess && rc == SEMD_OK) rc = hip_fail(he, "tuning run");
      (void)hipStreamSynchronize(stream);
      (void)hipFree(X);
      (void)hipFree(out);
      if (rc == SEMD_OK && best > 0) t.solve_target = best;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == SEMD_OK) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune = t;
  }
  return rc;
}

// Text form of the table:
//   semd-tune <abi> <gfx arch>
//   latency|throughput <bucket bound> <threads> <samples per thread>
//   stream-solve <unfolded solve blocks per workgroup slot>
int semd_tune_get(char* buf, size_t cap, size_t* needed) {
  g_err[0] = 0;
  if (!needed) return fail(SEMD_EINVAL, "needed is NULL");
  hipDeviceProp_t prop{};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(SEMD_EDEVICE, "no device");
  std::string text = "semd-tune " + std::to_string(SEMD_ABI_VERSION) + " " + prop.gcnArchName +
                     "\n";
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (int r = 0; r < 2; ++r)
      for (int b = 0; b < kNBuckets; ++b)
        if (g_tune.set[r][b])
          text += std::string(r == 0 ? "latency " : "throughput ") +
                  std::to_string(kBuckets[b]) + " " + std::to_string(g_tune.cls[r][b].nt) + " " +
                  std::to_string(g_tune.cls[r][b].c) + "\n";
    if (g_tune.solve_target > 0)
      text += "stream-solve " + std::to_string(g_tune.solve_target) + "\n";
  }
  *needed = text.size() + 1;
  if (buf && cap > 0) {
    const size_t k = std::min(cap - 1, text.size());
    std::memcpy(buf, text.data(), k);
    buf[k] = 0;
    if (cap < text.size() + 1) return fail(SEMD_EINVAL, "buffer of %zu bytes is short", cap);
  }
  return SEMD_OK;
}

int semd_tune_set(const char* text) {
  g_err[0] = 0;
  if (!text) return fail(SEMD_EINVAL, "text is NULL");
  hipDeviceProp_t prop{};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(SEMD_EDEVICE, "no device");
  TuneTable t{};
  const char* p = text;
  int abi = 0;
  char arch[96] = "";
  int used = 0;
  if (std::sscanf(p, "semd-tune %d %95s%n", &abi, arch, &used) != 2)
    return fail(SEMD_EINVAL, "not a tuning table");
  if (abi != SEMD_ABI_VERSION || std::strcmp(arch, prop.gcnArchName) != 0)
    return fail(SEMD_EINVAL, "tuning table is for abi %d on %s, not abi %d on %s", abi, arch,
                SEMD_ABI_VERSION, prop.gcnArchName);
  p += used;
  for (;;) {
    char word[16] = "";
    if (std::sscanf(p, "%15s%n", word, &used) != 1) break;
    p += used;
    if (std::strcmp(word, "stream-solve") == 0) {
      int target = 0;
      if (std::sscanf(p, "%d%n", &target, &used) != 1)
        return fail(SEMD_EINVAL, "malformed tuning entry");
      p += used;
      if (target < 1 || target > kMaxSolveTarget)
        return fail(SEMD_EINVAL, "invalid tuning entry stream-solve %d", target);
      t.solve_target = target;
      continue;
    }
    int bound = 0, nt = 0, c = 0;
    if (std::sscanf(p, "%d %d %d%n", &bound, &nt, &c, &used) != 3)
      return fail(SEMD_EINVAL, "malformed tuning entry");
    p += used;
    const int r = std::strcmp(word, "latency") == 0 ? 0
                  : std::strcmp(word, "throughput") == 0 ? 1
                                                          : -1;
    int b = -1;
    for (int i = 0; i < kNBuckets; ++i)
      if (kBuckets[i] == bound) b = i;
    const semd::ResidentClass cls{nt, c};
    if (r < 0 || b < 0 || !class_compiled(cls) || nt * c < bound)
      return fail(SEMD_EINVAL, "invalid tuning entry %s %d %d %d", word, bound, nt, c);
    t.cls[r][b] = cls;
    t.set[r][b] = true;
  }
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune = t;
  return SEMD_OK;
}

int semd_tune_reset(void) {
  g_err[0] = 0;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune = TuneTable{};
  return SEMD_OK;
}

size_t semd_workspace_bytes(const int64_t* dims, int ndim, const semd_params* p) {
  g_err[0] = 0;
  Shape sh;
  if (check_single(dims, ndim, p, &sh)) return 0;
  return single_layout(sh.L, p->path).bytes;
}

int semd_decompose_ex(const double* signal, const int64_t* dims, int ndim, const semd_params* p,
                      double* imfs_out, int32_t* n_imfs_out, void* workspace, size_t ws_bytes,
                      hipStream_t stream) {
  g_err[0] = 0;
  Shape sh;
  int rc = check_single(dims, ndim, p, &sh);
  if (rc) return rc;
  if (!signal || !imfs_out) return fail(SEMD_EINVAL, "NULL signal or output");
  const size_t need = single_layout(sh.L, p->path).bytes;
  const semd::WorkItem w = make_work(signal, imfs_out, n_imfs_out, sh, p->transition_len,
                                     sd_of(p));
  if (workspace) {
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
      return fail(SEMD_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
      return fail(SEMD_EINVAL, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    return run_single(w, p->max_imfs, p->sift_iters, p->path,
                      static_cast<unsigned char*>(workspace), stream);
  }
  unsigned char* ws = nullptr;
  if (dev_alloc(reinterpret_cast<void**>(&ws), need, stream) != hipSuccess)
    return fail(SEMD_ENOMEM, "workspace of %zu bytes", need);
  rc = run_single(w, p->max_imfs, p->sift_iters, p->path, ws, stream);
  (void)hipFreeAsync(ws, stream);
  return rc;
}

int semd_decompose_ex_noalloc(const double* signal, const int64_t* dims, int ndim,
                              const semd_params* p, double* imfs_out, int32_t* n_imfs_out,
                              hipStream_t stream) {
  g_err[0] = 0;
  Shape sh;
  int rc = check_single(dims, ndim, p, &sh);
  if (rc) return rc;
  if (!signal || !imfs_out) return fail(SEMD_EINVAL, "NULL signal or output");
  const size_t need = single_layout(sh.L, p->path).bytes;
  if (need > kScratchBytes)
    return fail(SEMD_EINVAL, "needs %zu bytes of workspace, the static scratch holds %zu", need,
                kScratchBytes);
  unsigned char* ws = nullptr;
  rc = scratch_for_current_device(&ws);
  if (rc) return rc;
  const semd::WorkItem w = make_work(signal, imfs_out, n_imfs_out, sh, p->transition_len,
                                     sd_of(p));
  return run_single(w, p->max_imfs, p->sift_iters, p->path, ws, stream);
}

size_t semd_noalloc_scratch_bytes(void) { return kScratchBytes; }

int semd_release_cached_memory(void) {
  g_err[0] = 0;
  std::lock_guard<std::mutex> lock(g_pool_dev_mu);
  for (int d = 0; d < kPoolDevices; ++d) {
    if (!g_mem_pool[d]) continue;
    g_pool_big[d] = 0;
    const hipError_t e = hipMemPoolTrimTo(g_mem_pool[d], 0);
    if (e != hipSuccess) return hip_fail(e, "hipMemPoolTrimTo");
  }
  return SEMD_OK;
}

int semd_profile_enable(int on) {
  g_err[0] = 0;
  std::lock_guard<std::mutex> lock(g_prof_mu);
  g_prof_on = on != 0;
  return SEMD_OK;
}

int semd_profile_reset(void) {
  g_err[0] = 0;
  prof_collect();
  std::lock_guard<std::mutex> lock(g_prof_mu);
  for (int k = 0; k < kPKinds; ++k) {
    g_prof_ms[k] = 0.0;
    g_prof_n[k] = 0;
  }
  return SEMD_OK;
}

int semd_profile_read(const char* kernel, int64_t* launches, double* total_ms) {
  g_err[0] = 0;
  if (!kernel || !launches || !total_ms)
    return fail(SEMD_EINVAL, "NULL kernel name or result pointer");
  int k = 0;
  while (k < kPKinds && std::strcmp(kernel, kProfNames[k]) != 0) ++k;
  if (k == kPKinds) return fail(SEMD_EINVAL, "no timed kernel named '%s'", kernel);
  prof_collect();
  std::lock_guard<std::mutex> lock(g_prof_mu);
  *launches = g_prof_n[k];
  *total_ms = g_prof_ms[k];
  return SEMD_OK;
}

int semd_decompose_trace(const double* signal, const int64_t* dims, int ndim,
                         const semd_params* p, double* imfs_out, int32_t* n_imfs_out,
                         int32_t* trace, int64_t trace_cap, hipStream_t stream) {
  g_err[0] = 0;
  Shape sh;
  int rc = check_single(dims, ndim, p, &sh);
  if (rc) return rc;
  if (!signal || !imfs_out || !trace) return fail(SEMD_EINVAL, "NULL signal, output or trace");
  if (trace_cap < 4 || trace_cap > INT32_MAX)
    return fail(SEMD_EINVAL, "trace_cap must be in [4, 2^31 - 1]");
  const size_t need = single_layout(sh.L, p->path).bytes;
  semd::WorkItem w = make_work(signal, imfs_out, n_imfs_out, sh, p->transition_len, sd_of(p));
  w.trace = trace;
  w.trace_cap = (int32_t)trace_cap;
  unsigned char* ws = nullptr;
  if (dev_alloc(reinterpret_cast<void**>(&ws), need, stream) != hipSuccess)
    return fail(SEMD_ENOMEM, "workspace of %zu bytes", need);
  rc = run_single(w, p->max_imfs, p->sift_iters, p->path, ws, stream);
  (void)hipFreeAsync(ws, stream);
  return rc;
}

int semd_decompose_slices(const double* signal, const int64_t* dims, int ndim,
                          const semd_params* p, double* imfs_out, int32_t* n_imfs_out,
                          hipStream_t stream) {
  g_err[0] = 0;
  int rc = check_params(p, false);
  if (rc) return rc;
  if (p->transition_len != 0)
    return fail(SEMD_EINVAL, "transition_len must be 0: slices are not serialized");
  if (!signal || !imfs_out) return fail(SEMD_EINVAL, "NULL signal or output");
  int64_t M, N;
  rc = parse_dims(dims, ndim, &M, &N);
  if (rc) return rc;
  if (N > (int64_t(1) << 24)) return fail(SEMD_EUNSUPPORTED, "%lld slices", (long long)N);
  rc = check_length(M, p->path, 0);
  if (rc) return rc;
  // column i is a signal of its own, writing its slots at column i of the
  // shared slot-major output
  const Shape col{M, 1, M};
  std::vector<semd::WorkItem> work;
  work.reserve((size_t)N);
  for (int64_t i = 0; i < N; ++i) {
    semd::WorkItem w = make_work(signal + i * M, imfs_out + i * M,
                                 n_imfs_out ? n_imfs_out + i : nullptr, col, 0, sd_of(p));
    w.slot_stride = M * N;
    work.push_back(w);
  }
  return run_work(work, p->max_imfs, p->sift_iters, p->path, stream);
}

int semd_decompose(const double* signal, const int64_t* dims, int ndim, int max_imfs,
                   int sift_iters, int boundary_rule, double* imfs_out, hipStream_t stream) {
  g_err[0] = 0;
  int64_t M, N;
  int rc = parse_dims(dims, ndim, &M, &N);
  if (rc) return rc;
  semd_params p{};
  p.transition_len = (int32_t)std::llround(0.2 * (double)M);
  p.max_imfs = max_imfs;
  p.sift_iters = sift_iters;
  p.boundary_rule = boundary_rule;
  p.ensemble = 1;
  return semd_decompose_ex(signal, dims, ndim, &p, imfs_out, nullptr, nullptr, 0, stream);
}

int semd_decompose_batch(const semd_item* items, int n, const semd_params* p,
                         hipStream_t stream) {
  g_err[0] = 0;
  int rc = check_params(p, false);
  if (rc) return rc;
  std::vector<Shape> shapes;
  rc = check_items(items, n, p->transition_len, p->path, shapes);
  if (rc) return rc;
  std::vector<semd::WorkItem> work;
  work.reserve(n);
  for (int i = 0; i < n; ++i)
    work.push_back(make_work(items[i].signal, items[i].imfs_out, items[i].n_imfs_out, shapes[i],
                             p->transition_len, sd_of(p), items[i].stats_out));
  return run_work(work, p->max_imfs, p->sift_iters, p->path, stream);
}

int semd_eemd_batch(const semd_item* items, int n, const semd_params* p, hipStream_t stream) {
  g_err[0] = 0;
  HostPhase hp(kHBatch);
  int rc = check_params(p, true);
  if (rc) return rc;
  std::vector<Shape> shapes;
  rc = check_items(items, n, p->transition_len, p->path, shapes);
  if (rc) return rc;
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(items[i].noise_sigma) || items[i].noise_sigma < 0)
      return fail(SEMD_EINVAL, "item %d: noise_sigma must be finite and >= 0", i);
  if (n == 0) return SEMD_OK;
  const int K = p->max_imfs, NR = p->ensemble;
  bool want_stats = false;
  for (int i = 0; i < n; ++i) want_stats |= items[i].stats_out != nullptr;
  // The realizations of consecutive items are decomposed in waves that fit
  // the budget (a third of the free device memory: larger waves take fewer
  // launches); one workspace, sized for the largest wave, serves them all.
  const size_t budget = std::max<size_t>(available_device_bytes() / 3, size_t(256) << 20);
  auto realizations = [&](int i0, int i1) {
    std::vector<semd::WorkItem> work;
    work.reserve((size_t)NR * (i1 - i0));
    for (int i = i0; i < i1; ++i)
      for (int m = 0; m < NR; ++m) {
        semd::WorkItem w = make_work(items[i].signal, nullptr, nullptr, shapes[i],
                                     p->transition_len, sd_of(p));
        w.beta = items[i].noise_sigma;
        w.key = semd::noise_key(p->seed, items[i].item_id, (uint64_t)m);
        w.flags = semd::kAddNoise;
        work.push_back(w);
      }
    return work;
  };
  struct Wave {
    int i0, i1;
    size_t slots, bytes;
  };
  std::vector<Wave> waves;
  size_t need = 0;
  for (int i0 = 0; i0 < n;) {
    size_t est = 0;
    int i1 = i0;
    while (i1 < n) {
      const size_t b = (size_t)NR * (sizeof(double) * (size_t)(K + 1) * shapes[i1].M *
                                         shapes[i1].N + stream_bytes(shapes[i1].L) +
                                     sizeof(int32_t));
      if (i1 > i0 && est + b > budget) break;
      est += b;
      ++i1;
    }
    Wave wv{i0, i1, 0, 0};
    for (int i = i0; i < i1; ++i) wv.slots += (size_t)NR * (K + 1) * shapes[i].M * shapes[i].N;
    wv.bytes = al256(sizeof(double) * std::max<size_t>(wv.slots, 1)) +
               al256(sizeof(int32_t) * (size_t)NR * (i1 - i0)) +
               (want_stats ? al256(sizeof(int64_t) * 3 * (size_t)NR * (i1 - i0)) : 0) +
               work_scratch_bytes(realizations(i0, i1), p->path);
    need = std::max(need, wv.bytes);
    waves.push_back(wv);
    i0 = i1;
  }
  unsigned char* ws = nullptr;
  if (dev_alloc(reinterpret_cast<void**>(&ws), need, stream) != hipSuccess)
    return fail(SEMD_ENOMEM, "EEMD workspace of %zu bytes", need);
  for (const Wave& wv : waves) {
    const int i0 = wv.i0, i1 = wv.i1;
    Carve cv{ws, need};
    double* buf = reinterpret_cast<double*>(cv.take(sizeof(double) * wv.slots));
    int32_t* cnt = reinterpret_cast<int32_t*>(cv.take(sizeof(int32_t) * (size_t)NR * (i1 - i0)));
    int64_t* wst = want_stats ? reinterpret_cast<int64_t*>(
                                    cv.take(sizeof(int64_t) * 3 * (size_t)NR * (i1 - i0)))
                              : nullptr;
    std::vector<semd::WorkItem> work = realizations(i0, i1);
    size_t so = 0, q = 0;
    for (int i = i0; i < i1; ++i) {
      const size_t per = (size_t)(K + 1) * shapes[i].M * shapes[i].N;
      for (int m = 0; m < NR; ++m, ++q) {
        work[q].out = buf + so + (size_t)m * per;
        work[q].n_imfs = cnt + (size_t)(i - i0) * NR + m;
        work[q].stats = items[i].stats_out ? wst + 3 * ((size_t)(i - i0) * NR + m) : nullptr;
      }
      so += (size_t)NR * per;
    }
    rc = run_work(work, K, p->sift_iters, p->path, stream, &cv);
    so = 0;
    for (int i = i0; i < i1 && rc == SEMD_OK; ++i) {
      const int64_t per = (int64_t)(K + 1) * shapes[i].M * shapes[i].N;
      hipError_t e = semd::launch_ensemble_mean(buf + so, NR, per, items[i].imfs_out, stream);
      if (e == hipSuccess && items[i].n_imfs_out)
        e = semd::launch_max_count(cnt + (size_t)(i - i0) * NR, NR, items[i].n_imfs_out, stream);
      if (e == hipSuccess && items[i].stats_out)
        e = semd::launch_sum_stats(wst + 3 * (size_t)(i - i0) * NR, NR, items[i].stats_out,
                                   stream);
      if (e != hipSuccess) rc = hip_fail(e, "ensemble mean launch");
      so += (size_t)NR * per;
    }
    if (rc) break;
  }
  (void)hipFreeAsync(ws, stream);
  return rc;
}

int semd_ceemdan_batch(const semd_item* items, int n, const semd_params* p,
                       hipStream_t stream) {
  g_err[0] = 0;
  int rc = check_params(p, true);
  if (rc) return rc;
  std::vector<Shape> shapes;
  rc = check_items(items, n, p->transition_len, p->path, shapes);
  if (rc) return rc;
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(items[i].noise_sigma) || items[i].noise_sigma < 0)
      return fail(SEMD_EINVAL, "item %d: noise_sigma (eps) must be finite and >= 0", i);
  const int K = p->max_imfs, NR = p->ensemble, S = p->sift_iters;
  const double sd = sd_of(p);
  const size_t budget = std::max<size_t>(available_device_bytes() / 4, size_t(256) << 20);
  // per item: residue, K mode slots, NR noise decompositions (K+1 slots),
  // NR stage outputs (2 slots), and the workspace of NR concurrent EMDs
  auto item_doubles = [&](int64_t L) {
    return (size_t)L * (1 + K + (size_t)NR * (K + 1) + (size_t)NR * 2);
  };
  int i0 = 0;
  while (i0 < n) {
    size_t bytes = 0;
    int i1 = i0;
    while (i1 < n) {
      const size_t b = sizeof(double) * item_doubles(shapes[i1].L) +
                       (size_t)NR * stream_bytes(shapes[i1].L) + sizeof(semd::CeemdanState);
      if (i1 > i0 && bytes + b > budget) break;
      bytes += b;
      ++i1;
    }
    const int nw = i1 - i0;
    size_t total = 0;
    std::vector<size_t> off(nw);
    for (int j = 0; j < nw; ++j) {
      off[j] = total;
      total += al256(sizeof(double) * item_doubles(shapes[i0 + j].L));
    }
    const size_t st_off = total;
    total += al256(sizeof(semd::CeemdanState) * (size_t)nw);
    unsigned char* arena = nullptr;
    if (dev_alloc(reinterpret_cast<void**>(&arena), total, stream) != hipSuccess)
      return fail(SEMD_ENOMEM, "CEEMDAN workspace of %zu bytes", total);
    auto* st = reinterpret_cast<semd::CeemdanState*>(arena + st_off);
    std::vector<semd::CeemdanJob> jobs(nw);
    std::vector<double*> E(nw);
    for (int j = 0; j < nw; ++j) {
      const Shape& sh = shapes[i0 + j];
      const int64_t L = sh.L;
      double* base = reinterpret_cast<double*>(arena + off[j]);
      semd::CeemdanJob& J = jobs[j];
      J.r = base;
      J.modes = base + L;
      E[j] = J.modes + (size_t)K * L;
      J.stage = E[j] + (size_t)NR * (K + 1) * L;
      J.out = items[i0 + j].imfs_out;
      J.n_out = items[i0 + j].n_imfs_out;
      J.st = st + j;
      J.M = sh.M;
      J.N = sh.N;
      J.L = L;
      J.slot_stride = sh.M * sh.N;
      J.D = p->transition_len;
      J.NR = NR;
      J.eps = items[i0 + j].noise_sigma;
    }
    void* d_jobs = nullptr;
    rc = upload(jobs.data(), sizeof(semd::CeemdanJob) * jobs.size(), stream, &d_jobs);
    if (rc) { (void)hipFreeAsync(arena, stream); return rc; }
    const auto* dj = static_cast<const semd::CeemdanJob*>(d_jobs);
    int64_t maxL = 0;
    for (int j = 0; j < nw; ++j) maxL = std::max(maxL, jobs[j].L);
    hipError_t e = hipSuccess;
    // r_0 = x, the serialized signal (Sec. 3.2)
    for (int j = 0; j < nw && e == hipSuccess; ++j)
      e = semd::launch_serialize(items[i0 + j].signal, shapes[i0 + j].M, shapes[i0 + j].N,
                                 p->transition_len, jobs[j].r, stream);
    if (e != hipSuccess) rc = hip_fail(e, "CEEMDAN serialize launch");
    // E_i(w_m): the full EMD of every noise realization
    if (rc == SEMD_OK) {
      std::vector<semd::WorkItem> work;
      for (int j = 0; j < nw; ++j) {
        const int64_t L = jobs[j].L;
        const Shape flat{L, 1, L};
        for (int m = 0; m < NR; ++m) {
          semd::WorkItem w = make_work(nullptr, E[j] + (size_t)m * (K + 1) * L, nullptr, flat, 0,
                                       sd);
          w.flags = semd::kNoSignal | semd::kAddNoise;
          w.beta = 1.0;
          w.key = semd::noise_key(p->seed, items[i0 + j].item_id, (uint64_t)m);
          work.push_back(w);
        }
      }
      rc = run_work(work, K, S, p->path, stream);
    }
    if (rc == SEMD_OK) {
      e = semd::launch_ceemdan_prep(dj, nw, K, stream);
      if (e != hipSuccess) rc = hip_fail(e, "CEEMDAN prep launch");
    }
    // stage i: the ensemble's first modes of r_{i-1} + beta_{i-1} noise_i,
    // noise_1 = w_m and noise_i = E_{i-1}(w_m), then their mean is mode i
    for (int stage = 1; stage <= K && rc == SEMD_OK; ++stage) {
      std::vector<semd::WorkItem> work;
      for (int j = 0; j < nw; ++j) {
        const int64_t L = jobs[j].L;
        const Shape flat{L, 1, L};
        for (int m = 0; m < NR; ++m) {
          semd::WorkItem w = make_work(jobs[j].r, const_cast<double*>(jobs[j].stage) +
                                                      (size_t)m * 2 * L,
                                       nullptr, flat, 0, sd);
          w.scale = &st[j].scale;
          if (stage == 1) {
            w.flags = semd::kAddNoise | semd::kScaleOnDevice;
            w.key = semd::noise_key(p->seed, items[i0 + j].item_id, (uint64_t)m);
          } else {
            w.flags = semd::kAddBuffer | semd::kScaleOnDevice;
            w.addend = E[j] + ((size_t)m * (K + 1) + (stage - 2)) * L;
          }
          work.push_back(w);
        }
      }
      rc = run_work(work, 1, S, p->path, stream);
      if (rc == SEMD_OK) {
        e = semd::launch_ceemdan_combine(dj, nw, maxL, stage, stream);
        if (e != hipSuccess) rc = hip_fail(e, "CEEMDAN combine launch");
      }
    }
    if (rc == SEMD_OK) {
      e = semd::launch_ceemdan_finish(dj, nw, K, stream);
      if (e != hipSuccess) rc = hip_fail(e, "CEEMDAN finish launch");
    }
    (void)hipFreeAsync(d_jobs, stream);
    (void)hipFreeAsync(arena, stream);
    if (rc) return rc;
    i0 = i1;
  }
  return SEMD_OK;
}

int semd_serialize(const double* X, const int64_t* dims, int ndim, int D, double* x,
                   hipStream_t stream) {
  g_err[0] = 0;
  if (!X || !x) return fail(SEMD_EINVAL, "NULL input or output");
  if (D < 0) return fail(SEMD_EINVAL, "D must be >= 0");
  Shape sh;
  int rc = shape_of(dims, ndim, D, &sh);
  if (rc) return rc;
  hipError_t e = semd::launch_serialize(X, sh.M, sh.N, D, x, stream);
  return e == hipSuccess ? SEMD_OK : hip_fail(e, "serialize launch");
}

int semd_deserialize(const double* y, const int64_t* dims, int ndim, int D, double* out,
                     hipStream_t stream) {
  g_err[0] = 0;
  if (!y || !out) return fail(SEMD_EINVAL, "NULL input or output");
  if (D < 0) return fail(SEMD_EINVAL, "D must be >= 0");
  Shape sh;
  int rc = shape_of(dims, ndim, D, &sh);
  if (rc) return rc;
  hipError_t e = semd::launch_deserialize(y, sh.M, sh.N, D, out, stream);
  return e == hipSuccess ? SEMD_OK : hip_fail(e, "deserialize launch");
}

int semd_extrema(const double* h, int64_t L, int32_t* imax, int32_t* imin, int32_t* counts,
                 hipStream_t stream) {
  g_err[0] = 0;
  if (!h || !imax || !imin || !counts) return fail(SEMD_EINVAL, "NULL pointer");
  if (L < 3 || L > semd::kResidentMaxL)
    return fail(SEMD_EINVAL, "L must be in [3, %d]", semd::kResidentMaxL);
  hipError_t e = semd::launch_extrema(h, (int)L, imax, imin, counts, stream);
  return e == hipSuccess ? SEMD_OK : hip_fail(e, "extrema launch");
}

int semd_noise(uint64_t seed, uint64_t item, uint64_t m, int64_t L, double* w,
               hipStream_t stream) {
  g_err[0] = 0;
  if (!w) return fail(SEMD_EINVAL, "NULL output");
  if (L < 0) return fail(SEMD_EINVAL, "L must be >= 0");
  if (L == 0) return SEMD_OK;
  hipError_t e = semd::launch_noise(semd::noise_key(seed, item, m), L, w, stream);
  return e == hipSuccess ? SEMD_OK : hip_fail(e, "noise launch");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Serving engine: continuous batching over the streaming kernels
// ---------------------------------------------------------------------------

#include <map>

struct semd_engine {
  struct Req {
    int64_t ticket;
    bool onchip;           // decomposed whole by one on-chip launch
    semd::StreamSig sig;   // streaming requests
    semd::WorkItem work;   // on-chip requests (workspace in the arena)
    int K, S;
    size_t off, bytes;
    bool loaded;           // streaming: h, r loaded; on-chip: launched
  };
  size_t budget = 0;
  int max_requests = 0;
  unsigned char* arena = nullptr;
  std::map<size_t, size_t> free_;  // offset -> bytes of free arena ranges
  std::vector<Req> reqs;           // resident requests, in table order
  bool dirty = true;               // tables differ from the requests
  void* d_tables = nullptr;        // current device tables (signals, tiles, blocks)
  int n_tiles = 0, n_blocks = 0, max_steps = 0;
  size_t o_til = 0, o_blk = 0;
  int32_t* d_done = nullptr;       // done flags of the last gathered step
  int32_t* h_done = nullptr;       // pinned copy
  int done_cap = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;            // a gather awaits processing
  std::vector<int64_t> pending_tickets;  // table order of that gather
  std::vector<int64_t> pending_onchip;   // on-chip requests launched in that step
  std::vector<int64_t> finished;   // tickets ready for poll
  int64_t next_ticket = 1;
  hipStream_t last_stream = nullptr;
  StepGraph graph;                 // the step on the current tables
  bool graph_ok = false;

  int alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return 0;
      }
    }
    return -1;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  void retire(int64_t t) {
    for (size_t j = 0; j < reqs.size(); ++j) {
      if (reqs[j].ticket == t) {
        release(reqs[j].off, reqs[j].bytes);
        if (!reqs[j].onchip) dirty = true;  // the streaming tables change
        reqs.erase(reqs.begin() + (ptrdiff_t)j);
        finished.push_back(t);
        break;
      }
    }
  }
  // Requests whose done flag was set in the last gathered step leave, and
  // the on-chip requests launched in that step (complete with it).
  void process_gather() {
    if (!pending) return;
    pending = false;
    for (size_t i = 0; i < pending_tickets.size(); ++i)
      if (h_done[i]) retire(pending_tickets[i]);
    for (const int64_t t : pending_onchip) retire(t);
    pending_onchip.clear();
  }
};

namespace {

std::mutex g_engine_mu;

int engine_check(const semd_item* it, const semd_params* p, Shape* sh) {
  int rc = check_params(p, false);
  if (rc) return rc;
  if (!it) return fail(SEMD_EINVAL, "item is NULL");
  std::vector<Shape> shapes;
  rc = check_items(it, 1, p->transition_len, p->path, shapes);
  if (rc) return rc;
  *sh = shapes[0];
  return SEMD_OK;
}

// Route of an engine request: on chip (whole decomposition in one launch)
// as semd_decompose_ex would route it, else streaming.
bool engine_onchip(const Shape& sh, const semd_params* p) {
  return p->path == SEMD_PATH_ONCHIP ||
         (p->path == SEMD_PATH_AUTO && sh.L <= semd::kResidentMaxL);
}

size_t engine_bytes(const Shape& sh, const semd_params* p) {
  if (engine_onchip(sh, p))
    return al256(sizeof(double) * (size_t)semd::resident_ws_doubles(sh.L));
  return al256(stream_bytes(sh.L));
}

// One on-chip launch per (K, S, launch shape) over a cohort of whole
// decompositions whose workspaces are set; shapes as for a single signal
// (semd_decompose_ex), so every result is bit-identical to its own call.
int launch_cohort(std::vector<semd_engine::Req*>& cohort, hipStream_t stream) {
  std::stable_sort(cohort.begin(), cohort.end(), [](const semd_engine::Req* a,
                                                    const semd_engine::Req* b) {
    if (a->K != b->K) return a->K < b->K;
    if (a->S != b->S) return a->S < b->S;
    return a->work.L > b->work.L;
  });
  std::vector<semd::WorkItem> items(cohort.size());
  for (size_t i = 0; i < cohort.size(); ++i) items[i] = cohort[i]->work;
  void* d = nullptr;
  int rc = upload(items.data(), items.size() * sizeof(semd::WorkItem), stream, &d);
  if (rc) return rc;
  auto same = [](const semd::ResidentClass& a, const semd::ResidentClass& b) {
    return a.nt == b.nt && a.c == b.c;
  };
  size_t i0 = 0;
  while (i0 < cohort.size() && rc == SEMD_OK) {
    const int K = cohort[i0]->K, S = cohort[i0]->S;
    const semd::ResidentClass cls = class_for(items[i0].L, 0);
    size_t i1 = i0;
    while (i1 < cohort.size() && cohort[i1]->K == K && cohort[i1]->S == S &&
           same(class_for(items[i1].L, 0), cls))
      ++i1;
    const hipError_t e = semd::launch_resident(static_cast<const semd::WorkItem*>(d) + i0,
                                               (int)(i1 - i0), items[i0].L, cls, K, S, stream);
    if (e != hipSuccess) rc = hip_fail(e, "engine on-chip launch");
    i0 = i1;
  }
  (void)hipFreeAsync(d, stream);
  return rc;
}

}  // namespace

extern "C" {

int semd_engine_create(size_t hbm_budget_bytes, int max_requests, semd_engine** out) {
  g_err[0] = 0;
  if (!out) return fail(SEMD_EINVAL, "out is NULL");
  if (max_requests < 1) return fail(SEMD_EINVAL, "max_requests must be >= 1");
  if (hbm_budget_bytes < (size_t(1) << 20)) return fail(SEMD_EINVAL, "budget below 1 MiB");
  auto* e = new semd_engine();
  e->budget = hbm_budget_bytes & ~size_t(255);
  e->max_requests = max_requests;
  if (hipMalloc(reinterpret_cast<void**>(&e->arena), e->budget) != hipSuccess) {
    delete e;
    return fail(SEMD_ENOMEM, "engine arena of %zu bytes", hbm_budget_bytes);
  }
  e->free_[0] = e->budget;
  e->done_cap = max_requests;
  if (hipMalloc(reinterpret_cast<void**>(&e->d_done), sizeof(int32_t) * max_requests) !=
          hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&e->h_done), sizeof(int32_t) * max_requests,
                    hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&e->ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipFree(e->arena);
    if (e->d_done) (void)hipFree(e->d_done);
    if (e->h_done) (void)hipHostFree(e->h_done);
    delete e;
    return fail(SEMD_ENOMEM, "engine flag buffers");
  }
  *out = e;
  return SEMD_OK;
}

int semd_engine_footprint(const semd_item* item, const semd_params* p, size_t* bytes) {
  g_err[0] = 0;
  if (!bytes) return fail(SEMD_EINVAL, "bytes is NULL");
  Shape sh;
  const int rc = engine_check(item, p, &sh);
  if (rc) return rc;
  *bytes = engine_bytes(sh, p);
  return SEMD_OK;
}

int semd_engine_admit(semd_engine* e, const semd_item* item, const semd_params* p,
                      int64_t* ticket) {
  g_err[0] = 0;
  if (!e || !ticket) return fail(SEMD_EINVAL, "NULL engine or ticket");
  std::lock_guard<std::mutex> lock(g_engine_mu);
  Shape sh;
  int rc = engine_check(item, p, &sh);
  if (rc) return rc;
  if ((int)e->reqs.size() >= e->max_requests)
    return fail(SEMD_EBUSY, "all %d request slots are taken", e->max_requests);
  const size_t bytes = engine_bytes(sh, p);
  if (bytes > e->budget)
    return fail(SEMD_ENOMEM, "request needs %zu bytes, more than the whole engine budget %zu",
                bytes, e->budget);
  size_t off = 0;
  if (e->alloc(bytes, &off))
    return fail(SEMD_EBUSY, "request needs %zu bytes, not free in the engine budget", bytes);
  semd::WorkItem w = make_work(item->signal, item->imfs_out, item->n_imfs_out, sh,
                               p->transition_len, sd_of(p), item->stats_out);
  semd_engine::Req r{};
  r.ticket = e->next_ticket++;
  r.onchip = engine_onchip(sh, p);
  r.K = p->max_imfs;
  r.S = p->sift_iters;
  if (r.onchip) {
    w.r = reinterpret_cast<double*>(e->arena + off);
    w.u = w.r + w.L;
    r.work = w;
  } else {
    r.sig = stream_sig(w, p->max_imfs, p->sift_iters, e->arena + off);
    e->dirty = true;
  }
  r.off = off;
  r.bytes = bytes;
  r.loaded = false;
  e->reqs.push_back(r);
  *ticket = r.ticket;
  return SEMD_OK;
}

int semd_engine_step(semd_engine* e, hipStream_t stream) {
  return semd_engine_step_n(e, 1, stream);
}

int semd_engine_step_n(semd_engine* e, int n_steps, hipStream_t stream) {
  g_err[0] = 0;
  if (!e) return fail(SEMD_EINVAL, "engine is NULL");
  if (n_steps < 1 || n_steps > SEMD_ENGINE_MAX_STEPS)
    return fail(SEMD_EINVAL, "n_steps %d outside [1, %d]", n_steps, SEMD_ENGINE_MAX_STEPS);
  std::lock_guard<std::mutex> lock(g_engine_mu);
  e->last_stream = stream;
  // on-chip requests admitted since the last step: whole decompositions,
  // launched together; they complete with this step
  std::vector<semd_engine::Req*> cohort;
  std::vector<int64_t> cohort_tickets;
  for (auto& r : e->reqs) {
    if (r.onchip && !r.loaded) {
      r.loaded = true;
      cohort.push_back(&r);
      cohort_tickets.push_back(r.ticket);
    }
  }
  if (!cohort.empty()) {
    const int rc = launch_cohort(cohort, stream);
    if (rc) return rc;
  }
  // streaming requests: one step each
  std::vector<semd_engine::Req*> sreqs;
  for (auto& r : e->reqs)
    if (!r.onchip) sreqs.push_back(&r);
  const int n = (int)sreqs.size();
  hipError_t he = hipSuccess;
  std::vector<int64_t> table_tickets;
  if (n > 0) {
    if (e->dirty) {
      std::vector<semd::StreamSig> sigs(n);
      std::vector<int2> new_tiles;
      for (int i = 0; i < n; ++i) {
        sigs[i] = sreqs[i]->sig;
        if (!sreqs[i]->loaded)
          for (int t = 0; t < sigs[i].ntiles; ++t) new_tiles.push_back(make_int2(i, t));
      }
      std::vector<int2> tiles;
      std::vector<int4> blocks;
      stream_tables(sigs, tiles, blocks);
      // new requests' tiles ride along after the blocks
      const size_t b_new = sizeof(int2) * new_tiles.size();
      size_t o_til, o_blk;
      std::vector<unsigned char> pack = pack_tables(sigs, tiles, blocks, &o_til, &o_blk);
      const size_t o_new = pack.size();
      pack.resize(o_new + std::max<size_t>(b_new, 8));
      std::memcpy(pack.data() + o_new, new_tiles.data(), b_new);
      void* d = nullptr;
      int rc = upload(pack.data(), pack.size(), stream, &d);
      if (rc) return rc;
      if (e->d_tables) (void)hipFreeAsync(e->d_tables, stream);
      e->d_tables = d;
      e->o_til = o_til;
      e->o_blk = o_blk;
      e->n_tiles = (int)tiles.size();
      e->n_blocks = (int)blocks.size();
      unsigned char* dp = static_cast<unsigned char*>(d);
      he = semd::st_load(reinterpret_cast<const semd::StreamSig*>(dp),
                         reinterpret_cast<const int2*>(dp + o_new), (int)new_tiles.size(), stream);
      for (auto* r : sreqs) r->loaded = true;
      e->dirty = false;
      e->graph_ok = false;
    }
    // ticket order of the table this step runs on (retirements below change
    // e->reqs, not the table)
    table_tickets.resize(n);
    for (int i = 0; i < n; ++i) table_tickets[i] = sreqs[i]->ticket;
    unsigned char* dp = static_cast<unsigned char*>(e->d_tables);
    const auto* d_sigs = reinterpret_cast<const semd::StreamSig*>(dp);
    // one sift of every resident request and the gather of their done
    // flags, captured once per table version and replayed every step
    sweep_retired_graphs();
    CaptureStream cs;
    if (he == hipSuccess) he = cs.open(stream);
    if (he == hipSuccess && !e->graph_ok) {
      const int nt = e->n_tiles, nb = e->n_blocks;
      int32_t* d_done = e->d_done;
      bool any_sd = false;
      for (const auto* r : sreqs) any_sd |= r->sig.sd > 0.0;
      he = e->graph.capture(cs.s, [&](hipStream_t s) {
        hipError_t le = semd::st_step(d_sigs, n, reinterpret_cast<const int2*>(dp + e->o_til),
                                      nt, reinterpret_cast<const int4*>(dp + e->o_blk), nb, s,
                                      any_sd);
        if (le == hipSuccess) le = semd::st_gather_done(d_sigs, n, d_done, s);
        return le;
      });
      e->graph_ok = he == hipSuccess;
    }
    // (a request that finishes within the replays idles through the rest:
    // every kernel returns at once on a finished signal)
    for (int k = 0; k < n_steps && he == hipSuccess; ++k) he = e->graph.launch(cs.s);
    if (he == hipSuccess) he = cs.join();
  }
  if (he != hipSuccess) return hip_fail(he, "engine step");
  // the previous step's flags: requests that finished then leave now
  if (e->pending) {
    if (hipEventSynchronize(e->ev) != hipSuccess) return fail(SEMD_EDEVICE, "event wait");
    e->process_gather();
  }
  if (n > 0 || !cohort_tickets.empty()) {
    if (n > 0)
      he = hipMemcpyAsync(e->h_done, e->d_done, sizeof(int32_t) * n, hipMemcpyDeviceToHost,
                          stream);
    if (he == hipSuccess) he = hipEventRecord(e->ev, stream);
    if (he == hipSuccess) {
      e->pending = true;
      e->pending_tickets = std::move(table_tickets);
      e->pending_onchip = std::move(cohort_tickets);
    }
  }
  if (he != hipSuccess) return hip_fail(he, "engine step");
  return SEMD_OK;
}

int semd_engine_poll(semd_engine* e, int64_t* done, int cap, int* n_done) {
  g_err[0] = 0;
  if (!e || !n_done || (cap > 0 && !done)) return fail(SEMD_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lock(g_engine_mu);
  if (e->pending && hipEventQuery(e->ev) == hipSuccess) e->process_gather();
  const int k = std::min<int>(cap, (int)e->finished.size());
  for (int i = 0; i < k; ++i) done[i] = e->finished[i];
  e->finished.erase(e->finished.begin(), e->finished.begin() + k);
  *n_done = k;
  return SEMD_OK;
}

int semd_engine_resident(semd_engine* e, int* n) {
  g_err[0] = 0;
  if (!e || !n) return fail(SEMD_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lock(g_engine_mu);
  *n = (int)e->reqs.size();
  return SEMD_OK;
}

int semd_engine_destroy(semd_engine* e) {
  g_err[0] = 0;
  if (!e) return SEMD_OK;
  std::lock_guard<std::mutex> lock(g_engine_mu);
  if (e->last_stream) {
    if (e->d_tables) (void)hipFreeAsync(e->d_tables, e->last_stream);
    (void)hipStreamSynchronize(e->last_stream);
  }
  (void)hipDeviceSynchronize();
  e->graph.retire(nullptr);
  sweep_retired_graphs();
  (void)hipFree(e->arena);
  (void)hipFree(e->d_done);
  (void)hipHostFree(e->h_done);
  (void)hipEventDestroy(e->ev);
  delete e;
  return SEMD_OK;
}

}  // extern "C"
