// Host side of the wkern C ABI: validation, geometry, plane ordering, tile
// schedule, device tables and the generate / grad entry points.
// The method and the data layout are described in include/wkern.h.
#include "wkern.h"

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "wkern_internal.h"

namespace {
// A roctx range over a scope (the entry points and, on the host side, the
// enqueueing of each stage): visible to rocprofv3 --marker-trace, no cost
// without a tool attached.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};
}  // namespace

using namespace wkern;

namespace {

thread_local std::string g_last_error;

void clear_error() { g_last_error.clear(); }

wkern_status fail(wkern_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  if (log_level() >= 2) fprintf(stderr, "wkern: error %d: %s\n", (int)s, buf);
  return s;
}

wkern_status hip_fail(hipError_t e, const char* what) {
  const wkern_status s =
      (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? WKERN_ERR_OUT_OF_MEMORY
                                                                  : WKERN_ERR_DEVICE;
  return fail(s, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

#define WK_HIP(call, what)                 \
  do {                                     \
    hipError_t e_ = (call);                \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// A kernel launch (through a launch_* helper); subject to WKERN_FAULT=launch.
#define WK_LAUNCH(call, what)                                                      \
  do {                                                                             \
    if (fault_hit("launch"))                                                       \
      return fail(WKERN_ERR_DEVICE, "%s: injected launch failure (WKERN_FAULT)", what); \
    WK_HIP(call, what);                                                            \
  } while (0)

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// The integer a C caller stored in an enum-typed field or argument.  C
// allows any int there, but C++ may not load a value outside the
// enumeration's range as the enum type, so the bits are read as an integer.
template <class E>
int32_t enum_bits(const E& e) {
  static_assert(sizeof(E) == sizeof(int32_t), "enum fields are 32-bit in this ABI");
  int32_t v;
  std::memcpy(&v, &e, sizeof v);
  return v;
}

// Validation shared by wkern_layout_desc and wkern_plan.
wkern_status validate(const wkern_desc* d) {
  if (!d) return fail(WKERN_ERR_INVALID_ARG, "desc is NULL");
  if (d->abi_version != WKERN_ABI_VERSION)
    return fail(WKERN_ERR_ABI_MISMATCH, "desc.abi_version %d, library %d", d->abi_version,
                WKERN_ABI_VERSION);
  if (d->image_size < 1) return fail(WKERN_ERR_INVALID_ARG, "image_size %d < 1", d->image_size);
  if (!(d->cellsize > 0.0) || !std::isfinite(d->cellsize))
    return fail(WKERN_ERR_INVALID_ARG, "cellsize must be finite and > 0");
  const double r_max = 0.5 * d->image_size * d->cellsize;
  if (!(r_max < 1.0)) return fail(WKERN_ERR_INVALID_ARG, "r_max = %g must be < 1", r_max);
  if (d->n_radial < 1 || d->n_radial > (1 << 20))
    return fail(WKERN_ERR_INVALID_ARG, "n_radial %d outside [1, 2^20]", d->n_radial);
  if (d->oversampling < 1 || d->oversampling > 64)
    return fail(WKERN_ERR_INVALID_ARG, "oversampling %d outside [1, 64]", d->oversampling);
  if (d->radial_refine < 1 || d->radial_refine > 16)
    return fail(WKERN_ERR_INVALID_ARG, "radial_refine %d outside [1, 16]", d->radial_refine);
  if (d->n_planes < 1 || d->n_planes > 65535)
    return fail(WKERN_ERR_INVALID_ARG, "n_planes %d outside [1, 65535]", d->n_planes);
  if (!d->support) return fail(WKERN_ERR_INVALID_ARG, "support is NULL");
  if (d->max_support < 1 || (d->max_support % 2) == 0)
    return fail(WKERN_ERR_INVALID_ARG, "max_support %d must be odd and >= 1", d->max_support);
  if ((int64_t)d->oversampling * d->max_support > 4096)
    return fail(WKERN_ERR_INVALID_ARG, "oversampling * max_support = %lld > 4096",
                (long long)d->oversampling * d->max_support);
  const int64_t nrho_max =
      (int64_t)d->radial_refine * d->oversampling * ((d->max_support - 1) / 2) + 4;
  if (nrho_max > kMaxRho)
    return fail(WKERN_ERR_INVALID_ARG, "radial line of %lld nodes exceeds %d",
                (long long)nrho_max, kMaxRho);
  const int32_t prec = enum_bits(d->precision), interp = enum_bits(d->interp);
  if (prec != WKERN_PREC_FP32 && prec != WKERN_PREC_BF16X6)
    return fail(WKERN_ERR_INVALID_ARG, "unknown precision %d", prec);
  if (interp != WKERN_INTERP_LINEAR && interp != WKERN_INTERP_CUBIC)
    return fail(WKERN_ERR_INVALID_ARG, "unknown interp %d", interp);
  for (int p = 0; p < d->n_planes; ++p) {
    const int s = d->support[p];
    if (s < 1 || (s % 2) == 0 || s > d->max_support)
      return fail(WKERN_ERR_INVALID_ARG, "support[%d] = %d must be odd in [1, %d]", p, s,
                  d->max_support);
  }
  if (d->mirror) {
    for (int p = 0; p < d->n_planes; ++p) {
      const int q = d->mirror[p];
      if (q == -1) continue;
      if (q < 0 || q >= d->n_planes || q == p)
        return fail(WKERN_ERR_INVALID_ARG, "mirror[%d] = %d is not -1 or another plane", p, q);
      if (d->mirror[q] != -1)
        return fail(WKERN_ERR_INVALID_ARG, "mirror[%d] = %d names a mirrored plane", p, q);
      if (d->support[q] != d->support[p])
        return fail(WKERN_ERR_INVALID_ARG, "mirror[%d] = %d: supports %d and %d differ", p, q,
                    d->support[p], d->support[q]);
    }
  }
  return WKERN_OK;
}

int32_t nrho_of(const wkern_desc* d, int s) {
  return d->radial_refine * d->oversampling * ((s - 1) / 2) + 4;
}

void layout_host(const wkern_desc* d, int64_t* offsets, int32_t* nrho) {
  int64_t acc = 0;
  const int64_t os2 = (int64_t)d->oversampling * d->oversampling;
  for (int p = 0; p < d->n_planes; ++p) {
    offsets[p] = acc;
    acc += os2 * d->support[p] * d->support[p];
    if (nrho) nrho[p] = nrho_of(d, d->support[p]);
  }
  offsets[d->n_planes] = acc;
}

// Restores the calling thread's current HIP device on scope exit.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

void wkern::set_last_error(const char* msg) { g_last_error = msg ? msg : ""; }

bool wkern::fault_hit(const char* site) {
  static std::mutex mu;
  static std::string armed;  // the WKERN_FAULT value the counter belongs to
  static int count = 0;
  const char* env = std::getenv("WKERN_FAULT");
  std::lock_guard<std::mutex> lock(mu);
  if (!env || !*env) {
    armed.clear();
    return false;
  }
  if (armed != env) {
    armed = env;
    count = 0;
  }
  const char* colon = std::strchr(env, ':');
  const size_t len = colon ? (size_t)(colon - env) : std::strlen(env);
  if (len != std::strlen(site) || std::strncmp(env, site, len) != 0) return false;
  const int nth = colon ? std::atoi(colon + 1) : 1;
  return ++count == nth;
}

int wkern::log_level() {
  const char* env = std::getenv("WKERN_LOG");
  return env ? std::atoi(env) : 0;
}

// One profiled launch: stage index and the events around it.
struct StageRecord {
  int stage;
  hipEvent_t start;
  hipEvent_t end;
};

struct wkern_plan_s {
  wkern_desc desc{};
  std::vector<int32_t> support;
  std::vector<int64_t> offsets;       // [P + 1]
  std::vector<int32_t> nrho;          // [P] caller order
  std::vector<int32_t> lineOffCaller; // [Pall + 1]
  std::vector<int32_t> mirror;        // [Pall] -1 or the source plane
  std::vector<int32_t> nrhoSorted;    // [P] computed planes, longest first
  std::vector<int32_t> perm;          // [P] sorted j -> caller p
  std::vector<int32_t> mirStart;      // [P + 1]
  std::vector<int32_t> mirList;       // mirrored planes grouped by source
  DevPlan dp{};
  // Every device allocation of the plan.  With canaries on (WKERN_CANARY at
  // plan creation) each one carries a guard band of kGuardBytes of
  // kGuardByte on both sides, checked by wkern_sync_status.
  struct Allocation {
    void* user;
    void* raw;
    size_t bytes;
    const char* what;
  };
  std::vector<Allocation> allocations;
  bool canary = false;
  static constexpr size_t kGuardBytes = 1024;
  static constexpr unsigned char kGuardByte = 0xA5;

  // pipeline chunks over the sorted planes
  int nChunks = 1;
  std::vector<int> chunkJ;   // [C + 1] sorted-plane boundaries
  std::vector<int> chunkU;   // [C + 1] resample-unit boundaries
  // contraction tile lists, one per variant, ordered by chunk
  Tile* d_tiles[kNumVariants] = {};
  std::vector<int> chunkT[kNumVariants];  // [C + 1] tile boundaries
  int variant = kWave32x64;
  float variantMs[kNumVariants] = {};
  bool tunedFromCache = false;
  // internal streams (default priority): sCompute is the capture stream of
  // the generation graph, sStore runs the resamples of a chunked pipeline
  hipStream_t sCompute = nullptr, sStore = nullptr;
  hipEvent_t evFork = nullptr, evJoinStore = nullptr;
  std::vector<hipEvent_t> evChunk;  // [C] compute of chunk c finished

  // captured generation graph, keyed by the caller's pointers
  bool useGraph = true;
  hipGraphExec_t graphExec = nullptr;
  const void* graphKey[3] = {nullptr, nullptr, nullptr};
  bool graphValid = false;

  // truncated generation scratch, allocated on its first call
  TruncScratch trunc{};
  bool truncReady = false;
  std::vector<int32_t> sortedPosOfCaller;  // [Pall] sorted index of the plane's source

  // adjoint scratch, allocated on the first wkern_grad call
  GradScratch grad{};
  bool gradReady = false;

  // gridding work-item table, allocated on the first wkern_grid call
  int32_t* gridChunks = nullptr;

  // radial-line engine: 0 matrix form (HT matrix on the matrix cores),
  // 1 projection-slice; the latter writes one K-chunk, so its spline and
  // line views carry nkc = 1
  int engine = WKERN_ENGINE_MATRIX;
  int psMode = 0;
  PsTables ps{};

  // stage profiling
  bool profiling = false;
  int profiledCalls = 0;
  std::vector<StageRecord> records;
  size_t recordsUsed = 0;

  ~wkern_plan_s() {
    for (auto& r : records) {
      (void)hipEventDestroy(r.start);
      (void)hipEventDestroy(r.end);
    }
    if (graphExec) (void)hipGraphExecDestroy(graphExec);
    for (hipEvent_t e : evChunk) (void)hipEventDestroy(e);
    if (evFork) (void)hipEventDestroy(evFork);
    if (evJoinStore) (void)hipEventDestroy(evJoinStore);
    if (sCompute) (void)hipStreamDestroy(sCompute);
    if (sStore) (void)hipStreamDestroy(sStore);
    for (const Allocation& a : allocations) (void)hipFree(a.raw);
  }

  template <class T>
  wkern_status alloc(T** ptr, size_t count, const char* what) {
    void* raw = nullptr;
    const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
    if (fault_hit("alloc")) {
      *ptr = nullptr;
      return fail(WKERN_ERR_OUT_OF_MEMORY, "%s: injected allocation failure (WKERN_FAULT)", what);
    }
    const size_t guard = canary ? kGuardBytes : 0;
    hipError_t e = hipMalloc(&raw, bytes + 2 * guard);
    if (e != hipSuccess) {
      *ptr = nullptr;
      return hip_fail(e, what);
    }
    if (guard) {
      // the whole block, so the guards hold the pattern before any kernel runs
      e = hipMemset(raw, kGuardByte, bytes + 2 * guard);
      if (e != hipSuccess) {
        (void)hipFree(raw);
        *ptr = nullptr;
        return hip_fail(e, "canary fill");
      }
    }
    void* user = (unsigned char*)raw + guard;
    allocations.push_back({user, raw, bytes, what});
    *ptr = (T*)user;
    return WKERN_OK;
  }

  template <class T>
  void release(T*& ptr) {
    if (!ptr) return;
    auto it = std::find_if(allocations.begin(), allocations.end(),
                           [&](const Allocation& a) { return a.user == (void*)ptr; });
    if (it != allocations.end()) {
      (void)hipFree(it->raw);
      allocations.erase(it);
    }
    ptr = nullptr;
  }

  template <class T>
  wkern_status upload(T** ptr, const std::vector<T>& host, const char* what) {
    wkern_status s = alloc(ptr, host.size(), what);
    if (s != WKERN_OK) return s;
    WK_HIP(hipMemcpy(*ptr, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice), what);
    return WKERN_OK;
  }

  // Event pair for one profiled launch (pooled across calls).
  wkern_status record_begin(int stage, hipStream_t st, StageRecord** rec) {
    *rec = nullptr;
    if (!profiling) return WKERN_OK;
    if (recordsUsed == records.size()) {
      StageRecord r{stage, nullptr, nullptr};
      WK_HIP(hipEventCreate(&r.start), "hipEventCreate");
      WK_HIP(hipEventCreate(&r.end), "hipEventCreate");
      records.push_back(r);
    }
    StageRecord* r = &records[recordsUsed++];
    r->stage = stage;
    WK_HIP(hipEventRecord(r->start, st), "hipEventRecord");
    *rec = r;
    return WKERN_OK;
  }
};

namespace {

wkern_status record_end(StageRecord* r, hipStream_t st) {
  if (r) WK_HIP(hipEventRecord(r->end, st), "hipEventRecord");
  return WKERN_OK;
}

// Tiles of one contraction variant over sorted planes [j0, j1): column
// blocks of the variant's width start at the chunk's first plane (the last
// block of a chunk stops at j1: tiles carry the chunk end and never store
// columns beyond it), row tiles of 32 * rb cover the block's longest line.
// Tiles that read the same screen columns over the same K-chunk form a
// group; a group is pinned to one XCD (workgroup i runs on XCD i % 8) and its
// tiles are dispatched back to back there, so the group's slice of the
// screen is read from HBM once and then served by that XCD's L2.
void build_tiles(int variant, int j0, int j1, const std::vector<int32_t>& nrhoSorted, int nkc,
                 int kchunk, std::vector<Tile>& out) {
  const ContractShape sh = contract_shape(variant);
  const int rowTile = 32 * sh.rb;
  std::vector<std::vector<Tile>> xcdQueue(kNumXcd);
  int group = 0;
  for (int c0 = 2 * j0; c0 < 2 * j1; c0 += sh.cols) {
    const int rows = nrhoSorted[c0 / 2];
    for (int kc = 0; kc < nkc; ++kc, ++group) {
      std::vector<Tile>& q = xcdQueue[group % kNumXcd];
      for (int r0 = 0; r0 < rows; r0 += rowTile) {
        const int rbN = std::min(sh.rb, (rows - r0 + 31) / 32);
        q.push_back(Tile{r0, c0, kc * kchunk, kc, rbN, {j1, 0, 0}});
      }
    }
  }
  size_t longest = 0;
  for (auto& q : xcdQueue) longest = std::max(longest, q.size());
  // interleave the per-XCD queues; short queues are padded with no-op
  // entries (row0 = -1)
  for (size_t m = 0; m < longest; ++m)
    for (int x = 0; x < kNumXcd; ++x)
      out.push_back(m < xcdQueue[x].size() ? xcdQueue[x][m]
                                           : Tile{-1, 0, 0, 0, 0, {0, 0, 0}});
}

// Pipeline chunks: consecutive runs of sorted planes with about equal cache
// bytes each (the resample of chunk c overlaps the screen, contraction and
// spline of chunk c + 1).
std::vector<int> make_chunks(const std::vector<int64_t>& bytesSorted, int want) {
  const int P = (int)bytesSorted.size();
  int64_t total = 0;
  for (int64_t b : bytesSorted) total += b;
  want = std::max(1, std::min(want, P));
  std::vector<int> cuts{0};
  int64_t acc = 0;
  for (int j = 0; j < P; ++j) {
    acc += bytesSorted[j];
    const int made = (int)cuts.size();
    if (made < want && acc * want >= total * made && j + 1 < P) cuts.push_back(j + 1);
  }
  cuts.push_back(P);
  return cuts;
}

}  // namespace

extern "C" {

int32_t wkern_abi_version(void) { return WKERN_ABI_VERSION; }

const char* wkern_strerror(wkern_status s) {
  switch (enum_bits(s)) {
    case WKERN_OK: return "success";
    case WKERN_ERR_INVALID_ARG: return "invalid argument";
    case WKERN_ERR_OUT_OF_MEMORY: return "out of memory";
    case WKERN_ERR_DEVICE: return "device or HIP runtime error";
    case WKERN_ERR_UNSUPPORTED: return "unsupported";
    case WKERN_ERR_ABI_MISMATCH: return "ABI version mismatch";
    case WKERN_ERR_NONFINITE: return "non-finite value in the generated kernels";
  }
  return "unknown status";
}

const char* wkern_last_error(void) { return g_last_error.c_str(); }

wkern_status wkern_layout_desc(const wkern_desc* d, int64_t* offsets, int32_t* nrho) {
  clear_error();
  wkern_status s = validate(d);
  if (s != WKERN_OK) return s;
  if (!offsets) return fail(WKERN_ERR_INVALID_ARG, "offsets is NULL");
  layout_host(d, offsets, nrho);
  return WKERN_OK;
}

wkern_status wkern_layout(wkern_plan_t plan, int64_t* offsets, int32_t* nrho) {
  clear_error();
  if (!plan) return fail(WKERN_ERR_INVALID_ARG, "plan is NULL");
  if (!offsets) return fail(WKERN_ERR_INVALID_ARG, "offsets is NULL");
  std::copy(plan->offsets.begin(), plan->offsets.end(), offsets);
  if (nrho) std::copy(plan->nrho.begin(), plan->nrho.end(), nrho);
  return WKERN_OK;
}

// Pipeline chunks, resample units and contraction tile lists for `want`
// chunks (rebuilt by wkern_set_chunks).
static wkern_status build_chunks(wkern_plan_s* pl, int want) {
  DevPlan& g = pl->dp;
  const int P = g.P;
  const std::vector<int32_t>& perm = pl->perm;
  // planes written by sorted plane j: itself and its mirrors
  auto written = [&](int j, std::vector<int>& out) {
    out.assign(1, perm[j]);
    for (int m = pl->mirStart[j]; m < pl->mirStart[j + 1]; ++m) out.push_back(pl->mirList[m]);
  };
  std::vector<int> wr;
  std::vector<int64_t> bytesSorted(P);
  for (int j = 0; j < P; ++j) {
    written(j, wr);
    bytesSorted[j] = 0;
    for (int p : wr) bytesSorted[j] += pl->offsets[p + 1] - pl->offsets[p];
  }
  pl->chunkJ = make_chunks(bytesSorted, want);
  pl->nChunks = (int)pl->chunkJ.size() - 1;

  // resample units: blocks of at most kUnitElems elements of one plane (a
  // multiple of 1024, so every wave chunk starts at a multiple of its size),
  // in chunk order
  const int64_t unitElems = kUnitElems;
  std::vector<ResampleUnit> units;
  pl->chunkU.assign(1, 0);
  for (int c = 0; c < pl->nChunks; ++c) {
    // the planes of a chunk in output address order: the cache is then
    // written front to back (measured 3% faster than in sorted-plane order)
    std::vector<int> ps;
    for (int j = pl->chunkJ[c]; j < pl->chunkJ[c + 1]; ++j) {
      written(j, wr);
      ps.insert(ps.end(), wr.begin(), wr.end());
    }
    std::sort(ps.begin(), ps.end());
    for (int p : ps) {
      const int64_t n = pl->offsets[p + 1] - pl->offsets[p];
      for (int64_t e0 = 0; e0 < n; e0 += unitElems)
        units.push_back(ResampleUnit{p, (int32_t)e0, (int32_t)std::min(n, e0 + unitElems), 0});
    }
    pl->chunkU.push_back((int)units.size());
  }
  g.nUnits = (int)units.size();
  wkern_status s;
  pl->release(g.units);
  if ((s = pl->upload(&g.units, units, "units")) != WKERN_OK) return s;

  for (int v = 0; v < kNumVariants; ++v) {
    std::vector<Tile> tiles;
    pl->chunkT[v].assign(1, 0);
    for (int c = 0; c < pl->nChunks; ++c) {
      build_tiles(v, pl->chunkJ[c], pl->chunkJ[c + 1], pl->nrhoSorted, g.nkc, g.kchunk, tiles);
      pl->chunkT[v].push_back((int)tiles.size());
    }
    pl->release(pl->d_tiles[v]);
    if ((s = pl->upload(&pl->d_tiles[v], tiles, "tiles")) != WKERN_OK) return s;
  }
  for (hipEvent_t e : pl->evChunk) (void)hipEventDestroy(e);
  pl->evChunk.assign(pl->nChunks, nullptr);
  for (auto& e : pl->evChunk)
    WK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
  return WKERN_OK;
}

// Persistent autotuner results.  WKERN_TUNE_CACHE names a text file with
// one line per tuned geometry, "<key> <variant> <ms of each variant>"; the
// key holds the device architecture, the HIP runtime version, the ABI
// version, variant count and kernel revision of this library, the precision
// and a bucket of the plan's geometry (padded Nr, K-chunk, computed planes
// and summed line lengths rounded up to powers of two, padded rows of M), so
// a new ROCm, library or kernel revision never reuses an entry.  Unset:
// nothing is read or written.
static std::string tune_key(const wkern_plan_s* pl, int device) {
  const char* path = std::getenv("WKERN_TUNE_CACHE");
  if (!path || !*path) return std::string();
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return std::string();
  int rt = 0;
  if (hipRuntimeGetVersion(&rt) != hipSuccess) return std::string();
  const DevPlan& g = pl->dp;
  int64_t sumRho = 0;
  for (int32_t n : pl->nrhoSorted) sumRho += n;
  auto pow2 = [](int64_t x) {
    int64_t v = 1;
    while (v < x) v <<= 1;
    return (long long)v;
  };
  std::string arch(prop.gcnArchName);
  for (char& c : arch)
    if (c == ' ') c = '_';
  char buf[384];
  snprintf(buf, sizeof(buf), "%s|hip%d|abi%d|nv%d|rev%d|prec%d|nr%d|kc%d|pc%lld|rows%d|rho%lld",
           arch.c_str(), rt, WKERN_ABI_VERSION, (int)kNumVariants, kKernelRevision, g.precision,
           g.NrPad, g.kchunk, pow2(g.P), g.rowsPad, pow2(sumRho));
  return std::string(buf);
}

static std::mutex g_tune_mu;

// Last entry of the cache file for `key` whose variant this precision
// supports; false if there is none (or no readable file).
static bool tune_lookup(const std::string& key, int precision, int* variant, float* ms) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  std::ifstream in(std::getenv("WKERN_TUNE_CACHE"));
  if (!in) return false;
  bool found = false;
  std::string line;
  while (std::getline(in, line)) {
    std::istringstream ls(line);
    std::string k;
    int v = -1;
    if (!(ls >> k >> v) || k != key || v < 0 || v >= kNumVariants ||
        !variant_supported(precision, v))
      continue;
    float t[kNumVariants];
    int n = 0;
    while (n < kNumVariants && (ls >> t[n])) ++n;
    if (n != kNumVariants) continue;
    *variant = v;
    std::copy(t, t + kNumVariants, ms);
    found = true;
  }
  return found;
}

static void tune_store(const std::string& key, int variant, const float* ms) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  std::ostringstream os;
  os.precision(9);  // a float survives the text round trip exactly
  os << key << ' ' << variant;
  for (int v = 0; v < kNumVariants; ++v) os << ' ' << ms[v];
  os << '\n';
  FILE* f = std::fopen(std::getenv("WKERN_TUNE_CACHE"), "a");
  if (!f) return;  // an unwritable cache only costs the next plan a re-tune
  const std::string text = os.str();
  std::fwrite(text.data(), 1, text.size(), f);
  std::fclose(f);
}

// The BF16 terms of M and the BF16-term screen buffer, for the split
// variants that stage them (built on the first selection of such a variant).
static wkern_status ensure_split_terms(wkern_plan_s* pl) {
  DevPlan& g = pl->dp;
  if (g.Msplit) return WKERN_OK;
  const size_t mElems = (size_t)g.rowsPad * g.NrPad;
  const size_t bElems = (size_t)g.colsPad * g.NrPad;
  wkern_status s;
  if ((s = pl->alloc(&g.Msplit, mElems * 3, "Msplit")) != WKERN_OK) return s;
  if ((s = pl->alloc(&g.Bsplit, bElems * 3, "screen buffer")) != WKERN_OK) {
    pl->release(g.Msplit);
    return s;
  }
  hipError_t e = hipMemset(g.Bsplit, 0, bElems * 3 * sizeof(uint16_t));
  if (e == hipSuccess) e = launch_hankel_matrix(g, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    pl->release(g.Msplit);
    pl->release(g.Bsplit);
    return hip_fail(e, "BF16 terms of the HT matrix");
  }
  return WKERN_OK;
}

static wkern_status build_plan(const wkern_desc* d, wkern_plan_s* pl) {
  const int P = d->n_planes;
  pl->desc = *d;
  pl->support.assign(d->support, d->support + P);
  pl->desc.support = pl->support.data();
  pl->offsets.resize(P + 1);
  pl->nrho.resize(P);
  layout_host(&pl->desc, pl->offsets.data(), pl->nrho.data());

  pl->mirror.assign(P, -1);
  if (d->mirror) pl->mirror.assign(d->mirror, d->mirror + P);
  pl->desc.mirror = pl->mirror.data();

  DevPlan& g = pl->dp;
  g.Pall = P;
  g.Nr = d->n_radial;
  g.NrPad = (int)round_up(d->n_radial, kNrAlign);
  g.os = d->oversampling;
  g.q = d->radial_refine;
  g.interp = d->interp == WKERN_INTERP_CUBIC ? 1 : 0;
  g.precision = d->precision == WKERN_PREC_BF16X6 ? 1 : 0;
  const double fov = d->image_size * d->cellsize;
  const double r_max = 0.5 * fov;
  const double du = 1.0 / fov;
  g.dr = r_max / d->n_radial;
  g.drho = du / ((double)d->radial_refine * d->oversampling);

  // computed planes (not mirrored), sorted by radial length, longest first
  // (ties: caller order)
  std::vector<int32_t> perm;
  for (int p = 0; p < P; ++p)
    if (pl->mirror[p] < 0) perm.push_back(p);
  std::stable_sort(perm.begin(), perm.end(),
                   [&](int a, int b) { return pl->nrho[a] > pl->nrho[b]; });
  const int Pc = (int)perm.size();
  g.P = Pc;
  std::vector<int32_t> nrhoSorted(Pc), lineOffSorted(Pc + 1);
  int64_t acc = 0;
  for (int j = 0; j < Pc; ++j) {
    nrhoSorted[j] = pl->nrho[perm[j]];
    lineOffSorted[j] = (int32_t)acc;
    acc += nrhoSorted[j];
  }
  lineOffSorted[Pc] = (int32_t)acc;
  g.lineTotal = (int)acc;
  std::vector<int32_t> sortedPos(P, -1);
  for (int j = 0; j < Pc; ++j) sortedPos[perm[j]] = j;
  // mirrored planes grouped by their source (sorted order)
  pl->mirStart.assign(Pc + 1, 0);
  for (int p = 0; p < P; ++p)
    if (pl->mirror[p] >= 0) ++pl->mirStart[sortedPos[pl->mirror[p]] + 1];
  for (int j = 0; j < Pc; ++j) pl->mirStart[j + 1] += pl->mirStart[j];
  pl->mirList.assign(pl->mirStart[Pc], 0);
  {
    std::vector<int32_t> fillPos(pl->mirStart.begin(), pl->mirStart.end() - 1);
    for (int p = 0; p < P; ++p)
      if (pl->mirror[p] >= 0) pl->mirList[fillPos[sortedPos[pl->mirror[p]]]++] = p;
  }
  pl->lineOffCaller.resize(P + 1);
  acc = 0;
  for (int p = 0; p < P; ++p) {
    pl->lineOffCaller[p] = (int32_t)acc;
    acc += pl->nrho[p];
  }
  pl->lineOffCaller[P] = (int32_t)acc;
  g.lineTotalAll = (int)acc;

  pl->nrhoSorted = nrhoSorted;
  g.nrhoSortedHost = pl->nrhoSorted.data();
  g.nrhoMax = nrhoSorted[0];
  g.rowsPad = (int)round_up(g.nrhoMax, kRowAlign);
  // column blocks of a chunk may run up to 512 columns (the widest tile) past
  // its last plane
  g.colsPad = (int)round_up(2 * (int64_t)Pc, kColAlign) + 512;

  // K-chunks: the longest power-of-two multiple of 256 dividing NrPad, <= 2048
  g.kchunk = kNrAlign;
  while (g.kchunk * 2 <= 2048 && g.NrPad % (g.kchunk * 2) == 0) g.kchunk *= 2;
  g.nkc = g.NrPad / g.kchunk;

  // resample table (caller order)
  std::vector<PlaneInfo> planes(P);
  const int os = d->oversampling;
  for (int p = 0; p < P; ++p) {
    const int S = d->support[p];
    PlaneInfo& pi = planes[p];
    const int src = pl->mirror[p] >= 0 ? pl->mirror[p] : p;
    pi.out_off = pl->offsets[p];
    pi.line_off = lineOffSorted[sortedPos[src]];
    pi.conj = pl->mirror[p] >= 0 ? 1 : 0;
    pi.line_off_caller = pl->lineOffCaller[p];
    pi.nrho = pl->nrho[p];
    pi.S = S;
    pi.h = (S - 1) / 2;
    pi.lim = (os * pi.h) * (os * pi.h);
    pi.invS = 1.0f / (float)S;
    magic_div24((uint32_t)std::max(S, 2), pi.magicS, pi.shiftS);
  }

  pl->perm = perm;
  pl->sortedPosOfCaller.resize(P);
  for (int p = 0; p < P; ++p)
    pl->sortedPosOfCaller[p] = sortedPos[pl->mirror[p] >= 0 ? pl->mirror[p] : p];

  // Thomas coefficients of the spline system: c'_0 = 1/2, c'_k = 1/(4 - c'_{k-1})
  std::vector<double> cprime(std::max(g.nrhoMax, 1));
  cprime[0] = 0.5;
  for (int k = 1; k < (int)cprime.size(); ++k) cprime[k] = 1.0 / (4.0 - cprime[k - 1]);

  // phi_i = r^2 / (1 + sqrt(1 - r^2)) in FP64, zero beyond Nr
  std::vector<double> phi(g.NrPad, 0.0);
  for (int i = 0; i < g.Nr; ++i) {
    const double r = (i + 0.5) * g.dr;
    phi[i] = r * r / (1.0 + std::sqrt(1.0 - r * r));
  }

  wkern_status s;
  if ((s = pl->upload(&g.phi, phi, "phi")) != WKERN_OK) return s;
  if ((s = pl->upload(&g.perm, perm, "perm")) != WKERN_OK) return s;
  if ((s = pl->upload(&g.nrhoSorted, nrhoSorted, "nrho")) != WKERN_OK) return s;
  if ((s = pl->upload(&g.lineOffSorted, lineOffSorted, "line offsets")) != WKERN_OK) return s;
  if ((s = pl->upload(&g.lineOffCaller, pl->lineOffCaller, "line offsets")) != WKERN_OK)
    return s;
  if ((s = pl->upload(&g.mirStart, pl->mirStart, "mirror table")) != WKERN_OK) return s;
  if ((s = pl->upload(&g.mirList, pl->mirList, "mirror table")) != WKERN_OK) return s;
  if ((s = pl->upload(&g.cprime, cprime, "spline table")) != WKERN_OK) return s;
  if ((s = pl->upload(&g.planes, planes, "plane table")) != WKERN_OK) return s;

  const size_t mElems = (size_t)g.rowsPad * g.NrPad;
  if ((s = pl->alloc(&g.M32, mElems, "M32")) != WKERN_OK) return s;
  // split plans: M's BF16 terms in the node-group-major layout the hybrid
  // variant stages
  if (g.precision == 1 && (s = pl->alloc(&g.MsplitG, mElems * 3, "MsplitG")) != WKERN_OK)
    return s;
  // the FP32 screen serves the FP32 path and the split path's FP32-operand
  // variants; the BF16 terms of M and of the screen, which only the other
  // split variants read, are built when such a variant is selected
  const size_t bElems = (size_t)g.colsPad * g.NrPad;
  if ((s = pl->alloc(&g.B32, bElems, "screen buffer")) != WKERN_OK) return s;
  WK_HIP(hipMemset(g.B32, 0, bElems * sizeof(float)), "hipMemset");
  if ((s = pl->alloc(&g.part, (size_t)g.nkc * g.lineTotal * 2, "partial sums")) != WKERN_OK)
    return s;
  if ((s = pl->alloc(&g.coef, (size_t)g.lineTotal * 2, "spline coefficients")) != WKERN_OK)
    return s;
  if ((s = pl->alloc(&g.status, 2, "status word")) != WKERN_OK) return s;
  {
    const int32_t clear[2] = {0, INT32_MAX};
    WK_HIP(hipMemcpy(g.status, clear, sizeof(clear), hipMemcpyHostToDevice), "status word");
  }

  WK_HIP(prepare_kernels(g), "kernel attributes");
  WK_HIP(prepare_resample_kernels(g), "kernel attributes");
  WK_HIP(launch_hankel_matrix(g, nullptr), "HT matrix launch");
  WK_HIP(hipDeviceSynchronize(), "HT matrix");

  // One chunk by default: measured on the batch workload, running the
  // resample of one chunk beside the contraction of the next slowed both
  // (the contraction is L2/HBM-bound as well), so the stages run in turn
  // unless wkern_set_chunks asks otherwise.
  if ((s = build_chunks(pl, 1)) != WKERN_OK) return s;
  WK_HIP(hipStreamCreateWithFlags(&pl->sCompute, hipStreamNonBlocking), "hipStreamCreate");
  WK_HIP(hipStreamCreateWithFlags(&pl->sStore, hipStreamNonBlocking), "hipStreamCreate");
  WK_HIP(hipEventCreateWithFlags(&pl->evFork, hipEventDisableTiming), "hipEventCreate");
  WK_HIP(hipEventCreateWithFlags(&pl->evJoinStore, hipEventDisableTiming), "hipEventCreate");

  // Autotune: time every candidate contraction variant on this plan's own
  // tile lists (timing does not depend on the screen values) and keep the
  // fastest, unless the tuning cache already holds this geometry.  The
  // candidates are the variants that read FP32 operands (every screen is
  // then the same FP32 kernel); the BF16-term variants stay selectable
  // through wkern_set_variant.
  const std::string key = tune_key(pl, d->device);
  if (!key.empty() && tune_lookup(key, g.precision, &pl->variant, pl->variantMs)) {
    pl->tunedFromCache = true;
  } else {
    hipEvent_t a, b;
    WK_HIP(hipEventCreate(&a), "hipEventCreate");
    WK_HIP(hipEventCreate(&b), "hipEventCreate");
    float best = 1e30f;
    for (int v = 0; v < kNumVariants; ++v) {
      if (!variant_supported(g.precision, v) || !variant_fp32_screen(g.precision, v)) {
        pl->variantMs[v] = -1.f;
        continue;
      }
      const int nt = pl->chunkT[v].back();
      float bestV = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        WK_HIP(hipEventRecord(a, pl->sCompute), "hipEventRecord");
        WK_HIP(launch_contract(g, v, pl->d_tiles[v], nt, pl->sCompute), "autotune launch");
        WK_HIP(hipEventRecord(b, pl->sCompute), "hipEventRecord");
        WK_HIP(hipEventSynchronize(b), "hipEventSynchronize");
        float ms = 0.f;
        WK_HIP(hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
        if (rep > 0) bestV = std::min(bestV, ms);
      }
      pl->variantMs[v] = bestV;
      if (bestV < best) {
        best = bestV;
        pl->variant = v;
      }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (!key.empty()) tune_store(key, pl->variant, pl->variantMs);
  }
  if (log_level() >= 1)
    fprintf(stderr, "wkern: plan P=%d (computed %d) Nr=%d os=%d precision=%d variant=%d (%s)\n",
            g.Pall, g.P, g.Nr, g.os, g.precision, pl->variant,
            pl->tunedFromCache ? "tuning cache" : "timed");
  return WKERN_OK;
}

wkern_status wkern_plan(const wkern_desc* d, wkern_plan_t* out) {
  clear_error();
  TraceRange tr("wkern_plan");
  if (!out) return fail(WKERN_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  wkern_status s = validate(d);
  if (s != WKERN_OK) return s;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev < 1) return fail(WKERN_ERR_DEVICE, "no HIP device available");
  if (d->device < 0 || d->device >= ndev)
    return fail(WKERN_ERR_DEVICE, "device %d not in [0, %d)", d->device, ndev);
  DeviceGuard guard(d->device);
  wkern_plan_s* pl = new (std::nothrow) wkern_plan_s();
  if (!pl) return fail(WKERN_ERR_OUT_OF_MEMORY, "plan allocation");
  {
    const char* env = std::getenv("WKERN_CANARY");
    pl->canary = env && std::atoi(env) != 0;
  }
  try {
    s = build_plan(d, pl);
  } catch (const std::bad_alloc&) {
    s = fail(WKERN_ERR_OUT_OF_MEMORY, "host allocation while planning");
  } catch (...) {
    s = fail(WKERN_ERR_DEVICE, "unexpected exception while planning");
  }
  if (s != WKERN_OK) {
    delete pl;
    return s;
  }
  *out = pl;
  return WKERN_OK;
}


static wkern_status check_gen_args(wkern_plan_t plan, const void* taper, const void* w,
                                   const void* out) {
  if (!plan) return fail(WKERN_ERR_INVALID_ARG, "plan is NULL");
  if (!taper) return fail(WKERN_ERR_INVALID_ARG, "taper is NULL");
  if (!w) return fail(WKERN_ERR_INVALID_ARG, "w is NULL");
  if (!out) return fail(WKERN_ERR_INVALID_ARG, "output is NULL");
  return WKERN_OK;
}

// The plan's tables as the spline and line-output kernels see them: the
// projection-slice engine leaves a single K-chunk.
static DevPlan lines_view(const wkern_plan_s* plan) {
  DevPlan v = plan->dp;
  if (plan->engine != WKERN_ENGINE_MATRIX) v.nkc = 1;
  return v;
}

// Radial lines of every computed plane with the selected engine (no
// profiling records): K-chunk partial sums in dp.part.
static wkern_status enqueue_lines(wkern_plan_t plan, const float* taper, const double* w,
                                  hipStream_t st) {
  const DevPlan& g = plan->dp;
  if (plan->engine == WKERN_ENGINE_MATRIX) {
    const int v = plan->variant;
    WK_LAUNCH(launch_screen(g, 0, g.P, taper, w, screen_layout(g.precision, v), st),
           "screen launch");
    WK_LAUNCH(launch_contract(g, v, plan->d_tiles[v], plan->chunkT[v].back(), st),
           "contraction launch");
  } else {
    WK_LAUNCH(launch_ps_lines(g, plan->ps, 0, g.P, taper, w, st), "projection-slice launch");
  }
  return WKERN_OK;
}

// Screen, contraction and spline of pipeline chunk c, then its resample.
static wkern_status enqueue_chunk(wkern_plan_t plan, int c, const float* taper, const double* w,
                                  void* out, hipStream_t compute, hipStream_t store,
                                  hipEvent_t handoff) {
  const DevPlan& g = plan->dp;
  const int j0 = plan->chunkJ[c], j1 = plan->chunkJ[c + 1];
  const int v = plan->variant;
  const int t0 = plan->chunkT[v][c], t1 = plan->chunkT[v][c + 1];
  StageRecord* r;
  wkern_status s;
  if (plan->engine == WKERN_ENGINE_MATRIX) {
    {
      TraceRange tr("wkern screen");
      if ((s = plan->record_begin(0, compute, &r)) != WKERN_OK) return s;
      WK_LAUNCH(launch_screen(g, j0, j1, taper, w, screen_layout(g.precision, v), compute),
             "screen launch");
      if ((s = record_end(r, compute)) != WKERN_OK) return s;
    }
    TraceRange tr("wkern contraction");
    if ((s = plan->record_begin(1, compute, &r)) != WKERN_OK) return s;
    WK_LAUNCH(launch_contract(g, v, plan->d_tiles[v] + t0, t1 - t0, compute), "contraction launch");
    if ((s = record_end(r, compute)) != WKERN_OK) return s;
  } else {
    TraceRange tr("wkern projection-slice lines");
    if ((s = plan->record_begin(1, compute, &r)) != WKERN_OK) return s;
    WK_LAUNCH(launch_ps_lines(g, plan->ps, j0, j1, taper, w, compute), "projection-slice launch");
    if ((s = record_end(r, compute)) != WKERN_OK) return s;
  }
  {
    TraceRange tr("wkern spline");
    if ((s = plan->record_begin(2, compute, &r)) != WKERN_OK) return s;
    WK_LAUNCH(launch_spline(lines_view(plan), j0, j1, compute), "spline launch");
    if ((s = record_end(r, compute)) != WKERN_OK) return s;
  }
  if (handoff) {
    WK_HIP(hipEventRecord(handoff, compute), "hipEventRecord");
    WK_HIP(hipStreamWaitEvent(store, handoff, 0), "hipStreamWaitEvent");
  }
  TraceRange tr("wkern resample");
  if ((s = plan->record_begin(3, store, &r)) != WKERN_OK) return s;
  WK_LAUNCH(launch_resample(g, plan->chunkU[c], plan->chunkU[c + 1], out, store),
         "resample launch");
  return record_end(r, store);
}

// The whole generation: compute stages on `origin`; with several pipeline
// chunks the resamples run on the plan's store stream, forked from and
// joined back into `origin`.
static wkern_status enqueue_all(wkern_plan_t plan, const float* taper, const double* w,
                                void* out, hipStream_t origin) {
  if (plan->nChunks == 1) return enqueue_chunk(plan, 0, taper, w, out, origin, origin, nullptr);
  WK_HIP(hipEventRecord(plan->evFork, origin), "hipEventRecord");
  WK_HIP(hipStreamWaitEvent(plan->sStore, plan->evFork, 0), "hipStreamWaitEvent");
  for (int c = 0; c < plan->nChunks; ++c) {
    wkern_status s =
        enqueue_chunk(plan, c, taper, w, out, origin, plan->sStore, plan->evChunk[c]);
    if (s != WKERN_OK) return s;
  }
  WK_HIP(hipEventRecord(plan->evJoinStore, plan->sStore), "hipEventRecord");
  WK_HIP(hipStreamWaitEvent(origin, plan->evJoinStore, 0), "hipStreamWaitEvent");
  return WKERN_OK;
}

// Capture enqueue_all on the plan's own stream into a graph for this pointer
// set (re-captured, and the executable updated or rebuilt, when the caller
// passes other buffers).
static wkern_status capture_graph(wkern_plan_t plan, const float* taper, const double* w,
                                  void* out) {
  hipGraph_t graph = nullptr;
  WK_HIP(hipStreamBeginCapture(plan->sCompute, hipStreamCaptureModeRelaxed),
         "hipStreamBeginCapture");
  wkern_status s = enqueue_all(plan, taper, w, out, plan->sCompute);
  if (s == WKERN_OK && fault_hit("capture"))
    s = fail(WKERN_ERR_DEVICE, "graph capture: injected failure (WKERN_FAULT)");
  hipError_t e = hipStreamEndCapture(plan->sCompute, &graph);
  if (s != WKERN_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  bool updated = false;
  if (plan->graphExec) {
    hipGraphExecUpdateResult res;
    hipGraphNode_t bad = nullptr;
    if (hipGraphExecUpdate(plan->graphExec, graph, &bad, &res) == hipSuccess &&
        res == hipGraphExecUpdateSuccess)
      updated = true;
    else {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(plan->graphExec);
      plan->graphExec = nullptr;
    }
  }
  if (!updated) {
    e = hipGraphInstantiate(&plan->graphExec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      plan->graphExec = nullptr;
      plan->graphValid = false;
      return hip_fail(e, "hipGraphInstantiate");
    }
  }
  (void)hipGraphDestroy(graph);
  plan->graphKey[0] = taper;
  plan->graphKey[1] = w;
  plan->graphKey[2] = out;
  plan->graphValid = true;
  return WKERN_OK;
}

wkern_status wkern_generate(wkern_plan_t plan, const float* taper, const double* w, void* out,
                            void* stream) {
  clear_error();
  TraceRange tr("wkern_generate");
  wkern_status s = check_gen_args(plan, taper, w, out);
  if (s != WKERN_OK) return s;
  DeviceGuard guard(plan->desc.device);
  hipStream_t st = (hipStream_t)stream;
  if (plan->profiling) {
    ++plan->profiledCalls;
    return enqueue_all(plan, taper, w, out, st);
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  WK_HIP(hipStreamIsCapturing(st, &cs), "hipStreamIsCapturing");
  if (!plan->useGraph || cs != hipStreamCaptureStatusNone)
    return enqueue_all(plan, taper, w, out, st);  // inside the caller's own capture
  if (!plan->graphValid || plan->graphKey[0] != taper || plan->graphKey[1] != w ||
      plan->graphKey[2] != out) {
    if ((s = capture_graph(plan, taper, w, out)) != WKERN_OK) return s;
  }
  WK_HIP(hipGraphLaunch(plan->graphExec, st), "hipGraphLaunch");
  return WKERN_OK;
}

wkern_status wkern_set_graph(wkern_plan_t plan, int32_t enable) {
  clear_error();
  if (!plan) return fail(WKERN_ERR_INVALID_ARG, "plan is NULL");
  plan->useGraph = enable != 0;
  return WKERN_OK;
}

static wkern_status ensure_trunc_scratch(wkern_plan_t plan) {
  if (plan->truncReady) return WKERN_OK;
  const DevPlan& g = plan->dp;
  TruncScratch& ts = plan->trunc;
  wkern_status s;
  if ((s = plan->alloc(&ts.hTrunc, (size_t)g.P, "truncation table")) != WKERN_OK ||
      (s = plan->alloc(&ts.unitStart, (size_t)g.Pall + 1, "truncation table")) != WKERN_OK ||
      (s = plan->alloc(&ts.unitPlane, (size_t)g.nUnits, "truncation table")) != WKERN_OK ||
      (s = plan->upload(&ts.sortedPos, plan->sortedPosOfCaller, "truncation table")) != WKERN_OK) {
    plan->release(ts.hTrunc);
    plan->release(ts.unitStart);
    plan->release(ts.unitPlane);
    plan->release(ts.sortedPos);
    return s;
  }
  plan->truncReady = true;
  return WKERN_OK;
}

wkern_status wkern_generate_truncated(wkern_plan_t plan, const float* taper, const double* w,
                                      double frac, void* out, int64_t out_capacity,
                                      int32_t* support_out, int64_t* offsets_out, void* stream) {
  clear_error();
  TraceRange tr("wkern_generate_truncated");
  wkern_status s = check_gen_args(plan, taper, w, out);
  if (s != WKERN_OK) return s;
  if (!support_out || !offsets_out) return fail(WKERN_ERR_INVALID_ARG, "layout output is NULL");
  if (!(frac > 0.0 && frac < 1.0)) return fail(WKERN_ERR_INVALID_ARG, "frac %g not in (0, 1)", frac);
  if (out_capacity < plan->offsets.back())
    return fail(WKERN_ERR_INVALID_ARG, "out_capacity %lld < %lld (untruncated cache)",
                (long long)out_capacity, (long long)plan->offsets.back());
  DeviceGuard guard(plan->desc.device);
  if ((s = ensure_trunc_scratch(plan)) != WKERN_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if ((s = enqueue_lines(plan, taper, w, st)) != WKERN_OK) return s;
  WK_LAUNCH(launch_resample_truncated(lines_view(plan), plan->trunc, frac, support_out, offsets_out,
                                   out, st),
         "truncated resample launch");
  return WKERN_OK;
}

wkern_status wkern_prepare_lines(wkern_plan_t plan, const float* taper, const double* w,
                                 double frac, int32_t* support_out, void* stream) {
  clear_error();
  TraceRange tr("wkern_prepare_lines");
  wkern_status s = check_gen_args(plan, taper, w, support_out);
  if (s != WKERN_OK) return s;
  if (!(frac >= 0.0 && frac < 1.0)) return fail(WKERN_ERR_INVALID_ARG, "frac %g not in [0, 1)", frac);
  DeviceGuard guard(plan->desc.device);
  if (frac > 0.0 && (s = ensure_trunc_scratch(plan)) != WKERN_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if ((s = enqueue_lines(plan, taper, w, st)) != WKERN_OK) return s;
  const DevPlan view = lines_view(plan);
  int32_t* hT = frac > 0.0 ? plan->trunc.hTrunc : nullptr;
  WK_LAUNCH(launch_spline(view, 0, view.P, st, frac, hT), "spline launch");
  WK_LAUNCH(launch_supports(view, hT, hT ? plan->trunc.sortedPos : nullptr, support_out, st),
         "supports launch");
  return WKERN_OK;
}

wkern_status wkern_grid(wkern_plan_t plan, const double* u, const double* v, const double* w,
                        const void* vis, int64_t n_records, const int32_t* order,
                        const int64_t* plane_start, const int32_t* support, const void* cache,
                        const int64_t* cache_offsets, int32_t grid_size, void* grid,
                        void* stream) {
  clear_error();
  TraceRange tr("wkern_grid");
  if (!plan) return fail(WKERN_ERR_INVALID_ARG, "plan is NULL");
  if (n_records < 0 || n_records > 0x7FFFFFFF)
    return fail(WKERN_ERR_INVALID_ARG, "n_records %lld out of range", (long long)n_records);
  if (grid_size < 2 || grid_size > 65536 || grid_size % 2)
    return fail(WKERN_ERR_INVALID_ARG, "grid_size %d must be even, 2 .. 65536", grid_size);
  if (n_records == 0) return WKERN_OK;  // nothing is read or written
  if (!u || !v || !w || !vis || !order || !plane_start || !support || !grid)
    return fail(WKERN_ERR_INVALID_ARG, "NULL argument");
  if (cache && !cache_offsets) return fail(WKERN_ERR_INVALID_ARG, "cache_offsets is NULL");
  DeviceGuard guard(plan->desc.device);
  wkern_status s;
  if (!plan->gridChunks &&
      (s = plan->alloc(&plan->gridChunks, (size_t)plan->dp.Pall + 1, "gridding table")) != WKERN_OK)
    return s;
  const double du = 1.0 / ((double)plan->desc.image_size * plan->desc.cellsize);
  WK_LAUNCH(launch_grid(lines_view(plan), plan->gridChunks, u, v, w, vis, n_records, order,
                     plane_start, support, cache, cache_offsets, grid_size, du, grid,
                     (hipStream_t)stream),
         "gridding launch");
  return WKERN_OK;
}

wkern_status wkern_set_profiling(wkern_plan_t plan, int32_t enable) {
  clear_error();
  if (!plan) return fail(WKERN_ERR_INVALID_ARG, "plan is NULL");
  plan->profiling = enable != 0;
  if (enable) {
    plan->recordsUsed = 0;
    plan->profiledCalls = 0;
  }
  return WKERN_OK;
}

wkern_status wkern_stage_times(wkern_plan_t plan, double* ms, int32_t* calls) {
  clear_error();
  if (!plan) return fail(WKERN_ERR_INVALID_ARG, "plan is NULL");
  if (!ms) return fail(WKERN_ERR_INVALID_ARG, "ms is NULL");
  DeviceGuard guard(plan->desc.device);
  for (int k = 0; k < 4; ++k) ms[k] = 0.0;
  for (size_t i = 0; i < plan->recordsUsed; ++i) {
    const StageRecord& r = plan->records[i];
    WK_HIP(hipEventSynchronize(r.end), "hipEventSynchronize");
    float t = 0.f;
    WK_HIP(hipEventElapsedTime(&t, r.start, r.end), "hipEventElapsedTime");
    ms[r.stage] += t;
  }
  if (calls) *calls = plan->profiledCalls;
  return WKERN_OK;
}

wkern_status wkern_plan_info(wkern_plan_t plan, int32_t* variant, int32_t* n_variants,
                            float* variant_ms, int32_t* chunks) {
  clear_error();
  if (!plan) return fail(WKERN_ERR_INVALID_ARG, "plan is NULL");
  if (variant) *variant = plan->variant;
  if (n_variants) *n_variants = kNumVariants;
  if (variant_ms)
    for (int v = 0; v < kNumVariants; ++v) variant_ms[v] = plan->variantMs[v];
  if (chunks) *chunks = plan->nChunks;
  return WKERN_OK;
}

// Workspace width of the projection-slice engine for one plane: the power of
// two at or above max(S, min_width, 2), doubled until the padded transform
// reaches the line's last node.
static int ps_width(int S, int minWidth, int pad, int nrho) {
  int n = 2;
  while (n < S || n < minWidth) n *= 2;
  while (pad * n / 2 < nrho) n *= 2;
  return n;
}

wkern_status wkern_set_engine(wkern_plan_t plan, int32_t engine, int32_t workspace_mode) {
  clear_error();
  if (!plan) return fail(WKERN_ERR_INVALID_ARG, "plan is NULL");
  if (engine != WKERN_ENGINE_MATRIX && engine != WKERN_ENGINE_PROJECTION_SLICE)
    return fail(WKERN_ERR_INVALID_ARG, "engine %d unknown", engine);
  if (workspace_mode != 0 && workspace_mode != 1)
    return fail(WKERN_ERR_INVALID_ARG, "workspace_mode %d not 0 or 1", workspace_mode);
  DeviceGuard guard(plan->desc.device);
  WK_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
  plan->graphValid = false;
  if (engine == WKERN_ENGINE_MATRIX) {
    plan->engine = engine;
    return WKERN_OK;
  }
  const DevPlan& g = plan->dp;
  const int pad = g.q * g.os;
  const int minWidth = workspace_mode == 0 ? plan->desc.max_support : 0;
  std::vector<int32_t> n(g.P);
  int maxN = 2;
  for (int j = 0; j < g.P; ++j) {
    n[j] = ps_width(plan->support[plan->perm[j]], minWidth, pad, plan->nrhoSorted[j]);
    maxN = std::max(maxN, n[j]);
  }
  const long long lmax = (long long)pad * maxN;
  if (lmax > kPsMaxL)
    return fail(WKERN_ERR_UNSUPPORTED, "padded transform %lld above %d", lmax, kPsMaxL);
  std::vector<double> cosTab((size_t)lmax);
  for (long long m = 0; m < lmax; ++m) cosTab[m] = std::cos(2.0 * M_PI * (double)m / (double)lmax);
  plan->release(plan->ps.n);
  plan->release(plan->ps.cosTab);
  wkern_status s;
  if ((s = plan->upload(&plan->ps.n, n, "projection-slice table")) != WKERN_OK) return s;
  if ((s = plan->upload(&plan->ps.cosTab, cosTab, "projection-slice table")) != WKERN_OK) return s;
  plan->ps.Lmax = (int)lmax;
  plan->ps.maxN = maxN;
  plan->ps.fov = (double)plan->desc.image_size * plan->desc.cellsize;
  plan->engine = engine;
  plan->psMode = workspace_mode;
  return WKERN_OK;
}

wkern_status wkern_set_variant(wkern_plan_t plan, int32_t variant) {
  clear_error();
  if (!plan) return fail(WKERN_ERR_INVALID_ARG, "plan is NULL");
  if (variant < 0 || variant >= kNumVariants)
    return fail(WKERN_ERR_INVALID_ARG, "variant %d not in [0, %d)", variant, kNumVariants);
  if (!variant_supported(plan->dp.precision, variant))
    return fail(WKERN_ERR_INVALID_ARG, "variant %d is not available for this precision", variant);
  DeviceGuard guard(plan->desc.device);
  if (!variant_fp32_screen(plan->dp.precision, variant)) {
    WK_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    wkern_status s = ensure_split_terms(plan);
    if (s != WKERN_OK) return s;
  }
  plan->variant = variant;
  plan->graphValid = false;
  return WKERN_OK;
}

wkern_status wkern_set_chunks(wkern_plan_t plan, int32_t chunks) {
  clear_error();
  if (!plan) return fail(WKERN_ERR_INVALID_ARG, "plan is NULL");
  if (chunks < 1) return fail(WKERN_ERR_INVALID_ARG, "chunks %d < 1", chunks);
  DeviceGuard guard(plan->desc.device);
  WK_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
  plan->graphValid = false;
  try {
    return build_chunks(plan, chunks);
  } catch (const std::bad_alloc&) {
    return fail(WKERN_ERR_OUT_OF_MEMORY, "host allocation");
  }
}

wkern_status wkern_generate_radial(wkern_plan_t plan, const float* taper, const double* w,
                                   void* lines, void* stream) {
  clear_error();
  TraceRange tr("wkern_generate_radial");
  wkern_status s = check_gen_args(plan, taper, w, lines);
  if (s != WKERN_OK) return s;
  DeviceGuard guard(plan->desc.device);
  hipStream_t st = (hipStream_t)stream;
  if ((s = enqueue_lines(plan, taper, w, st)) != WKERN_OK) return s;
  WK_LAUNCH(launch_lines_out(lines_view(plan), lines, st), "lines launch");
  return WKERN_OK;
}

wkern_status wkern_grad(wkern_plan_t plan, const float* taper, const double* w,
                        const void* grad_out, float* grad_taper, double* grad_w, void* stream) {
  clear_error();
  TraceRange tr("wkern_grad");
  wkern_status s = check_gen_args(plan, taper, w, grad_out);
  if (s != WKERN_OK) return s;
  if (!grad_taper || !grad_w) return fail(WKERN_ERR_INVALID_ARG, "gradient output is NULL");
  if (plan->desc.oversampling > 32)
    return fail(WKERN_ERR_UNSUPPORTED, "gradient needs oversampling <= 32");
  if (plan->engine != WKERN_ENGINE_MATRIX)
    return fail(WKERN_ERR_UNSUPPORTED, "the adjoint covers the matrix-form engine only");
  DeviceGuard guard(plan->desc.device);
  const DevPlan& g = plan->dp;
  if (!plan->gradReady) {
    GradScratch& gs = plan->grad;
    const size_t lt = (size_t)g.lineTotal;
    const size_t pn = (size_t)g.P * g.NrPad;
    if ((s = plan->alloc(&gs.mom, (size_t)g.lineTotalAll * 4, "adjoint moments")) != WKERN_OK ||
        (s = plan->alloc(&gs.gy, lt, "adjoint lines")) != WKERN_OK ||
        (s = plan->alloc(&gs.ure, pn, "adjoint screen")) != WKERN_OK ||
        (s = plan->alloc(&gs.wterm, pn, "adjoint screen")) != WKERN_OK ||
        (s = plan->alloc(&gs.momfx, (size_t)g.lineTotalAll * 8, "adjoint moments")) != WKERN_OK ||
        (s = plan->alloc(&gs.amax, (size_t)g.Pall, "adjoint maxima")) != WKERN_OK) {
      // release what was allocated, so that a later call starts clean
      plan->release(gs.mom);
      plan->release(gs.gy);
      plan->release(gs.ure);
      plan->release(gs.wterm);
      plan->release(gs.momfx);
      plan->release(gs.amax);
      return s;
    }
    plan->gradReady = true;
  }
  WK_LAUNCH(launch_grad(g, plan->grad, taper, w, grad_out, grad_taper, grad_w, (hipStream_t)stream),
         "gradient launch");
  return WKERN_OK;
}

// Compare every guard band of the plan's allocations with the fill pattern
// after the device has drained.  The first changed band is reported (and
// refilled, so that a later check starts clean); WKERN_FAULT=canary changes
// one byte of the first allocation's trailing band first, from the host,
// to test this path without an overrun.
static wkern_status check_canaries(wkern_plan_t plan) {
  using A = wkern_plan_s;
  WK_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
  if (!plan->allocations.empty() && fault_hit("canary")) {
    const A::Allocation& a = plan->allocations.front();
    const unsigned char bad = (unsigned char)~A::kGuardByte;
    WK_HIP(hipMemcpy((unsigned char*)a.user + a.bytes + 7, &bad, 1, hipMemcpyHostToDevice),
           "canary fault");
  }
  std::vector<unsigned char> band(A::kGuardBytes);
  for (const A::Allocation& a : plan->allocations) {
    unsigned char* sides[2] = {(unsigned char*)a.raw, (unsigned char*)a.user + a.bytes};
    for (int side = 0; side < 2; ++side) {
      WK_HIP(hipMemcpy(band.data(), sides[side], A::kGuardBytes, hipMemcpyDeviceToHost),
             "canary read");
      size_t k = 0;
      while (k < A::kGuardBytes && band[k] == A::kGuardByte) ++k;
      if (k == A::kGuardBytes) continue;
      WK_HIP(hipMemset(sides[side], A::kGuardByte, A::kGuardBytes), "canary refill");
      return fail(WKERN_ERR_DEVICE,
                  "canary overwritten %s the %s buffer (%zu bytes): byte %zu of the guard band",
                  side ? "after" : "before", a.what, a.bytes, k);
    }
  }
  return WKERN_OK;
}

wkern_status wkern_sync_status(wkern_plan_t plan, void* stream) {
  clear_error();
  if (!plan) return fail(WKERN_ERR_INVALID_ARG, "plan is NULL");
  DeviceGuard guard(plan->desc.device);
  hipStream_t st = (hipStream_t)stream;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  WK_HIP(hipStreamIsCapturing(st, &cs), "hipStreamIsCapturing");
  if (cs != hipStreamCaptureStatusNone)
    return fail(WKERN_ERR_INVALID_ARG, "stream is being captured; the status word needs a wait");
  int32_t word[2] = {0, INT32_MAX};
  WK_HIP(hipMemcpyAsync(word, plan->dp.status, sizeof(word), hipMemcpyDeviceToHost, st),
         "status read");
  WK_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
  if (plan->canary) {
    wkern_status cs2 = check_canaries(plan);
    if (cs2 != WKERN_OK) return cs2;
  }
  if (word[0] == 0) return WKERN_OK;
  const int32_t clear[2] = {0, INT32_MAX};
  WK_HIP(hipMemcpy(plan->dp.status, clear, sizeof(clear), hipMemcpyHostToDevice), "status clear");
  if (word[0] & kStatusNonFinite)
    return fail(WKERN_ERR_NONFINITE,
                "non-finite radial line value; first affected plane %d (caller order)", word[1]);
  return fail(WKERN_ERR_DEVICE, "device status word 0x%x", (unsigned)word[0]);
}

wkern_status wkern_destroy(wkern_plan_t plan) {
  clear_error();
  if (!plan) return WKERN_OK;
  wkern_status s = WKERN_OK;
  {
    DeviceGuard guard(plan->desc.device);
    (void)hipDeviceSynchronize();
    if (plan->canary) s = check_canaries(plan);
    delete plan;
  }
  return s;
}

}  // extern "C"
