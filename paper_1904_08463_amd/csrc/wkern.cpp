// Host side of the wkern C ABI: validation, geometry, plane ordering, tile
// schedule, device tables and the generate / grad entry points.
// The method and the data layout are described in include/wkern.h.
#include "wkern.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "wkern_internal.h"

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

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

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
  if (d->precision != WKERN_PREC_FP32 && d->precision != WKERN_PREC_BF16X6)
    return fail(WKERN_ERR_INVALID_ARG, "unknown precision %d", (int)d->precision);
  if (d->interp != WKERN_INTERP_LINEAR && d->interp != WKERN_INTERP_CUBIC)
    return fail(WKERN_ERR_INVALID_ARG, "unknown interp %d", (int)d->interp);
  for (int p = 0; p < d->n_planes; ++p) {
    const int s = d->support[p];
    if (s < 1 || (s % 2) == 0 || s > d->max_support)
      return fail(WKERN_ERR_INVALID_ARG, "support[%d] = %d must be odd in [1, %d]", p, s,
                  d->max_support);
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

struct wkern_plan_s {
  wkern_desc desc{};
  std::vector<int32_t> support;
  std::vector<int64_t> offsets;       // [P + 1]
  std::vector<int32_t> nrho;          // [P] caller order
  std::vector<int32_t> lineOffCaller; // [P + 1]
  std::vector<int32_t> nrhoSorted;    // [P] longest first
  DevPlan dp{};
  int32_t* d_lineOffCaller = nullptr;
  std::vector<void*> allocations;
  // stage profiling: one set of 5 events per profiled generate call
  bool profiling = false;
  std::vector<std::array<hipEvent_t, 5>> events;
  size_t eventsUsed = 0;

  ~wkern_plan_s() {
    for (auto& ev : events)
      for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (void* ptr : allocations) (void)hipFree(ptr);
  }

  template <class T>
  wkern_status alloc(T** ptr, size_t count, const char* what) {
    void* raw = nullptr;
    const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
    hipError_t e = hipMalloc(&raw, bytes);
    if (e != hipSuccess) {
      *ptr = nullptr;
      return hip_fail(e, what);
    }
    allocations.push_back(raw);
    *ptr = (T*)raw;
    return WKERN_OK;
  }

  template <class T>
  wkern_status upload(T** ptr, const std::vector<T>& host, const char* what) {
    wkern_status s = alloc(ptr, host.size(), what);
    if (s != WKERN_OK) return s;
    WK_HIP(hipMemcpy(*ptr, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice), what);
    return WKERN_OK;
  }
};

extern "C" {

int32_t wkern_abi_version(void) { return WKERN_ABI_VERSION; }

const char* wkern_strerror(wkern_status s) {
  switch (s) {
    case WKERN_OK: return "success";
    case WKERN_ERR_INVALID_ARG: return "invalid argument";
    case WKERN_ERR_OUT_OF_MEMORY: return "out of memory";
    case WKERN_ERR_DEVICE: return "device or HIP runtime error";
    case WKERN_ERR_UNSUPPORTED: return "unsupported";
    case WKERN_ERR_ABI_MISMATCH: return "ABI version mismatch";
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

static wkern_status build_plan(const wkern_desc* d, wkern_plan_s* pl) {
  const int P = d->n_planes;
  pl->desc = *d;
  pl->support.assign(d->support, d->support + P);
  pl->desc.support = pl->support.data();
  pl->offsets.resize(P + 1);
  pl->nrho.resize(P);
  layout_host(&pl->desc, pl->offsets.data(), pl->nrho.data());

  DevPlan& g = pl->dp;
  g.P = P;
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

  // planes sorted by radial length, longest first (ties: caller order)
  std::vector<int32_t> perm(P);
  for (int p = 0; p < P; ++p) perm[p] = p;
  std::stable_sort(perm.begin(), perm.end(),
                   [&](int a, int b) { return pl->nrho[a] > pl->nrho[b]; });
  std::vector<int32_t> nrhoSorted(P), lineOffSorted(P + 1);
  int64_t acc = 0;
  for (int j = 0; j < P; ++j) {
    nrhoSorted[j] = pl->nrho[perm[j]];
    lineOffSorted[j] = (int32_t)acc;
    acc += nrhoSorted[j];
  }
  lineOffSorted[P] = (int32_t)acc;
  g.lineTotal = (int)acc;
  std::vector<int32_t> sortedPos(P);
  for (int j = 0; j < P; ++j) sortedPos[perm[j]] = j;
  pl->lineOffCaller.resize(P + 1);
  acc = 0;
  for (int p = 0; p < P; ++p) {
    pl->lineOffCaller[p] = (int32_t)acc;
    acc += pl->nrho[p];
  }
  pl->lineOffCaller[P] = (int32_t)acc;

  pl->nrhoSorted = nrhoSorted;
  g.nrhoSortedHost = pl->nrhoSorted.data();
  g.nrhoMax = nrhoSorted[0];
  g.rowsPad = (int)round_up(g.nrhoMax, kRowAlign);
  g.colsPad = (int)round_up(2 * (int64_t)P, kColAlign);

  // K-chunks: the longest power-of-two multiple of 256 dividing NrPad, <= 2048
  g.kchunk = kNrAlign;
  while (g.kchunk * 2 <= 2048 && g.NrPad % (g.kchunk * 2) == 0) g.kchunk *= 2;
  g.nkc = g.NrPad / g.kchunk;

  // contraction tiles: 32 rows x 64 columns (32 planes) per wave, staircase
  // over the sorted planes: a column block needs the rows of its longest line.
  // Tiles that read the same screen columns over the same K-chunk form a
  // group; a group is pinned to one XCD (workgroup i runs on XCD i % 8) and
  // its tiles are dispatched back to back there, so the group's slice of the
  // screen is read from HBM once and then served by that XCD's L2.
  std::vector<std::vector<Tile>> xcdQueue(kNumXcd);
  const int colTile = 64;
  int group = 0;
  for (int c0 = 0; c0 < 2 * P; c0 += colTile) {
    const int rows = nrhoSorted[c0 / 2];
    for (int kc = 0; kc < g.nkc; ++kc, ++group) {
      std::vector<Tile>& q = xcdQueue[group % kNumXcd];
      for (int r0 = 0; r0 < rows; r0 += 32) q.push_back(Tile{r0, c0, kc * g.kchunk, kc});
    }
  }
  std::vector<Tile> tiles;
  size_t longest = 0;
  for (auto& q : xcdQueue) longest = std::max(longest, q.size());
  // interleave the per-XCD queues; a short queue is padded by repeating its
  // last tile index as a no-op marker (row0 = -1)
  for (size_t m = 0; m < longest; ++m)
    for (int x = 0; x < kNumXcd; ++x)
      tiles.push_back(m < xcdQueue[x].size() ? xcdQueue[x][m] : Tile{-1, 0, 0, 0});
  g.nTiles = (int)tiles.size();

  // resample units: blocks of at most 65536 elements of one plane (multiples of
  // 256, so every wave chunk starts 64-aligned)
  const int64_t unitElems = 65536;
  std::vector<ResampleUnit> units;
  std::vector<PlaneInfo> planes(P);
  const int os = d->oversampling;
  for (int p = 0; p < P; ++p) {
    const int S = d->support[p];
    PlaneInfo& pi = planes[p];
    pi.out_off = pl->offsets[p];
    pi.line_off = lineOffSorted[sortedPos[p]];
    pi.nrho = pl->nrho[p];
    pi.S = S;
    pi.h = (S - 1) / 2;
    pi.lim = (os * pi.h) * (os * pi.h);
    pi.invS = 1.0f / (float)S;
    const int64_t n = (int64_t)os * os * S * S;
    for (int64_t e0 = 0; e0 < n; e0 += unitElems)
      units.push_back(ResampleUnit{p, (int32_t)e0, (int32_t)std::min(n, e0 + unitElems), 0});
  }
  g.nUnits = (int)units.size();

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
  if ((s = pl->upload(&pl->d_lineOffCaller, pl->lineOffCaller, "line offsets")) != WKERN_OK)
    return s;
  if ((s = pl->upload(&g.cprime, cprime, "spline table")) != WKERN_OK) return s;
  if ((s = pl->upload(&g.planes, planes, "plane table")) != WKERN_OK) return s;
  if ((s = pl->upload(&g.tiles, tiles, "tiles")) != WKERN_OK) return s;
  if ((s = pl->upload(&g.units, units, "units")) != WKERN_OK) return s;

  const size_t mElems = (size_t)g.rowsPad * g.NrPad;
  if ((s = pl->alloc(&g.M32, mElems, "M32")) != WKERN_OK) return s;
  if ((s = pl->alloc(&g.Msplit, mElems * 3, "Msplit")) != WKERN_OK) return s;
  const size_t bElems = (size_t)g.colsPad * g.NrPad;
  if (g.precision == 0) {
    if ((s = pl->alloc(&g.B32, bElems, "screen buffer")) != WKERN_OK) return s;
    WK_HIP(hipMemset(g.B32, 0, bElems * sizeof(float)), "hipMemset");
  } else {
    if ((s = pl->alloc(&g.Bsplit, bElems * 3, "screen buffer")) != WKERN_OK) return s;
    WK_HIP(hipMemset(g.Bsplit, 0, bElems * 3 * sizeof(uint16_t)), "hipMemset");
  }
  if ((s = pl->alloc(&g.part, (size_t)g.nkc * g.lineTotal * 2, "partial sums")) != WKERN_OK)
    return s;
  if ((s = pl->alloc(&g.coef, (size_t)g.lineTotal * 2, "spline coefficients")) != WKERN_OK)
    return s;

  WK_HIP(launch_hankel_matrix(g, nullptr), "HT matrix launch");
  WK_HIP(hipDeviceSynchronize(), "HT matrix");
  return WKERN_OK;
}

wkern_status wkern_plan(const wkern_desc* d, wkern_plan_t* out) {
  clear_error();
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

wkern_status wkern_generate(wkern_plan_t plan, const float* taper, const double* w, void* out,
                            void* stream) {
  clear_error();
  wkern_status s = check_gen_args(plan, taper, w, out);
  if (s != WKERN_OK) return s;
  DeviceGuard guard(plan->desc.device);
  hipStream_t st = (hipStream_t)stream;
  const DevPlan& g = plan->dp;
  hipEvent_t* ev = nullptr;
  if (plan->profiling) {
    if (plan->eventsUsed == plan->events.size()) {
      std::array<hipEvent_t, 5> set{};
      for (auto& e : set) WK_HIP(hipEventCreate(&e), "hipEventCreate");
      plan->events.push_back(set);
    }
    ev = plan->events[plan->eventsUsed++].data();
  }
  if (ev) WK_HIP(hipEventRecord(ev[0], st), "hipEventRecord");
  WK_HIP(launch_screen(g, taper, w, st), "screen launch");
  if (ev) WK_HIP(hipEventRecord(ev[1], st), "hipEventRecord");
  WK_HIP(launch_contract(g, st), "contraction launch");
  if (ev) WK_HIP(hipEventRecord(ev[2], st), "hipEventRecord");
  WK_HIP(launch_spline(g, st), "spline launch");
  if (ev) WK_HIP(hipEventRecord(ev[3], st), "hipEventRecord");
  WK_HIP(launch_resample(g, out, st), "resample launch");
  if (ev) WK_HIP(hipEventRecord(ev[4], st), "hipEventRecord");
  return WKERN_OK;
}

wkern_status wkern_set_profiling(wkern_plan_t plan, int32_t enable) {
  clear_error();
  if (!plan) return fail(WKERN_ERR_INVALID_ARG, "plan is NULL");
  plan->profiling = enable != 0;
  if (enable) plan->eventsUsed = 0;
  return WKERN_OK;
}

wkern_status wkern_stage_times(wkern_plan_t plan, double* ms, int32_t* calls) {
  clear_error();
  if (!plan) return fail(WKERN_ERR_INVALID_ARG, "plan is NULL");
  if (!ms) return fail(WKERN_ERR_INVALID_ARG, "ms is NULL");
  DeviceGuard guard(plan->desc.device);
  for (int k = 0; k < 4; ++k) ms[k] = 0.0;
  for (size_t c = 0; c < plan->eventsUsed; ++c) {
    auto& ev = plan->events[c];
    WK_HIP(hipEventSynchronize(ev[4]), "hipEventSynchronize");
    for (int k = 0; k < 4; ++k) {
      float t = 0.f;
      WK_HIP(hipEventElapsedTime(&t, ev[k], ev[k + 1]), "hipEventElapsedTime");
      ms[k] += t;
    }
  }
  if (calls) *calls = (int32_t)plan->eventsUsed;
  return WKERN_OK;
}

wkern_status wkern_generate_radial(wkern_plan_t plan, const float* taper, const double* w,
                                   void* lines, void* stream) {
  clear_error();
  wkern_status s = check_gen_args(plan, taper, w, lines);
  if (s != WKERN_OK) return s;
  DeviceGuard guard(plan->desc.device);
  hipStream_t st = (hipStream_t)stream;
  const DevPlan& g = plan->dp;
  WK_HIP(launch_screen(g, taper, w, st), "screen launch");
  WK_HIP(launch_contract(g, st), "contraction launch");
  WK_HIP(launch_lines_out(g, plan->d_lineOffCaller, lines, st), "lines launch");
  return WKERN_OK;
}

wkern_status wkern_grad(wkern_plan_t plan, const float* taper, const double* w,
                        const void* grad_out, float* grad_taper, double* grad_w, void* stream) {
  clear_error();
  wkern_status s = check_gen_args(plan, taper, w, grad_out);
  if (s != WKERN_OK) return s;
  if (!grad_taper || !grad_w) return fail(WKERN_ERR_INVALID_ARG, "gradient output is NULL");
  (void)stream;
  return fail(WKERN_ERR_UNSUPPORTED, "gradient not built yet");
}

wkern_status wkern_destroy(wkern_plan_t plan) {
  clear_error();
  if (!plan) return WKERN_OK;
  {
    DeviceGuard guard(plan->desc.device);
    (void)hipDeviceSynchronize();
    delete plan;
  }
  return WKERN_OK;
}

}  // extern "C"
