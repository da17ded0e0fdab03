// Comparison path: the standard w-projection kernel generation by 2D FFT
// (Lucas, Skipper & Scaife 2019, section 3 and Algorithm 1), on the GPU.
// For each plane: the IAA-kernel times the w-kernel on an N x N image-domain
// workspace (workspace undersampling, section 4.2: N is a power of two at
// or above the kernel width), zero padding to L = os N, a 2D FFT (rocFFT
// through hipFFT, FP32), and extraction of the oversampled kernel cache in
// the same layout and circular support as wkern_generate.  It exists to be
// timed against the Hankel path on the same device and inputs.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>
#include <vector>

#include "wkern.h"
#include "wkern_internal.h"

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

wkern_status ffail(wkern_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  wkern::set_last_error(buf);
  return s;
}

#define FF_HIP(call, what)                                                              \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return ffail(e_ == hipErrorOutOfMemory ? WKERN_ERR_OUT_OF_MEMORY : WKERN_ERR_DEVICE, \
                   "%s: %s", what, hipGetErrorString(e_));                              \
  } while (0)

#define FF_FFT(call, what)                                                  \
  do {                                                                      \
    hipfftResult r_ = (call);                                               \
    if (r_ != HIPFFT_SUCCESS) return ffail(WKERN_ERR_DEVICE, "%s: hipfft status %d", what, (int)r_); \
  } while (0)

struct FftPlane {
  int64_t out_off;
  int32_t S;
  int32_t h;
  int32_t lim;
  int32_t pad;  // os^2 S^2, the plane's element count
};

// Workspace of one batch: sample (kx, ky) of the L x L transform input holds
// the image-domain kernel at pixel offset (lx, ly) = (kx, ky) taken modulo L
// into [-L/2, L/2), i.e. the centred N x N workspace zero padded and shifted
// so that l = 0 sits at index 0.  Inside the open disc lx^2 + ly^2 < (N/2)^2
// (the image's circular region, r < r_max) the value is
//   tau(r) exp(+j 2 pi w phi(r)) dl^2,   r = dl sqrt(lx^2 + ly^2),
// with tau linearly interpolated between the midpoint radial samples and
// the transform's area element dl^2 folded in.
__global__ void k_fft_fill(int N, int L, int g0, const int32_t* __restrict__ planeIdx,
                           const double* __restrict__ w, const float* __restrict__ taper, int Nr,
                           double dl, double dr, float2* __restrict__ work) {
  const size_t LL = (size_t)L * L;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= LL) return;
  const int b = blockIdx.y;
  const int p = planeIdx[g0 + b];
  const int ky = (int)(e / (size_t)L);
  const int kx = (int)(e - (size_t)ky * L);
  const int lx = kx < L / 2 ? kx : kx - L;
  const int ly = ky < L / 2 ? ky : ky - L;
  const int half = N / 2;
  float2 v = make_float2(0.f, 0.f);
  if (lx >= -half && lx < half && ly >= -half && ly < half && lx * lx + ly * ly < half * half) {
    const double r2 = (double)(lx * lx + ly * ly) * dl * dl;
    const double phi = r2 / (1.0 + sqrt(1.0 - r2));
    double t = w[p] * phi;
    t -= rint(t);
    const float th = (float)t;
    const float dph = (float)((t - (double)th) * kTwoPi);
    float sn, cs;
    sincospif(2.0f * th, &sn, &cs);
    const float c2 = cs - dph * sn;
    const float s2 = sn + dph * cs;
    const double ti = sqrt(r2) / dr - 0.5;
    double tau;
    if (ti <= 0.0) {
      tau = taper[0];
    } else {
      const int i = (int)ti;
      if (i >= Nr - 1) {
        tau = taper[Nr - 1];
      } else {
        const double f = ti - i;
        tau = (1.0 - f) * (double)taper[i] + f * (double)taper[i + 1];
      }
    }
    const float a = (float)(tau * dl * dl);
    v = make_float2(a * c2, a * s2);
  }
  work[(size_t)b * LL + e] = v;
}

// Kernel cache of the batch's planes: sample (fv, fu, b, a) at uv offset
// (X, Y) = (os (a - h) - fu, os (b - h) - fv) grid cells of du / os is
// transform bin (X mod L, Y mod L); zero outside X^2 + Y^2 <= (os h)^2.
// L = os N need not be a power of two.
__global__ void k_fft_extract(int os, int L, int g0, const int32_t* __restrict__ planeIdx,
                              const FftPlane* __restrict__ info,
                              const float2* __restrict__ work, float2* __restrict__ out) {
  const int b = blockIdx.y;
  const int p = planeIdx[g0 + b];
  const FftPlane pi = info[p];
  const int S = pi.S;
  const int n = os * os * S * S;
  const float2* src = work + (size_t)b * L * L;
  float2* dst = out + pi.out_off;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const int a = e % S;
    const int R = e / S;
    const int bb = R % S;
    const int F = R / S;
    const int fu = F % os;
    const int fv = F / os;
    const int X = os * (a - pi.h) - fu;
    const int Y = os * (bb - pi.h) - fv;
    float2 v = make_float2(0.f, 0.f);
    if (X * X + Y * Y <= pi.lim) {
      const int xm = ((X % L) + L) % L;
      const int ym = ((Y % L) + L) % L;
      v = src[(size_t)ym * L + xm];
    }
    dst[e] = v;
  }
}

// Mirrored planes (section 4.1): the cache of plane p is the conjugate of
// its source plane's.
__global__ void k_conj_copy(int nm, const int32_t* __restrict__ mir, const int32_t* __restrict__ src,
                            const FftPlane* __restrict__ info, float2* __restrict__ out) {
  const int m = blockIdx.y;
  if (m >= nm) return;
  const FftPlane pd = info[mir[m]];
  const FftPlane ps = info[src[m]];
  const int n = (int)(pd.pad);  // element count of the plane
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const float2 v = out[ps.out_off + e];
    out[pd.out_off + e] = make_float2(v.x, -v.y);
  }
}

int next_pow2(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

}  // namespace

struct FftGroup {
  int N = 0;
  int L = 0;
  int batch = 0;  // planes per transform batch
  std::vector<int32_t> planes;
  int first = 0;  // offset of this group's planes in the device plane list
  hipfftHandle full = 0;
  hipfftHandle rem = 0;
  bool hasFull = false, hasRem = false;
};

struct wkern_fft2d_s {
  wkern_desc desc{};
  std::vector<int32_t> support;
  std::vector<int32_t> mirror;
  std::vector<int64_t> offsets;
  int nMirror = 0;
  int32_t* dMir = nullptr;     // mirrored planes
  int32_t* dMirSrc = nullptr;  // their sources
  double dl0 = 0.0;  // FOV, divided by N per group
  double dr = 0.0;
  std::vector<FftGroup> groups;
  float2* work = nullptr;
  int32_t* dPlanes = nullptr;
  FftPlane* dInfo = nullptr;

  ~wkern_fft2d_s() {
    for (auto& g : groups) {
      if (g.hasFull) (void)hipfftDestroy(g.full);
      if (g.hasRem) (void)hipfftDestroy(g.rem);
    }
    if (work) (void)hipFree(work);
    if (dPlanes) (void)hipFree(dPlanes);
    if (dInfo) (void)hipFree(dInfo);
    if (dMir) (void)hipFree(dMir);
    if (dMirSrc) (void)hipFree(dMirSrc);
  }
};

static wkern_status make_fft(hipfftHandle* h, int L, int batch) {
  int n[2] = {L, L};
  FF_FFT(hipfftPlanMany(h, 2, n, nullptr, 1, L * L, nullptr, 1, L * L, HIPFFT_C2C, batch),
         "hipfftPlanMany");
  return WKERN_OK;
}

static wkern_status build_fft(const wkern_desc* d, int mode, size_t budget, wkern_fft2d_s* pl) {
  const int P = d->n_planes;
  pl->desc = *d;
  pl->support.assign(d->support, d->support + P);
  pl->desc.support = pl->support.data();
  pl->mirror.assign(P, -1);
  if (d->mirror) pl->mirror.assign(d->mirror, d->mirror + P);
  pl->desc.mirror = pl->mirror.data();
  pl->offsets.resize(P + 1);
  wkern_status s = wkern_layout_desc(&pl->desc, pl->offsets.data(), nullptr);
  if (s != WKERN_OK) return s;
  const double fov = d->image_size * d->cellsize;
  pl->dl0 = fov;
  pl->dr = 0.5 * fov / d->n_radial;
  const int os = d->oversampling;

  // group planes by workspace size
  std::vector<int> ws(P);
  for (int p = 0; p < P; ++p)
    ws[p] = next_pow2(mode == 0 ? d->max_support : d->support[p]);
  std::vector<int> sizes(ws);
  std::sort(sizes.begin(), sizes.end());
  sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
  std::vector<int32_t> order;
  size_t maxLL = 0;
  for (int N : sizes) {
    FftGroup g;
    g.N = N;
    g.L = os * N;
    if ((int64_t)g.L > 16384)
      return ffail(WKERN_ERR_UNSUPPORTED, "2D transform of %d^2 too large", g.L);
    for (int p = 0; p < P; ++p)
      if (ws[p] == N && pl->mirror[p] < 0) g.planes.push_back(p);
    if (g.planes.empty()) continue;
    g.first = (int)order.size();
    order.insert(order.end(), g.planes.begin(), g.planes.end());
    const size_t LL = (size_t)g.L * g.L;
    g.batch = (int)std::max<size_t>(1, std::min<size_t>(g.planes.size(), budget / (LL * 8)));
    // every sample offset |X| <= os h + os - 1 must stay below L / 2 (no
    // aliasing of the extracted bins): N >= S + 1 guarantees it
    for (int p : g.planes) {
      const int h = (d->support[p] - 1) / 2;
      if (2 * (os * h + os - 1) >= g.L)
        return ffail(WKERN_ERR_INVALID_ARG, "plane %d: support %d does not fit workspace %d", p,
                     d->support[p], N);
    }
    maxLL = std::max(maxLL, LL * (size_t)g.batch);
    pl->groups.push_back(g);
  }
  for (auto& g : pl->groups) {
    const int nb = (int)g.planes.size();
    if (nb >= g.batch) {
      if ((s = make_fft(&g.full, g.L, g.batch)) != WKERN_OK) return s;
      g.hasFull = true;
    }
    if (nb % g.batch) {
      if ((s = make_fft(&g.rem, g.L, nb % g.batch)) != WKERN_OK) return s;
      g.hasRem = true;
    }
  }
  FF_HIP(hipMalloc(&pl->work, maxLL * sizeof(float2)), "workspace");
  FF_HIP(hipMalloc(&pl->dPlanes, order.size() * sizeof(int32_t)), "plane list");
  FF_HIP(hipMemcpy(pl->dPlanes, order.data(), order.size() * sizeof(int32_t),
                   hipMemcpyHostToDevice),
         "plane list");
  std::vector<FftPlane> info(P);
  for (int p = 0; p < P; ++p) {
    const int S = d->support[p];
    const int h = (S - 1) / 2;
    info[p] = FftPlane{pl->offsets[p], S, h, (os * h) * (os * h), os * os * S * S};
  }
  FF_HIP(hipMalloc(&pl->dInfo, P * sizeof(FftPlane)), "plane table");
  FF_HIP(hipMemcpy(pl->dInfo, info.data(), P * sizeof(FftPlane), hipMemcpyHostToDevice),
         "plane table");
  std::vector<int32_t> mir, src;
  for (int p = 0; p < P; ++p)
    if (pl->mirror[p] >= 0) {
      mir.push_back(p);
      src.push_back(pl->mirror[p]);
    }
  pl->nMirror = (int)mir.size();
  if (pl->nMirror > 0) {
    FF_HIP(hipMalloc(&pl->dMir, mir.size() * sizeof(int32_t)), "mirror table");
    FF_HIP(hipMalloc(&pl->dMirSrc, src.size() * sizeof(int32_t)), "mirror table");
    FF_HIP(hipMemcpy(pl->dMir, mir.data(), mir.size() * sizeof(int32_t), hipMemcpyHostToDevice),
           "mirror table");
    FF_HIP(hipMemcpy(pl->dMirSrc, src.data(), src.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice),
           "mirror table");
  }
  return WKERN_OK;
}

extern "C" {

wkern_status wkern_fft2d_plan(const wkern_desc* d, int32_t workspace_mode,
                              int64_t workspace_bytes, wkern_fft2d_t* out) {
  wkern::set_last_error("");
  if (!out) return ffail(WKERN_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!d) return ffail(WKERN_ERR_INVALID_ARG, "desc is NULL");
  if (workspace_mode != 0 && workspace_mode != 1)
    return ffail(WKERN_ERR_INVALID_ARG, "workspace_mode %d not 0 or 1", workspace_mode);
  if (workspace_bytes <= 0) workspace_bytes = (int64_t)2 << 30;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return ffail(WKERN_ERR_DEVICE, "no HIP device available");
  if (d->device < 0 || d->device >= ndev) return ffail(WKERN_ERR_DEVICE, "bad device");
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(d->device);
  wkern_fft2d_s* pl = new (std::nothrow) wkern_fft2d_s();
  wkern_status s = pl ? WKERN_OK : ffail(WKERN_ERR_OUT_OF_MEMORY, "plan");
  if (s == WKERN_OK) {
    try {
      s = build_fft(d, workspace_mode, (size_t)workspace_bytes, pl);
    } catch (const std::bad_alloc&) {
      s = ffail(WKERN_ERR_OUT_OF_MEMORY, "host allocation");
    }
  }
  (void)hipSetDevice(prev);
  if (s != WKERN_OK) {
    delete pl;
    return s;
  }
  *out = pl;
  return WKERN_OK;
}

wkern_status wkern_fft2d_generate(wkern_fft2d_t plan, const float* taper, const double* w,
                                  void* out, void* stream) {
  wkern::set_last_error("");
  if (!plan || !taper || !w || !out) return ffail(WKERN_ERR_INVALID_ARG, "NULL argument");
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(plan->desc.device);
  hipStream_t st = (hipStream_t)stream;
  const int os = plan->desc.oversampling;
  for (auto& g : plan->groups) {
    const int nb = (int)g.planes.size();
    const double dl = plan->dl0 / g.N;
    const size_t LL = (size_t)g.L * g.L;
    for (int b0 = 0; b0 < nb; b0 += g.batch) {
      const int cnt = std::min(g.batch, nb - b0);
      hipfftHandle h = cnt == g.batch ? g.full : g.rem;
      dim3 gf((unsigned)((LL + 255) / 256), cnt);
      hipLaunchKernelGGL(k_fft_fill, gf, dim3(256), 0, st, g.N, g.L, g.first + b0,
                         plan->dPlanes, w, taper, plan->desc.n_radial, dl, plan->dr, plan->work);
      FF_HIP(hipGetLastError(), "fill launch");
      FF_FFT(hipfftSetStream(h, st), "hipfftSetStream");
      FF_FFT(hipfftExecC2C(h, (hipfftComplex*)plan->work, (hipfftComplex*)plan->work,
                           HIPFFT_FORWARD),
             "hipfftExecC2C");
      dim3 ge(64, cnt);
      hipLaunchKernelGGL(k_fft_extract, ge, dim3(256), 0, st, os, g.L, g.first + b0,
                         plan->dPlanes, plan->dInfo, plan->work, (float2*)out);
      FF_HIP(hipGetLastError(), "extract launch");
    }
  }
  for (int m0 = 0; m0 < plan->nMirror; m0 += 65535) {
    const int cnt = std::min(65535, plan->nMirror - m0);
    hipLaunchKernelGGL(k_conj_copy, dim3(16, cnt), dim3(256), 0, st, cnt, plan->dMir + m0,
                       plan->dMirSrc + m0, plan->dInfo, (float2*)out);
    FF_HIP(hipGetLastError(), "conjugate copy launch");
  }
  (void)hipSetDevice(prev);
  return WKERN_OK;
}

wkern_status wkern_fft2d_destroy(wkern_fft2d_t plan) {
  if (!plan) return WKERN_OK;
  (void)hipSetDevice(plan->desc.device);
  (void)hipDeviceSynchronize();
  delete plan;
  return WKERN_OK;
}

}  // extern "C"
