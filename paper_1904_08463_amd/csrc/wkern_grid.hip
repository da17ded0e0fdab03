// Gridding with the generated kernels: the step of Algorithm 2 that consumes
// each w-plane's kernel.  Every visibility record adds V K (V conj(K) when
// its w is negative, section 4.1) to the S x S grid cells around it, K being
// the nearest oversampled sub-kernel of its plane:
//   x = u / du + N/2, i = floor(x), f = floor((x - i) os + 1/2) (f = os moves
//   to i + 1, f = 0); cell i + a - h gets sample a of sub-kernel f;
// the same in v.  Cells outside the N x N grid are skipped.
//
// Two consumers: the fused one evaluates every kernel value from the plane's
// spline intervals in LDS while gridding, so the oversampled cache is never
// written to HBM; the other reads a cache made by wkern_generate(_truncated).
// Work items are runs of up to kGridChunk records of one plane (the records
// in the partition's sorted order); a persistent grid of workgroups walks
// them, the threads of a workgroup covering one record's footprint at a
// time.  Sums use FP32 atomics, so their order (and last bits) vary from run
// to run.
#include "wkern_internal.h"
#include "wkern_radial.h"

namespace wkern {

namespace {

constexpr int kGridChunk = 64;
constexpr int kGridThreads = 256;

// Work-item layout: plane m owns ceil(count_m / kGridChunk) items starting at
// chunkStart[m]; one block of 1024 threads, a fixed-order scan.
__global__ __launch_bounds__(1024) void k_grid_layout(int P, const int64_t* __restrict__ planeStart,
                                                      int32_t* __restrict__ chunkStart) {
  __shared__ int32_t sc[1024];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < P; base += 1024) {
    const int m = base + (int)threadIdx.x;
    int32_t c = 0;
    if (m < P) c = (int32_t)((planeStart[m + 1] - planeStart[m] + kGridChunk - 1) / kGridChunk);
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
      const int32_t t = (int)threadIdx.x >= d ? sc[threadIdx.x - d] : 0;
      __syncthreads();
      sc[threadIdx.x] += t;
      __syncthreads();
    }
    if (m < P) chunkStart[m] = carry + sc[threadIdx.x] - c;
    __syncthreads();
    if (threadIdx.x == 1023) carry += sc[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) chunkStart[P] = carry;
}

// Cell and sub-kernel of one coordinate, in FP64 with the operations (and
// roundings) written out: no contraction into fused multiply-adds.
__device__ __forceinline__ void grid_position(double u, double du, int N, int os, int& i, int& f) {
  const double x = __dadd_rn(__ddiv_rn(u, du), 0.5 * (double)N);
  const double fl = floor(x);
  i = (int)fl;
  f = (int)floor(__dadd_rn(__dmul_rn(__dsub_rn(x, fl), (double)os), 0.5));
  if (f == os) {
    i += 1;
    f = 0;
  }
}

template <bool kFused>
__global__ __launch_bounds__(kGridThreads) void k_grid(
    int P, int N, double du, int os, float q, const PlaneInfo* __restrict__ planes,
    const float4* __restrict__ coef, const float2* __restrict__ cache,
    const int64_t* __restrict__ cacheOff, const double* __restrict__ u,
    const double* __restrict__ v, const double* __restrict__ w, const float2* __restrict__ vis,
    const int32_t* __restrict__ order, const int64_t* __restrict__ planeStart,
    const int32_t* __restrict__ support, const int32_t* __restrict__ chunkStart,
    float* __restrict__ grid) {
  extern __shared__ float4 sc[];
  const int total = chunkStart[P];
  for (int c = blockIdx.x; c < total; c += gridDim.x) {
    int lo = 0, hi = P - 1;  // last plane with chunkStart[m] <= c
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (chunkStart[mid] <= c) lo = mid;
      else hi = mid - 1;
    }
    const int m = lo;
    const int64_t r0 = planeStart[m] + (int64_t)(c - chunkStart[m]) * kGridChunk;
    const int64_t r1 = min(planeStart[m + 1], r0 + kGridChunk);
    const PlaneInfo pi = planes[m];
    const int S = support[m];
    const int h = (S - 1) / 2;
    const int lim = (os * h) * (os * h);
    const int nmax = pi.nrho - 2;
    const float invS = 1.0f / (float)S;
    if (kFused) {
      __syncthreads();  // the previous item is done with sc
      const float4* src = coef + (size_t)pi.line_off * 2;
      for (int k = threadIdx.x; k < pi.nrho * 2; k += kGridThreads) sc[k] = src[k];
      __syncthreads();
    }
    const int cells = S * S;
    for (int64_t r = r0; r < r1; ++r) {
      const int k = order[r];
      int iu, fu, iv, fv;
      grid_position(u[k], du, N, os, iu, fu);
      grid_position(v[k], du, N, os, iv, fv);
      // the cache already holds a mirrored plane's conjugate; the lines do not
      const bool cj = (w[k] < 0.0) != (kFused && pi.conj != 0);
      const float2 V = vis[k];
      for (int e = threadIdx.x; e < cells; e += kGridThreads) {
        int a;
        const int b = div_small(e, S, invS, a);
        const int x = iu - h + a;
        const int y = iv - h + b;
        if ((unsigned)x >= (unsigned)N || (unsigned)y >= (unsigned)N) continue;
        const int X = os * (a - h) - fu;
        const int Y = os * (b - h) - fv;
        f32x2 val;
        if (kFused) {
          if (X * X + Y * Y > lim) continue;
          val = cache_value(X, Y, lim, q, nmax, sc);
        } else {
          const float2 cv = cache[cacheOff[m] + ((int64_t)(fv * os + fu) * S + b) * S + a];
          if (cv.x == 0.f && cv.y == 0.f) continue;
          val.x = cv.x;
          val.y = cv.y;
        }
        if (cj) val.y = -val.y;
        float* g = grid + 2 * ((int64_t)y * N + x);
        atomicAdd(g, V.x * val.x - V.y * val.y);
        atomicAdd(g + 1, V.x * val.y + V.y * val.x);
      }
    }
  }
}

// Supports of the planes after prepare_lines: truncated (from the spline's
// decision, section 3.1) or as planned.
__global__ void k_supports(int Pall, const int32_t* __restrict__ hTrunc,
                           const int32_t* __restrict__ sortedPos,
                           const PlaneInfo* __restrict__ planes, int32_t* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= Pall) return;
  out[p] = hTrunc ? 2 * hTrunc[sortedPos[p]] + 1 : planes[p].S;
}

}  // namespace

hipError_t launch_supports(const DevPlan& p, const int32_t* hTrunc, const int32_t* sortedPos,
                           int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_supports, dim3((p.Pall + 255) / 256), dim3(256), 0, s, p.Pall, hTrunc,
                     sortedPos, p.planes, out);
  return hipGetLastError();
}

hipError_t launch_grid(const DevPlan& p, int32_t* chunkStart, const double* u, const double* v,
                       const double* w, const void* vis, int64_t n, const int32_t* order,
                       const int64_t* planeStart, const int32_t* support, const void* cache,
                       const int64_t* cacheOff, int N, double du, void* grid, hipStream_t s) {
  hipLaunchKernelGGL(k_grid_layout, dim3(1), dim3(1024), 0, s, p.Pall, planeStart, chunkStart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t items = n / kGridChunk + p.Pall;  // upper bound
  const int blocks = (int)(items < 8192 ? items : 8192);
  if (cache) {
    hipLaunchKernelGGL(k_grid<false>, dim3(blocks), dim3(kGridThreads), 0, s, p.Pall, N, du, p.os,
                       (float)p.q, p.planes, p.coef, (const float2*)cache, cacheOff, u, v, w,
                       (const float2*)vis, order, planeStart, support, chunkStart, (float*)grid);
  } else {
    const size_t shm = (size_t)2 * p.nrhoMax * sizeof(float4);
    hipLaunchKernelGGL(k_grid<true>, dim3(blocks), dim3(kGridThreads), shm, s, p.Pall, N, du, p.os,
                       (float)p.q, p.planes, p.coef, (const float2*)nullptr, cacheOff, u, v, w,
                       (const float2*)vis, order, planeStart, support, chunkStart, (float*)grid);
  }
  return hipGetLastError();
}

}  // namespace wkern
