// Resample of the radial lines into the oversampled kernel cache (section
// 4.4, Algorithm 2) and the truncated layout (section 3.1).
#include "wkern_internal.h"
#include "wkern_radial.h"

namespace wkern {

namespace {

// --------------------------------------------------------------------------
// Oversampled kernel cache (section 4.4, Algorithm 2).  Each block writes
// the elements [e0, e1) of one plane, e = ((fv os + fu) S + b) S + a; the
// plane's spline intervals are staged in LDS.  Stores are coalesced
// (consecutive lanes, consecutive elements) and non-temporal: the cache is
// written once and read by a later consumer.
//
// Radius in units of the radial node spacing: t = q sqrt(d2), d2 = X^2 + Y^2
// (an integer, exact in FP32).  Rounding t itself to FP32 would cost up to
// ulp(t) ~ 6e-5 nodes at t ~ 1000; instead sqrt(d2) = s + c with s from the
// hardware reciprocal square root and the Newton correction
// c = (d2 - s^2) / (2 s) formed with an exact fma residual, and the interval
// fraction u = (q s - k) + q c keeps ~1e-7 absolute accuracy.  k is the
// truncation of q s: a value that lands one node early or late only moves
// u slightly outside [0, 1), where the neighbouring cubic piece agrees.
// --------------------------------------------------------------------------

// Writes elements [e0, e1) of one plane (its spline intervals already in sc).
__device__ __forceinline__ void resample_range(const PlaneInfo& pi, int e0, int e1, int os,
                                               float invOs, float q,
                                               const float4* __restrict__ sc,
                                               float2* __restrict__ out) {
  f32x2* o = (f32x2*)(out + pi.out_off);
  const int S = pi.S;
  const int h = pi.h;
  const int nmax = pi.nrho - 2;
  const int lane = threadIdx.x & 63;
  if (S >= 64) {
    // Each wave takes 64-element chunks wave, wave + 4, ...; the chunk's first
    // element is decoded once (wave-uniform) and advanced by 256 elements per
    // step; within a chunk a row boundary is crossed at most once.
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int e = e0 + 64 * wave;
    int R = e / S;
    int a0 = e - R * S;
    int F = R / S;
    int b0 = R - F * S;
    int fv0 = F / os;
    int fu0 = F - fv0 * os;
    const int stepA = 256 % S;
    const int stepR = 256 / S;
    for (; e < e1; e += 256) {
      if (e + lane < e1) {
        int a = a0 + lane;
        int b = b0, fu = fu0, fv = fv0;
        if (a >= S) {
          a -= S;
          b += 1;
          if (b == S) {
            b = 0;
            fu += 1;
            if (fu == os) {
              fu = 0;
              fv += 1;
            }
          }
        }
        const int X = os * (a - h) - fu;
        const int Y = os * (b - h) - fv;
        f32x2 v = cache_value(X, Y, pi.lim, q, nmax, sc);
        v.y = pi.conj ? -v.y : v.y;
        __builtin_nontemporal_store(v, o + e + lane);
      }
      a0 += stepA;
      int c = stepR;
      if (a0 >= S) {
        a0 -= S;
        c += 1;
      }
      b0 += c;
      if (b0 >= S) {
        b0 -= S;
        fu0 += 1;
        if (fu0 == os) {
          fu0 = 0;
          fv0 += 1;
        }
      }
    }
  } else {
    for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
      int a, b, fu;
      const int R = div_small(e, S, pi.invS, a);
      const int F = div_small(R, S, pi.invS, b);
      const int fv = div_small(F, os, invOs, fu);
      const int X = os * (a - h) - fu;
      const int Y = os * (b - h) - fv;
      f32x2 v = cache_value(X, Y, pi.lim, q, nmax, sc);
      v.y = pi.conj ? -v.y : v.y;
      __builtin_nontemporal_store(v, o + e);
    }
  }
}

__global__ __launch_bounds__(256) void k_resample(const ResampleUnit* __restrict__ units,
                                                  const PlaneInfo* __restrict__ planes,
                                                  const float4* __restrict__ coef, int os,
                                                  float invOs, float q,
                                                  float2* __restrict__ out) {
  extern __shared__ float4 sc[];
  const ResampleUnit u = units[blockIdx.x];
  const PlaneInfo pi = planes[u.p];
  const float4* src = coef + (size_t)pi.line_off * 2;
  for (int k = threadIdx.x; k < pi.nrho * 2; k += 256) sc[k] = src[k];
  __syncthreads();
  resample_range(pi, u.e0, u.e1, os, invOs, q, sc, out);
}

// Truncated layout (section 3.1, Algorithm 2): one block of 1024 threads.
// Plane p (caller order) takes the half-width its source line was truncated
// to; writes supports, the exclusive prefix sums of os^2 S^2 (offsets) and
// of the per-plane resample units (unitStart, units of kUnitElems).
constexpr int kUnitElems = 65536;

__global__ __launch_bounds__(1024) void k_trunc_layout(int Pall, int os,
                                                       const int32_t* __restrict__ hSorted,
                                                       const int32_t* __restrict__ sortedPos,
                                                       int32_t* __restrict__ supportOut,
                                                       int64_t* __restrict__ offsetsOut,
                                                       int32_t* __restrict__ unitStart) {
  __shared__ int64_t sBytes[1024];
  __shared__ int32_t sUnits[1024];
  __shared__ int64_t carryB;
  __shared__ int32_t carryU;
  if (threadIdx.x == 0) {
    carryB = 0;
    carryU = 0;
  }
  __syncthreads();
  for (int base = 0; base < Pall; base += 1024) {
    const int p = base + (int)threadIdx.x;
    int64_t n = 0;
    int32_t nu = 0;
    if (p < Pall) {
      const int S = 2 * hSorted[sortedPos[p]] + 1;
      supportOut[p] = S;
      n = (int64_t)os * os * S * S;
      nu = (int32_t)((n + kUnitElems - 1) / kUnitElems);
    }
    sBytes[threadIdx.x] = n;
    sUnits[threadIdx.x] = nu;
    __syncthreads();
    // inclusive scan (Hillis-Steele) in a fixed order
    for (int d = 1; d < 1024; d <<= 1) {
      int64_t tb = 0;
      int32_t tu = 0;
      if ((int)threadIdx.x >= d) {
        tb = sBytes[threadIdx.x - d];
        tu = sUnits[threadIdx.x - d];
      }
      __syncthreads();
      sBytes[threadIdx.x] += tb;
      sUnits[threadIdx.x] += tu;
      __syncthreads();
    }
    if (p < Pall) {
      offsetsOut[p] = carryB + sBytes[threadIdx.x] - n;
      unitStart[p] = carryU + sUnits[threadIdx.x] - nu;
    }
    __syncthreads();
    if (threadIdx.x == 1023) {
      carryB += sBytes[1023];
      carryU += sUnits[1023];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    offsetsOut[Pall] = carryB;
    unitStart[Pall] = carryU;
  }
}

// Resample of a truncated layout: a fixed grid walks the units; unit u
// belongs to the plane found by binary search in unitStart.
__global__ __launch_bounds__(256) void k_resample_trunc(int Pall, const PlaneInfo* __restrict__ planes,
                                                        const int32_t* __restrict__ supportOut,
                                                        const int64_t* __restrict__ offsetsOut,
                                                        const int32_t* __restrict__ unitStart,
                                                        const float4* __restrict__ coef, int os,
                                                        float invOs, float q,
                                                        float2* __restrict__ out) {
  extern __shared__ float4 sc[];
  const int total = unitStart[Pall];
  for (int u = blockIdx.x; u < total; u += gridDim.x) {
    int lo = 0, hi = Pall - 1;  // last p with unitStart[p] <= u
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (unitStart[mid] <= u) lo = mid;
      else hi = mid - 1;
    }
    const int p = lo;
    PlaneInfo pi = planes[p];
    const int S = supportOut[p];
    pi.S = S;
    pi.h = (S - 1) / 2;
    pi.lim = (os * pi.h) * (os * pi.h);
    pi.invS = 1.0f / (float)S;
    pi.out_off = offsetsOut[p];
    const int n = os * os * S * S;
    const int e0 = (u - unitStart[p]) * kUnitElems;
    const int e1 = min(n, e0 + kUnitElems);
    __syncthreads();  // the previous unit is done with sc
    const float4* src = coef + (size_t)pi.line_off * 2;
    for (int k = threadIdx.x; k < pi.nrho * 2; k += 256) sc[k] = src[k];
    __syncthreads();
    resample_range(pi, e0, e1, os, invOs, q, sc, out);
  }
}

}  // namespace

hipError_t launch_resample(const DevPlan& p, int u0, int u1, void* out, hipStream_t s) {
  if (u1 <= u0) return hipSuccess;
  const size_t shm = (size_t)2 * p.nrhoMax * sizeof(float4);
  hipLaunchKernelGGL(k_resample, dim3(u1 - u0), dim3(256), shm, s, p.units + u0, p.planes,
                     p.coef, p.os, 1.0f / (float)p.os, (float)p.q, (float2*)out);
  return hipGetLastError();
}

hipError_t launch_resample_truncated(const DevPlan& p, const TruncScratch& ts, double frac,
                                     int32_t* supportOut, int64_t* offsetsOut, void* out,
                                     hipStream_t s) {
  hipError_t e = launch_spline(p, 0, p.P, s, frac, ts.hTrunc);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_trunc_layout, dim3(1), dim3(1024), 0, s, p.Pall, p.os, ts.hTrunc,
                     ts.sortedPos, supportOut, offsetsOut, ts.unitStart);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t shm = (size_t)2 * p.nrhoMax * sizeof(float4);
  hipLaunchKernelGGL(k_resample_trunc, dim3(2048), dim3(256), shm, s, p.Pall, p.planes, supportOut,
                     offsetsOut, ts.unitStart, p.coef, p.os, 1.0f / (float)p.os, (float)p.q,
                     (float2*)out);
  return hipGetLastError();
}

}  // namespace wkern
