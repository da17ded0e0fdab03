// Radial position and spline value of a kernel sample, shared by the
// resample, its adjoint and the fused gridder (device code only).
#pragma once

#include <hip/hip_runtime.h>

namespace wkern {

typedef float f32x2 __attribute__((ext_vector_type(2)));

// Interval index k and fraction u of the sample at integer offsets (X, Y):
// t = q sqrt(X^2 + Y^2) in units of the radial node spacing.
__device__ __forceinline__ void radial_pos(int d2, float q, int nmax, int& k, float& uu) {
  const float d2f = (float)d2;
  const float r = __builtin_amdgcn_rsqf(d2f);
  const bool nz = d2 > 0;
  const float sq = nz ? d2f * r : 0.f;
  const float res = fmaf(-sq, sq, d2f);
  const float corr = nz ? 0.5f * res * r : 0.f;
  k = min((int)(q * sq), nmax);
  uu = fmaf(q, corr, fmaf(q, sq, -(float)k));
}

// Exact n / d for n < 2^24 and d < 2^16 from an FP32 reciprocal estimate
// (off by at most one) and one integer correction.
__device__ __forceinline__ int div_small(int n, int d, float inv, int& rem) {
  int qt = (int)((float)n * inv);
  int r = n - __mul24(qt, d);  // 0 <= qt, d < 2^24: the 24-bit multiply is exact
  if (r < 0) {
    qt -= 1;
    r += d;
  } else if (r >= d) {
    qt += 1;
    r -= d;
  }
  rem = r;
  return qt;
}

// Kernel value at integer oversampled offsets (X, Y) from the power-form
// spline intervals sc ([2k] re, [2k + 1] im); zero outside the circular
// support X^2 + Y^2 <= lim.
__device__ __forceinline__ f32x2 cache_value(int X, int Y, int lim, float q, int nmax,
                                             const float4* __restrict__ sc) {
  const int d2 = X * X + Y * Y;
  f32x2 v = {0.f, 0.f};
  if (d2 <= lim) {
    int k;
    float uu;
    radial_pos(d2, q, nmax, k, uu);
    const float4 cr = sc[2 * k];
    const float4 ci = sc[2 * k + 1];
    v.x = fmaf(uu, fmaf(uu, fmaf(uu, cr.w, cr.z), cr.y), cr.x);
    v.y = fmaf(uu, fmaf(uu, fmaf(uu, ci.w, ci.z), ci.y), ci.x);
  }
  return v;
}

}  // namespace wkern
