// Radial position of a cache sample, shared by the forward resample and its
// adjoint (device code only).
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

}  // namespace wkern
