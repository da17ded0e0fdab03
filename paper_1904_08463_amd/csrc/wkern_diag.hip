// Store ceilings of the device: a buffer written with a constant pattern in
// the two store structures the kernel-cache writers can take, for comparing
// the resample's HBM rate with what plain stores reach on the same device.
#include "wkern.h"
#include "wkern_internal.h"

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// One 16-byte store per lane, then the wave ends (blocks of 256 lanes in
// address order).
__global__ __launch_bounds__(256) void k_store_oneshot(f32x4* __restrict__ out, int64_t n16) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n16) out[i] = f32x4{0.f, 0.f, 0.f, 0.f};
}

// The resample's structure: a block of 256 lanes walks a unit of
// kUnitElems complex64 (256 KB) in steps of 4 KB, one 16-byte store per lane
// per step, and the units go to the XCDs in runs of kXcdRun (block b, the
// slot-th on XCD b mod 8, takes unit ((slot / run) 8 + b mod 8) run +
// slot mod run), as in k_resample.
__global__ __launch_bounds__(256) void k_store_units(f32x4* __restrict__ out, int64_t n16,
                                                     int64_t nUnits) {
  constexpr int64_t kUnit16 = (int64_t)wkern::kUnitElems / 2;  // 16-byte items per unit
  constexpr int64_t run = wkern::kXcdRun;
  const int64_t slot = blockIdx.x / wkern::kNumXcd, xcd = blockIdx.x % wkern::kNumXcd;
  const int64_t unit = ((slot / run) * wkern::kNumXcd + xcd) * run + slot % run;
  if (unit >= nUnits) return;
  const int64_t base = unit * kUnit16;
  const int64_t end = base + kUnit16 < n16 ? base + kUnit16 : n16;
  for (int64_t i = base + threadIdx.x; i < end; i += 256) out[i] = f32x4{0.f, 0.f, 0.f, 0.f};
}

}  // namespace

extern "C" wkern_status wkern_store_ceiling(void* buf, int64_t bytes, int32_t pattern,
                                            void* stream) {
  wkern::set_last_error("");
  if (!buf || bytes <= 0 || bytes % 16 != 0 || ((uintptr_t)buf & 15) != 0) {
    wkern::set_last_error("buf must be non-NULL and 16-byte aligned, bytes a positive multiple of 16");
    return WKERN_ERR_INVALID_ARG;
  }
  if (pattern != 0 && pattern != 1) {
    wkern::set_last_error("pattern must be 0 (one store per lane) or 1 (unit walk)");
    return WKERN_ERR_INVALID_ARG;
  }
  const int64_t n16 = bytes / 16;
  hipStream_t s = (hipStream_t)stream;
  if (pattern == 0) {
    const int64_t blocks = (n16 + 255) / 256;
    if (blocks > 0x7FFFFFFF) {
      wkern::set_last_error("buffer too large for one launch");
      return WKERN_ERR_INVALID_ARG;
    }
    hipLaunchKernelGGL(k_store_oneshot, dim3((uint32_t)blocks), dim3(256), 0, s, (f32x4*)buf, n16);
  } else {
    const int64_t unit16 = (int64_t)wkern::kUnitElems / 2;
    const int64_t nUnits = (n16 + unit16 - 1) / unit16;
    const int64_t runs = wkern::kNumXcd * (int64_t)wkern::kXcdRun;
    const int64_t per = (nUnits + runs - 1) / runs * wkern::kXcdRun;  // blocks per XCD
    if (per * wkern::kNumXcd > 0x7FFFFFFF) {
      wkern::set_last_error("buffer too large for one launch");
      return WKERN_ERR_INVALID_ARG;
    }
    hipLaunchKernelGGL(k_store_units, dim3((uint32_t)(per * wkern::kNumXcd)), dim3(256), 0, s,
                       (f32x4*)buf, n16, nUnits);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    wkern::set_last_error(hipGetErrorString(e));
    return WKERN_ERR_DEVICE;
  }
  return WKERN_OK;
}
