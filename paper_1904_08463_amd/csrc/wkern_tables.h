// Device tables the resampler reads: one entry per plane and one per block
// of cache elements (shared by the host plan code and the kernels).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wkern {

// Per-plane table used by the resampler (caller order).
struct PlaneInfo {
  int64_t out_off;    // complex64 offset of the plane's cache
  int32_t line_off;   // offset of its (or its source plane's) radial line, sorted order
  int32_t nrho;       // radial nodes
  int32_t S;          // full width
  int32_t h;          // half width
  int32_t lim;        // (os h)^2
  float invS;         // 1 / S (estimate for the exact small division)
  int32_t conj;       // 1: mirrored plane, written as the conjugate of its source
  int32_t line_off_caller;  // offset of its own line in the caller-order layout
  uint32_t magicS;    // x / S = umulhi(x, magicS) >> shiftS for 0 <= x < 2^24 (S >= 2)
  int32_t shiftS;
};

// Multiplier and shift that divide every 0 <= x < 2^24 by d >= 2 exactly:
// x / d = umulhi(x, m) >> sh.  With L = max(32, 24 + ceil(log2 d)) and
// m = ceil(2^L / d), x m / 2^L exceeds x / d by less than x / 2^L < 2^-(L-24)
// <= 1 / d, which cannot carry it past the next integer.
__host__ __device__ inline void magic_div24(uint32_t d, uint32_t& m, int32_t& sh) {
  int l = 0;
  while ((1u << l) < d) ++l;
  const int L = l + 24 > 32 ? l + 24 : 32;
  m = (uint32_t)((((uint64_t)1 << L) + d - 1) / d);
  sh = L - 32;
}

// Resample units: blocks of at most this many consecutive elements of one
// plane (the full cache's units, and the truncated layout's), 256 KB of
// complex64; a multiple of 1024, so every wave's chunk of a step starts at a
// multiple of its size.  With each XCD walking its own eighth of the units
// (a plane's intervals then come from that XCD's L2), 32 K elements write
// the batch cache in 5.41-5.44 ms, against 5.44-5.45 for 24 K, 5.48-5.50 for
// 48 K, 5.63 for 16 K and 5.66 for 64 K (one box, bit-identical caches).
constexpr int kUnitElems = 32768;

// Runs of consecutive resample units dealt to the XCDs in turn (k_resample).
constexpr int kXcdRun = 64;

// One block of output elements [e0, e1) of plane p (plane-local indices).
struct ResampleUnit {
  int32_t p;
  int32_t e0;
  int32_t e1;
  int32_t pad;
};

}  // namespace wkern
