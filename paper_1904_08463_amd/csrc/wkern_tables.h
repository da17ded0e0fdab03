// Device tables the resampler reads: one entry per plane and one per block
// of cache elements (shared by the host plan code and the kernels).
#pragma once

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
};

// One block of output elements [e0, e1) of plane p (plane-local indices).
struct ResampleUnit {
  int32_t p;
  int32_t e0;
  int32_t e1;
  int32_t pad;
};

}  // namespace wkern
