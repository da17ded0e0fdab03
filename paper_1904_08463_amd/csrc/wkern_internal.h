// Internal declarations shared by the host plan code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wkern_tables.h"

namespace wkern {

// Sets the calling thread's detail string returned by wkern_last_error().
void set_last_error(const char* msg);

// Host-side fault injection: WKERN_FAULT = "<site>[:<n>]" makes the n-th
// (default first) event at that site after the variable was set fail once
// ("alloc": a device allocation, "launch": a kernel launch, "capture": the
// graph capture of wkern_generate).  Unset or empty: never.
bool fault_hit(const char* site);
// WKERN_LOG: 0 (default, silent), 1 plan summaries, 2 also every error.
int log_level();

// Radial K-chunk accumulated in FP32 inside the matrix cores before it is
// added to an FP64 running sum.
constexpr int kSubChunk = 128;
// Granularity of the padded radial-node count (a multiple of kSubChunk).
constexpr int kNrAlign = 256;
// Rows of M are padded to this multiple (largest row tile).
constexpr int kRowAlign = 128;
// Columns (plane x {re, im}) are padded to this multiple (largest column tile).
constexpr int kColAlign = 128;
// Largest radial line a plane may have (sets the spline's LDS footprint).
constexpr int kMaxRho = 2048;
// Accelerator complex dies (XCDs) of an MI355X; consecutive workgroups are
// dispatched round-robin over them.
constexpr int kNumXcd = 8;
// Revision of the contraction kernels' code, part of the autotuner cache key:
// raised whenever a variant's code changes its speed, so that a stored choice
// made with older kernels is timed again.
constexpr int kKernelRevision = 4;

// Warm-up length of the truncated spline recurrences; the neglected start
// value is damped by (2 - sqrt 3)^16 ~ 7e-10, far below the FP32 rounding of
// the stored coefficients (6e-8).  The recurrences' serial latency is most
// of the spline's time: 32 nodes cost about 25% more.
constexpr int kSplineWarm = 16;

// One contraction tile: rows [row0, row0 + rows), sorted columns
// [col0, col0 + cols), radial nodes [k0, k0 + kchunk).  row0 < 0 marks a
// padding entry that does nothing.
struct Tile {
  int32_t row0;
  int32_t col0;
  int32_t k0;
  int32_t kc;   // index of the K-chunk (partial-sum slot)
  int32_t rbN;  // 32-row blocks this tile computes
  int32_t pad[3];  // pad[0]: end (exclusive, sorted) of the planes it may store
};

// Contraction variants (candidates of the plan-time autotuner).
enum ContractVariant {
  kWave32x64 = 0,   // one wave per tile of 32 rows x 64 columns, direct loads
  kWave32x128 = 1,  // one wave per tile of 32 rows x 128 columns, direct loads
  kLds128x128 = 2,  // 4 waves, up to 128 rows of M staged in LDS, 128 columns
  kLds64x256 = 3,   // 4 waves, up to 64 rows of M staged in LDS, 256 columns
  // split-BF16 only: M rows and screen columns through a ring of LDS stages
  // filled by direct global-to-LDS loads
  kRing128x128 = 4,
  kRing64x256 = 5,
  kRing32x512 = 6,
  // the same ring fed with FP32 M and FP32 screen columns: split into BF16
  // terms in registers (split-BF16, two thirds of the operand bytes) or
  // multiplied on the FP32 matrix cores (FP32)
  kRingF128x128 = 7,
  kRingF64x256 = 8,
  // the 64 x 256 FP32-operand ring on 8 waves of 32 x 64 (two waves per SIMD)
  kRingF64x256W8 = 9,
  // split-BF16 only: M as its plan-time BF16 terms (group-major MsplitG),
  // the FP32 screen split in registers; 8 waves of 64 rows x 32 columns, so
  // every screen value is split by one wave and M by none
  kRingH64x256 = 10,
  // the same tile with operands staged through registers and the running
  // sum held as an FP32 two-sum pair (split-BF16 only)
  kRingR64x256 = 11,
  // the same tile with the screen loaded straight into registers by the
  // lanes that use it, M's terms through a deep LDS ring, one barrier every
  // 4 stages, and an FP64 running sum of the 00 product (the small products
  // in FP32 over the K-chunk) (split-BF16 only)
  kRingW64x256 = 12,
  kNumVariants = 13
};

// Tile geometry of a variant: rows per tile = 32 * rb, columns per tile.
struct ContractShape {
  int rb;
  int cols;
  int pad;
};
ContractShape contract_shape(int variant);
// The BF16-term ring variants exist for the split-BF16 contraction only.
inline bool variant_supported(int precision, int variant) {
  if (variant == kRingH64x256 || variant == kRingR64x256 || variant == kRingW64x256)
    return precision == 1;
  return variant < kRing128x128 || variant >= kRingF128x128 || precision == 1;
}
// Whether a variant reads the FP32 screen (B32) rather than its BF16 terms.
inline bool variant_fp32_screen(int precision, int variant) {
  return precision == 0 || variant >= kRingF128x128;
}
// Layout of the screen a variant reads: its BF16 terms (Bsplit), the FP32
// screen column-major (B32[col][NrPad]) or node-group-major
// (B32[NrPad / 16][colsPad][16], so that the 16 nodes of a stage of all
// columns are one contiguous block).
enum ScreenLayout { kScreenTerms = 0, kScreenColumns = 1, kScreenGroups = 2 };
inline ScreenLayout screen_layout(int precision, int variant) {
  if (!variant_fp32_screen(precision, variant)) return kScreenTerms;
  return variant == kRingW64x256 && precision == 1 ? kScreenGroups : kScreenColumns;
}

// Planes of a pipeline chunk start at multiples of this (in sorted order),
// so no contraction column block straddles two chunks.
constexpr int kChunkAlign = 128;

struct DevPlan {
  // geometry
  int P;           // computed planes (sorted order)
  int Pall;        // all planes, mirrored ones included (caller order)
  int lineTotalAll;  // sum of nrho over all planes
  int Nr, NrPad, os, q, nrhoMax, rowsPad, colsPad, lineTotal, nkc, kchunk;
  int interp;     // 0 linear, 1 cubic
  int precision;  // 0 fp32, 1 bf16x6
  double dr, drho;
  // device tables
  double* phi;            // [NrPad]
  float* M32;             // [rowsPad][NrPad]
  uint16_t* Msplit;       // [rowsPad][NrPad/8][3][8]
  uint16_t* MsplitG;      // [NrPad/8][3][rowsPad][8]: the same terms, node-group major
  int32_t* perm;          // [P] sorted j -> caller p
  int32_t* nrhoSorted;    // [P]
  int32_t* lineOffSorted; // [P + 1]
  double* cprime;         // [nrhoMax] Thomas coefficients
  const int32_t* nrhoSortedHost;  // [P] host copy of nrhoSorted
  PlaneInfo* planes;      // [Pall] caller order
  int32_t* mirStart;      // [P + 1] mirrored planes of sorted plane j: mirList[mirStart[j] ..]
  int32_t* mirList;       // [Pall - P] caller indices
  int32_t* lineOffCaller; // [Pall + 1]
  ResampleUnit* units;
  int nUnits;
  // scratch
  float* B32;             // [colsPad][NrPad], or [NrPad/16][colsPad][16] (kScreenGroups)
  uint16_t* Bsplit;       // [colsPad][NrPad/8][3][8]
  double* part;           // [nkc][lineTotal][2]
  float4* coef;           // [lineTotal][2]
  // device status word: [0] flag bits (kStatusNonFinite), [1] smallest
  // caller index of a plane whose radial line held a non-finite value
  int32_t* status;
};

// Bits of the device status word.
constexpr int32_t kStatusNonFinite = 1;

// Scratch of the adjoint (allocated on the first gradient call).
struct GradScratch {
  double2* mom;   // [lineTotal][4] coefficient moments
  double2* gy;    // [lineTotal] gradient of the radial lines
  double* ure;    // [P][NrPad] Re u
  double* wterm;  // [P][NrPad] 2 pi phi tau Im u
  unsigned long long* momfx;  // [lineTotalAll][8] fixed-point moments
  uint32_t* amax;             // [Pall] max |G| per plane (FP32 bits)
};

hipError_t launch_grad(const DevPlan& p, const GradScratch& gs, const float* taper,
                       const double* w, const void* gout, float* gtau, double* gw,
                       hipStream_t s);
hipError_t launch_hankel_matrix(const DevPlan& p, hipStream_t s);
hipError_t prepare_kernels(const DevPlan& p);
// Write the screen of sorted planes [j0, j1) in the given layout.
hipError_t launch_screen(const DevPlan& p, int j0, int j1, const float* taper, const double* w,
                         ScreenLayout layout, hipStream_t s);
hipError_t launch_contract(const DevPlan& p, int variant, const Tile* tiles, int nTiles,
                           hipStream_t s);
hipError_t launch_spline(const DevPlan& p, int j0, int j1, hipStream_t s, double frac = 0.0,
                         int32_t* hTrunc = nullptr);

// Scratch of the truncated generation (allocated on its first call).
struct TruncScratch {
  int32_t* hTrunc;     // [P] truncated half-widths (sorted order)
  int32_t* sortedPos;  // [Pall] caller plane -> sorted index of its source
  int32_t* unitStart;  // [Pall + 1] prefix sums of resample units
  int32_t* unitPlane;  // [nUnits] plane of each truncated unit (at most the
                       // untruncated count, supports only shrink)
};
hipError_t launch_resample_truncated(const DevPlan& p, const TruncScratch& ts, double frac,
                                     int32_t* supportOut, int64_t* offsetsOut, void* out,
                                     hipStream_t s);
hipError_t launch_resample(const DevPlan& p, int u0, int u1, void* out, hipStream_t s);
// Kernel attributes of the resample kernels that depend on the plan.
hipError_t prepare_resample_kernels(const DevPlan& p);
hipError_t launch_lines_out(const DevPlan& p, void* lines, hipStream_t s);

// Plane supports after wkern_prepare_lines (truncated when hTrunc is given).
hipError_t launch_supports(const DevPlan& p, const int32_t* hTrunc, const int32_t* sortedPos,
                           int32_t* out, hipStream_t s);
// Gridding with the plan's kernels: fused (cache == nullptr, values from the
// spline intervals) or from a kernel cache; chunkStart is [Pall + 1] scratch.
hipError_t launch_grid(const DevPlan& p, int32_t* chunkStart, const double* u, const double* v,
                       const double* w, const void* vis, int64_t n, const int32_t* order,
                       const int64_t* planeStart, const int32_t* support, const void* cache,
                       const int64_t* cacheOff, int N, double du, void* grid, hipStream_t s);

// Tables of the projection-slice engine (built when the engine is selected).
struct PsTables {
  int32_t* n;       // [P] workspace width N_ws of sorted plane j (a power of two)
  double* cosTab;   // [Lmax] cos(2 pi m / Lmax), Lmax = q os max N_ws
  int Lmax;
  int maxN;
  double fov;       // image_size * cellsize
};
// Largest padded transform length the engine's LDS tables hold.
constexpr int kPsMaxL = 8192;
// Radial lines of sorted planes [j0, j1) by projection and padded transform,
// written to K-chunk 0 of the partial-sum buffer.
hipError_t launch_ps_lines(const DevPlan& p, const PsTables& t, int j0, int j1,
                           const float* taper, const double* w, hipStream_t s);

}  // namespace wkern
