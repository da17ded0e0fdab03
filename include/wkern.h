/*
 * wkern.h -- w-projection convolution-kernel generation on AMD Instinct MI355X
 * (gfx950), C ABI.
 *
 * Method: Lucas, Skipper & Scaife (2019), "Fast W-Projection for Wide-field
 * Imaging", section 4 and Algorithm 2.  For every w-plane the library
 *   1. evaluates the radially symmetric image-domain convolution kernel
 *      s(r) = tau(r) * G(r, w) on radial nodes, with G the w-projection
 *      screen of section 2.5 (equation wproj_G):
 *          G = exp(-j 2 pi w (sqrt(1 - r^2) - 1)) = exp(+j 2 pi w phi(r)),
 *          phi(r) = r^2 / (1 + sqrt(1 - r^2)), formed in FP64;
 *   2. takes it to the uv plane with the order-0 Hankel transform (section
 *      4.3, equation ht) applied as the product of a discrete HT matrix,
 *      built once per plan, with the sampled screen:
 *          K_p(rho_k) = sum_i M[k, i] s_p(r_i),
 *          M[k, i]    = 2 pi J0(2 pi rho_k r_i) r_i dr,
 *          r_i = (i + 1/2) dr, dr = r_max / Nr, r_max = image_size*cellsize/2,
 *          rho_k = k du / (q os), du = 1 / (image_size * cellsize),
 *          k = 0 .. q os h_p + 3;
 *   3. interpolates the radial line with a cubic spline (s'(0) = 0, natural
 *      at the last node) or linearly (section 4.3.2) onto the oversampled
 *      kernel cache over the circular support (section 4.4, Algorithm 2).
 *
 * Output layout (kernel cache).  Plane p (caller order) of odd full width
 * S_p (half-width h_p = (S_p - 1) / 2) occupies os*os*S_p*S_p complex64
 * values starting at offsets[p] (prefix sum, see wkern_layout):
 *     out[offsets[p] + ((fv*os + fu)*S_p + b)*S_p + a],  fv, fu in [0, os),
 *     b, a in [0, S_p), holds K_p at uv offset ((a - h) - fu/os,
 *     (b - h) - fv/os) cells, i.e. X = os (a - h) - fu, Y = os (b - h) - fv,
 *     radius rho = du sqrt(X^2 + Y^2) / os, when X^2 + Y^2 <= (os h)^2, and
 *     exactly 0 outside that disc.
 * complex64 = two floats (re, im), the layout of C99 float _Complex and of
 * torch.complex64.
 *
 * Conventions.
 * - Every call returns a wkern_status.  No C++ exception crosses the ABI.
 *   On any error a detail string is available from wkern_last_error() (per
 *   thread, valid until the next call on that thread).
 * - Host-side validation completes before anything is enqueued: on an error
 *   status from a generating call nothing has been written.
 * - Device pointers are HIP device pointers on the plan's device.  The
 *   caller owns every buffer it passes; the plan owns its own tables and
 *   scratch.  Buffers must not alias each other.
 * - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls on
 *   one plan must not overlap in time: a plan serves one stream at a time.
 * - Generating calls are asynchronous with respect to the host.
 * - A plan keeps a device status word.  The spline step, which reads every
 *   radial-line value, flags a non-finite one (a NaN or infinite taper
 *   sample or w gives one); wkern_sync_status reports and clears it.
 *
 * Environment (read by the host code at each call):
 * - WKERN_TUNE_CACHE=<file>: the plan-time autotuner's results persist in
 *   this text file, one line per device architecture, HIP runtime version,
 *   library ABI version and kernel revision, and geometry bucket; a plan
 *   whose key is present
 *   takes the stored choice instead of timing the candidates.  Unset: every
 *   plan times them.
 * - WKERN_LOG=<level>: 0 silent (default), 1 a summary line per plan on
 *   stderr, 2 also every error detail.
 * - WKERN_FAULT=<site>[:<n>]: test hook.  The n-th (default first) event at
 *   the site after the variable took this value fails once: "alloc" (a device
 *   allocation of the library: OUT_OF_MEMORY), "launch" (a kernel launch of a
 *   generating call: DEVICE), "capture" (the graph capture of wkern_generate:
 *   DEVICE), "canary" (the canary check of wkern_sync_status finds one byte
 *   changed, written there by the host).  A failed call releases what it
 *   allocated and leaves the plan usable.
 * - WKERN_CANARY=1 (debug, read by wkern_plan): every device allocation of
 *   the plan, including the scratch allocated on the first truncated,
 *   gradient and gridding calls, gets a 1 KiB guard band of 0xA5 bytes on
 *   each side; wkern_sync_status compares all of them with the pattern and
 *   returns DEVICE naming the buffer whose band changed (an overrun of the
 *   library's own scratch).  The caller's output has no band inside it:
 *   plane blocks are contiguous, so an overrun of one lands in its
 *   neighbour, and around the whole buffer the caller can place its own.
 *   Costs 2 KiB per allocation and a synchronous check per status read.
 */
#ifndef WKERN_H
#define WKERN_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WKERN_ABI_VERSION 3

typedef enum {
  WKERN_OK = 0,
  WKERN_ERR_INVALID_ARG = 1,   /* argument fails validation; nothing enqueued */
  WKERN_ERR_OUT_OF_MEMORY = 2, /* device or host allocation failed */
  WKERN_ERR_DEVICE = 3,        /* no usable device or a HIP runtime error */
  WKERN_ERR_UNSUPPORTED = 4,   /* valid request outside what the library implements */
  WKERN_ERR_ABI_MISMATCH = 5,  /* desc->abi_version != WKERN_ABI_VERSION */
  WKERN_ERR_NONFINITE = 6      /* a radial line held a non-finite value (wkern_sync_status) */
} wkern_status;

/* Arithmetic of the Hankel contraction (step 2).  The phase is always formed
 * in FP64.  FP32: M and s rounded to FP32, FP32 matrix-core products.
 * BF16X6: each operand as three BF16 terms (x = x0 + x1 + x2), combined
 * with six BF16 matrix-core products (02, 11, 20, 01, 10, 00).  The
 * screen's terms are an exact split of its FP32 value; M's terms are an
 * exact split of its FP32 value (ringf variants) or split at plan time from
 * its FP64 value (the others).  Both paths accumulate in FP32 over
 * sub-chunks of 128 radial nodes; the sub-chunk sums go into an FP64
 * running sum or, in ringr64x256, into an FP32 pair formed with an exact
 * two-sum (about 48 bits; measured at the same error).  ringw64x256 (the
 * autotuner's usual choice) adds only the 00 product's sub-chunk sums to
 * the FP64 running sum and keeps the five small products in FP32 over the
 * whole K-chunk (at most 2048 nodes; emulated at the same error). */
typedef enum { WKERN_PREC_FP32 = 0, WKERN_PREC_BF16X6 = 1 } wkern_precision;

/* Interpolation of the radial line (section 4.3.2). */
typedef enum { WKERN_INTERP_LINEAR = 0, WKERN_INTERP_CUBIC = 1 } wkern_interp;

typedef struct wkern_plan_s* wkern_plan_t; /* opaque, owned by the library */

/* Problem description; arguments follow the paper's statement of the
 * problem: per-plane w (Algorithm 2), image and cell size (section 5,
 * imager settings), IAA taper (Algorithm 2), maximum support (section 4.2
 * and section 5 settings), oversampling (section 3.1), interpolation type
 * (section 4.3.2). */
typedef struct {
  int32_t abi_version;     /* must be WKERN_ABI_VERSION */
  int32_t image_size;      /* N pixels; FOV = N * cellsize; r_max = FOV / 2 */
  double cellsize;         /* radians, direction-cosine increment; r_max < 1 */
  int32_t n_radial;        /* Nr >= 1: midpoint nodes over [0, r_max] */
  int32_t oversampling;    /* os in [1, 64] */
  int32_t radial_refine;   /* q in [1, 16]; 1 = spacing du/os (section 4.4) */
  int32_t n_planes;        /* P >= 1: w-planes x channels */
  const int32_t* support;  /* host [P]: odd full widths, 1 <= S_p <= max_support */
  int32_t max_support;     /* odd, >= 1; os * max_support <= 4096 */
  wkern_precision precision;
  wkern_interp interp;
  int32_t device;          /* HIP device ordinal */
  /* host [P] or NULL.  Absolute w-term (section 4.1): K(-w) = conj K(w) for
   * a real taper.  mirror[p] = q >= 0 declares that w[p] = -w[q]; plane p is
   * then not computed but written as the exact conjugate of plane q, and
   * w[p] is not read.  q must have mirror[q] = -1 and S_q = S_p.
   * mirror[p] = -1 (or a NULL table): plane p is computed from w[p]. */
  const int32_t* mirror;
} wkern_desc;

/* Version of the ABI this library was built with (== WKERN_ABI_VERSION). */
int32_t wkern_abi_version(void);

/* Layout of the kernel cache for a description, on the host only (no device
 * is touched).  offsets: host [P + 1], complex elements, offsets[P] = total.
 * nrho: host [P] radial nodes per plane (q os h_p + 4), may be NULL.
 * Errors: WKERN_ERR_INVALID_ARG / WKERN_ERR_ABI_MISMATCH as for wkern_plan. */
wkern_status wkern_layout_desc(const wkern_desc* d, int64_t* offsets, int32_t* nrho);

/* Build a plan: validates d, computes the geometry in FP64, the discrete HT
 * matrix M (section 4.3: computed once) on the device with FP64 J0, the
 * plane order and tile schedule, and allocates all scratch.  Synchronous.
 * The description (including `support`) is copied; the caller keeps
 * ownership of d.  On error *out is set to NULL and nothing leaks.
 * Errors: INVALID_ARG (a field out of range, a NULL pointer, an even or too
 * large support, r_max >= 1), ABI_MISMATCH, DEVICE (no such device / HIP
 * failure), OUT_OF_MEMORY. */
wkern_status wkern_plan(const wkern_desc* d, wkern_plan_t* out);

/* Same layout as wkern_layout_desc for the plan's description. */
wkern_status wkern_layout(wkern_plan_t plan, int64_t* offsets, int32_t* nrho);

/* Generate every plane's kernel cache (steps 1-3).
 * taper: device float [Nr], tau at r_i (caller owned, read only).
 * w:     device double [P], w of each plane in wavelengths (read only).
 * out:   device complex64 [offsets[P]] (written completely, zeros included).
 * The launches of one call are captured once into a HIP graph per
 * (taper, w, out) pointer set and replayed with a single graph launch on
 * later calls (see wkern_set_graph); when `stream` is itself being captured
 * by the caller, or profiling is on, the kernels are launched directly.
 * Asynchronous on `stream`.  Errors: INVALID_ARG (NULL plan or pointer),
 * DEVICE (launch or capture failure). */
wkern_status wkern_generate(wkern_plan_t plan, const float* taper, const double* w,
                            void* out, void* stream);

/* Generation with the truncation step of Algorithm 2 (section 3.1: the
 * 1D conv-kernel is cut where its amplitude falls below a fraction of its
 * maximum).  The plan's support S_p is plane p's maximum.  Every line is
 * computed for it; k* is the last radial node with
 * |K_p(rho_k)| >= frac * max_k |K_p(rho_k)| (FP64); the plane gets the
 * half-width h_p = min(ceil(k* / (q os)), (S_p - 1) / 2) and its cache is
 * sampled from the spline through the full line, over the circular support
 * of h_p.  A mirrored plane takes its source's support.
 * frac:        in (0, 1), e.g. 0.01.
 * out:         device complex64 [out_capacity]; the planes are packed in
 *              caller order at offsets_out (elements beyond offsets_out[P]
 *              are not written).
 * out_capacity: >= the untruncated cache size (offsets[P] of wkern_layout),
 *              so no truncation outcome can overflow it.
 * support_out: device int32 [P] (written): the truncated full widths.
 * offsets_out: device int64 [P + 1] (written): prefix sums of os^2 S^2.
 * Asynchronous on `stream` (the layout is known once the stream reaches
 * this point).  Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
wkern_status wkern_generate_truncated(wkern_plan_t plan, const float* taper, const double* w,
                                      double frac, void* out, int64_t out_capacity,
                                      int32_t* support_out, int64_t* offsets_out, void* stream);

/* Steps 1-2 only: the radial lines, for inspection and tests.
 * lines: device complex128 (two doubles) [sum_p nrho[p]], plane p's line at
 * the prefix sum of nrho over planes before p (caller order); line p holds
 * K_p(rho_k), k = 0 .. nrho[p] - 1.  Asynchronous on `stream`. */
wkern_status wkern_generate_radial(wkern_plan_t plan, const float* taper, const double* w,
                                   void* lines, void* stream);

/* Gradient of a real loss L of the kernel cache (reverse of steps 1-3; the
 * paper has no gradient, this is the chain rule through the steps above).
 * grad_out:   device complex64 [offsets[P]], dL/dRe + j dL/dIm of each value.
 * grad_taper: device float [Nr] (written), dL/dtau_i.
 * grad_w:     device double [P] (written), dL/dw_p.  For a mirrored plane p
 *             (mirror[p] = q) the cache is a function of w[q]: its share of
 *             the gradient is folded into grad_w[q] and grad_w[p] = 0.
 * Every reduction runs in a fixed order (bit-reproducible).  The plan's
 * gradient scratch is allocated on the first call.  Asynchronous on
 * `stream`.  Errors: INVALID_ARG, UNSUPPORTED (oversampling > 32),
 * OUT_OF_MEMORY, DEVICE. */
wkern_status wkern_grad(wkern_plan_t plan, const float* taper, const double* w,
                        const void* grad_out, float* grad_taper, double* grad_w,
                        void* stream);

/* -------------------------------------------------------------------------
 * Gridding with the kernels (Algorithm 2, last step of each w-plane): every
 * visibility record adds V K to the S x S grid cells around it, K the nearest
 * oversampled sub-kernel of the record's plane, conjugated when the record's
 * w is negative (section 4.1).  Grid: N x N cells of du = 1 / (image_size
 * cellsize); cell (ix, iy) holds uv = ((ix - N/2) du, (iy - N/2) du), row
 * major (v, then u).  A record at x = u / du + N/2 uses cell i = floor(x) and
 * sub-kernel f = floor((x - i) os + 1/2) (f = os moves to i + 1, f = 0); cell
 * i + a - h receives sample a of sub-kernel f (both axes; FP64).  Cells
 * outside the grid are skipped.
 * ------------------------------------------------------------------------- */

/* Steps 1-3 without the resample: the radial lines and their spline
 * coefficients stay in the plan for a fused wkern_grid, so no kernel cache
 * is written.  frac > 0 applies the truncation rule of
 * wkern_generate_truncated; frac == 0 keeps the planned supports.
 * support_out: device int32 [P] (written): the supports wkern_grid should
 * use.  Asynchronous on `stream`.  Errors: INVALID_ARG, OUT_OF_MEMORY,
 * DEVICE. */
wkern_status wkern_prepare_lines(wkern_plan_t plan, const float* taper, const double* w,
                                 double frac, int32_t* support_out, void* stream);

/* u, v, w:      device double [n_records], wavelengths.
 * vis:          device complex64 [n_records].
 * order, plane_start: the partition (wkern_wpartition) over the plan's P
 *               planes: plane m grids records order[plane_start[m] ..
 *               plane_start[m + 1] - 1].  plane_start (device int64
 *               [P + 1]) starts at 0 and does not decrease; order (device
 *               int32 [plane_start[P]]) holds indices in [0, n_records), a
 *               subset of the records or all of them.  Both are read on the
 *               device as given.
 * support:      device int32 [P], odd widths; each at most the planned one.
 * cache:        NULL: fused, the kernel values come from the spline
 *               coefficients of the plan's last wkern_prepare_lines or
 *               generate call (same stream, same taper and w); otherwise a
 *               device complex64 kernel cache with plane m at
 *               cache_offsets[m] (device int64 [P + 1]) laid out
 *               [os][os][S][S] with S = support[m] (what wkern_generate /
 *               wkern_generate_truncated write).
 * grid_size:    N, even.
 * grid:         device complex64 [N][N], accumulated into (the caller clears
 *               it); FP32 atomic sums, so the last bits depend on timing.
 * n_records = 0 is a no-op (the record pointers may then be NULL).
 * Asynchronous on `stream`.  Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
wkern_status wkern_grid(wkern_plan_t plan, const double* u, const double* v, const double* w,
                        const void* vis, int64_t n_records, const int32_t* order,
                        const int64_t* plane_start, const int32_t* support, const void* cache,
                        const int64_t* cache_offsets, int32_t grid_size, void* grid,
                        void* stream);

/* Engine of the radial-line step (steps 1-2).
 * WKERN_ENGINE_MATRIX (default): the discrete HT matrix times the sampled
 *   screen on the matrix cores (section 4.3), in the plan's precision.
 * WKERN_ENGINE_PROJECTION_SLICE: the paper's own route (section 4.3.1,
 *   Algorithm 2): the IConv-kernel on an N x N image workspace (pixel
 *   l = (x - N/2) FOV/N, zero outside the open disc r < r_max, the taper
 *   linear in r between its samples), projected onto one axis and
 *   transformed with zero padding by q os, in FP64.  N is the power of two at
 *   or above max(S_p, 2) (workspace_mode 1, per plane) or max(max_support, 2)
 *   (workspace_mode 0), doubled until q os N / 2 >= nrho; q os N must not
 *   exceed 8192.  It is a different discretisation of the same transform:
 *   its line equals, sample for sample, the v = 0 row of the 2D FFT of that
 *   workspace, not the matrix form's line.
 * Both engines feed the same spline and resample.  wkern_grad supports the
 * matrix engine only.  Synchronises the plan's device; the captured graph is
 * rebuilt on the next call.  Errors: INVALID_ARG, UNSUPPORTED,
 * OUT_OF_MEMORY, DEVICE. */
typedef enum { WKERN_ENGINE_MATRIX = 0, WKERN_ENGINE_PROJECTION_SLICE = 1 } wkern_engine;
wkern_status wkern_set_engine(wkern_plan_t plan, int32_t engine, int32_t workspace_mode);

/* Stage timing of wkern_generate with HIP events recorded on the call's own
 * stream around each stage (0 screen, 1 contraction, 2 spline, 3 resample);
 * recording adds no synchronisation.  enable != 0 clears and starts
 * accumulation, enable == 0 stops it.  Errors: INVALID_ARG, DEVICE. */
wkern_status wkern_set_profiling(wkern_plan_t plan, int32_t enable);

/* Waits for the recorded events and returns the summed milliseconds of each
 * stage (ms: host double [4]) and the number of profiled generate calls
 * (calls: host, may be NULL).  Errors: INVALID_ARG, DEVICE. */
wkern_status wkern_stage_times(wkern_plan_t plan, double* ms, int32_t* calls);

/* Tuning state of a plan.  variant: the Hankel-contraction kernel variant
 * the plan-time autotuner chose (it times every candidate on the plan's own
 * tile lists, or takes the tuning cache's entry); n_variants: number of
 * variants; variant_ms: host float [n_variants], the measured time of each
 * (-1 for a variant that was not a candidate; may be NULL); chunks: number of
 * pipeline chunks (the resample of one chunk of planes overlaps the screen,
 * contraction and spline of the next).  Any output pointer may be NULL.
 * Errors: INVALID_ARG. */
wkern_status wkern_plan_info(wkern_plan_t plan, int32_t* variant, int32_t* n_variants,
                             float* variant_ms, int32_t* chunks);

/* enable != 0 (the default): wkern_generate replays a captured HIP graph;
 * 0: it launches the kernels one by one.  Errors: INVALID_ARG. */
wkern_status wkern_set_graph(wkern_plan_t plan, int32_t enable);

/* Override the autotuner's choice of contraction variant (0 <= variant <
 * n_variants).  All variants compute the same products in the same order
 * per output element; they differ in tiling, in how operands reach LDS and,
 * for ringr64x256 and ringw64x256, in the running sum (an FP32 two-sum pair;
 * FP64 for the 00 product only), so results can differ in the last bits.  The
 * autotuner's candidates are the variants that stage FP32 operands or M's
 * plan-time BF16 terms with the FP32 screen.  Indices: 0 wave32x64,
 * 1 wave32x128, 2 lds128x128, 3 lds64x256, 4 ring128x128, 5 ring64x256,
 * 6 ring32x512 (4-6 split-BF16 only), 7 ringf128x128, 8 ringf64x256,
 * 9 ringf64x256w8, 10 ringh64x256, 11 ringr64x256, 12 ringw64x256 (10-12
 * split-BF16 only); a variant the plan's precision cannot run is
 * INVALID_ARG.  Selecting a split-BF16 variant that stages BF16 terms
 * builds those terms (M's and a screen buffer) on its first selection
 * (synchronous then).  Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
wkern_status wkern_set_variant(wkern_plan_t plan, int32_t variant);

/* Re-split the batch into `chunks` pipeline chunks of about equal cache
 * size (clamped to the number of planes; 1 = the stages run one after the
 * other on the caller's stream).  Synchronous: waits for the plan's device
 * first.  Errors: INVALID_ARG (chunks < 1), DEVICE, OUT_OF_MEMORY. */
wkern_status wkern_set_chunks(wkern_plan_t plan, int32_t chunks);

/* Device status word of the plan: waits for `stream`, reads the word, and
 * clears it.  WKERN_OK: no flag since the last read.  WKERN_ERR_NONFINITE: a
 * generating call since then produced a non-finite radial-line value; the
 * detail (wkern_last_error) names the first affected plane in caller order,
 * and the affected planes' caches are unspecified.  With canaries on
 * (WKERN_CANARY) it first waits for the whole device and checks every guard
 * band: DEVICE, with the buffer named, if one changed (the band is refilled,
 * so the next read reports later overruns only).  Not allowed while
 * `stream` is being captured (INVALID_ARG).  Errors: INVALID_ARG, DEVICE. */
wkern_status wkern_sync_status(wkern_plan_t plan, void* stream);

/* Release the plan and everything it owns.  Synchronises the plan's device
 * first.  NULL is accepted and ignored.  With canaries on (WKERN_CANARY at
 * plan creation) the guard bands are checked first: DEVICE, with the buffer
 * named, if one changed; the plan is released all the same. */
wkern_status wkern_destroy(wkern_plan_t plan);

/* Static description of a status code. */
const char* wkern_strerror(wkern_status s);

/* Detail of the last error on the calling thread ("" if none). */
const char* wkern_last_error(void);

/* ---------------------------------------------------------------------------
 * Comparison path: the standard algorithm (section 3, Algorithm 1).  For
 * each plane the IAA-kernel times the w-kernel on an N x N image-domain
 * workspace, zero padded by the oversampling factor to L = os N, a 2D FFT
 * (rocFFT through hipFFT, FP32) and extraction of the kernel cache, with the
 * same output layout, sample offsets and circular support as wkern_generate.
 * Workspace undersampling (section 4.2): N is a power of two at or above
 * the kernel's full width.  The taper samples at r_i are interpolated
 * linearly in r onto the workspace pixels; pixels outside the open disc
 * r < r_max are zero.  It is kept beside the Hankel path to be timed
 * against it; it is not the method this library accelerates.
 * ------------------------------------------------------------------------- */
typedef struct wkern_fft2d_s* wkern_fft2d_t;

/* workspace_mode 0: one N for all planes, the power of two at or above
 * max_support (the setting the paper's imager used, sections 5 and 6.4);
 * 1: per plane, the power of two at or above S_p.  workspace_bytes: device
 * memory for batched transforms (<= 0: 2 GiB); planes are transformed in
 * batches that fit it.  Uses d's geometry, supports and device; precision
 * and interp are ignored.  Errors: INVALID_ARG, UNSUPPORTED (L > 16384),
 * DEVICE, OUT_OF_MEMORY. */
wkern_status wkern_fft2d_plan(const wkern_desc* d, int32_t workspace_mode,
                              int64_t workspace_bytes, wkern_fft2d_t* out);

/* Same arguments and output as wkern_generate.  Asynchronous on `stream`. */
wkern_status wkern_fft2d_generate(wkern_fft2d_t plan, const float* taper, const double* w,
                                  void* out, void* stream);

/* Release the comparison plan (synchronises its device first). */
wkern_status wkern_fft2d_destroy(wkern_fft2d_t plan);

/* -------------------------------------------------------------------------
 * w-plane partition of visibility records: the first three steps of
 * Algorithm 2 (sort by increasing absolute w-term, divide into M equally
 * sized w-planes, average or median w-term per plane; Algorithm 1 is the
 * same with signed w).  The plane w-terms come back in device memory, ready
 * to be passed as `w` to wkern_generate / wkern_generate_truncated.
 *
 * Conventions: plane m holds the sorted positions
 * [floor(m n / M), floor((m + 1) n / M)); records with equal keys keep their
 * input order (stable); -0.0 sorts as +0.0 and every NaN after all numbers.
 * With absolute = 1 the key and the statistic are |w| (a record with w < 0
 * is gridded with the conjugate kernel, section 4.1); with absolute = 0 they
 * are w.  The mean sums in a fixed order (bit-reproducible); the median of
 * an even count is the mean of the two middle values.
 * ------------------------------------------------------------------------- */
typedef enum { WKERN_WSTAT_MEAN = 0, WKERN_WSTAT_MEDIAN = 1 } wkern_wstat;

/* Device workspace wkern_wpartition needs for n_records records on the
 * current device.  Errors: INVALID_ARG, UNSUPPORTED (n_records > 2^31 - 1),
 * DEVICE. */
wkern_status wkern_wpartition_workspace(int64_t n_records, size_t* bytes);

/* w:           device double [n_records], w-terms in wavelengths.
 * n_planes:    M, 1 <= M <= n_records.
 * absolute:    1: Algorithm 2 (|w|); 0: Algorithm 1 (signed w).
 * stat:        WKERN_WSTAT_MEAN or WKERN_WSTAT_MEDIAN.
 * workspace:   caller-owned device memory of at least
 *              wkern_wpartition_workspace(n_records) bytes, 256-byte aligned;
 *              its contents are scratch.
 * order:       device int32 [n_records] (written): record indices in sorted
 *              order; plane m's records are order[plane_start[m] ..
 *              plane_start[m + 1] - 1].
 * plane_start: device int64 [M + 1] (written).
 * w_plane:     device double [M] (written): the plane w-terms (|w| when
 *              absolute = 1).
 * Asynchronous on `stream`; allocates nothing.  Errors: INVALID_ARG (NULL
 * pointer, M out of range, short or misaligned workspace), UNSUPPORTED
 * (n_records > 2^31 - 1), DEVICE. */
wkern_status wkern_wpartition(const double* w, int64_t n_records, int32_t n_planes,
                              int32_t absolute, int32_t stat, void* workspace,
                              size_t workspace_bytes, int32_t* order, int64_t* plane_start,
                              double* w_plane, void* stream);

/* -------------------------------------------------------------------------
 * Diagnostics.
 * ------------------------------------------------------------------------- */

/* Store ceiling of the device, for comparison with the resample's HBM write
 * rate (its bound): writes `bytes` of zeros to buf (device, 16-byte aligned,
 * bytes a positive multiple of 16) in one of the store structures a kernel
 * writer can take.  pattern 0: one 16-byte store per lane, after which the
 * wave ends (blocks of 256 lanes in address order; the fastest plain-store
 * structure measured on this device); pattern 1: the resample's structure, a
 * block of 256 lanes walking a 256 KB unit in 4 KB steps, the units dealt
 * to the XCDs in runs of 64.  Asynchronous on
 * `stream`.  Errors: INVALID_ARG, DEVICE. */
wkern_status wkern_store_ceiling(void* buf, int64_t bytes, int32_t pattern, void* stream);

/* wkern_wpartition without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the keys, record indices and sort storage live in
 * a static 64 MiB device array of the library, held on each device it runs on
 * until the process ends; nothing is allocated.  Same arguments, results and
 * errors as wkern_wpartition minus the workspace, on the current device;
 * additionally INVALID_ARG for n_records above 2^20 (1048576), the most the
 * array holds.  Every call on a device shares that device's array: calls
 * that overlap in time on one device (other streams, other threads) race
 * and must be serialised by the caller.  Asynchronous on `stream`. */
wkern_status wkern_wpartition_noalloc(const double* w, int64_t n_records, int32_t n_planes,
                                      int32_t absolute, int32_t stat, int32_t* order,
                                      int64_t* plane_start, double* w_plane, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* WKERN_H */
