/* A plain C99 consumer of the wkern C ABI: no C++, no Python and no torch in
 * the process, only the public header, the HIP runtime's C API and
 * libwkern.so.  tests/test_gpu_c_consumer.py builds it with gcc, writes the
 * problem, runs it and checks what it writes against the FP64 oracle.
 *
 * Usage: wkern_c_consumer <problem file> <result file>
 *
 * Problem file (native byte order):
 *   int32  image_size, n_radial, oversampling, radial_refine, n_planes,
 *          max_support, precision, interp, has_mirror
 *   double cellsize
 *   int32  support[P]
 *   int32  mirror[P]            (only when has_mirror != 0)
 *   float  taper[Nr]
 *   double w[P]
 * Result file:
 *   int64  offsets[P + 1]       (complex elements)
 *   int32  nrho[P]
 *   float  cache[2 offsets[P]]  (re, im of every element, from wkern_generate)
 *   double lines[2 sum nrho]    (re, im of every radial node, from
 *                                wkern_generate_radial)
 *
 * Besides the result it checks, and reports through its exit status:
 *   - wkern_layout_desc (host only) and wkern_layout of the plan agree;
 *   - a second wkern_generate call (a replay of the captured graph) writes
 *     the same bytes as the first;
 *   - wkern_sync_status reports no non-finite value;
 *   - a description with n_radial = 0 fails with WKERN_ERR_INVALID_ARG, a
 *     detail string and a NULL plan; wkern_destroy(NULL) is accepted.
 * Exit status 0: every call succeeded and every check held. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "wkern.h"

static int fail_hip(const char* what, hipError_t e) {
  fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
  return 1;
}

static int fail_wk(const char* what, wkern_status s) {
  fprintf(stderr, "%s: %s (%s)\n", what, wkern_strerror(s), wkern_last_error());
  return 1;
}

static int read_all(FILE* f, void* dst, size_t bytes) {
  return fread(dst, 1, bytes, f) == bytes ? 0 : 1;
}

static int write_all(FILE* f, const void* src, size_t bytes) {
  return fwrite(src, 1, bytes, f) == bytes ? 0 : 1;
}

int main(int argc, char** argv) {
  int32_t hdr[9];
  double cellsize = 0.0;
  int32_t *support = NULL, *mirror = NULL, *nrho = NULL;
  float* taper = NULL;
  double* w = NULL;
  int64_t *offsets = NULL, *offsets_desc = NULL;
  float *cache = NULL, *cache2 = NULL;
  double* lines = NULL;
  void *d_taper = NULL, *d_w = NULL, *d_out = NULL, *d_lines = NULL;
  wkern_plan_t plan = NULL;
  wkern_desc d;
  wkern_status s;
  hipError_t e;
  FILE* f;
  int rc = 1, P, Nr, p;
  int64_t total, sum_nrho = 0;

  if (argc != 3) {
    fprintf(stderr, "usage: %s <problem file> <result file>\n", argv[0]);
    return 2;
  }
  f = fopen(argv[1], "rb");
  if (!f || read_all(f, hdr, sizeof(hdr)) || read_all(f, &cellsize, sizeof(cellsize))) {
    fprintf(stderr, "cannot read the problem header from %s\n", argv[1]);
    return 2;
  }
  Nr = hdr[1];
  P = hdr[4];
  if (Nr < 1 || P < 1 || Nr > (1 << 20) || P > (1 << 20)) {
    fprintf(stderr, "problem sizes out of range: Nr %d, P %d\n", Nr, P);
    return 2;
  }
  support = (int32_t*)malloc((size_t)P * sizeof(int32_t));
  mirror = (int32_t*)malloc((size_t)P * sizeof(int32_t));
  nrho = (int32_t*)malloc((size_t)P * sizeof(int32_t));
  taper = (float*)malloc((size_t)Nr * sizeof(float));
  w = (double*)malloc((size_t)P * sizeof(double));
  offsets = (int64_t*)malloc((size_t)(P + 1) * sizeof(int64_t));
  offsets_desc = (int64_t*)malloc((size_t)(P + 1) * sizeof(int64_t));
  if (!support || !mirror || !nrho || !taper || !w || !offsets || !offsets_desc ||
      read_all(f, support, (size_t)P * sizeof(int32_t)) ||
      (hdr[8] && read_all(f, mirror, (size_t)P * sizeof(int32_t))) ||
      read_all(f, taper, (size_t)Nr * sizeof(float)) ||
      read_all(f, w, (size_t)P * sizeof(double))) {
    fprintf(stderr, "cannot read the problem body from %s\n", argv[1]);
    goto done;
  }
  fclose(f);
  f = NULL;

  memset(&d, 0, sizeof(d));
  d.abi_version = WKERN_ABI_VERSION;
  d.image_size = hdr[0];
  d.cellsize = cellsize;
  d.n_radial = Nr;
  d.oversampling = hdr[2];
  d.radial_refine = hdr[3];
  d.n_planes = P;
  d.support = support;
  d.max_support = hdr[5];
  d.precision = (wkern_precision)hdr[6];
  d.interp = (wkern_interp)hdr[7];
  d.device = 0;
  d.mirror = hdr[8] ? mirror : NULL;

  /* the error path of a C caller: an invalid description, no plan */
  {
    wkern_desc bad = d;
    wkern_plan_t none = (wkern_plan_t)&bad; /* must be overwritten with NULL */
    bad.n_radial = 0;
    s = wkern_plan(&bad, &none);
    if (s != WKERN_ERR_INVALID_ARG || none != NULL || wkern_last_error()[0] == '\0') {
      fprintf(stderr, "invalid description: status %d, plan %p, detail '%s'\n", (int)s,
              (void*)none, wkern_last_error());
      goto done;
    }
    if ((s = wkern_destroy(NULL)) != WKERN_OK) {
      fail_wk("wkern_destroy(NULL)", s);
      goto done;
    }
  }

  if ((s = wkern_layout_desc(&d, offsets_desc, NULL)) != WKERN_OK) {
    fail_wk("wkern_layout_desc", s);
    goto done;
  }
  if ((s = wkern_plan(&d, &plan)) != WKERN_OK) {
    fail_wk("wkern_plan", s);
    goto done;
  }
  if ((s = wkern_layout(plan, offsets, nrho)) != WKERN_OK) {
    fail_wk("wkern_layout", s);
    goto done;
  }
  if (memcmp(offsets, offsets_desc, (size_t)(P + 1) * sizeof(int64_t)) != 0) {
    fprintf(stderr, "wkern_layout and wkern_layout_desc disagree\n");
    goto done;
  }
  total = offsets[P];
  for (p = 0; p < P; ++p) sum_nrho += nrho[p];

  if ((e = hipMalloc(&d_taper, (size_t)Nr * sizeof(float))) != hipSuccess ||
      (e = hipMalloc(&d_w, (size_t)P * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&d_out, (size_t)total * 2 * sizeof(float))) != hipSuccess ||
      (e = hipMalloc(&d_lines, (size_t)sum_nrho * 2 * sizeof(double))) != hipSuccess) {
    fail_hip("hipMalloc", e);
    goto done;
  }
  if ((e = hipMemcpy(d_taper, taper, (size_t)Nr * sizeof(float), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(d_w, w, (size_t)P * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess) {
    fail_hip("hipMemcpy to the device", e);
    goto done;
  }
  cache = (float*)malloc((size_t)total * 2 * sizeof(float));
  cache2 = (float*)malloc((size_t)total * 2 * sizeof(float));
  lines = (double*)malloc((size_t)sum_nrho * 2 * sizeof(double));
  if (!cache || !cache2 || !lines) {
    fprintf(stderr, "out of host memory\n");
    goto done;
  }

  /* first call (captures the graph), then a replay; the null stream */
  if ((s = wkern_generate(plan, (const float*)d_taper, (const double*)d_w, d_out, NULL)) !=
      WKERN_OK) {
    fail_wk("wkern_generate", s);
    goto done;
  }
  if ((e = hipMemcpy(cache, d_out, (size_t)total * 2 * sizeof(float), hipMemcpyDeviceToHost)) !=
      hipSuccess) {
    fail_hip("hipMemcpy of the cache", e);
    goto done;
  }
  if ((e = hipMemset(d_out, 0xFF, (size_t)total * 2 * sizeof(float))) != hipSuccess) {
    fail_hip("hipMemset", e);
    goto done;
  }
  if ((s = wkern_generate(plan, (const float*)d_taper, (const double*)d_w, d_out, NULL)) !=
      WKERN_OK) {
    fail_wk("wkern_generate (replay)", s);
    goto done;
  }
  if ((e = hipMemcpy(cache2, d_out, (size_t)total * 2 * sizeof(float), hipMemcpyDeviceToHost)) !=
      hipSuccess) {
    fail_hip("hipMemcpy of the replayed cache", e);
    goto done;
  }
  if (memcmp(cache, cache2, (size_t)total * 2 * sizeof(float)) != 0) {
    fprintf(stderr, "the graph replay wrote different bytes\n");
    goto done;
  }
  if ((s = wkern_generate_radial(plan, (const float*)d_taper, (const double*)d_w, d_lines,
                                 NULL)) != WKERN_OK) {
    fail_wk("wkern_generate_radial", s);
    goto done;
  }
  if ((e = hipMemcpy(lines, d_lines, (size_t)sum_nrho * 2 * sizeof(double),
                     hipMemcpyDeviceToHost)) != hipSuccess) {
    fail_hip("hipMemcpy of the lines", e);
    goto done;
  }
  if ((s = wkern_sync_status(plan, NULL)) != WKERN_OK) {
    fail_wk("wkern_sync_status", s);
    goto done;
  }

  f = fopen(argv[2], "wb");
  if (!f || write_all(f, offsets, (size_t)(P + 1) * sizeof(int64_t)) ||
      write_all(f, nrho, (size_t)P * sizeof(int32_t)) ||
      write_all(f, cache, (size_t)total * 2 * sizeof(float)) ||
      write_all(f, lines, (size_t)sum_nrho * 2 * sizeof(double))) {
    fprintf(stderr, "cannot write %s\n", argv[2]);
    goto done;
  }
  if (fclose(f) != 0) {
    f = NULL;
    fprintf(stderr, "cannot close %s\n", argv[2]);
    goto done;
  }
  f = NULL;
  printf("c consumer: %d planes, %lld cache elements, %lld line nodes\n", P, (long long)total,
         (long long)sum_nrho);
  rc = 0;

done:
  if (f) fclose(f);
  if (plan && (s = wkern_destroy(plan)) != WKERN_OK) rc = fail_wk("wkern_destroy", s);
  if (d_taper) (void)hipFree(d_taper);
  if (d_w) (void)hipFree(d_w);
  if (d_out) (void)hipFree(d_out);
  if (d_lines) (void)hipFree(d_lines);
  free(support);
  free(mirror);
  free(nrho);
  free(taper);
  free(w);
  free(offsets);
  free(offsets_desc);
  free(cache);
  free(cache2);
  free(lines);
  return rc;
}
