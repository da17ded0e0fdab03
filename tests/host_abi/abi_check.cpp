// Host-only exercise of the C ABI's validation, layout and error paths, built
// with AddressSanitizer and UndefinedBehaviorSanitizer (see
// tests/test_host_sanitizers.py).  Nothing here reaches a device: every call
// either fails validation or needs no device.  Exit status 0 = all checks
// passed; a sanitizer report aborts with a non-zero status.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "wkern.h"

static int g_failed = 0;

#define CHECK(cond)                                                        \
  do {                                                                     \
    if (!(cond)) {                                                         \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
      ++g_failed;                                                          \
    }                                                                      \
  } while (0)

static wkern_desc base_desc(std::vector<int32_t>& sup) {
  wkern_desc d;
  std::memset(&d, 0, sizeof(d));
  d.abi_version = WKERN_ABI_VERSION;
  d.image_size = 128;
  d.cellsize = 7.8125e-4;
  d.n_radial = 64;
  d.oversampling = 4;
  d.radial_refine = 1;
  d.n_planes = (int32_t)sup.size();
  d.support = sup.data();
  d.max_support = 31;
  d.precision = WKERN_PREC_BF16X6;
  d.interp = WKERN_INTERP_CUBIC;
  d.device = 0;
  d.mirror = nullptr;
  return d;
}

// Layout of random valid descriptions against a prefix sum computed here.
static void random_layouts() {
  std::mt19937 rng(1904);
  for (int trial = 0; trial < 400; ++trial) {
    const int os = 1 + (int)(rng() % 16);
    const int q = 1 + (int)(rng() % 4);
    int maxS = 1 + 2 * (int)(rng() % 64);
    while (os * maxS > 4096 || q * os * ((maxS - 1) / 2) + 4 > 2048) maxS -= 2;
    const int P = 1 + (int)(rng() % 300);
    std::vector<int32_t> sup(P), mir(P, -1);
    for (int p = 0; p < P; ++p) sup[p] = 1 + 2 * (int)(rng() % ((maxS + 1) / 2));
    // mirror some planes onto earlier planes of the same support
    for (int p = 1; p < P; ++p)
      if (rng() % 4 == 0) {
        const int src = (int)(rng() % p);
        if (mir[src] == -1) {
          mir[p] = src;
          sup[p] = sup[src];
        }
      }
    wkern_desc d = base_desc(sup);
    d.oversampling = os;
    d.radial_refine = q;
    d.max_support = maxS;
    d.mirror = mir.data();
    std::vector<int64_t> offs(P + 1, -1);
    std::vector<int32_t> nrho(P, -1);
    CHECK(wkern_layout_desc(&d, offs.data(), nrho.data()) == WKERN_OK);
    int64_t acc = 0;
    for (int p = 0; p < P; ++p) {
      CHECK(offs[p] == acc);
      CHECK(nrho[p] == q * os * ((sup[p] - 1) / 2) + 4);
      acc += (int64_t)os * os * sup[p] * sup[p];
    }
    CHECK(offs[P] == acc);
    // NULL nrho is allowed
    CHECK(wkern_layout_desc(&d, offs.data(), nullptr) == WKERN_OK);
  }
}

// Each invalid field: INVALID_ARG (or ABI_MISMATCH), a detail string, and
// wkern_plan leaves *out NULL without touching a device.
static void invalid_descriptions() {
  std::vector<int32_t> sup = {7, 9, 31};
  struct Bad {
    const char* what;
    void (*apply)(wkern_desc&, std::vector<int32_t>&, std::vector<int32_t>&);
    wkern_status expect;
  };
  const Bad bad[] = {
      {"abi", [](wkern_desc& d, auto&, auto&) { d.abi_version = 1; }, WKERN_ERR_ABI_MISMATCH},
      {"image_size", [](wkern_desc& d, auto&, auto&) { d.image_size = 0; }, WKERN_ERR_INVALID_ARG},
      {"cellsize", [](wkern_desc& d, auto&, auto&) { d.cellsize = -1.0; }, WKERN_ERR_INVALID_ARG},
      {"r_max", [](wkern_desc& d, auto&, auto&) { d.cellsize = 0.02; }, WKERN_ERR_INVALID_ARG},
      {"n_radial", [](wkern_desc& d, auto&, auto&) { d.n_radial = 0; }, WKERN_ERR_INVALID_ARG},
      {"os", [](wkern_desc& d, auto&, auto&) { d.oversampling = 65; }, WKERN_ERR_INVALID_ARG},
      {"q", [](wkern_desc& d, auto&, auto&) { d.radial_refine = 0; }, WKERN_ERR_INVALID_ARG},
      {"planes", [](wkern_desc& d, auto&, auto&) { d.n_planes = 0; }, WKERN_ERR_INVALID_ARG},
      {"support", [](wkern_desc& d, auto&, auto&) { d.support = nullptr; }, WKERN_ERR_INVALID_ARG},
      {"even", [](wkern_desc&, auto& s, auto&) { s[1] = 8; }, WKERN_ERR_INVALID_ARG},
      {"large", [](wkern_desc&, auto& s, auto&) { s[2] = 33; }, WKERN_ERR_INVALID_ARG},
      {"maxS", [](wkern_desc& d, auto&, auto&) { d.max_support = 30; }, WKERN_ERR_INVALID_ARG},
      {"os*S", [](wkern_desc& d, auto&, auto&) { d.oversampling = 64; d.max_support = 65; },
       WKERN_ERR_INVALID_ARG},
      {"precision", [](wkern_desc& d, auto&, auto&) { d.precision = (wkern_precision)9; },
       WKERN_ERR_INVALID_ARG},
      {"interp", [](wkern_desc& d, auto&, auto&) { d.interp = (wkern_interp)9; },
       WKERN_ERR_INVALID_ARG},
      {"mirror self", [](wkern_desc& d, auto&, auto& m) { m[1] = 1; d.mirror = m.data(); },
       WKERN_ERR_INVALID_ARG},
      {"mirror range", [](wkern_desc& d, auto&, auto& m) { m[1] = 3; d.mirror = m.data(); },
       WKERN_ERR_INVALID_ARG},
      {"mirror chain", [](wkern_desc& d, auto& s, auto& m) {
         s[1] = s[0]; s[2] = s[0]; m[1] = 0; m[2] = 1; d.mirror = m.data(); },
       WKERN_ERR_INVALID_ARG},
      {"mirror support", [](wkern_desc& d, auto&, auto& m) { m[2] = 0; d.mirror = m.data(); },
       WKERN_ERR_INVALID_ARG},
  };
  for (const Bad& b : bad) {
    std::vector<int32_t> s = sup, m(sup.size(), -1);
    wkern_desc d = base_desc(s);
    b.apply(d, s, m);
    int64_t offs[4];
    const wkern_status st = wkern_layout_desc(&d, offs, nullptr);
    if (st != b.expect) std::fprintf(stderr, "case %s: status %d\n", b.what, (int)st);
    CHECK(st == b.expect);
    CHECK(std::strlen(wkern_last_error()) > 0);
    wkern_plan_t plan = (wkern_plan_t)0x1;
    CHECK(wkern_plan(&d, &plan) == b.expect);
    CHECK(plan == nullptr);
  }
  CHECK(wkern_layout_desc(nullptr, nullptr, nullptr) == WKERN_ERR_INVALID_ARG);
  std::vector<int32_t> s = sup;
  wkern_desc d = base_desc(s);
  CHECK(wkern_layout_desc(&d, nullptr, nullptr) == WKERN_ERR_INVALID_ARG);
  CHECK(wkern_plan(&d, nullptr) == WKERN_ERR_INVALID_ARG);
}

// Every entry point that takes a plan refuses NULL before anything else.
static void null_plan() {
  float f = 0.f;
  double x = 0.0;
  int32_t i = 0;
  int64_t l = 0;
  char buf[16];
  const wkern_status inv = WKERN_ERR_INVALID_ARG;
  CHECK(wkern_layout(nullptr, &l, &i) == inv);
  CHECK(wkern_generate(nullptr, &f, &x, buf, nullptr) == inv);
  CHECK(wkern_generate_truncated(nullptr, &f, &x, 0.01, buf, 1, &i, &l, nullptr) == inv);
  CHECK(wkern_generate_radial(nullptr, &f, &x, buf, nullptr) == inv);
  CHECK(wkern_grad(nullptr, &f, &x, buf, &f, &x, nullptr) == inv);
  CHECK(wkern_prepare_lines(nullptr, &f, &x, 0.0, &i, nullptr) == inv);
  CHECK(wkern_grid(nullptr, &x, &x, &x, buf, 1, &i, &l, &i, nullptr, nullptr, 2, buf, nullptr) ==
        inv);
  CHECK(wkern_set_engine(nullptr, 0, 0) == inv);
  CHECK(wkern_set_profiling(nullptr, 1) == inv);
  double ms[4];
  CHECK(wkern_stage_times(nullptr, ms, &i) == inv);
  float vms[16];
  CHECK(wkern_plan_info(nullptr, &i, &i, vms, &i) == inv);
  CHECK(wkern_set_graph(nullptr, 1) == inv);
  CHECK(wkern_set_variant(nullptr, 0) == inv);
  CHECK(wkern_set_chunks(nullptr, 1) == inv);
  CHECK(wkern_sync_status(nullptr, nullptr) == inv);
  CHECK(wkern_destroy(nullptr) == WKERN_OK);
}

static void strings() {
  for (int s = 0; s <= 7; ++s) {
    const char* t = wkern_strerror((wkern_status)s);
    CHECK(t != nullptr && std::strlen(t) > 0);
  }
  CHECK(std::strcmp(wkern_strerror(WKERN_ERR_NONFINITE), "unknown status") != 0);
  CHECK(wkern_abi_version() == WKERN_ABI_VERSION);
  // a successful call clears the detail string
  std::vector<int32_t> s = {5};
  wkern_desc d = base_desc(s);
  int64_t offs[2];
  CHECK(wkern_layout_desc(nullptr, offs, nullptr) == WKERN_ERR_INVALID_ARG);
  CHECK(std::strlen(wkern_last_error()) > 0);
  CHECK(wkern_layout_desc(&d, offs, nullptr) == WKERN_OK);
  CHECK(std::strlen(wkern_last_error()) == 0);
}

int main() {
  random_layouts();
  invalid_descriptions();
  null_plan();
  strings();
  if (g_failed) {
    std::fprintf(stderr, "%d checks failed\n", g_failed);
    return 1;
  }
  std::printf("host ABI checks passed\n");
  return 0;
}
