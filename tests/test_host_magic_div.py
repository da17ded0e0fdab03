"""The multiply-shift division the resample decodes with (magic_div24 in
the library's resample tables): x / d == umulhi(x, m) >> sh for every
0 <= x < 2^24 and 2 <= d <= 4095 (the widths and oversampling factors a plan
accepts).  Checked exactly by a host program: every divisor at every
multiple boundary (k d - 1, k d) up to 2^24, at the top of the range and at
random points, and a few divisors over every x."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PROGRAM = r"""
#include <cstdio>
#include <cstdint>
#include <random>
#include "wkern_tables.h"
using wkern::magic_div24;
static inline uint32_t q_of(uint32_t x, uint32_t m, int sh) {
  return (uint32_t)(((uint64_t)x * m) >> 32) >> sh;
}
int main() {
  const uint32_t top = 1u << 24;
  std::mt19937 rng(1904);
  long checks = 0;
  for (uint32_t d = 2; d <= 4095; ++d) {
    uint32_t m; int32_t sh;
    magic_div24(d, m, sh);
    auto check = [&](uint32_t x) {
      ++checks;
      if (q_of(x, m, sh) != x / d) { std::printf("FAIL d=%u x=%u\n", d, x); return false; }
      return true;
    };
    for (uint32_t k = d; k < top; k += d)
      if (!check(k - 1) || !check(k)) return 1;
    for (uint32_t x = top - 1; x > top - 2 * d; --x)
      if (!check(x)) return 1;
    for (int i = 0; i < 2000; ++i)
      if (!check(rng() % top)) return 1;
  }
  for (uint32_t d : {3u, 7u, 8u, 255u, 4095u}) {
    uint32_t m; int32_t sh;
    magic_div24(d, m, sh);
    for (uint32_t x = 0; x < top; ++x)
      if (q_of(x, m, sh) != x / d) { std::printf("FAIL d=%u x=%u\n", d, x); return 1; }
    checks += top;
  }
  std::printf("ok %ld\n", checks);
  return 0;
}
"""


def test_magic_division_exact():
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    cc = HIPCC if os.path.exists(HIPCC) else shutil.which("hipcc")
    with tempfile.TemporaryDirectory() as tmp:
        src = os.path.join(tmp, "magic.cpp")
        exe = os.path.join(tmp, "magic")
        with open(src, "w") as fh:
            fh.write(PROGRAM)
        inc = os.path.join(ROOT, "paper_1904_08463_amd", "csrc")
        r = subprocess.run([cc, "-O2", "-std=c++17", "-x", "c++", "-D__HIP_PLATFORM_AMD__",
                            "-I/opt/rocm/include", f"-I{inc}", src, "-o", exe],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stdout + r.stderr
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
        assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr
