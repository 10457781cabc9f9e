"""The kernels' division by run-time constants (multiply-high and shift, as
built by make_fastdiv) against plain integer division, on the host: every
divisor up to 4096 and a spread of large ones, numerators at and around every
multiple boundary they can meet plus the largest supported numerator."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROG = r"""
#include <cstdint>
#include <cstdio>
#include "hf_device.hpp"
using namespace hf;
static int check(uint32_t d, uint32_t n) {
  const FastDiv f = make_fastdiv(d);
  if (fdiv(n, f) != n / d) { std::printf("FAIL d=%u n=%u got %u\n", d, n, fdiv(n, f)); return 1; }
  return 0;
}
int main() {
  const uint32_t nmax = 0x7FFFFFFFu;
  int bad = 0;
  uint64_t checked = 0;
  for (uint32_t d = 1; d <= 4096 && !bad; ++d) {
    for (uint32_t n = 0; n < 3 * d + 5; ++n) { bad |= check(d, n); ++checked; }
    for (uint64_t q = 1; q * d <= nmax && !bad; q = q * 3 + 1) {
      const uint64_t m = q * d;
      for (int e = -2; e <= 2; ++e) {
        const int64_t n = (int64_t)m + e;
        if (n >= 0 && n <= nmax) { bad |= check(d, (uint32_t)n); ++checked; }
      }
    }
    bad |= check(d, nmax);
  }
  const uint32_t big[] = {4097u, 65535u, 65536u, 65537u, 3136u * 64u, 1000003u, 16777216u, 16777217u,
                          0x3FFFFFFFu, 0x40000000u, 0x40000001u, 0x7FFFFFFEu, 0x7FFFFFFFu};
  for (uint32_t d : big) {
    for (uint32_t n = 0; n < 1000; ++n) bad |= check(d, n);
    for (uint64_t m = d; m <= nmax; m += (m / 7 + 1) * (uint64_t)d) {
      for (int e = -1; e <= 1; ++e) {
        const int64_t n = (int64_t)m + e;
        if (n >= 0 && n <= nmax) bad |= check(d, (uint32_t)n);
      }
    }
    bad |= check(d, nmax);
  }
  std::printf("%s %llu\n", bad ? "FAIL" : "OK", (unsigned long long)checked);
  return bad;
}
"""


def test_fastdiv_matches_integer_division():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "fd.hip")
        exe = os.path.join(d, "fd")
        open(src, "w").write(PROG)
        # built like the library (host and gfx950 device code); only host code runs
        subprocess.check_call(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "--offload-arch=gfx950",
                               "-I", os.path.join(ROOT, "paper_2007_01277_amd", "csrc"), src, "-o", exe])
        out = subprocess.run([exe], capture_output=True, text=True)
        assert out.returncode == 0 and out.stdout.startswith("OK"), out.stdout
