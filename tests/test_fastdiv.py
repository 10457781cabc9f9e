"""The kernels' division by run-time constants (multiply-high and shift, as
built by make_fastdiv) against plain integer division, on the host: every
divisor up to 4096 and a spread of large ones, numerators at and around every
multiple boundary they can meet plus the largest supported numerator.  The
same for the remainder of make_fastmod / fmod32, whose numerators span all
32 bits and whose divisors reach 2^32 - 1."""
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


PROG_MOD = r"""
#include <cstdint>
#include <cstdio>
#include "hf_device.hpp"
using namespace hf;
static int check(uint32_t d, uint32_t n) {
  const FastMod f = make_fastmod(d);
  if (fmod32(n, f) != n % d) { std::printf("FAIL d=%u n=%u got %u\n", d, n, fmod32(n, f)); return 1; }
  return 0;
}
static int around(uint32_t d, uint64_t m) {
  int bad = 0;
  for (int e = -2; e <= 2; ++e) {
    const int64_t n = (int64_t)m + e;
    if (n >= 0 && n <= 0xFFFFFFFFll) bad |= check(d, (uint32_t)n);
  }
  return bad;
}
int main() {
  int bad = 0;
  for (uint32_t d = 1; d <= 4096 && !bad; ++d) {
    for (uint32_t n = 0; n < 3 * d + 5; ++n) bad |= check(d, n);
    for (uint64_t q = 1; q * d <= 0xFFFFFFFFull; q = q * 3 + 1) bad |= around(d, q * d);
    const uint64_t top = 0xFFFFFFFFull / d * d;  // the largest multiple below 2^32
    bad |= around(d, top);
    bad |= check(d, 0xFFFFFFFFu);
  }
  const uint32_t big[] = {4097u, 4099u, 65535u, 65536u, 65537u, 1000003u, 8388608u, 16777216u, 16777217u,
                          0x3FFFFFFFu, 0x40000000u, 0x7FFFFFFFu, 0x80000000u, 0x80000001u, 0xAAAAAAABu,
                          0xFFFFFFFEu, 0xFFFFFFFFu};
  for (uint32_t d : big) {
    for (uint32_t n = 0; n < 1000; ++n) bad |= check(d, n);
    for (uint64_t m = d; m <= 0xFFFFFFFFull; m += (m / 7 + 1) * (uint64_t)d) bad |= around(d, m);
    bad |= around(d, 0xFFFFFFFFull / d * d);
    bad |= check(d, 0xFFFFFFFFu);
  }
  // a pseudo-random spread of divisors and numerators (xorshift32)
  uint32_t x = 2463534242u;
  for (int i = 0; i < 2000000 && !bad; ++i) {
    x ^= x << 13; x ^= x >> 17; x ^= x << 5;
    uint32_t d = x >> (x & 31);
    if (d == 0) d = 1;
    x ^= x << 13; x ^= x >> 17; x ^= x << 5;
    bad |= check(d, x);
  }
  std::printf("%s\n", bad ? "FAIL" : "OK");
  return bad;
}
"""


def test_fastmod_matches_integer_remainder():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "fm.hip")
        exe = os.path.join(d, "fm")
        open(src, "w").write(PROG_MOD)
        subprocess.check_call(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "--offload-arch=gfx950",
                               "-I", os.path.join(ROOT, "paper_2007_01277_amd", "csrc"), src, "-o", exe])
        out = subprocess.run([exe], capture_output=True, text=True)
        assert out.returncode == 0 and out.stdout.startswith("OK"), out.stdout
