"""Index division of the kernels (host logic, no GPU): the exact multiply-high
division used for region coordinates (any 32-bit dividend) and the
table-driven one used inside boxes (dividend and divisor below 2^16), compiled
from the library's own header and compared with integer division."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2311_12133_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PROG = r"""
#include <cstdio>
#include <cstdint>
#include "interp_dev.h"
using namespace hpez;
int main() {
  uint64_t bad = 0, checked = 0;
  // exact division: every divisor up to 2^16 against dividends at and around
  // multiples of it, at the top of the 32-bit range and a pseudo-random spread
  uint64_t z = 0x9E3779B97F4A7C15ull;
  for (uint32_t d = 1; d <= 65536; d++) {
    const XDivisor m = xmagic(d);
    const uint32_t top = 0xFFFFFFFFu;
    uint32_t ns[12] = {0u, 1u, d - 1u, d, d + 1u, top, top - 1u, top - (top % d),
                       top - (top % d) - 1u, 0x80000000u, 0x7FFFFFFFu, 16777216u};
    for (int k = 0; k < 12; k++) { checked++; bad += xdiv(ns[k], m) != ns[k] / d; }
    for (int k = 0; k < 64; k++) {
      z ^= z << 13; z ^= z >> 7; z ^= z << 17;
      const uint32_t n = (uint32_t)z;
      checked++; bad += xdiv(n, m) != n / d;
    }
  }
  // large divisors with random dividends
  for (int k = 0; k < 4000000; k++) {
    z ^= z << 13; z ^= z >> 7; z ^= z << 17;
    const uint32_t d = (uint32_t)(z >> 32) | 1u, n = (uint32_t)z;
    checked++; bad += xdiv(n, xmagic(d)) != n / d;
  }
  // the table multipliers: every dividend below 2^16, every divisor in the table
  for (uint32_t d = 2; d <= kMagicMax; d++) {
    const uint32_t m = (uint32_t)(0xFFFFFFFFull / d + 1);
    for (uint32_t n = 0; n < 65536; n++) {
      checked++;
      bad += (uint32_t)(((uint64_t)n * m) >> 32) != n / d;
    }
  }
  printf("%llu %llu\n", (unsigned long long)checked, (unsigned long long)bad);
  return bad != 0;
}
"""


def test_index_division(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    src = tmp_path / "div.cpp"
    src.write_text(PROG)
    exe = tmp_path / "div"
    r = subprocess.run([HIPCC, "-O2", "-std=c++17", "-I", CSRC, "-I",
                        os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    checked, bad = (int(v) for v in out.stdout.split())
    assert checked > 600_000_000 and bad == 0, out.stdout
