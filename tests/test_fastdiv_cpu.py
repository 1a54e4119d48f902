"""Host check of the multiply-and-shift division the grid kernels use for
their index arithmetic (gabp_internal.h: fast_div / fdiv): a small program
built from the library's own header on the host (no GPU) compares it with
the hardware quotient for every divisor up to 4096 against every numerator
below 70000 and random ones up to 2^31 - 1, and for random divisors up to
2^31 - 1."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

PROGRAM = r"""
#include "gabp_internal.h"
#include <cstdio>
#include <random>
using namespace gabp;
int main() {
  std::mt19937_64 rng(1);
  long bad = 0, checked = 0;
  auto check = [&](int n, int d, const FastDiv &f) {
    if (n < 0) return;
    ++checked;
    if (fdiv(n, f) != n / d) ++bad;
  };
  for (int d = 1; d <= 4096; ++d) {
    const FastDiv f = fast_div(d);
    for (int n = 0; n < 70000; ++n) check(n, d, f);
    for (int k = 0; k < 2000; ++k) check((int)(rng() & 0x7fffffff), d, f);
    const int top = 0x7fffffff / d * d;
    check(0x7fffffff, d, f); check(top, d, f); check(top - 1, d, f);
  }
  for (int k = 0; k < 20000; ++k) {
    const int d = 1 + (int)(rng() % 0x7ffffffe);
    const FastDiv f = fast_div(d);
    for (int j = 0; j < 50; ++j) check((int)(rng() & 0x7fffffff), d, f);
    check(d, d, f); check(d - 1, d, f); check(0x7fffffff, d, f);
  }
  std::printf("%ld %ld\n", checked, bad);
  return bad != 0;
}
"""


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_fast_division_equals_integer_division(tmp_path):
    src = tmp_path / "fastdiv.hip"
    src.write_text(PROGRAM)
    exe = tmp_path / "fastdiv"
    subprocess.run([HIPCC, "--offload-host-only", "-std=c++17", "-O2",
                    "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_0810_1119_amd", "csrc"),
                    str(src), "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    checked, bad = int(out[0]), int(out[1])
    assert checked > 290_000_000 and bad == 0
