"""The compile-time roots of unity of the mixed-radix register z pass against libm.

The kernel's twiddles cos(2 pi m / N), sin(2 pi m / N) are constant expressions evaluated by
the compiler (reflection to [0, pi/4], then a Taylor series).  This host program evaluates the
same functions for every N <= 512 and every m in [-N, 2N] and compares them with the 80-bit
long-double cosl / sinl.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1903_09802_amd", "csrc")

PROGRAM = r"""
#include "zpass_mr.h"
#include <cmath>
#include <cstdio>
int main() {
  const long double two_pi = 6.283185307179586476925286766559005768L;
  double worst = 0.0;
  int bad_n = 0, bad_m = 0;
  for (int N = 1; N <= 512; ++N)
    for (int m = -N; m <= 2 * N; ++m) {
      const long double a = two_pi * (long double)m / (long double)N;
      const double ec = std::fabs(dda::cx_cos2pi(m, N) - (double)cosl(a));
      const double es = std::fabs(dda::cx_sin2pi(m, N) - (double)sinl(a));
      const double e = ec > es ? ec : es;
      if (e > worst) { worst = e; bad_n = N; bad_m = m; }
    }
  std::printf("%.6e %d %d\n", worst, bad_n, bad_m);
  return 0;
}
"""


def test_compile_time_roots_match_libm(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = tmp_path / "roots.hip"
    src.write_text(PROGRAM)
    exe = tmp_path / "roots"
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", f"-I{CSRC}", str(src), "-o", str(exe)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    worst, n, m = float(out[0]), int(out[1]), int(out[2])
    # a few units in the last place of values of magnitude <= 1
    assert worst < 5e-16, (worst, n, m)
