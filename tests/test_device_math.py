"""CPU check of the device-side FP64 exponential of the stage epilogues
(`exp_nonpos` in csrc/kernels_common.hpp, a host-and-device function): built
for the host with hipcc from the library's own header and compared with the C
library's exp on 400k points of [-760, 0] (the Maxwellian's arguments, section
3.4) and on the special values. Skipped where hipcc is absent."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2103_14890_amd", "csrc")

PROGRAM = r"""
#include <cmath>
#include <cstdio>
#include <random>
#include "kernels_common.hpp"
int main() {
  const double c[17] = QCOLL_EXP_CONSTANTS;
  std::mt19937_64 g(7);
  std::uniform_real_distribution<double> wide(-760.0, 0.0), near(-5.0, 0.0);
  double worst = 0.0;
  long bad_sub = 0;
  for (int i = 0; i < 400000; ++i) {
    const double x = (i & 1) ? wide(g) : near(g);
    const double a = qcoll::exp_nonpos(x, c), b = std::exp(x);
    if (b < 2.2250738585072014e-308) {            // subnormal or zero results: absolute error
      if (std::fabs(a - b) > 4 * 4.9406564584124654e-324) ++bad_sub;
      continue;
    }
    const double rel = std::fabs(a - b) / b;
    if (rel > worst) worst = rel;
  }
  std::printf("%.6e %ld %.17g %.17g %d %.17g\n", worst, bad_sub, qcoll::exp_nonpos(0.0, c),
              qcoll::exp_nonpos(-1.0, c) - std::exp(-1.0), std::isnan(qcoll::exp_nonpos(NAN, c)) ? 1 : 0,
              qcoll::exp_nonpos(-800.0, c));
  return 0;
}
"""


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_exp_nonpos_matches_libm(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    src = tmp_path / "exp_check.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "exp_check"
    subprocess.run([hipcc, "-O2", "-std=c++17", f"-I{CSRC}", f"-I{os.path.join(ROOT, 'include')}", str(src), "-o",
                    str(exe)], check=True, capture_output=True, timeout=300)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=60).stdout.split()
    worst, bad_sub, at0, dm1, isnan, big = float(out[0]), int(out[1]), float(out[2]), float(out[3]), int(out[4]), \
        float(out[5])
    assert worst <= 4 * 2.0 ** -53, worst          # within 4 units in the last place
    assert bad_sub == 0
    assert at0 == 1.0 and abs(dm1) <= 2 ** -53 and isnan == 1 and big == 0.0
