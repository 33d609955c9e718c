"""The FP64 arctangent and logarithm the propagation uses (csrc/kfdev.h,
written out so the build kernels hold fewer registers than around the
library routines), checked on the CPU against the host C library: the
arctangent within 8 ulp over arguments spanning 2^-30 .. 2^30 of both signs,
the logarithm within 4 ulp over positive arguments from subnormal to 2^1020,
exact special values.  The header's functions
are __host__ __device__; a host-only compile runs them here."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PROGRAM = r"""
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include "kfdev.h"
static double ulps(double a, double b) {
  if (a == b) return 0;
  int64_t ia, ib;
  memcpy(&ia, &a, 8);
  memcpy(&ib, &b, 8);
  if ((ia < 0) != (ib < 0)) return 1e300;
  return (double)llabs(ia - ib);
}
int main() {
  std::mt19937_64 g(20171106);
  double worst = 0;
  for (int i = 0; i < 2000000; ++i) {
    const double x = std::ldexp(std::uniform_real_distribution<double>(-1, 1)(g),
                                std::uniform_int_distribution<int>(-30, 30)(g));
    const double d = ulps(kfdev::k_atan(x), std::atan(x));
    if (d > worst) worst = d;
  }
  // the reduction boundaries and their neighbours
  const double edges[] = {0.05, 0.1, 0.2, 0.4, 1.0, 20.0};
  for (double e : edges)
    for (int k = -2; k <= 2; ++k) {
      double x = e;
      for (int s = 0; s < (k < 0 ? -k : k); ++s) x = std::nextafter(x, k < 0 ? 0.0 : 1e9);
      const double d = ulps(kfdev::k_atan(x), std::atan(x));
      if (d > worst) worst = d;
    }
  printf("%.0f\n", worst);
  double wl = 0;
  for (int i = 0; i < 2000000; ++i) {
    const double y = std::ldexp(std::uniform_real_distribution<double>(0.5, 1)(g),
                                std::uniform_int_distribution<int>(-1070, 1020)(g));
    const double d = ulps(kfdev::k_log(y), std::log(y));
    if (d > wl) wl = d;
  }
  // the scattering term's range: x/X0 over the incidence times 1/beta^2
  for (int i = 0; i < 200000; ++i) {
    const double y = std::uniform_real_distribution<double>(0.005, 2.0)(g);
    const double d = ulps(kfdev::k_log(y), std::log(y));
    if (d > wl) wl = d;
  }
  printf("%.0f\n", wl);
  printf("%d %d %d %.17g\n", (int)(std::isinf(kfdev::k_log(0.0)) && kfdev::k_log(0.0) < 0),
         (int)std::isnan(kfdev::k_log(-1.0)), (int)std::isinf(kfdev::k_log((double)INFINITY)), kfdev::k_log(1.0));
  printf("%.17g %.17g %d %.17g %.17g %d\n", kfdev::k_atan((double)INFINITY), kfdev::k_atan(-(double)INFINITY),
         (int)std::isnan(kfdev::k_atan((double)NAN)), kfdev::k_atan(0.0), kfdev::k_atan(1.0),
         (int)std::signbit(kfdev::k_atan(-0.0)));
  return 0;
}
"""


@pytest.fixture(scope="module")
def program(tmp_path_factory):
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("kfdev_math")
    src = d / "atan_check.cpp"
    src.write_text(PROGRAM)
    exe = d / "atan_check"
    cmd = [HIPCC, "-O2", "-std=c++17", "--cuda-host-only", "-I", os.path.join(ROOT, "paper_1711_06571_amd", "csrc"),
           "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    return str(exe)


def test_atan_matches_the_host_library(program):
    out = subprocess.run([program], check=True, capture_output=True, text=True).stdout.split("\n")
    worst = float(out[0])
    assert worst <= 8, f"k_atan off by {worst} ulp"
    inf_p, inf_m, nan, zero, one, negzero = out[3].split()
    assert float(inf_p) == 1.5707963267948966 and float(inf_m) == -1.5707963267948966
    assert nan == "1" and float(zero) == 0.0 and negzero == "1"
    assert abs(float(one) - 0.78539816339744831) <= 2e-16


def test_log_matches_the_host_library(program):
    out = subprocess.run([program], check=True, capture_output=True, text=True).stdout.split("\n")
    worst = float(out[1])
    assert worst <= 4, f"k_log off by {worst} ulp"
    neg_inf_at_zero, nan_below_zero, inf_at_inf, log_one = out[2].split()
    assert neg_inf_at_zero == "1" and nan_below_zero == "1" and inf_at_inf == "1" and float(log_one) == 0.0
