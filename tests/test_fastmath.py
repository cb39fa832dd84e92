"""Accuracy of the pair kernels' exponential, compiled for the host.

``exp_neg`` is a ``__host__ __device__`` function; the same source is built
here with g++ and compared with the C library's ``exp`` (correctly rounded to
within 1 ulp on glibc) over the argument range the kernels see.
"""
import os
import subprocess
import tempfile

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2210_03699_amd", "csrc")

SRC = r"""
#include <cstdio>
#include <cmath>
#include <cstdlib>
#include "fastmath.h"
int main(int argc, char** argv) {
  double worst = 0, worst_x = 0;
  long n = 2000000;
  for (long i = 0; i <= n; ++i) {
    double x = 60.0 * (double)i / n;           // kappa R up to 60
    double a = ibim::exp_neg(x), b = std::exp(-x);
    double rel = std::fabs(a - b) / b;
    if (rel > worst) { worst = rel; worst_x = x; }
  }
  // exact points
  std::printf("%.3e %.17g %.17g %.17g\n", worst, worst_x, ibim::exp_neg(0.0), ibim::exp_neg(800.0));
  return 0;
}
"""


def test_exp_neg_relative_error():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.cpp")
        exe = os.path.join(d, "t")
        open(src, "w").write(SRC)
        subprocess.run(["g++", "-O2", "-std=c++17", "-mfma", "-I", HDR, src, "-o", exe],
                       check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    worst = float(out[0])
    assert worst < 4e-16, out          # a few ulp
    assert float(out[2]) == 1.0        # e^0
    assert float(out[3]) == 0.0        # underflow
