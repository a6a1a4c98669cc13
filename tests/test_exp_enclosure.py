"""The FP64 exp enclosure of the pixel kernels, compiled for the host from the same
header, checked against long double references (x86 80-bit, 64-bit mantissa).

Pins (Table "Bounds for operations Exp, Div and Ind" needs e_dn <= exp(x) <= e_up and
an upper bound of the chord slope): dn <= exp(x) <= up with relative width <= 2^-42 for
x >= -700 (each side 2^-44 from the computed value), the [0, 2^-1000] enclosure below; (e^h - 1)/h <= phi with relative excess
<= 2^-43 on [0, 1/2]; exact values at 0.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2503_00308_amd", "csrc", "ar_expm.h")

PROG = r"""
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <random>
using std::fma; using std::fmax; using std::fabs; using std::rint; using std::ldexp;
#define AR_HD inline
#include "ar_expm.h"
static const double tab[ar::kExpTableLen] = AR_EXP_TABLE;
int main() {
  std::mt19937_64 g(12345);
  std::uniform_real_distribution<double> ux(-745.0, 20.0), us(-1.0, 1.0), uh(0.0, 0.5);
  long bad = 0; double worst = 0.0, worst_phi = 0.0;
  auto check = [&](double x) {
    double dn, up; ar::exp_encl(x, dn, up, tab);
    long double e = expl((long double)x);
    if (!((long double)dn <= e && e <= (long double)up)) { if (bad < 5) printf("BAD x=%.17g dn=%.17g up=%.17g\n", x, dn, up); ++bad; }
    if (x >= -700.0) { double w = (double)(((long double)up - (long double)dn) / e); if (w > worst) worst = w; }
    else if (!(dn == 0.0 && up == 0x1p-1000)) ++bad;
    double d1, u1, d2, u2, phi;
    ar::exp_triple(x, x * 0.5, 0.0, d1, u1, d2, u2, phi, tab);
    if (d1 != dn || u1 != up) ++bad;
  };
  for (long i = 0; i < 3000000; ++i) check(ux(g));
  for (long i = 0; i < 1000000; ++i) check(us(g));
  const double edge[] = {0.0, -0.0, -1e-300, -0x1p-1074, -0.34657359027997264, -0.3465735902799727,
                         -700.0, -700.0000000000001, -708.3, -744.9, -745.0, -746.0, -1e6, 1.0, 5.0};
  for (double x : edge) check(x);
  for (long i = 0; i < 1000000; ++i) {
    double h = (i == 0) ? 0.0 : (i == 1 ? 0.5 : uh(g));
    double phi = ar::expm1_over_x_up(h, tab);
    long double t = (h == 0.0) ? 1.0L : expm1l((long double)h) / (long double)h;
    if (!((long double)phi >= t)) { if (bad < 5) printf("BAD phi h=%.17g\n", h); ++bad; }
    double ex = (double)(((long double)phi - t) / t); if (ex > worst_phi) worst_phi = ex;
    double d1, u1, d2, u2, p3; ar::exp_triple(-1.0, -2.0, h, d1, u1, d2, u2, p3, tab);
    if (p3 != phi) ++bad;
  }
  printf("bad %ld worst_width %.3e worst_phi_excess %.3e\n", bad, worst, worst_phi);
  return bad != 0;
}
"""


def test_exp_enclosure_against_long_double(tmp_path):
    src = tmp_path / "t.cpp"
    src.write_text(PROG)
    exe = tmp_path / "t"
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-I", os.path.dirname(HDR), str(src),
                    "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    last = r.stdout.strip().splitlines()[-1].split()
    assert float(last[3]) <= 2.0 ** -42   # dn, up are each 2^-44 from the value
    assert float(last[5]) <= 2.0 ** -43
