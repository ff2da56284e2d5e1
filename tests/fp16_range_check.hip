// Host-side check of the FP16 storage test of the block multipliers
// (segprec.h: lfits, lnarrow): every multiplier accepted by lfits narrows to
// a finite FP16 value within half an FP16 ulp, and the values at and beyond
// the range edge (and non-finite ones) are refused.  Built for the host only
// by tests/test_fp16_range.py; prints one line per failure, exits 1 on any.
#include <cmath>
#include <cstdio>
#include <random>

#include "segprec.h"

using vdc::c16;
using vdc::c64;

static int fails = 0;

static void expect(bool ok, const char* what, double re, double im) {
  if (!ok) {
    std::printf("FAIL %s at (%.17g, %.17g)\n", what, re, im);
    ++fails;
  }
}

// |x - fp16(x)| allowed by round-to-nearest: half an ulp of x (normal range)
// or half the smallest subnormal spacing below 2^-14.
static double half_ulp(double x) {
  const double a = std::fabs(x);
  if (a < 6.103515625e-05) return 0.5 * 5.9604644775390625e-08;
  int e;
  std::frexp(a, &e);                 // a = m 2^e, m in [0.5, 1)
  return std::ldexp(1.0, e - 1 - 10) * 0.5;
}

int main() {
  const double edge[][2] = {{6.0e4, 0.0}, {0.0, 6.0e4}, {-6.0e4, 1.0}, {1.0, -6.0e4},
                            {65504.0, 0.0}, {7.0e4, 7.0e4}, {NAN, 0.0}, {0.0, INFINITY}};
  for (const auto& v : edge) expect(!vdc::lfits<float>(c64{v[0], v[1]}), "accepted", v[0], v[1]);
  for (const auto& v : edge) expect(vdc::lfits<double>(c64{v[0], v[1]}), "FP64 refused", v[0], v[1]);
  const double inside[][2] = {{59999.99, -59999.99}, {0.0, 0.0}, {1e-9, -1e-9}, {1.0, 0.5}};
  std::mt19937_64 rng(7);
  std::uniform_real_distribution<double> lg(-9.0, std::log10(59999.99));
  std::uniform_int_distribution<int> sg(0, 1);
  for (int k = 0; k < 200004; ++k) {
    double re, im;
    if (k < 4) {
      re = inside[k][0];
      im = inside[k][1];
    } else {
      re = (sg(rng) ? 1 : -1) * std::pow(10.0, lg(rng));
      im = (sg(rng) ? 1 : -1) * std::pow(10.0, lg(rng));
    }
    const c64 a{re, im};
    expect(vdc::lfits<float>(a), "refused", re, im);
    const c16 h = vdc::lnarrow<float>(a);
    const double hr = (double)(float)h.x, hi = (double)(float)h.y;
    expect(std::isfinite(hr) && std::isfinite(hi), "non-finite FP16", re, im);
    // narrowing goes through FP32: allow the FP32 rounding on top
    expect(std::fabs(hr - re) <= half_ulp(re) * (1.0 + 1e-6) + std::fabs(re) * 6e-8,
           "real part rounding", re, im);
    expect(std::fabs(hi - im) <= half_ulp(im) * (1.0 + 1e-6) + std::fabs(im) * 6e-8,
           "imaginary part rounding", re, im);
  }
  std::printf("%s (%d failures)\n", fails ? "FAIL" : "OK", fails);
  return fails ? 1 : 0;
}
