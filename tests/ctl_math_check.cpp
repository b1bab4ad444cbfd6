// ctl_math_check.cpp -- accuracy of the controller's double-precision log,
// sine and cosine (paper_2604_27193_amd/csrc/ctl_math.h) over the argument
// ranges that reach them, against the C library's long double functions (64
// significant bits: their own error is about 1/2000 of a double's ulp).
// Built and run by tests/test_ctl_math_host.py on the CPU (the functions are
// __host__ __device__ with explicit fused operations, so the host evaluates
// them bit for bit as the device does).  Prints the largest errors in units
// in the last place of the double result.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>

#include "ctl_math.h"

static double ulp_err(double got, long double ref) {
  const double r = static_cast<double>(ref);
  if (r == 0.0) return got == 0.0 ? 0.0 : INFINITY;
  int e;
  std::frexp(r, &e);  // |r| in [2^(e-1), 2^e): ulp 2^(e-53)
  return static_cast<double>(std::fabs(static_cast<long double>(got) - ref) /
                             std::ldexp(1.0L, e - 53));
}

int main() {
  double el = 0.0, es = 0.0, ec = 0.0;
  double worst_l = 0.0, worst_s = 0.0, worst_c = 0.0;
  auto check_log = [&](double a) {
    const double e = ulp_err(aeb::ctl_log(a), logl(static_cast<long double>(a)));
    if (!(e <= el)) {
      el = e;
      worst_l = a;
    }
  };
  auto check_sincos = [&](double x) {
    double s, c;
    aeb::ctl_sincos(x, &s, &c);
    const double e1 = ulp_err(s, sinl(static_cast<long double>(x)));
    const double e2 = ulp_err(c, cosl(static_cast<long double>(x)));
    if (!(e1 <= es)) {
      es = e1;
      worst_s = x;
    }
    if (!(e2 <= ec)) {
      ec = e2;
      worst_c = x;
    }
  };
  std::mt19937_64 rng(20260415);
  // the generator's uniforms: (k + 1/2) 2^-52, k < 2^52; the smallest and the
  // largest, the neighbourhoods of 1/2, sqrt(1/2) and 1, and random k drawn
  // log-uniformly and uniformly
  const uint64_t top = (uint64_t(1) << 52) - 1;
  auto unit = [](uint64_t k) { return (static_cast<double>(k) + 0.5) * 0x1p-52; };
  for (uint64_t k = 0; k < 4096; ++k) {
    check_log(unit(k));
    check_log(unit(top - k));
    check_log(unit((uint64_t(1) << 51) + k - 2048));
  }
  const double sh = std::sqrt(0.5);
  double y = sh;
  for (int j = 0; j < 4096; ++j) y = std::nextafter(y, 0.0);
  for (int j = 0; j < 8192; ++j, y = std::nextafter(y, 1.0)) check_log(y);
  for (int j = 0; j < 4000000; ++j) {
    const double lg = -52.0 * std::ldexp(static_cast<double>(rng() >> 11), -53);
    check_log(unit(static_cast<uint64_t>(std::ldexp(1.0, 52) * std::exp2(lg)) & top));
    check_log(unit((rng() >> 12) & top));
  }
  // angles 2 pi u: random, and the neighbourhoods of the multiples of pi/4
  // (quadrant switches and zeros of the sine and cosine)
  const double two_pi = 6.283185307179586;
  for (int j = 0; j < 4000000; ++j) check_sincos(two_pi * unit((rng() >> 12) & top));
  for (int q = 0; q <= 8; ++q) {
    double x = static_cast<double>(q * (3.14159265358979323846L / 4.0L));
    for (int j = 0; j < 2048 && x > 0.0; ++j) x = std::nextafter(x, 0.0);
    for (int j = 0; j < 4096; ++j, x = std::nextafter(x, 10.0))
      if (x > 0.0 && x < two_pi) check_sincos(x);
  }
  check_sincos(two_pi * unit(0));
  check_sincos(two_pi * unit(top));
  std::printf("log max ulp %.4f at %a\n", el, worst_l);
  std::printf("sin max ulp %.4f at %a\n", es, worst_s);
  std::printf("cos max ulp %.4f at %a\n", ec, worst_c);
  return 0;
}
