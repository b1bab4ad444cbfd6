// ctl_math.h -- double-precision natural logarithm, sine and cosine for the
// controller's exact stage decision (the Box-Muller radius and angle of the
// measurement noise, Sec. VIII's controller assessment), written for the
// argument ranges that reach them:
//   ctl_log(a)        a in [2^-53, 1]  (the generator's uniforms)
//   ctl_sincos(x)     x in [0, 2 pi)   (2 pi times a uniform)
// A general-purpose library routine carries a reduction for arguments of any
// size; inlined into the integration kernel its temporaries cost registers,
// and so a wavefront per SIMD, on every step.  These need a few registers.
//
// Methods (textbook, constants derived from pi and ln 2 in exact arithmetic):
//   log:  a = m 2^e with m in [sqrt(1/2), sqrt(2)); log m = 2 atanh(f),
//         f = (m - 1) / (m + 1), |f| <= 0.1716, by its odd series to f^23
//         (next term below 1e-17 relative), arranged so that the exact m - 1
//         leads; e ln 2 with ln 2 split so that e * LN2_HI is exact.
//   sin, cos: x = n pi/2 + r, |r| <= pi/4, n the nearest integer to 2x/pi,
//         r by a three-part pi/2 (each product n * part exact for n <= 4) as
//         a head and a tail; Taylor polynomials of sin r to r^17 and cos r to
//         r^18 (remainders below 1e-19 relative on |r| <= pi/4) with the
//         tail's first-order term; the quadrant n mod 4 selects and signs them.
// Both are accurate to about one unit in the last place (the host test
// measures the largest error against the C library over dense samples of the
// ranges).  Everything is __host__ __device__ with explicit fused operations,
// so host and device give the same bits.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace aeb {

// The constants live in a table read through a volatile pointer at each use,
// inside the rarely taken exact stage: as literals the compiler hoists them
// out of the integration loop and holds them in registers for the whole
// kernel.
namespace ctlm {
constexpr double TAB[] = {
    // 0-2: pi/2 = PIO2_1 + PIO2_2 + PIO2_3 (each product n * part exact for n <= 4)
    0x1.921fb54400000p+0, 0x1.0b4611a600000p-34, 0x1.3198a2e037073p-69,
    // 3: 2/pi; 4, 5: ln 2 = LN2_HI + LN2_LO (e * LN2_HI exact); 6: sqrt(1/2)
    0x1.45f306dc9c883p-1, 0x1.62e42fefa3800p-1, 0x1.ef35793c76730p-45, 0x1.6a09e667f3bccp-1,
    // 7-17: 1/23, 1/21, ..., 1/3 (the atanh series)
    0x1.642c8590b2164p-5, 0x1.8618618618618p-5, 0x1.af286bca1af28p-5, 0x1.e1e1e1e1e1e1ep-5,
    0x1.1111111111111p-4, 0x1.3b13b13b13b14p-4, 0x1.745d1745d1746p-4, 0x1.c71c71c71c71cp-4,
    0x1.2492492492492p-3, 0x1.999999999999ap-3, 0x1.5555555555555p-2,
    // 18-25: 1/17!, -1/15!, 1/13!, ..., -1/3! (sine)
    0x1.952c77030ad4ap-49, -0x1.ae7f3e733b81fp-41, 0x1.6124613a86d09p-33, -0x1.ae64567f544e4p-26,
    0x1.71de3a556c734p-19, -0x1.a01a01a01a01ap-13, 0x1.1111111111111p-7, -0x1.5555555555555p-3,
    // 26-33: -1/18!, 1/16!, ..., 1/4! (cosine)
    -0x1.6827863b97d97p-53, 0x1.ae7f3e733b81fp-45, -0x1.93974a8c07c9dp-37, 0x1.1eed8eff8d898p-29,
    -0x1.27e4fb7789f5cp-22, 0x1.a01a01a01a01ap-16, -0x1.6c16c16c16c17p-10, 0x1.5555555555555p-5};
enum { PIO2_1, PIO2_2, PIO2_3, TWO_OVER_PI, LN2_HI, LN2_LO, SQRT_HALF, LOG_P, SIN_P = 18,
       COS_P = 26, TAB_N = 34 };
static_assert(sizeof(TAB) / sizeof(TAB[0]) == TAB_N, "table size");
}  // namespace ctlm

__host__ __device__ inline double ctl_log(double a) {
  const volatile double* t = ctlm::TAB;
  int e;
  double m = std::frexp(a, &e);  // m in [1/2, 1)
  if (m < t[ctlm::SQRT_HALF]) {
    m = m * 2.0;  // exact
    e -= 1;
  }
  // with g = m - 1 (exact) and f = g / (2 + g) = (m - 1) / (m + 1):
  // log m = 2f + f R, R = 2 f^2 (1/3 + f^2/5 + ...), written
  // g - (g^2/2 - f (g^2/2 + R)) (2f = g - f g), so that the exact g leads and
  // only the small corrections carry rounding
  const double g = m - 1.0;
  const double f = g / (2.0 + g);
  const double z = f * f;
  // 1/3 + z/5 + z^2/7 + ... + z^10/23
  double p = t[ctlm::LOG_P];
  for (int j = 1; j < 11; ++j) p = fma(p, z, t[ctlm::LOG_P + j]);
  const double R = 2.0 * (z * p);
  const double h = 0.5 * (g * g);
  const double de = static_cast<double>(e);
  return de * t[ctlm::LN2_HI] - ((h - (f * (h + R) + de * t[ctlm::LN2_LO])) - g);
}

__host__ __device__ inline void ctl_sincos(double x, double* sn, double* cs) {
  const volatile double* t = ctlm::TAB;
  const double n = std::rint(x * t[ctlm::TWO_OVER_PI]);
  // r = x - n pi/2 as rh + rl: x - n PIO2_1 is exact (n <= 4, |r| <= pi/4),
  // the subtraction of n PIO2_2 is split exactly (|a| >= |w|), then n PIO2_3
  const double a = x - n * t[ctlm::PIO2_1];
  const double w = n * t[ctlm::PIO2_2];
  const double rh = a - w;
  const double rl = ((a - rh) - w) - n * t[ctlm::PIO2_3];
  const double z = rh * rh;
  // sin(rh + rl) = rh + rh^3 (-1/3! + z/5! - ... + z^7/17!) + rl (1 - z/2)
  double ps = t[ctlm::SIN_P];
  for (int j = 1; j < 8; ++j) ps = fma(ps, z, t[ctlm::SIN_P + j]);
  const double s = rh + fma(rh * z, ps, rl - 0.5 * z * rl);
  // cos(rh + rl) = 1 - z/2 + z^2 (1/4! - z/6! + ... - z^7/18!) - rh rl, with
  // 1 - z/2 rounded to u and its rounding error carried
  double pc = t[ctlm::COS_P];
  for (int j = 1; j < 8; ++j) pc = fma(pc, z, t[ctlm::COS_P + j]);
  const double hz = 0.5 * z;
  const double u = 1.0 - hz;
  const double c = u + (((1.0 - u) - hz) + (z * z * pc - rh * rl));
  // quadrant: x = n pi/2 + r
  const int q = static_cast<int>(n) & 3;
  const double ss = (q & 1) ? c : s, cc = (q & 1) ? s : c;
  *sn = (q & 2) ? -ss : ss;
  *cs = ((q + 1) & 2) ? -cc : cc;
}

}  // namespace aeb
