// Sine and cosine of the float64 phases of the operator.  For |x| < 2^20
// (k r and k n.d of any surface here) x = n pi/2 + y with a three-part
// Cody-Waite reduction (pi/2 split into two 33-bit parts, exact in n * part,
// and a remainder) and |y| <= pi/4; sin y and cos y by their Taylor series to
// y^15 and y^16 (the first omitted terms are below 7e-17 and 3e-18 on
// [-pi/4, pi/4]); the quadrant n mod 4 permutes and signs them.  Larger
// arguments take the library sincos (phase_sincos), or are the caller's to
// route elsewhere (phase_sincos_near, branch-free, for loops whose callers
// check the range of their arguments up front).
#pragma once

#include <hip/hip_runtime.h>

namespace bem {

constexpr double kPhaseNear = 1048576.0;   // 2^20

// Valid for |x| < kPhaseNear only.
__device__ inline void phase_sincos_near(double x, double* s, double* c) {
  const double n = rint(x * 0.6366197723675814);   // 2/pi
  double y = fma(-n, 1.5707963267341256, x);
  y = fma(-n, 6.077100506303966e-11, y);
  y = fma(-n, 2.0222662487959506e-21, y);
  const double y2 = y * y;
  double ps = -7.647163731819816e-13;   // -1/15!
  ps = fma(ps, y2, 1.6059043836821613e-10);   // +1/13!
  ps = fma(ps, y2, -2.505210838544172e-08);   // -1/11!
  ps = fma(ps, y2, 2.7557319223985893e-06);   // +1/9!
  ps = fma(ps, y2, -0.0001984126984126984);   // -1/7!
  ps = fma(ps, y2, 0.008333333333333333);   // +1/5!
  ps = fma(ps, y2, -0.16666666666666666);   // -1/3!
  const double sy = fma(ps * y2, y, y);
  double pc = 4.779477332387385e-14;   // 1/16!
  pc = fma(pc, y2, -1.1470745597729725e-11);   // -1/14!
  pc = fma(pc, y2, 2.08767569878681e-09);   // +1/12!
  pc = fma(pc, y2, -2.755731922398589e-07);   // -1/10!
  pc = fma(pc, y2, 2.48015873015873e-05);   // +1/8!
  pc = fma(pc, y2, -0.001388888888888889);   // -1/6!
  pc = fma(pc, y2, 0.041666666666666664);   // +1/4!
  pc = fma(pc, y2, -0.5);
  const double cy = fma(pc, y2, 1.0);
  const int q = (int)n & 3;
  const double sa = (q & 1) ? cy : sy, ca = (q & 1) ? sy : cy;
  *s = (q & 2) ? -sa : sa;
  *c = ((q + 1) & 2) ? -ca : ca;
}

__device__ inline void phase_sincos(double x, double* s, double* c) {
  if (!(fabs(x) < kPhaseNear)) {
    sincos(x, s, c);
    return;
  }
  phase_sincos_near(x, s, c);
}

}  // namespace bem
