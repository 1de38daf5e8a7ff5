// e^{i theta} in FP64 for the propagators' phase factors, from the Taylor
// series of sin and cos (no library calls, so that the constants are few and
// the result does not depend on a math library's rounding).
#pragma once

#include <hip/hip_runtime.h>

namespace icwf {

// e^{i theta} for |theta| <= pi/4 by the Taylor series of sin and cos in
// u = theta^2, to degrees 15 and 16: the first dropped terms are below
// (pi/4)^17/17! = 5e-17 and (pi/4)^18/18! = 2e-18, under half an ulp of
// the results.  Horner's rule from the highest power.
__device__ inline double2 expi_small(double th) {
    const double u = th * th;
    double s = -1.0 / 1307674368000.0;   // -1/15!
    s = fma(s, u, 1.0 / 6227020800.0);   // +1/13!
    s = fma(s, u, -1.0 / 39916800.0);    // -1/11!
    s = fma(s, u, 1.0 / 362880.0);       // +1/9!
    s = fma(s, u, -1.0 / 5040.0);        // -1/7!
    s = fma(s, u, 1.0 / 120.0);          // +1/5!
    s = fma(s, u, -1.0 / 6.0);           // -1/3!
    double c = 1.0 / 20922789888000.0;   // +1/16!
    c = fma(c, u, -1.0 / 87178291200.0); // -1/14!
    c = fma(c, u, 1.0 / 479001600.0);    // +1/12!
    c = fma(c, u, -1.0 / 3628800.0);     // -1/10!
    c = fma(c, u, 1.0 / 40320.0);        // +1/8!
    c = fma(c, u, -1.0 / 720.0);         // -1/6!
    c = fma(c, u, 1.0 / 24.0);           // +1/4!
    c = fma(c, u, -0.5);                 // -1/2!
    return make_double2(fma(u, c, 1.0), fma(th * u, s, th));
}

// e^{i theta} for any theta: theta = k pi/2 + r with k = rint(2 theta/pi),
// r = theta - k pi/2 by the three-term split of pi/2 of Cody and Waite (three
// doubles whose sum is pi/2 to 160 bits; each product is exact inside its
// FMA), so |r| <= pi/4 up to rounding; then e^{i theta} = i^k e^{i r}.  The
// absolute error stays at a few 1e-16 for |theta| < 2^30, far beyond any
// phase a time step takes.
__device__ inline double2 expi(double th) {
    const double k = rint(th * 0.63661977236758134308);
    double r = fma(-k, 1.5707963267948966, th);      // pi/2 rounded to a double
    r = fma(-k, 6.123233995736766e-17, r);           // pi/2 minus that, rounded
    r = fma(-k, -1.4973849048591698e-33, r);         // the remainder, rounded
    const double2 e = expi_small(r);
    const double k4 = k - 4.0 * floor(0.25 * k);     // k mod 4
    // i^k (c + i s): k = 0: (c, s), 1: (-s, c), 2: (-c, -s), 3: (s, -c)
    const bool odd = k4 == 1.0 || k4 == 3.0;
    const double a = odd ? e.y : e.x, b = odd ? e.x : e.y;
    return make_double2((k4 == 1.0 || k4 == 2.0) ? -a : a, k4 >= 2.0 ? -b : b);
}

}  // namespace icwf
