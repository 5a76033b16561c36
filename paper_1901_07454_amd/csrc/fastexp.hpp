// fastexp.hpp -- e^x and e^x - 1 of one argument with a short dependency chain.
//
// Cody and Waite's argument reduction: x = k ln2 + r with k = rint(x log2 e)
// and |r| <= ln2/2, ln2 split into a high part with 11 trailing zero bits (so
// k ln2_hi is exact for |k| < 2^11) and the rest.  Then
// u = e^r - 1 = r + r^2 q(r) with q the Taylor series of (e^r - 1 - r)/r^2 to
// degree 12 (coefficients 1/(i+2)!; truncation below 1e-19 for
// |r| <= ln2/2), evaluated by Estrin's scheme: pairs, then quadruples with
// r^2, octets with r^4, and r^8, four dependent steps after r instead of
// twelve.  e^x = 2^k (1 + u) and e^x - 1 = 2^k u + (2^k - 1), each with one
// final rounding.  Every
// product-sum is an explicit fma, so the host and the device round alike.
// Valid for |x| < 700 (the callers' arguments stay far inside).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace arbmi {

struct ExpPair {
    double e;    // e^x
    double em1;  // e^x - 1
};

__host__ __device__ inline ExpPair exp_pair(double x) {
    const double k = rint(x * 1.4426950408889634);   // log2(e)
    double r = fma(-k, 0x1.62e42fefa3800p-1, x);      // ln2, high part
    r = fma(-k, 0x1.ef35793c76730p-45, r);            // ln2, low part
    // e^r - 1 = r + r^2 q(r), q(r) = sum_{i=0}^{12} r^i / (i+2)!
    const double r2 = r * r, r4 = r2 * r2, r8 = r4 * r4;
    const double a0 = fma(0x1.5555555555555p-3, r, 0x1.0000000000000p-1);    // 1/2!, 1/3!
    const double a1 = fma(0x1.1111111111111p-7, r, 0x1.5555555555555p-5);    // 1/4!, 1/5!
    const double a2 = fma(0x1.a01a01a01a01ap-13, r, 0x1.6c16c16c16c17p-10);  // 1/6!, 1/7!
    const double a3 = fma(0x1.71de3a556c734p-19, r, 0x1.a01a01a01a01ap-16);  // 1/8!, 1/9!
    const double a4 = fma(0x1.ae64567f544e4p-26, r, 0x1.27e4fb7789f5cp-22);  // 1/10!, 1/11!
    const double a5 = fma(0x1.6124613a86d09p-33, r, 0x1.1eed8eff8d898p-29);  // 1/12!, 1/13!
    const double a6 = 0x1.93974a8c07c9dp-37;                                  // 1/14!
    const double b0 = fma(a1, r2, a0), b1 = fma(a3, r2, a2), b2 = fma(a5, r2, a4);
    const double d0 = fma(b1, r4, b0), d1 = fma(a6, r4, b2);
    const double q = fma(d1, r8, d0);
    const double u = fma(r2, q, r);          // e^r - 1
    const int ki = int(k);
    const double s = ldexp(1.0, ki);         // 2^k
    ExpPair out;
    out.e = fma(s, u, s);
    out.em1 = (ki == 0) ? u : fma(s, u, s - 1.0);
    return out;
}

}  // namespace arbmi
