// Natural logarithm in FP64 for the column solves' equation of state.
//
// The column solves take two logarithms per layer and pass (interface
// pressures for the layer-mean pressure, and the power of the equation of
// state); the device library's FP64 logarithm carries a double-double
// reduction of about a hundred instructions, which made the logarithms most of
// the solves' FP64 work.  This one follows the classical atanh reduction used
// by the fdlibm logarithm (Sun Microsystems, 1993):
//
//   x = 2^e m, m in [sqrt(1/2), sqrt(2)),  f = m - 1 (exact),
//   s = f / (2 + f),  log(1 + f) = 2 atanh(s) = 2 s + s R(s^2),
//   R(z) = 2z/3 + 2z^2/5 + ... + 2z^10/21   (|s| <= 0.1716: the first omitted
//                                            term is below 2^-59 of the result),
//   log(1 + f) = f - (f^2/2 - s (f^2/2 + R))   (since 2 s = f - s f),
//   log x = e ln2_hi + (log(1 + f) + e ln2_lo),
//
// with the leading term f exact and the rounding of the small correction
// terms well below an ulp of the result; ln 2 is split into a head with 32
// significant bits (e ln2_hi exact for |e| < 2^21) and the rounded tail
// (hex literals below: ln 2 to 60 digits, head truncated to 32 bits).
// Measured against the host library on about 10^6 arguments, subnormal ones
// included: at most one ulp.  Straight-line code (no call of the library's
// logarithm, whose registers would lower the solves' occupancy): 0 gives
// -inf, negative arguments and NaN give NaN, and so does +inf (which no
// finite column produces; the solves' non-finite check reports it).
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>

namespace fv3 {

__host__ __device__ inline double flog(double x)
{
    constexpr double LN2_HI = 0x1.62e42fee00000p-1, LN2_LO = 0x1.a39ef35793c76p-33;
    int e;
    double m = std::frexp(x, &e);   // [1/2, 1)
    if (m < 0x1.6a09e667f3bcdp-1) {  // sqrt(1/2)
        m *= 2.0;
        e -= 1;
    }
    const double f = m - 1.0;
    const double s = f / (2.0 + f);
    const double z = s * s;
    double r = 2.0 / 21.0;
    r = std::fma(r, z, 2.0 / 19.0);
    r = std::fma(r, z, 2.0 / 17.0);
    r = std::fma(r, z, 2.0 / 15.0);
    r = std::fma(r, z, 2.0 / 13.0);
    r = std::fma(r, z, 2.0 / 11.0);
    r = std::fma(r, z, 2.0 / 9.0);
    r = std::fma(r, z, 2.0 / 7.0);
    r = std::fma(r, z, 2.0 / 5.0);
    r = std::fma(r, z, 2.0 / 3.0);
    r *= z;
    const double hf = 0.5 * f * f;
    const double de = (double)e;
    const double corr = hf - std::fma(s, hf + r, de * LN2_LO);
    const double y = de * LN2_HI - (corr - f);
    return x > 0.0 ? y : (x == 0.0 ? -INFINITY : NAN);
}

}  // namespace fv3
