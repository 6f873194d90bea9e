// wcc_rn.hpp -- correctly rounded binary64 division and square root for
// device code.
//
// The binary64 quotient the compiler emits (a reciprocal refined by Newton
// steps, then one correction, with range scaling) and the library square root
// are faithful, within one unit in the last place, but not always the
// correctly rounded result.  When the exact value lies very near the midpoint
// of two binary64 neighbours they can return the farther one.  This was
// observed for a denominator just below a power of two, a density of
// 0.125 (1 - 4e-16) in Sod's problem, where one quotient came out one unit
// low.  The CPU reference divides and takes square roots with IEEE binary64
// operations, so one such unit in one cell is enough to end bit-identical
// results.  The helpers below take the hardware result and fix its last bit
// from the exact remainder that a fused multiply-add gives.
//
// Domain: the result is correctly rounded where the remainder is exact, i.e.
// |numerator| >= 2^-969 with a quotient of normal magnitude (division), or
// 2^-960 <= x < 2^1000 (square root).  Zero, infinite and NaN operands and
// results are the IEEE ones; elsewhere (subnormal quotients, tiny numerators,
// huge or tiny square root operands) the result is within one unit in the
// last place.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wcc {

// Correctly rounded a / b.
__device__ __forceinline__ double div_rn(double a, double b) {
  const double q = a / b;
  // a - q b, exact for a faithful q and |a| >= 2^-969
  const double r = __builtin_fma(-q, b, a);
  // the neighbour of q on the side of a / b = q + r / b: one step up in
  // magnitude when r / b has the sign of q
  const int hi = __double2hiint(r) ^ __double2hiint(b) ^ __double2hiint(q);
  const double qn = __longlong_as_double(__double_as_longlong(q) + (hi >= 0 ? 1LL : -1LL));
  const double rn = __builtin_fma(-qn, b, a);
  // |remainder| = |b| x distance to a / b: take the nearer.  A tie would need
  // b a power of two, where the quotient is exact and r = 0.  Zero and NaN
  // quotients keep q (r is 0 or NaN there, and the comparison fails), and so
  // do infinite ones: after an overflow r is infinite and the neighbour, the
  // largest finite number, would compare nearer.
  return (__builtin_fabs(rn) < __builtin_fabs(r) && __builtin_fabs(a) >= 0x1p-969 && __builtin_isfinite(q)) ? qn
                                                                                                           : q;
}

// Correctly rounded sqrt(x).
__device__ __forceinline__ double sqrt_rn(double x) {
  const double s = __builtin_sqrt(x);
  // x - s^2, exact where it matters (near the thresholds below)
  const double r = __builtin_fma(-s, s, x);
  // With u the spacing of binary64 numbers just above s, sqrt(x) lies past
  // the midpoint to s + u iff r > s u; with d the spacing just below s (u,
  // or u / 2 when s is a power of two), it lies before the midpoint to s - d
  // iff r <= -s d.  (x - s^2 and s u are multiples of the same grid.)
  const long long si = __double_as_longlong(s);
  const double pe = __longlong_as_double(si & 0x7ff0000000000000LL);   // 2^exponent(s)
  const double su = s * (pe * 0x1p-52);
  const double sd = (si & 0x000fffffffffffffLL) == 0 ? 0.5 * su : su;
  const bool ok = x >= 0x1p-960 && x < 0x1p1000;
  const double up = __longlong_as_double(si + 1), dn = __longlong_as_double(si - 1);
  return !ok ? s : (r > su ? up : (r <= -sd ? dn : s));
}

}  // namespace wcc
