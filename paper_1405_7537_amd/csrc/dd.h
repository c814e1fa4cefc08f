// Double-double arithmetic for the device: the extended precision that the
// paper asks for in the tip of the arrowhead inverse (Sec. 2.1, 2.3).  A
// value is hi + lo with |lo| <= ulp(hi)/2.  The
// error-free transformations are Knuth's TwoSum, Dekker's FastTwoSum and the
// FMA-based TwoProd; the library is compiled with -ffp-contract=off so that
// none of these sequences is re-associated or fused behind our back.
#pragma once
#include <hip/hip_runtime.h>

namespace dpr1 {

struct dd {
  double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}

// requires |a| >= |b| (or a == 0)
__device__ __forceinline__ dd fast_two_sum(double a, double b) {
  double s = a + b;
  double e = b - (s - a);
  return {s, e};
}

__device__ __forceinline__ dd two_prod(double a, double b) {
  double p = a * b;
  double e = __builtin_fma(a, b, -p);
  return {p, e};
}

// Sum of two double-doubles whose hi parts have the same sign (no
// cancellation): relative error about 2^-104.
__device__ __forceinline__ dd dd_add_same(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  s.lo += a.lo + b.lo;
  return fast_two_sum(s.hi, s.lo);
}

// Accurate sum for arbitrary signs (both parts through TwoSum).
__device__ __forceinline__ dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ dd dd_neg(dd a) { return {-a.hi, -a.lo}; }

__device__ __forceinline__ dd dd_mul_d(dd a, double b) {
  dd p = two_prod(a.hi, b);
  p.lo = __builtin_fma(a.lo, b, p.lo);
  return fast_two_sum(p.hi, p.lo);
}

__device__ __forceinline__ dd dd_mul(dd a, dd b) {
  dd p = two_prod(a.hi, b.hi);
  p.lo = __builtin_fma(a.hi, b.lo, p.lo);
  p.lo = __builtin_fma(a.lo, b.hi, p.lo);
  return fast_two_sum(p.hi, p.lo);
}

// a / b: one correction step after the leading quotient (relative error a
// few units of 2^-104).
__device__ __forceinline__ dd dd_div(dd a, dd b) {
  double q1 = a.hi / b.hi;
  dd p = dd_mul_d(b, q1);
  dd r = two_sum(a.hi, -p.hi);
  r.lo += a.lo - p.lo;
  double q2 = (r.hi + r.lo) / b.hi;
  return fast_two_sum(q1, q2);
}

// a / zeta^2 with zeta^2 formed exactly as a double-double.  zeta is first
// scaled by a power of two into [1, 2) (and a by its square): for |zeta|
// below about 2^-484 the low part of the unscaled square would be a
// subnormal number and lose bits.
__device__ __forceinline__ dd dd_div_sq(dd a, double zeta) {
  const int e = ilogb(zeta);
  const double zs = ldexp(zeta, -e);
  const dd as = {ldexp(a.hi, -2 * e), ldexp(a.lo, -2 * e)};
  return dd_div(as, two_prod(zs, zs));
}

}  // namespace dpr1
