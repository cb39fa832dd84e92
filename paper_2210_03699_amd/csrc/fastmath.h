// Elementary functions for the pair kernels, written for the value ranges
// the kernels need (no special-value handling).
#pragma once

#if defined(__HIPCC__)
#define IBIM_HD __host__ __device__
#else
#define IBIM_HD
#endif

#include <cmath>

namespace ibim {

// e^{-x} for finite x >= 0 (x = kappa R).  Cody-Waite reduction
// -x = k ln2 + r, |r| <= ln2/2, then e^r by a degree-11 polynomial whose
// coefficients interpolate e^r at the Chebyshev nodes of [-0.3466, 0.3466]
// (relative error below 2e-17 before rounding), and 2^k by ldexp.  Underflow
// for large x returns 0 through ldexp.
IBIM_HD inline double exp_neg(double x) {
  const double kLog2e = 1.4426950408889634;
  const double kLn2Hi = 6.93147180369123816490e-01;  // ln 2, high 32 bits
  const double kLn2Lo = 1.90821492927058770002e-10;  // ln 2 - kLn2Hi
  const double k = rint(-x * kLog2e);
  const double r = fma(-k, kLn2Lo, fma(-k, kLn2Hi, -x));
  double p = 2.5110049204818658e-08;
  p = fma(p, r, 2.763265472252779e-07);
  p = fma(p, r, 2.755724088722987e-06);
  p = fma(p, r, 2.4801485441561313e-05);
  p = fma(p, r, 0.00019841269890076403);
  p = fma(p, r, 0.0013888888952352863);
  p = fma(p, r, 0.008333333333319589);
  p = fma(p, r, 0.04166666666648795);
  p = fma(p, r, 0.1666666666666668);
  p = fma(p, r, 0.5000000000000019);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)k);
}

// e^{-x} in float32 for x >= 0, from the hardware base-2 exponential.
IBIM_HD inline float exp_neg_f32(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_exp2f(-x * 1.44269504088896341f);
#else
  return std::exp2(-x * 1.44269504088896341f);
#endif
}

#if defined(__HIPCC__)
// e^{-kappa R} for finite R >= 0 in the symmetric float64 pair kernel, by
// Tang's table-driven method (ACM TOMS 15, 1989) with a table of 64 entries:
// y = -64 kappa R / ln 2 is split as y = n + f, n = 64 m + j integer,
// |f| <= 1/2, so that e^{-kappa R} = 2^m 2^{j/64} 2^{f/64}.  The nearest
// integer n comes from adding 1.5 2^52 in the fused multiply-add that forms
// y (the low word of the sum is n), f from a second fused multiply-add, and
// 2^{f/64} - 1 from its Taylor polynomial of degree 5 (truncation below
// 3.6e-17 relative).  Entry j of the table, 2^{j/64}, is held by lane j of
// the wavefront and read with ds_bpermute, so every lane must be active.
// ds_bpermute selects lane (address / 4) mod 64 and ignores the higher
// address bits, so the address is n * 4 with no masking.  The factor 2^m
// goes into the exponent field: lane j keeps its entry's high word minus
// j * 2^14, and adding n * 2^14 = m * 2^20 + j * 2^14 (mod 2^32) to the
// permuted word leaves the entry's high word plus m * 2^20.  This holds while
// 2^m 2^{j/64} stays a normal number: kappa R <= 708 (callers check it).
struct ExpWave {
  double c;     // -64 kappa / ln 2
  int lo, hi;   // this lane's entry 2^{lane/64}: low word, high word - lane * 2^14
};
__device__ inline ExpWave exp_wave_init(double kappa) {
  ExpWave w;
  w.c = -kappa * 92.33248261689366;  // 64 / ln 2
  const int lane = (int)(threadIdx.x & 63);
  const double t = exp2((double)lane * 0.015625);
  w.lo = __double2loint(t);
  w.hi = (int)((unsigned)__double2hiint(t) - ((unsigned)lane << 14));
  return w;
}
__device__ __forceinline__ double exp_neg_wave(double R, const ExpWave& w) {
  const double kShift = 6755399441055744.0;  // 1.5 2^52
  const double s = fma(R, w.c, kShift);
  const unsigned n = (unsigned)__double2loint(s);
  const double f = fma(R, w.c, -(s - kShift));
  double p = fma(f, 1.2417843701716925e-12, 5.732851688640402e-10);
  p = fma(p, f, 2.1173137155464776e-07);
  p = fma(p, f, 5.86490495505617e-05);
  p = fma(p, f, 0.010830424696249145);
  p *= f;
  const int addr = (int)(n << 2);
  const unsigned hi = (unsigned)__builtin_amdgcn_ds_bpermute(addr, w.hi) + (n << 14);
  const double T = __hiloint2double((int)hi, __builtin_amdgcn_ds_bpermute(addr, w.lo));
  return fma(T, p, T);
}

// 1/sqrt(x) for finite x > 0: hardware estimate and one third-order
// correction y (1 + e/2 + 3 e^2/8), e = 1 - x y^2.
__device__ inline double rsqrt_pos(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
#else
  return 1.0 / std::sqrt(x);
#endif
}
#endif

}  // namespace ibim
