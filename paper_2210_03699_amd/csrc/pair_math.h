// Per-pair kernel evaluations shared by the float64 and mixed-precision
// pair kernels and by the near-pair fix-up.
//
// For target x = P(y_k) with normal n_k and source P(y_m) with normal n_m,
// r = x - P(y_m), e = e^{-kR}, t = e (1 + kR), the kernels of
// eq. (Kij-kernels) times 4 pi are
//   K11 = (r.n_m)(1 - c1 t)/R^3,   K12 = (1 - e)/R,
//   K21 = [(1 - t)(n_k.n_m - 3 q/R^2) + k^2 e q]/R^3,  q = (r.n_k)(r.n_m),
//   K22 = -(r.n_k)(1 - c2 t)/R^3,
// (K21 uses (kR)^2/R^2 = k^2 to fold the cubic term of 1 - e(1 + kR + (kR)^2/3)),
// and the contributions of one source with amplitudes (a1, a2) = w (u1, u2)
// to the two rows are d1 = K11 a1 - K12 a2, d2 = K21 a1 - K22 a2.
#pragma once

#include <hip/hip_runtime.h>

#include "fastmath.h"

namespace ibim {

struct PairConsts {
  double c1, c2, kappa, kappa2;
};

struct PairConstsF {
  float c1, c2, kappa, kappa2;
};

// float64.  kAccumulate: add the contributions straight into (s1, s2) with
// fused multiply-adds; otherwise write them to (s1, s2).
template <bool kAccumulate>
__device__ __forceinline__ void pair_f64(double x, double y, double z, double nxk, double nyk,
                                         double nzk, double px, double py, double pz, double nxm,
                                         double nym, double nzm, double a1, double a2,
                                         const PairConsts& c, double& s1, double& s2) {
  const double rx = x - px, ry = y - py, rz = z - pz;
  const double R2 = fma(rz, rz, fma(ry, ry, rx * rx));
  const double iR = rsqrt_pos(R2);
  const double R = R2 * iR;
  const double iR2 = iR * iR;
  const double iR3 = iR2 * iR;
  const double kr = c.kappa * R;
  const double e = exp_neg(kr);
  const double te = fma(e, kr, e);
  const double rny = fma(rz, nzm, fma(ry, nym, rx * nxm));
  const double rnx = fma(rz, nzk, fma(ry, nyk, rx * nxk));
  const double nn = fma(nzk, nzm, fma(nyk, nym, nxk * nxm));
  const double A1 = a1 * iR3;
  const double A2 = a2 * iR3;
  const double g11 = rny * fma(-c.c1, te, 1.0);
  const double g12 = (1.0 - e) * R2;
  const double phi2 = 1.0 - te;
  const double q = rnx * rny;
  const double g21 = fma(phi2, fma(q * iR2, -3.0, nn), c.kappa2 * e * q);
  const double g22 = rnx * fma(-c.c2, te, 1.0);
  if (kAccumulate) {
    s1 = fma(g11, A1, fma(-g12, A2, s1));
    s2 = fma(g21, A1, fma(g22, A2, s2));
  } else {
    s1 = fma(g11, A1, -g12 * A2);
    s2 = fma(g21, A1, g22 * A2);
  }
}

// float32 from the difference r = x - P(y_m), every operation explicit
// (fused multiply-adds written out), so that every kernel including this
// header computes bit-identical values when its translation unit is compiled
// without automatic contraction.
__device__ __forceinline__ void pair_f32_r(float rx, float ry, float rz, float nxk, float nyk,
                                           float nzk, float nxm, float nym, float nzm, float a1,
                                           float a2, const PairConstsF& c, float& d1, float& d2) {
  const float R2 = __fmaf_rn(rz, rz, __fmaf_rn(ry, ry, rx * rx));
  const float iR = __builtin_amdgcn_rsqf(R2);
  const float R = R2 * iR;
  const float iR2 = iR * iR;
  const float iR3 = iR2 * iR;
  const float kr = c.kappa * R;
  const float e = exp_neg_f32(kr);
  const float te = __fmaf_rn(e, kr, e);
  const float rny = __fmaf_rn(rz, nzm, __fmaf_rn(ry, nym, rx * nxm));
  const float rnx = __fmaf_rn(rz, nzk, __fmaf_rn(ry, nyk, rx * nxk));
  const float nn = __fmaf_rn(nzk, nzm, __fmaf_rn(nyk, nym, nxk * nxm));
  const float A1 = a1 * iR3;
  const float A2 = a2 * iR3;
  const float g11 = rny * __fmaf_rn(-c.c1, te, 1.0f);
  const float g12 = (1.0f - e) * R2;
  const float phi2 = 1.0f - te;
  const float q = rnx * rny;
  const float g21 = __fmaf_rn(phi2, __fmaf_rn(q * iR2, -3.0f, nn), (c.kappa2 * e) * q);
  const float g22 = rnx * __fmaf_rn(-c.c2, te, 1.0f);
  d1 = __fmaf_rn(g11, A1, -(g12 * A2));
  d2 = __fmaf_rn(g21, A1, g22 * A2);
}

// float32 from the two points (pair_f32_r of their difference).
__device__ __forceinline__ void pair_f32(float x, float y, float z, float nxk, float nyk,
                                         float nzk, float px, float py, float pz, float nxm,
                                         float nym, float nzm, float a1, float a2,
                                         const PairConstsF& c, float& d1, float& d2) {
  pair_f32_r(x - px, y - py, z - pz, nxk, nyk, nzk, nxm, nym, nzm, a1, a2, c, d1, d2);
}

// float32, both directions of one pair for the symmetric kernel: fixed node f
// (target k) and rotating node m.  (d1, d2): contribution to k from m with
// m's amplitudes (am1, am2); (c1, c2): contribution to m from k with k's
// amplitudes (ak1, ak2).  With r' = -r the reverse pair has r'.n_k = -r.n_m
// and r'.n_m = -r.n_k.  Every operation explicit, as in pair_f32.
// kUnit: lengths in units of the Debye length 1/kappa (kappa = 1 in the
// formulas, which saves two multiplications).
// pair_f32_sym_r takes the difference r = x_k - P_m and its R2 = |r|^2
// (formed as pair_f32_sym forms them) from the caller.
template <bool kUnit = false>
__device__ __forceinline__ void pair_f32_sym_r(float rx, float ry, float rz, float R2, float nxk,
                                               float nyk, float nzk, float ak1, float ak2,
                                               float nxm, float nym, float nzm, float am1,
                                               float am2, const PairConstsF& c, float& d1,
                                               float& d2, float& c1, float& c2) {
  const float iR = __builtin_amdgcn_rsqf(R2);
  const float R = R2 * iR;
  const float iR2 = iR * iR;
  const float iR3 = iR2 * iR;
  const float kr = kUnit ? R : c.kappa * R;
  const float e = exp_neg_f32(kr);
  const float rny = __fmaf_rn(rz, nzm, __fmaf_rn(ry, nym, rx * nxm));
  const float rnx = __fmaf_rn(rz, nzk, __fmaf_rn(ry, nyk, rx * nxk));
  const float nn = __fmaf_rn(nzk, nzm, __fmaf_rn(nyk, nym, nxk * nxm));
  // t3 = e (1 + kR)/R^3, u = 1/R^3 - t3; (1 - c t)/R^3 = 1/R^3 - c t3,
  // (1 - e)/R = 1/R - e/R, K21 = n_k.n_m u + q (k^2 e/R^3 - 3 u/R^2)
  const float eiR3 = e * iR3;
  const float t3 = __fmaf_rn(eiR3, kr, eiR3);
  const float u = iR3 - t3;
  const float f1 = __fmaf_rn(-c.c1, t3, iR3);
  const float f2 = __fmaf_rn(-c.c2, t3, iR3);
  const float g12 = __fmaf_rn(-e, iR, iR);
  const float q = rnx * rny;
  const float k2e = kUnit ? eiR3 : c.kappa2 * eiR3;
  const float g21 = __fmaf_rn(nn, u, q * __fmaf_rn(u * iR2, -3.0f, k2e));
  const float g11 = rny * f1, g22 = rnx * f2;
  d1 = __fmaf_rn(g11, am1, -(g12 * am2));
  d2 = __fmaf_rn(g21, am1, g22 * am2);
  const float h11 = -rnx * f1, h22 = -rny * f2;
  c1 = __fmaf_rn(h11, ak1, -(g12 * ak2));
  c2 = __fmaf_rn(g21, ak1, h22 * ak2);
}

template <bool kUnit = false>
__device__ __forceinline__ void pair_f32_sym(float xk, float yk, float zk, float nxk, float nyk,
                                             float nzk, float ak1, float ak2, float xm, float ym,
                                             float zm, float nxm, float nym, float nzm, float am1,
                                             float am2, const PairConstsF& c, float& d1,
                                             float& d2, float& c1, float& c2) {
  const float rx = xk - xm, ry = yk - ym, rz = zk - zm;
  const float R2 = __fmaf_rn(rz, rz, __fmaf_rn(ry, ry, rx * rx));
  pair_f32_sym_r<kUnit>(rx, ry, rz, R2, nxk, nyk, nzk, ak1, ak2, nxm, nym, nzm, am1, am2, c, d1,
                        d2, c1, c2);
}

}  // namespace ibim
