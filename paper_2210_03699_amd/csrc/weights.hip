// Correction weights of the CTR2 rule, computed on the device.
//
// For a correction entry (target row k, grid plane with shift (alpha, beta)
// and line-point signed distance eta) the weight of a kernel with leading
// term s0(y) = l(y/|y|)/|y| (Theorem 2.1; with the signs of s0^(11), s0^(22)
// and the factor kappa^2 of s0^(21) that the kernels' limits give) is
//   omega[s0; alpha, beta] = sum_k a_k omega[cos(k psi)/|y|] + b_k omega[sin(k psi)/|y|]
// (Section 2.4.2).  l is pi-periodic, so only even k occur.  Each basis weight
// is the limit of eq. (single_correction_weight), i.e. minus the regularised
// punctured lattice sum Z_k(alpha, beta) of e^{ik psi}/|y| over Z^2 - (alpha, beta),
// which an Ewald split evaluates exactly:
//   Z_k = sum_{n != 0} e^{ik psi(n-a)} Q(s, pi|n-a|^2)/|n-a|
//       + (-i)^k sum_{m != 0} e^{ik psi(m)} e^{-2 pi i m.a} Q(s, pi|m|^2)/|m|
//       - 2 [k = 0] - e^{ik psi(-a)} P(s, pi|a|^2)/|a|,        s = (k+1)/2,
// Q, P the regularised incomplete gamma functions.  Instead of tabulating
// basis weights and interpolating them, the GPU evaluates this for every
// entry directly: one wavefront per entry, the lanes splitting the theta
// samples, the Fourier modes and the lattice points.  Only the modes up to the
// last significant one are summed, over a lattice just wide enough for it.
#include <hip/hip_runtime.h>

#include <cmath>

#include <cstdint>

#include "fastmath.h"
#include "weights.h"

namespace ibim {
namespace {

constexpr int kWave = 64;
constexpr int kModes = 41;    // even modes 0, 2, ..., 80
constexpr int kSamples = 128; // samples of l on [0, pi)
// Lattice half-width of both sums for the highest mode in use: points with
// |n_i| > L lie at distance >= L + 1/2, where Q(s, pi r^2)/r < 3e-22 for every
// s = j + 1/2 up to the highest significant mode j (L = 4 up to j = 4, 5 up
// to j = 18, 6 up to j = 40).
constexpr int kLatMax = 6;
__device__ inline int lattice_halfwidth(int jhi) { return jhi <= 4 ? 4 : (jhi <= 18 ? 5 : kLatMax); }
// Modes whose coefficients (of l11, and of l21) are all below this fraction
// of that function's largest coefficient are dropped: with
// |omega[e^{ik psi}/|y|]| < 25 over the cell, the dropped terms total below
// 1e-13 of the largest coefficient.
constexpr double kModeCut = 1e-16;
constexpr int kWavesPerBlock = 4;
// Reciprocals 1/(m + 3/2) of the gamma recurrences (x^s/Gamma(s+1) steps
// from s to s + 1); indices reach kModes + the series length of step 4.
constexpr int kRecip = 256;
constexpr int kSeries = kRecip - kModes;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Side of the widest lattice.
constexpr int kLatSide = 2 * kLatMax + 1;

// The reciprocal-lattice terms that do not depend on the entry, per point m
// of the widest lattice ((m1 + kLatMax) * kLatSide + m2 + kLatMax):
// [0] = (Q(1/2, pi|m|^2), x^(1/2) e^-x / Gamma(3/2) at x = pi|m|^2),
// [1] = (x, 1/|m|), [2] = -e^{2i psi(m)} (the factor (-i)^2 of a mode step).
// Only the phase e^{-2 pi i m.a} remains per entry (a product of per-entry
// tables of e^{-2 pi i m1 alpha} and e^{-2 pi i m2 beta}).  Filled before every
// weights launch on the same stream; the values never change, so launches
// on other streams that read it meanwhile see the same bits.
__device__ double2 recip_terms[kLatSide * kLatSide][3];

__global__ void recip_terms_kernel() {
  const int t = threadIdx.x;
  if (t >= kLatSide * kLatSide) return;
  const int n1 = t / kLatSide - kLatMax, n2 = t % kLatSide - kLatMax;
  if (n1 == 0 && n2 == 0) {
    recip_terms[t][0] = make_double2(0.0, 0.0);
    recip_terms[t][1] = make_double2(0.0, 0.0);
    recip_terms[t][2] = make_double2(0.0, 0.0);
    return;
  }
  const double y1 = n1, y2 = n2;
  const double r2 = y1 * y1 + y2 * y2;
  const double ir = rsqrt_pos(r2);
  const double r = r2 * ir;
  const double x = kPiD * r2;
  const double sx = 1.7724538509055160 * r;  // sqrt(x)
  const double zr = y1 * ir, zi = y2 * ir;
  recip_terms[t][0] = make_double2(erfc(sx), 1.1283791670955126 * sx * exp(-x));
  recip_terms[t][1] = make_double2(x, ir);
  recip_terms[t][2] = make_double2(-(zr * zr - zi * zi), -(2.0 * zr * zi));
}

__global__ __launch_bounds__(kWave* kWavesPerBlock, 4) void weights_kernel(WeightArgs a) {
  // (cos, sin) of pi q / kSamples, q < 2 kSamples: the sample angles and,
  // at even q, the angles 2 pi m / kSamples of the transform
  __shared__ double2 cs_t[2 * kSamples];
  __shared__ double l11s[kWavesPerBlock][kSamples], l21s[kWavesPerBlock][kSamples];
  __shared__ double2 coef[kWavesPerBlock][kModes][2];  // (a11, b11), (a21, b21) of mode 2j
  // folded samples of step 2: [parity of j][p][0] = (A of l11, of l21),
  // [..][1] = (B of l11, of l21); mid = (U_h, V_h) at p = kSamples / 4
  __shared__ double2 fold[kWavesPerBlock][2][kSamples / 4][2];
  __shared__ double2 mid[kWavesPerBlock][2];
  // (cos, sin) of -2 pi n alpha and of -2 pi n beta, n = -kLatMax .. kLatMax:
  // the phase e^{-2 pi i m.a} of reciprocal point m is a product of two
  __shared__ double2 phase[kWavesPerBlock][2][kLatSide];
  __shared__ double rs[kRecip];

  const int lane = threadIdx.x % kWave;
  const int wv = threadIdx.x / kWave;
  // angles are multiples of pi: sincospi reduces them exactly
  for (int q = threadIdx.x; q < 2 * kSamples; q += blockDim.x) {
    double sq, cq;
    sincospi((double)q / kSamples, &sq, &cq);
    cs_t[q] = make_double2(cq, sq);
  }
  for (int m = threadIdx.x; m < kRecip; m += blockDim.x) rs[m] = 1.0 / (m + 1.5);
  __syncthreads();

  // A wavefront past the last entry recomputes the last entry and discards
  // it, so every wavefront reaches every block barrier.
  const int64_t e_raw = (int64_t)blockIdx.x * kWavesPerBlock + wv;
  const bool valid = e_raw < a.nnz;
  const int64_t e = valid ? e_raw : a.nnz - 1;

  const int32_t k = a.rowid[e];
  // K-reg entries (axis -1) run the same steps on harmless values and are
  // written as the regularised constants at the end
  const bool kreg = a.axis[e] < 0;
  const int ax = kreg ? 0 : a.axis[e];
  const int ia = (ax + 1) % 3, ib = (ax + 2) % 3;
  const double al = a.alpha[e], be = a.beta[e], eta = kreg ? 0.0 : a.eta[e];
  const double* tau = a.tau + 6 * (int64_t)k;
  const double t1a = tau[ia], t1b = tau[ib], t2a = tau[3 + ia], t2b = tau[3 + ib];
  const double d1 = 1.0 / (1.0 - eta * a.kap1[k]);
  const double d2 = 1.0 / (1.0 - eta * a.kap2[k]);
  const double k1 = a.kap1[k], k2 = a.kap2[k];
  const double c11 = (a.eps_out / a.eps_in - 1.0) / (8.0 * kPiD);
  const double c21 = a.kappa * a.kappa / (8.0 * kPiD);

  // 1. samples of l11, l21 at theta_p = pi p / kSamples
#pragma unroll 1
  for (int p = lane; p < kSamples; p += kWave) {
    const double c = cs_t[p].x, s = cs_t[p].y;
    double v0 = (t1a * c + t1b * s) * d1;
    double v1 = (t2a * c + t2b * s) * d2;
    double vn2 = v0 * v0 + v1 * v1;
    double vn = sqrt(vn2);
    double qf = k1 * v0 * v0 + k2 * v1 * v1;
    l11s[wv][p] = c11 * qf / (vn2 * vn);
    l21s[wv][p] = c21 / vn;
  }
  if (lane < 2 * kLatSide) {
    const int d = lane / kLatSide, n = lane % kLatSide - kLatMax;
    double sp, cp;
    sincospi(-2.0 * n * (d ? be : al), &sp, &cp);
    phase[wv][d][n + kLatMax] = make_double2(cp, sp);
  }
  __syncthreads();

  // 2. Fourier coefficients of the even modes: lane j owns mode k = 2j, whose
  //    basis functions at theta_p are cos and sin of 2 pi j p / N (N = kSamples).
  //    Samples p and N - p pair up (cos equal, sin of opposite sign): with
  //    U_p = l_p + l_{N-p}, V_p = l_p - l_{N-p},
  //      sum_p l_p cos = l_0 + (-1)^j l_{N/2} + sum_{p=1}^{N/2-1} U_p cos,
  //      sum_p l_p sin = sum_{p=1}^{N/2-1} V_p sin.
  //    Then p and N/2 - p pair up as well: the angle of N/2 - p is pi j minus
  //    that of p, so with s = (-1)^j its cos is s cos and its sin is -s sin:
  //      sum cos = U_{N/4} cos(pi j / 2) + sum_{p=1}^{N/4-1} (U_p + s U_{N/2-p}) cos,
  //      sum sin = V_{N/4} sin(pi j / 2) + sum_{p=1}^{N/4-1} (V_p - s V_{N/2-p}) sin.
  //    The folded sums A = U_p + s U_{N/2-p}, B = V_p - s V_{N/2-p} are formed
  //    once for both signs (lane p), and the angle 2 pi j p / N is entry
  //    2 j p mod 2N of the table.
  {
    const int p = lane;  // 1 .. N/4 - 1, and N/4 for the middle term
    const double* L1 = l11s[wv];
    const double* L2 = l21s[wv];
    if (p > 0 && p < kSamples / 4) {
      const int h = kSamples / 2;
      const double u1 = L1[p] + L1[kSamples - p], v1 = L1[p] - L1[kSamples - p];
      const double u2 = L2[p] + L2[kSamples - p], v2 = L2[p] - L2[kSamples - p];
      const double w1 = L1[h - p] + L1[h + p], x1 = L1[h - p] - L1[h + p];
      const double w2 = L2[h - p] + L2[h + p], x2 = L2[h - p] - L2[h + p];
      fold[wv][0][p][0] = make_double2(u1 + w1, u2 + w2);
      fold[wv][0][p][1] = make_double2(v1 - x1, v2 - x2);
      fold[wv][1][p][0] = make_double2(u1 - w1, u2 - w2);
      fold[wv][1][p][1] = make_double2(v1 + x1, v2 + x2);
    } else if (p == kSamples / 4) {
      const int q = 3 * kSamples / 4;
      mid[wv][0] = make_double2(L1[p] + L1[q], L2[p] + L2[q]);
      mid[wv][1] = make_double2(L1[p] - L1[q], L2[p] - L2[q]);
    }
  }
  __syncthreads();
  if (lane < kModes) {
    const int j = lane;
    const double sg = (j & 1) ? -1.0 : 1.0;
    double a11 = l11s[wv][0] + sg * l11s[wv][kSamples / 2];
    double a21 = l21s[wv][0] + sg * l21s[wv][kSamples / 2];
    double b11 = 0.0, b21 = 0.0;
    {
      const double2 cs = cs_t[(kSamples / 2 * j) & (2 * kSamples - 1)];
      const double2 U = mid[wv][0], V = mid[wv][1];
      a11 = fma(U.x, cs.x, a11);
      a21 = fma(U.y, cs.x, a21);
      b11 = fma(V.x, cs.y, b11);
      b21 = fma(V.y, cs.y, b21);
    }
    const double2(*fj)[2] = fold[wv][j & 1];
    int q = 0;
#pragma unroll
    for (int p = 1; p < kSamples / 4; ++p) {
      q = (q + 2 * j) & (2 * kSamples - 1);
      const double2 cs = cs_t[q];
      const double2 A = fj[p][0], B = fj[p][1];
      a11 = fma(A.x, cs.x, a11);
      a21 = fma(A.y, cs.x, a21);
      b11 = fma(B.x, cs.y, b11);
      b21 = fma(B.y, cs.y, b21);
    }
    double f = (j == 0) ? 1.0 / kSamples : 2.0 / kSamples;
    coef[wv][j][0] = make_double2(a11 * f, b11 * f);
    coef[wv][j][1] = make_double2(a21 * f, b21 * f);
  }
  __syncthreads();
  // highest significant mode (wave-uniform): a mode counts if one of its
  // coefficients of l11 (or of l21) exceeds kModeCut of the largest
  // coefficient of the same function (the two scales differ by ~10^3)
  double m11 = 0.0, m21 = 0.0;
  if (lane < kModes) {
    const double2 c1 = coef[wv][lane][0], c2 = coef[wv][lane][1];
    m11 = fmax(fabs(c1.x), fabs(c1.y));
    m21 = fmax(fabs(c2.x), fabs(c2.y));
  }
  double x11 = m11, x21 = m21;
  for (int off = kWave / 2; off > 0; off >>= 1) {
    x11 = fmax(x11, __shfl_xor(x11, off, kWave));
    x21 = fmax(x21, __shfl_xor(x21, off, kWave));
  }
  const unsigned long long sig =
      __ballot(lane < kModes && (m11 > kModeCut * x11 || m21 > kModeCut * x21));
  const int jmax = sig ? 64 - __clzll((long long)sig) : 1;
  const int lat = lattice_halfwidth(jmax - 1);
  const int side = 2 * lat + 1, pts = side * side;  // pts includes the origin, skipped
  // q / side by a float reciprocal: q < 169 and (q + 1/2)/side stays at
  // least 1/26 away from an integer, far above the float rounding
  const float inv_side = 1.0f / (float)side;

  // 3. lattice sums, accumulated straight into the two weights
  double acc11 = 0.0, acc21 = 0.0;
  const double two_over_sqrtpi = 1.1283791670955126;
  const double sqrtpi = 1.7724538509055160;
#pragma unroll 1
  for (int idx = lane; idx < 2 * pts; idx += kWave) {
    const int recip = idx >= pts;
    const int q = recip ? idx - pts : idx;
    const int qd = (int)(((float)q + 0.5f) * inv_side);
    const int n1 = qd - lat, n2 = q - qd * side - lat;
    if (n1 == 0 && n2 == 0) continue;
    double Q, term, x, ir, z2r, z2i, pr, pi;
    if (!recip) {
      const double y1 = n1 - al, y2 = n2 - be;
      const double r2 = y1 * y1 + y2 * y2;
      ir = rsqrt_pos(r2);
      const double r = r2 * ir;
      x = kPiD * r2;
      const double sx = sqrtpi * r;              // sqrt(x)
      Q = erfc(sx);                              // Q(1/2, x)
      term = two_over_sqrtpi * sx * exp(-x);     // x^s e^-x / Gamma(s+1), s = 1/2
      const double zr = y1 * ir, zi = y2 * ir;
      z2r = zr * zr - zi * zi;                   // e^{2i psi}
      z2i = 2.0 * zr * zi;
      pr = 1.0;
      pi = 0.0;
    } else {
      const double2* t = recip_terms[(n1 + kLatMax) * kLatSide + n2 + kLatMax];
      const double2 t0 = t[0], t1 = t[1], t2 = t[2];
      Q = t0.x;
      term = t0.y;
      x = t1.x;
      ir = t1.y;
      z2r = t2.x;  // e^{2i psi} times (-i)^2 = -1 per mode step
      z2i = t2.y;
      const double2 e1 = phase[wv][0][n1 + kLatMax], e2 = phase[wv][1][n2 + kLatMax];
      pr = e1.x * e2.x - e1.y * e2.y;
      pi = e1.x * e2.y + e1.y * e2.x;
    }
    double wr = pr * ir, wi = pi * ir;  // phase * e^{ik psi} / r, k = 0
    for (int j = 0; j < jmax; ++j) {
      const double cr = wr * Q, ci = wi * Q;
      const double2 c1 = coef[wv][j][0], c2 = coef[wv][j][1];
      acc11 = fma(c1.x, cr, fma(c1.y, ci, acc11));
      acc21 = fma(c2.x, cr, fma(c2.y, ci, acc21));
      Q += term;                 // Q(s + 1, x) = Q(s, x) + x^s e^-x / Gamma(s + 1)
      term *= x * rs[j];         // s = j + 1/2 -> j + 3/2
      const double nr = fma(wr, z2r, -wi * z2i);
      const double ni = fma(wr, z2i, wi * z2r);
      wr = nr;
      wi = ni;
    }
  }

  // 4. constant term and the punctured node (lane j owns mode 2j)
  const double r0 = sqrt(al * al + be * be);
  if (lane == 0) {
    acc11 += coef[wv][0][0].x * (-2.0);
    acc21 += coef[wv][0][1].x * (-2.0);
  }
  if (r0 == 0.0) {
    if (lane == 0) {  // limit of -P(1/2, pi r^2)/r; higher modes vanish
      acc11 += coef[wv][0][0].x * (-2.0);
      acc21 += coef[wv][0][1].x * (-2.0);
    }
  } else if (lane < jmax) {
    // P(s, x0) = x0^s e^-x0 / Gamma(s + 1) * sum_l x0^l / ((s+1)...(s+l)),
    // s = j + 1/2; |a| <= 1/sqrt(2) keeps x0 <= pi/2, so the series has
    // converged to 1e-18 long before kSeries terms.
    const int j = lane;
    const double x0 = kPiD * r0 * r0;
    double pref = two_over_sqrtpi * sqrtpi * r0 * exp(-x0);
    for (int t = 0; t < j; ++t) pref *= x0 * rs[t];
    double sum = 0.0, tt = 1.0;
    for (int l = 0; l < kSeries; ++l) {
      sum += tt;
      tt *= x0 * rs[j + l];
      if (tt < 1e-18 * sum) break;
    }
    const double Pv = pref * sum;
    // e^{i 2j psi(-a)}
    const double ur = -al / r0, ui = -be / r0;
    const double u2r = ur * ur - ui * ui, u2i = 2.0 * ur * ui;
    double zkr = 1.0, zki = 0.0;
    for (int t = 0; t < j; ++t) {
      double nr = zkr * u2r - zki * u2i;
      double ni = zkr * u2i + zki * u2r;
      zkr = nr;
      zki = ni;
    }
    const double cr = -zkr * Pv / r0, ci = -zki * Pv / r0;
    const double2 c1 = coef[wv][j][0], c2 = coef[wv][j][1];
    acc11 += c1.x * cr + c1.y * ci;
    acc21 += c2.x * cr + c2.y * ci;
  }

  const double z11 = wave_sum(acc11);
  const double z21 = wave_sum(acc21);
  if (lane == 0 && valid) {
    const double wm = a.w[a.col[e]];
    const double h2 = a.h * a.h, h3 = h2 * a.h;
    double* B = a.blocks + 4 * e;
    if (kreg) {
      a.om11[e] = 0.0;
      a.om21[e] = 0.0;
      B[0] = 0.0;
      B[1] = -h3 * a.c12 * wm;
      B[2] = 0.0;
      B[3] = 0.0;
    } else {
      const double om11 = -z11, om21 = -z21;
      a.om11[e] = om11;
      a.om21[e] = om21;
      B[0] = h2 * om11 * wm;
      B[1] = -h3 * (a.kappa / (4.0 * kPiD)) * wm;
      B[2] = h2 * om21 * wm;
      B[3] = h2 * (a.eps_in / a.eps_out) * om11 * wm;
    }
  }
}

}  // namespace

double kreg_constant(double kappa, double tau) {
  if (kappa == 0.0) return 0.0;
  const double x = kappa * tau;
  // numerator e^{-x} - 1 + x, by its series where it would cancel
  const double num =
      x < 1e-2 ? x * x * (0.5 - x * (1.0 / 6.0 - x * (1.0 / 24.0 - x / 120.0))) : std::expm1(-x) + x;
  return num / (2.0 * kPiD * kappa * tau * tau);
}

hipError_t launch_weights(const WeightArgs& a, hipStream_t stream) {
  if (a.nnz == 0) return hipSuccess;
  const int64_t blocks = (a.nnz + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL(recip_terms_kernel, dim3(1), dim3(192), 0, stream);
  hipLaunchKernelGGL(weights_kernel, dim3((unsigned)blocks), dim3(kWave * kWavesPerBlock), 0,
                     stream, a);
  return hipGetLastError();
}

}  // namespace ibim
