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
// samples, the Fourier modes and the lattice points.
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
// Lattice half-width of both sums.  The first omitted points lie at distance
// >= 6.5; there Q(s, pi r^2)/r < 3e-22 even for the highest mode (s = 40.5).
constexpr int kLat = 6;
constexpr int kSide = 2 * kLat + 1;
constexpr int kPts = kSide * kSide;  // includes the origin, skipped
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

__global__ __launch_bounds__(kWave* kWavesPerBlock) void weights_kernel(WeightArgs a) {
  __shared__ double cos_t[kSamples], sin_t[kSamples];
  __shared__ double l11s[kWavesPerBlock][kSamples], l21s[kWavesPerBlock][kSamples];
  __shared__ double2 coef[kWavesPerBlock][kModes][2];  // (a11, b11), (a21, b21) of mode 2j
  __shared__ double rs[kRecip];

  const int lane = threadIdx.x % kWave;
  const int wv = threadIdx.x / kWave;
  // angles are multiples of pi: sincospi reduces them exactly
  for (int q = threadIdx.x; q < kSamples; q += blockDim.x)
    sincospi(2.0 * q / kSamples, &sin_t[q], &cos_t[q]);
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
    double c, s;
    sincospi((double)p / kSamples, &s, &c);
    double v0 = (t1a * c + t1b * s) * d1;
    double v1 = (t2a * c + t2b * s) * d2;
    double vn2 = v0 * v0 + v1 * v1;
    double vn = sqrt(vn2);
    double qf = k1 * v0 * v0 + k2 * v1 * v1;
    l11s[wv][p] = c11 * qf / (vn2 * vn);
    l21s[wv][p] = c21 / vn;
  }
  __syncthreads();

  // 2. Fourier coefficients of the even modes: lane j owns mode k = 2j.
  //    cos(2j theta_p) = cos(2 pi (j p mod N) / N).
  if (lane < kModes) {
    const int j = lane;
    double a11 = 0.0, b11 = 0.0, a21 = 0.0, b21 = 0.0;
#pragma unroll 1
    for (int p = 0; p < kSamples; ++p) {
      int q = (j * p) & (kSamples - 1);
      double cq = cos_t[q], sq = sin_t[q];
      a11 += l11s[wv][p] * cq;
      b11 += l11s[wv][p] * sq;
      a21 += l21s[wv][p] * cq;
      b21 += l21s[wv][p] * sq;
    }
    double f = (j == 0) ? 1.0 / kSamples : 2.0 / kSamples;
    coef[wv][j][0] = make_double2(a11 * f, b11 * f);
    coef[wv][j][1] = make_double2(a21 * f, b21 * f);
  }
  __syncthreads();
  // highest significant mode (wave-uniform): lane j holds the largest
  // coefficient of mode 2j; a mode counts if it exceeds 1e-18 of the largest
  double mj = 0.0;
  if (lane < kModes) {
    const double2 c1 = coef[wv][lane][0], c2 = coef[wv][lane][1];
    mj = fmax(fmax(fabs(c1.x), fabs(c1.y)), fmax(fabs(c2.x), fabs(c2.y)));
  }
  double mx = mj;
  for (int off = kWave / 2; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, kWave));
  const unsigned long long sig = __ballot(lane < kModes && mj > 1e-18 * mx);
  const int jmax = sig ? 64 - __clzll((long long)sig) : 1;

  // 3. lattice sums, accumulated straight into the two weights
  double acc11 = 0.0, acc21 = 0.0;
  const double two_over_sqrtpi = 1.1283791670955126;
  const double sqrtpi = 1.7724538509055160;
#pragma unroll 1
  for (int idx = lane; idx < 2 * kPts; idx += kWave) {
    const int recip = idx >= kPts;
    const int q = recip ? idx - kPts : idx;
    const int n1 = q / kSide - kLat, n2 = q % kSide - kLat;
    if (n1 == 0 && n2 == 0) continue;
    double y1, y2, pr, pi, sg;
    if (!recip) {
      y1 = n1 - al;
      y2 = n2 - be;
      pr = 1.0;
      pi = 0.0;
      sg = 1.0;
    } else {
      y1 = n1;
      y2 = n2;
      sincospi(-2.0 * (n1 * al + n2 * be), &pi, &pr);
      sg = -1.0;  // (-i)^k = (-1)^(k/2) for even k
    }
    const double r2 = y1 * y1 + y2 * y2;
    const double ir = rsqrt_pos(r2);
    const double r = r2 * ir;
    const double x = kPiD * r2;
    const double sx = sqrtpi * r;                 // sqrt(x)
    double Q = erfc(sx);                          // Q(1/2, x)
    double term = two_over_sqrtpi * sx * exp(-x);  // x^s e^-x / Gamma(s+1), s = 1/2
    const double zr = y1 * ir, zi = y2 * ir;
    // e^{2i psi}, times (-i)^2 = -1 per mode step for the reciprocal sum
    const double z2r = (zr * zr - zi * zi) * sg, z2i = 2.0 * zr * zi * sg;
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
  hipLaunchKernelGGL(weights_kernel, dim3((unsigned)blocks), dim3(kWave * kWavesPerBlock), 0,
                     stream, a);
  return hipGetLastError();
}

}  // namespace ibim
