// Treecode summation of the dense pair sum on the device.
//
// Interpolation in the source variable.  On the bounding box of a cluster C
// take the tensor Chebyshev points s_p (second kind, `order` per dimension)
// and the Lagrange basis L_p(y) = l_i(y_x) l_j(y_y) l_k(y_z).  Every kernel of
// the pair sum is a derivative of
//   FA = (1 - c1 e^{-kR})/R,  FB = (1 - e^{-kR})/R,  FC = (1 - c2 e^{-kR})/R
// (times 1/(4 pi)): K11 = d/dn_y FA, K12 = FB, K21 = d/dn_x d/dn_y FB,
// K22 = d/dn_x FC.  Replacing F(x, y) by sum_p F(x, s_p) L_p(y) gives, for
// the sources of C,
//   sum_m K11 a1_m - K12 a2_m  ~  sum_p FA(x, s_p) Q1_p - FB(x, s_p) Q2_p,
//   sum_m K21 a1_m - K22 a2_m  ~  sum_p d/dn_x FB(x, s_p) Q1_p - d/dn_x FC(x, s_p) Q2_p,
// with the proxy charges Q1_p = sum_m a1_m n_m . grad L_p(y_m) and
// Q2_p = sum_m a2_m L_p(y_m).  The basis is evaluated in barycentric form and
// its derivative through the differentiation matrix of the Chebyshev points
// (l_i' = sum_q l_q D_qi, exact for polynomials of this degree).  Every
// cluster of more than proxy_cost * n^3 nodes (tree.h) carries proxies (a
// target-proxy evaluation costs about a quarter of a direct pair in the
// mixed form and under half in float64, so proxies pay off below n^3
// nodes); its charges come from its children's proxies by the exact
// transfer of bbFMM's upward pass (below) and directly from the sources of
// children without proxies.
//
// One workgroup per work item (part of the lists of a batch of 256 targets,
// one target per lane) runs through its proxy clusters and then its direct
// source ranges, staging both in LDS; the finishing kernel adds a batch's
// parts in a fixed order, so results are reproducible.  All arithmetic is
// float64 except, in the mixed form, the target-proxy evaluations (float32
// kernels on float64-formed differences, summed in float32 over one line of
// n proxies and then in float64) and the direct pairs at distance r_near or
// more (float32 kernels on float64-formed differences, summed in float64);
// direct pairs nearer than r_near, where the float32 kernels lose accuracy,
// stay float64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "context.h"
#include "pair_math.h"
#include "treecode.h"

namespace ibim {
namespace {

constexpr int kUpSrc = 64;  // sources per round of the proxy-charge kernel

struct TreeArgs {
  const int32_t *perm, *pos, *bstart, *fcol, *nlo, *nhi, *xrow, *xcol, *dstart, *dend, *kid,
      *mlist, *ibatch, *ifar0, *ifar1, *inear0, *inear1, *iorder, *pcol, *pown;
  const double *pbox, *cheb;
  const double *tx, *ty, *tz, *tnx, *tny, *tnz, *tw;
  double *ta1, *ta2, *pq, *S, *rowS, *colS;
  const double* u;
  PairConsts pc;
  int32_t M;
  int order;
  float rnear2;  // mixed form: direct pairs with float32 R^2 below this stay float64
};

TreeArgs make_args(const TreeDevice& T, const DeviceProblem& P, const double* u) {
  TreeArgs a;
  a.perm = T.perm; a.pos = T.pos; a.bstart = T.bstart; a.fcol = T.fcol;
  a.nlo = T.nlo; a.nhi = T.nhi; a.xrow = T.xrow; a.xcol = T.xcol;
  a.dstart = T.dstart; a.dend = T.dend; a.kid = T.kid; a.mlist = T.mlist;
  a.ibatch = T.ibatch; a.ifar0 = T.ifar0; a.ifar1 = T.ifar1; a.inear0 = T.inear0;
  a.inear1 = T.inear1; a.iorder = T.iorder; a.pcol = T.pcol; a.pown = T.pown;
  a.pbox = T.pbox; a.cheb = T.cheb;
  a.tx = T.tx; a.ty = T.ty; a.tz = T.tz; a.tnx = T.tnx; a.tny = T.tny; a.tnz = T.tnz;
  a.tw = T.tw;
  a.ta1 = T.ta1; a.ta2 = T.ta2; a.pq = T.pq; a.S = T.S; a.rowS = T.rowS; a.colS = T.colS;
  a.u = u;
  a.pc = PairConsts{P.eps_out / P.eps_in, P.eps_in / P.eps_out, P.kappa, P.kappa * P.kappa};
  a.M = T.M;
  a.order = T.order;
  a.rnear2 = (float)(T.rnear * T.rnear);
  return a;
}

// a1 = w u1, a2 = w u2 in tree order
__global__ void tree_gather_kernel(TreeArgs a) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.M) return;
  const int32_t k = a.perm[t];
  const double w = a.tw[t];
  a.ta1[t] = w * a.u[k];
  a.ta2[t] = w * a.u[a.M + k];
}

// Barycentric Lagrange basis of the Chebyshev points at t into l[0..n)
// (t equal to a point gives the unit vector).
__device__ inline void cheb_basis(double t, const double* tch, const double* wch, int n,
                                  double* l) {
  int hit = -1;
  for (int i = 0; i < n; ++i)
    if (t == tch[i]) hit = i;
  if (hit >= 0) {
    for (int i = 0; i < n; ++i) l[i] = i == hit ? 1.0 : 0.0;
    return;
  }
  double sum = 0.0;
  for (int i = 0; i < n; ++i) {
    const double v = wch[i] / (t - tch[i]);
    l[i] = v;
    sum += v;
  }
  const double is = 1.0 / sum;
  for (int i = 0; i < n; ++i) l[i] *= is;
}

__device__ inline void load_cheb(const TreeArgs& a, double* tch, double* wch, double* dch) {
  const int n = a.order, tid = threadIdx.x;
  if (tid < n) {
    tch[tid] = a.cheb[tid];
    wch[tid] = a.cheb[n + tid];
  }
  if (dch && tid < n * n) dch[tid] = a.cheb[2 * n + tid];
}

// Proxy charges of one cluster per workgroup from the sources of
// [dstart, dend) (zero when empty).  PER proxies per thread.
template <int PER>
__global__ __launch_bounds__(256) void tree_p2m_kernel(TreeArgs a) {
  __shared__ double tch[kTreeMaxOrder], wch[kTreeMaxOrder], dch[kTreeMaxOrder * kTreeMaxOrder];
  __shared__ double bl[kUpSrc][3][kTreeMaxOrder];  // l_i(y_d)
  __shared__ double bd[kUpSrc][3][kTreeMaxOrder];  // d l_i / d y_d
  __shared__ double sv[kUpSrc][4];                 // a1 n_x, a1 n_y, a1 n_z, a2
  const int slot = blockIdx.x, tid = threadIdx.x;
  const int n = a.order, n2 = n * n, n3 = n2 * n;
  const int32_t s = a.dstart[slot], e = a.dend[slot];
  const double* box = a.pbox + 6 * (size_t)slot;
  load_cheb(a, tch, wch, dch);
  double Q1[PER], Q2[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) Q1[r] = Q2[r] = 0.0;
  for (int32_t c0 = s; c0 < e; c0 += kUpSrc) {
    __syncthreads();
    if (tid < 3 * kUpSrc) {
      const int j = tid / 3, d = tid % 3;
      const int32_t m = c0 + j;
      if (m < e) {
        const double y = d == 0 ? a.tx[m] : (d == 1 ? a.ty[m] : a.tz[m]);
        const double lo = box[d], hi = box[3 + d];
        const double half = 0.5 * (hi - lo);
        double* l = bl[j][d];
        cheb_basis((y - 0.5 * (lo + hi)) / half, tch, wch, n, l);
        const double ih = 1.0 / half;
        for (int i = 0; i < n; ++i) {
          double dl = 0.0;
          for (int q = 0; q < n; ++q) dl = fma(l[q], dch[q * n + i], dl);
          bd[j][d][i] = dl * ih;
        }
        if (d == 0) {
          const double w = a.ta1[m];
          sv[j][0] = w * a.tnx[m];
          sv[j][1] = w * a.tny[m];
          sv[j][2] = w * a.tnz[m];
          sv[j][3] = a.ta2[m];
        }
      }
    }
    __syncthreads();
    const int cnt = min(kUpSrc, (int)(e - c0));
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int p = tid + 256 * r;
      if (p < n3) {
        const int i = p / n2, jj = (p / n) % n, k = p % n;
        double q1 = Q1[r], q2 = Q2[r];
        for (int j = 0; j < cnt; ++j) {
          const double lx = bl[j][0][i], ly = bl[j][1][jj], lz = bl[j][2][k];
          const double dx = bd[j][0][i], dy = bd[j][1][jj], dz = bd[j][2][k];
          const double lyz = ly * lz;
          q2 = fma(lx * lyz, sv[j][3], q2);
          q1 = fma(sv[j][0] * dx, lyz, q1);
          q1 = fma(sv[j][1] * lx, dy * lz, q1);
          q1 = fma(sv[j][2] * lx, ly * dz, q1);
        }
        Q1[r] = q1;
        Q2[r] = q2;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int p = tid + 256 * r;
    if (p < n3) {
      a.pq[2 * ((size_t)slot * n3 + p)] = Q1[r];
      a.pq[2 * ((size_t)slot * n3 + p) + 1] = Q2[r];
    }
  }
}

// Adds to the charges of the clusters mlist[off + blockIdx.x] those of their
// children with proxies.  The parent's basis polynomials are reproduced
// exactly by the child's interpolation, so
//   L_p(y) = sum_q L_p(s_q^child) L_q^child(y)  and  Q_p += sum_q L_p(s_q^child) Q_q^child
// for both charges (the gradient charges too, by differentiating the identity).
// The tensor transfer is applied one dimension at a time.
__global__ __launch_bounds__(256) void tree_m2m_kernel(TreeArgs a, int off) {
  constexpr int kN3 = kTreeMaxOrder * kTreeMaxOrder * kTreeMaxOrder;
  __shared__ double tch[kTreeMaxOrder], wch[kTreeMaxOrder];
  __shared__ double Sm[3][kTreeMaxOrder][kTreeMaxOrder];  // Sm[d][p][q] = l_p(child point q)
  __shared__ double A[kN3], B[kN3];
  const int slot = a.mlist[off + blockIdx.x], tid = threadIdx.x;
  const int n = a.order, n2 = n * n, n3 = n2 * n;
  const double* pb = a.pbox + 6 * (size_t)slot;
  load_cheb(a, tch, wch, nullptr);
  for (int c = 0; c < 2; ++c) {
    const int ch = a.kid[2 * slot + c];
    if (ch < 0) continue;  // uniform
    const double* cb = a.pbox + 6 * (size_t)ch;
    __syncthreads();
    if (tid < 3 * n) {
      const int d = tid / n, q = tid % n;
      const double cmid = 0.5 * (cb[d] + cb[3 + d]), chalf = 0.5 * (cb[3 + d] - cb[d]);
      const double pmid = 0.5 * (pb[d] + pb[3 + d]), phalf = 0.5 * (pb[3 + d] - pb[d]);
      double l[kTreeMaxOrder];
      cheb_basis((cmid + chalf * tch[q] - pmid) / phalf, tch, wch, n, l);
      for (int p = 0; p < n; ++p) Sm[d][p][q] = l[p];
    }
    for (int chg = 0; chg < 2; ++chg) {
      __syncthreads();
      for (int idx = tid; idx < n3; idx += 256) B[idx] = a.pq[2 * ((size_t)ch * n3 + idx) + chg];
      __syncthreads();
      // x: A[px][qy][qz] = sum_qx Sx[px][qx] B[qx][qy][qz]
      for (int idx = tid; idx < n3; idx += 256) {
        const int px = idx / n2, rest = idx % n2;
        double v = 0.0;
        for (int q = 0; q < n; ++q) v = fma(Sm[0][px][q], B[q * n2 + rest], v);
        A[idx] = v;
      }
      __syncthreads();
      // y: B[px][py][qz] = sum_qy Sy[py][qy] A[px][qy][qz]
      for (int idx = tid; idx < n3; idx += 256) {
        const int px = idx / n2, py = (idx / n) % n, qz = idx % n;
        double v = 0.0;
        for (int q = 0; q < n; ++q) v = fma(Sm[1][py][q], A[px * n2 + q * n + qz], v);
        B[idx] = v;
      }
      __syncthreads();
      // z, added to the parent's charges
      for (int idx = tid; idx < n3; idx += 256) {
        const int base = idx - idx % n, pz = idx % n;
        double v = 0.0;
        for (int q = 0; q < n; ++q) v = fma(Sm[2][pz][q], B[base + q], v);
        a.pq[2 * ((size_t)slot * n3 + idx) + chg] += v;
      }
    }
  }
}

// Far field of one proxy point given R^2 = |x - s_p|^2 and rn = (x - s_p).n_k
// (formed from per-axis terms of the proxy grid).  With e = e^{-kR},
// t = e (1 + kR) and the point's charges (Q1, Q2):
//   FA Q1 - FB Q2 = [(1 - c1 e) Q1 - (1 - e) Q2]/R = [A + e B]/R,
//   d/dn_x FB Q1 - d/dn_x FC Q2 = (rn/R^3)[(1 - c2 t) Q2 - (1 - t) Q1] = (rn/R^3)[-A + t D],
// A = Q1 - Q2, B = Q2 - c1 Q1, D = Q1 - c2 Q2 formed once per point.
__device__ __forceinline__ void far_eval(double R2, double rn, double A, double B, double D,
                                         const PairConsts& c, double& S1, double& S2) {
  const double iR = rsqrt_pos(R2);
  const double R = R2 * iR;
  const double kr = c.kappa * R;
  const double e = exp_neg(kr);
  const double te = fma(e, kr, e);
  const double iR3 = iR * iR * iR;
  S1 = fma(iR, fma(e, B, A), S1);
  S2 = fma(rn * iR3, fma(te, D, -A), S2);
}

// far_eval in float32 (the mixed form): hardware reciprocal square root and
// base-2 exponential, every operation explicit.
__device__ __forceinline__ void far_eval_f32(float R2, float rn, float A, float B, float D,
                                             const PairConstsF& c, float& S1, float& S2) {
  const float iR = __builtin_amdgcn_rsqf(R2);
  const float R = R2 * iR;
  const float kr = c.kappa * R;
  const float e = exp_neg_f32(kr);
  const float te = __fmaf_rn(e, kr, e);
  const float iR3 = iR * iR * iR;
  S1 = __fmaf_rn(iR, __fmaf_rn(e, B, A), S1);
  S2 = __fmaf_rn(rn * iR3, __fmaf_rn(te, D, -A), S2);
}

// One work item: part of one batch's far clusters and direct ranges.  kN is
// the order when it is fixed at compile time (the float64 form at the
// default order 8: 3-4% faster), else 0.
template <bool kMixed, int kN>
__global__ __launch_bounds__(256) void tree_item_kernel(TreeArgs a) {
  // LDS: near sources as 8 arrays of 256, or (same buffer) the combined
  // charges (A, B, D interleaved) of a proxy cluster, as many x-planes of its
  // grid at a time as fit; the grid axes separately
  __shared__ double sh[8][256];
  __shared__ float shf[kMixed ? 5 : 1][256];  // mixed form: n_m, a1, a2 of the near sources
  __shared__ double ax[3][kTreeMaxOrder];
  const int it = a.iorder[blockIdx.x];
  const int b = a.ibatch[it];
  const int tid = threadIdx.x;
  const int32_t t0 = a.bstart[b], nt = a.bstart[b + 1] - t0;
  const int32_t t = t0 + min(tid, nt - 1);
  const double x = a.tx[t], y = a.ty[t], z = a.tz[t];
  const double nxk = a.tnx[t], nyk = a.tny[t], nzk = a.tnz[t];
  const int n = kN > 0 ? kN : a.order, n2 = n * n, n3 = n2 * n;
  // x-planes of the proxy grid whose charges fit in the LDS buffer at once
  const int planes = max(1, (kMixed ? 4096 : 2048) / (3 * n2));
  double* qs = &sh[0][0];
  float* qf = reinterpret_cast<float*>(&sh[0][0]);
  double S1 = 0.0, S2 = 0.0;
  const PairConstsF pcf{(float)a.pc.c1, (float)a.pc.c2, (float)a.pc.kappa, (float)a.pc.kappa2};
  const float nxf = (float)nxk, nyf = (float)nyk, nzf = (float)nzk;
  float rzf[kTreeMaxOrder];  // mixed form: z - Z_k of the current cluster
  // proxy clusters: points (X_i, Y_j, Z_k), so R^2 and r.n_k are built from
  // per-axis terms: (x - X_i)^2 + (y - Y_j)^2 once per (i, j), plus (z - Z_k)^2
  for (int32_t f = a.ifar0[it]; f < a.ifar1[it]; ++f) {
    const int slot = a.fcol[f];
    const size_t base = (size_t)slot * n3;
    for (int i0 = 0; i0 < n; i0 += planes) {
      const int i1 = min(n, i0 + planes);
      __syncthreads();
      if (i0 == 0 && tid < 3 * n) {
        const int d = tid / n, i = tid % n;
        const double* bx = a.pbox + 6 * (size_t)slot;
        ax[d][i] = 0.5 * (bx[d] + bx[3 + d]) + 0.5 * (bx[3 + d] - bx[d]) * a.cheb[i];
      }
      for (int q = tid; q < (i1 - i0) * n2; q += 256) {
        const double q1 = a.pq[2 * (base + (size_t)i0 * n2 + q)];
        const double q2 = a.pq[2 * (base + (size_t)i0 * n2 + q) + 1];
        if (kMixed) {
          qf[3 * q] = (float)(q1 - q2);
          qf[3 * q + 1] = (float)fma(-a.pc.c1, q1, q2);
          qf[3 * q + 2] = (float)fma(-a.pc.c2, q2, q1);
        } else {
          qs[3 * q] = q1 - q2;
          qs[3 * q + 1] = fma(-a.pc.c1, q1, q2);
          qs[3 * q + 2] = fma(-a.pc.c2, q2, q1);
        }
      }
      __syncthreads();
      if (kMixed) {
        if (i0 == 0) {
#pragma unroll
          for (int k = 0; k < kTreeMaxOrder; ++k) rzf[k] = k < n ? (float)(z - ax[2][k]) : 0.0f;
        }
        for (int i = i0; i < i1; ++i) {
          const float rx = (float)(x - ax[0][i]);
          const float rx2 = rx * rx, rxn = rx * nxf;
          for (int j = 0; j < n; ++j) {
            const float ry = (float)(y - ax[1][j]);
            const float axy = __fmaf_rn(ry, ry, rx2), bxy = __fmaf_rn(ry, nyf, rxn);
            const float* q = qf + 3 * (((i - i0) * n + j) * n);
            float s1 = 0.0f, s2 = 0.0f;
#pragma unroll
            for (int k = 0; k < (kN > 0 ? kN : kTreeMaxOrder); ++k) {
              if (kN > 0 || k < n)
                far_eval_f32(__fmaf_rn(rzf[k], rzf[k], axy), __fmaf_rn(rzf[k], nzf, bxy),
                             q[3 * k], q[3 * k + 1], q[3 * k + 2], pcf, s1, s2);
            }
            S1 += (double)s1;
            S2 += (double)s2;
          }
        }
      } else {
        for (int i = i0; i < i1; ++i) {
          const double rx = x - ax[0][i];
          const double rx2 = rx * rx, rxn = rx * nxk;
          for (int j = 0; j < n; ++j) {
            const double ry = y - ax[1][j];
            const double axy = fma(ry, ry, rx2), bxy = fma(ry, nyk, rxn);
            const double* q = qs + 3 * (((i - i0) * n + j) * n);
            for (int k = 0; k < n; ++k) {
              const double rz = z - ax[2][k];
              far_eval(fma(rz, rz, axy), fma(rz, nzk, bxy), q[3 * k], q[3 * k + 1],
                       q[3 * k + 2], a.pc, S1, S2);
            }
          }
        }
      }
    }
  }
  // direct ranges, pairs of N_k skipped
  int32_t p = a.xrow[t];
  const int32_t pe = a.xrow[t + 1];
  for (int32_t r = a.inear0[it]; r < a.inear1[it]; ++r) {
    const int32_t lo = a.nlo[r], hi = a.nhi[r];
    while (p < pe && a.xcol[p] < lo) ++p;
    int32_t nxt = p < pe ? a.xcol[p] : INT32_MAX;
    for (int32_t c0 = lo; c0 < hi; c0 += 256) {
      const int cnt = min(256, (int)(hi - c0));
      __syncthreads();
      if (tid < cnt) {
        const int32_t m = c0 + tid;
        sh[0][tid] = a.tx[m];
        sh[1][tid] = a.ty[m];
        sh[2][tid] = a.tz[m];
        sh[3][tid] = a.tnx[m];
        sh[4][tid] = a.tny[m];
        sh[5][tid] = a.tnz[m];
        sh[6][tid] = a.ta1[m];
        sh[7][tid] = a.ta2[m];
        if (kMixed) {
          shf[0][tid] = (float)a.tnx[m];
          shf[1][tid] = (float)a.tny[m];
          shf[2][tid] = (float)a.tnz[m];
          shf[3][tid] = (float)a.ta1[m];
          shf[4][tid] = (float)a.ta2[m];
        }
      }
      __syncthreads();
      for (int j = 0; j < cnt; ++j) {
        double d1, d2;
        if (kMixed) {
          const float rx = (float)(x - sh[0][j]), ry = (float)(y - sh[1][j]),
                      rz = (float)(z - sh[2][j]);
          float e1, e2;
          pair_f32_r(rx, ry, rz, nxf, nyf, nzf, shf[0][j], shf[1][j], shf[2][j], shf[3][j],
                     shf[4][j], pcf, e1, e2);
          d1 = (double)e1;
          d2 = (double)e2;
          const bool near = __fmaf_rn(rz, rz, __fmaf_rn(ry, ry, rx * rx)) < a.rnear2;
          if (__any(near)) {  // wave-uniform: the float64 pair for the lanes that need it
            double g1, g2;
            pair_f64<false>(x, y, z, nxk, nyk, nzk, sh[0][j], sh[1][j], sh[2][j], sh[3][j],
                            sh[4][j], sh[5][j], sh[6][j], sh[7][j], a.pc, g1, g2);
            d1 = near ? g1 : d1;
            d2 = near ? g2 : d2;
          }
        } else {
          pair_f64<false>(x, y, z, nxk, nyk, nzk, sh[0][j], sh[1][j], sh[2][j], sh[3][j],
                          sh[4][j], sh[5][j], sh[6][j], sh[7][j], a.pc, d1, d2);
        }
        const bool ex = c0 + j == nxt;
        if (ex) {
          ++p;
          nxt = p < pe ? a.xcol[p] : INT32_MAX;
        }
        S1 += ex ? 0.0 : d1;
        S2 += ex ? 0.0 : d2;
      }
    }
  }
  a.S[(size_t)it * 2 * kTreeBatch + tid] = S1;
  a.S[(size_t)it * 2 * kTreeBatch + kTreeBatch + tid] = S2;
}

// float64, both directions of one pair from the difference r = x_k - P_m:
// (d1, d2) the contribution to k from m with m's amplitudes (am1, am2),
// (c1, c2) the one to m from k with k's (ak1, ak2); the reverse pair has
// r' = -r, so r'.n_k = -r.n_m and r'.n_m = -r.n_k, and R, the exponential,
// n_k.n_m and q = (r.n_k)(r.n_m) are shared.  With u = (1 - e(1 + kR))/R^3
// and t3 = e(1 + kR)/R^3 the kernel factors are 1/R^3 - c t3 and
// K21 = n_k.n_m u + q (k^2 e/R^3 - 3 u/R^2).
__device__ __forceinline__ void pair_f64_sym_r(double rx, double ry, double rz, double nxk,
                                               double nyk, double nzk, double ak1, double ak2,
                                               double nxm, double nym, double nzm, double am1,
                                               double am2, const PairConsts& c, double& d1,
                                               double& d2, double& c1, double& c2) {
  const double R2 = fma(rz, rz, fma(ry, ry, rx * rx));
  const double iR = rsqrt_pos(R2);
  const double R = R2 * iR;
  const double iR2 = iR * iR;
  const double iR3 = iR2 * iR;
  const double kr = c.kappa * R;
  const double e = exp_neg(kr);
  const double rny = fma(rz, nzm, fma(ry, nym, rx * nxm));
  const double rnx = fma(rz, nzk, fma(ry, nyk, rx * nxk));
  const double nn = fma(nzk, nzm, fma(nyk, nym, nxk * nxm));
  const double eiR3 = e * iR3;
  const double t3 = fma(eiR3, kr, eiR3);
  const double u = iR3 - t3;
  const double f1 = fma(-c.c1, t3, iR3);
  const double f2 = fma(-c.c2, t3, iR3);
  const double g12 = fma(-e, iR, iR);  // (1 - e)/R
  const double q = rnx * rny;
  const double g21 = fma(nn, u, q * fma(u * iR2, -3.0, c.kappa2 * eiR3));
  const double g11 = rny * f1, g22 = rnx * f2;
  d1 = fma(g11, am1, -g12 * am2);
  d2 = fma(g21, am1, g22 * am2);
  const double h11 = -rnx * f1, h22 = -rny * f2;
  c1 = fma(h11, ak1, -g12 * ak2);
  c2 = fma(g21, ak1, h22 * ak2);
}

// Two-way pairs of leaves, one workgroup each: the targets of batch b =
// pown[q] (one per lane) against the sources of batch b' = pcol[q], both
// directions from one evaluation (the pairs hold no pair of N_k): float64,
// or in the mixed form float32 on float64-formed differences (float64 for
// the lanes whose pair is nearer than r_near).  Row sums go to rowS[q].  The sources are
// swept as in the symmetric direct kernel: in phase p wave w takes the 64
// sources of sub-block (w + p) mod 4, lane l source (l + s) mod 64 at step
// s, so each source's column sum in LDS receives one add per step from one
// lane, in a fixed order; colS[q] takes them at the end.
// b < b', so b is never the ragged last batch.
template <bool kMixed>
__global__ __launch_bounds__(256) void tree_pair_kernel(TreeArgs a) {
  __shared__ double sh[8][256];
  __shared__ float shf[kMixed ? 5 : 1][256];
  __shared__ double cs1[256], cs2[256];
  const int q = blockIdx.x;
  const int b = a.pown[q], b2 = a.pcol[q];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int32_t t0 = a.bstart[b], nt = a.bstart[b + 1] - t0;
  const int32_t t = t0 + min(tid, nt - 1);
  const bool valid = tid < nt;
  const double x = a.tx[t], y = a.ty[t], z = a.tz[t];
  const double nxk = a.tnx[t], nyk = a.tny[t], nzk = a.tnz[t];
  const float nxf = (float)nxk, nyf = (float)nyk, nzf = (float)nzk;
  const double ak1d = a.ta1[t], ak2d = a.ta2[t];
  const float ak1 = (float)ak1d, ak2 = (float)ak2d;
  const PairConstsF pcf{(float)a.pc.c1, (float)a.pc.c2, (float)a.pc.kappa, (float)a.pc.kappa2};
  const int32_t c0 = a.bstart[b2];
  const int cnt = a.bstart[b2 + 1] - c0;
  if (tid < cnt) {
    const int32_t m = c0 + tid;
    sh[0][tid] = a.tx[m];
    sh[1][tid] = a.ty[m];
    sh[2][tid] = a.tz[m];
    sh[3][tid] = a.tnx[m];
    sh[4][tid] = a.tny[m];
    sh[5][tid] = a.tnz[m];
    sh[6][tid] = a.ta1[m];
    sh[7][tid] = a.ta2[m];
    if (kMixed) {
      shf[0][tid] = (float)a.tnx[m];
      shf[1][tid] = (float)a.tny[m];
      shf[2][tid] = (float)a.tnz[m];
      shf[3][tid] = (float)a.ta1[m];
      shf[4][tid] = (float)a.ta2[m];
    }
  }
  cs1[tid] = cs2[tid] = 0.0;
  __syncthreads();
  double S1 = 0.0, S2 = 0.0;
  for (int ph = 0; ph < 4; ++ph) {
    const int sb = ((wv + ph) & 3) * 64;
    for (int st = 0; st < 64; ++st) {
      const int j = sb + ((lane + st) & 63);
      const bool live = j < cnt;  // sources past a ragged partner batch do not exist
      const int jj = live ? j : 0;
      double d1, d2, g1, g2;
      if (!kMixed) {
        pair_f64_sym_r(x - sh[0][jj], y - sh[1][jj], z - sh[2][jj], nxk, nyk, nzk, ak1d, ak2d,
                       sh[3][jj], sh[4][jj], sh[5][jj], sh[6][jj], sh[7][jj], a.pc, d1, d2, g1,
                       g2);
      }
      const float rx = (float)(x - sh[0][jj]), ry = (float)(y - sh[1][jj]),
                  rz = (float)(z - sh[2][jj]);
      const float R2 = __fmaf_rn(rz, rz, __fmaf_rn(ry, ry, rx * rx));
      if (kMixed) {
        float e1, e2, f1, f2;
        pair_f32_sym_r(rx, ry, rz, R2, nxf, nyf, nzf, ak1, ak2, shf[0][jj], shf[1][jj],
                       shf[2][jj], shf[3][jj], shf[4][jj], pcf, e1, e2, f1, f2);
        d1 = (double)e1;
        d2 = (double)e2;
        g1 = (double)f1;
        g2 = (double)f2;
      }
      const bool near = kMixed && R2 < a.rnear2;
      if (kMixed && __any(near)) {  // wave-uniform: the float64 pair both ways where needed
        double h1, h2, k1, k2;
        pair_f64<false>(x, y, z, nxk, nyk, nzk, sh[0][jj], sh[1][jj], sh[2][jj], sh[3][jj],
                        sh[4][jj], sh[5][jj], sh[6][jj], sh[7][jj], a.pc, h1, h2);
        pair_f64<false>(sh[0][jj], sh[1][jj], sh[2][jj], sh[3][jj], sh[4][jj], sh[5][jj], x, y,
                        z, nxk, nyk, nzk, ak1d, ak2d, a.pc, k1, k2);
        d1 = near ? h1 : d1;
        d2 = near ? h2 : d2;
        g1 = near ? k1 : g1;
        g2 = near ? k2 : g2;
      }
      if (live) {
        S1 += d1;
        S2 += d2;
        if (valid) {  // one lane per source and step: the adds to a slot come in step order
          atomicAdd(&cs1[j], g1);
          atomicAdd(&cs2[j], g2);
        }
      }
    }
    __syncthreads();  // the next phase's sub-block was this phase's of another wave
  }
  a.rowS[(size_t)q * 2 * kTreeBatch + tid] = S1;
  a.rowS[(size_t)q * 2 * kTreeBatch + kTreeBatch + tid] = S2;
  if (tid < cnt) {
    a.colS[(size_t)q * 2 * kTreeBatch + tid] = cs1[tid];
    a.colS[(size_t)q * 2 * kTreeBatch + kTreeBatch + tid] = cs2[tid];
  }
}

struct TreeFinishArgs {
  const double* u;
  const double* S;
  const double *rowS, *colS;
  const int32_t* perm;
  const int32_t* istart;
  const int32_t *prow, *inrow, *incol;
  const int32_t* crow;
  const int32_t* ccol;
  const double* blocks;
  int32_t M;
  double lam1, lam2, scale;
  double* out;
};

// One thread per tree position (so that the partial sums of a batch are
// read coalesced), writing its node's row.
__global__ void tree_finish_kernel(TreeFinishArgs a) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.M) return;
  const int32_t M = a.M, k = a.perm[t];
  const int b = t / kTreeBatch, l = t % kTreeBatch;
  double s1 = 0.0, s2 = 0.0;
  for (int32_t it = a.istart[b]; it < a.istart[b + 1]; ++it) {
    s1 += a.S[(size_t)it * 2 * kTreeBatch + l];
    s2 += a.S[(size_t)it * 2 * kTreeBatch + kTreeBatch + l];
  }
  // two-way pairs: row sums of this batch's own pairs, column sums of those
  // of lower batches with it
  for (int32_t q = a.prow[b]; q < a.prow[b + 1]; ++q) {
    s1 += a.rowS[(size_t)q * 2 * kTreeBatch + l];
    s2 += a.rowS[(size_t)q * 2 * kTreeBatch + kTreeBatch + l];
  }
  for (int32_t i = a.inrow[b]; i < a.inrow[b + 1]; ++i) {
    const double* c = a.colS + (size_t)a.incol[i] * 2 * kTreeBatch;
    s1 += c[l];
    s2 += c[kTreeBatch + l];
  }
  double o1 = a.lam1 * a.u[k] + a.scale * s1;
  double o2 = a.lam2 * a.u[M + k] + a.scale * s2;
  for (int32_t e = a.crow[k]; e < a.crow[k + 1]; ++e) {
    const int32_t m = a.ccol[e];
    const double* B = a.blocks + 4 * (size_t)e;
    const double v1 = a.u[m], v2 = a.u[M + m];
    o1 += B[0] * v1 + B[1] * v2;
    o2 += B[2] * v1 + B[3] * v2;
  }
  a.out[k] = o1;
  a.out[M + k] = o2;
}

template <class T>
hipError_t up(T** dst, const std::vector<T>& v, size_t* bytes, hipStream_t s) {
  *bytes += v.size() * sizeof(T);
  return upload(dst, v.data(), v.size(), s);
}

}  // namespace

void TreeDevice::release() {
  dfree(perm); dfree(pos); dfree(bstart);
  dfree(dstart); dfree(dend); dfree(kid); dfree(mlist);
  dfree(ibatch); dfree(ifar0); dfree(ifar1); dfree(inear0); dfree(inear1); dfree(istart);
  dfree(iorder); dfree(prow); dfree(pcol); dfree(pown); dfree(inrow); dfree(incol);
  dfree(rowS); dfree(colS);
  dfree(fcol); dfree(nlo); dfree(nhi); dfree(xrow); dfree(xcol);
  dfree(pbox); dfree(cheb);
  dfree(tx); dfree(ty); dfree(tz); dfree(tnx); dfree(tny); dfree(tnz); dfree(tw);
  dfree(ta1); dfree(ta2); dfree(pq); dfree(S);
}

hipError_t tree_upload(const TreePlan& pl, const DeviceProblem& P, const double* hpx,
                       const double* hpy, const double* hpz, const double* hnx, const double* hny,
                       const double* hnz, const double* hw, TreeDevice* T, hipStream_t s) {
  TreeDevice& d = *T;
  d.M = pl.M;
  d.order = pl.order;
  d.n_batches = (int)pl.bstart.size() - 1;
  d.n_slots = (int)pl.pstart.size();
  d.mlevel = pl.mlevel;
  d.n_items = (int)pl.ibatch.size();
  d.n_pairs = (int)pl.pcol.size();
  const int n = pl.order, n3 = n * n * n;
  // Chebyshev points of the second kind, barycentric weights, differentiation matrix
  std::vector<double> cheb(2 * n + n * n);
  for (int i = 0; i < n; ++i) {
    cheb[i] = std::cos(kPi * i / (n - 1));
    cheb[n + i] = ((i % 2) ? -1.0 : 1.0) * ((i == 0 || i == n - 1) ? 0.5 : 1.0);
  }
  for (int q = 0; q < n; ++q) {
    double diag = 0.0;
    for (int i = 0; i < n; ++i) {
      if (i == q) continue;
      const double v = (cheb[n + i] / cheb[n + q]) / (cheb[q] - cheb[i]);
      cheb[2 * n + q * n + i] = v;  // l_i'(t_q)
      diag -= v;
    }
    cheb[2 * n + q * n + q] = diag;
  }
  const int32_t M = pl.M;
  std::vector<double> g[7];
  const double* src[7] = {hpx, hpy, hpz, hnx, hny, hnz, hw};
  for (int c = 0; c < 7; ++c) {
    g[c].resize(M);
    for (int32_t t = 0; t < M; ++t) g[c][t] = src[c][pl.perm[t]];
  }
  size_t& by = d.bytes;
  by = 0;
  hipError_t e = hipSuccess;
#define TUP(dst, vec) \
  if (e == hipSuccess) e = up(&d.dst, vec, &by, s)
  TUP(perm, pl.perm);
  TUP(pos, pl.pos);
  TUP(bstart, pl.bstart);
  TUP(dstart, pl.dstart);
  TUP(dend, pl.dend);
  TUP(kid, pl.kid);
  TUP(mlist, pl.mlist);
  TUP(ibatch, pl.ibatch);
  TUP(ifar0, pl.ifar0);
  TUP(ifar1, pl.ifar1);
  TUP(inear0, pl.inear0);
  TUP(inear1, pl.inear1);
  TUP(istart, pl.istart);
  TUP(iorder, pl.iorder);
  TUP(prow, pl.prow);
  TUP(pcol, pl.pcol);
  TUP(pown, pl.pown);
  TUP(inrow, pl.inrow);
  TUP(incol, pl.incol);
  TUP(fcol, pl.fcol);
  TUP(nlo, pl.nlo);
  TUP(nhi, pl.nhi);
  TUP(xrow, pl.xrow);
  TUP(xcol, pl.xcol);
  TUP(pbox, pl.pbox);
  TUP(cheb, cheb);
  TUP(tx, g[0]);
  TUP(ty, g[1]);
  TUP(tz, g[2]);
  TUP(tnx, g[3]);
  TUP(tny, g[4]);
  TUP(tnz, g[5]);
  TUP(tw, g[6]);
#undef TUP
  if (e == hipSuccess) e = dalloc(&d.ta1, (size_t)M);
  if (e == hipSuccess) e = dalloc(&d.ta2, (size_t)M);
  if (e == hipSuccess) e = dalloc(&d.pq, (size_t)d.n_slots * n3 * 2);
  if (e == hipSuccess) e = dalloc(&d.S, (size_t)d.n_items * 2 * kTreeBatch);
  if (e == hipSuccess) e = dalloc(&d.rowS, (size_t)d.n_pairs * 2 * kTreeBatch);
  if (e == hipSuccess) e = dalloc(&d.colS, (size_t)d.n_pairs * 2 * kTreeBatch);
  by += (2 * (size_t)M + ((size_t)d.n_items + 2 * (size_t)d.n_pairs) * 2 * kTreeBatch +
         (size_t)d.n_slots * n3 * 2) *
        sizeof(double);
  // the host vectors above are temporaries
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

hipError_t launch_tree_sum(const TreeDevice& T, const DeviceProblem& P, const double* u,
                           hipStream_t s) {
  const TreeArgs a = make_args(T, P, u);
  hipLaunchKernelGGL(tree_gather_kernel, dim3((unsigned)((T.M + 255) / 256)), dim3(256), 0, s, a);
  if (T.n_slots > 0) {
    const int n3 = T.order * T.order * T.order, per = (n3 + 255) / 256;
    const dim3 g((unsigned)T.n_slots);
    if (per <= 1)
      hipLaunchKernelGGL(tree_p2m_kernel<1>, g, dim3(256), 0, s, a);
    else if (per <= 2)
      hipLaunchKernelGGL(tree_p2m_kernel<2>, g, dim3(256), 0, s, a);
    else if (per <= 4)
      hipLaunchKernelGGL(tree_p2m_kernel<4>, g, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL(tree_p2m_kernel<8>, g, dim3(256), 0, s, a);
    for (size_t hh = 1; hh + 1 < T.mlevel.size(); ++hh) {
      const int off = T.mlevel[hh], cnt = T.mlevel[hh + 1] - off;
      if (cnt > 0)
        hipLaunchKernelGGL(tree_m2m_kernel, dim3((unsigned)cnt), dim3(256), 0, s, a, off);
    }
  }
  const dim3 gi((unsigned)T.n_items);
  if (T.mixed) {
    // the float32 far field is faster with the order left to run time (86
    // against 102 VGPRs, one more wave per SIMD)
    hipLaunchKernelGGL((tree_item_kernel<true, 0>), gi, dim3(256), 0, s, a);
    if (T.n_pairs > 0)
      hipLaunchKernelGGL(tree_pair_kernel<true>, dim3((unsigned)T.n_pairs), dim3(256), 0, s, a);
  } else {
    if (T.order == 8)
      hipLaunchKernelGGL((tree_item_kernel<false, 8>), gi, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((tree_item_kernel<false, 0>), gi, dim3(256), 0, s, a);
    if (T.n_pairs > 0)
      hipLaunchKernelGGL(tree_pair_kernel<false>, dim3((unsigned)T.n_pairs), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_tree_finish(const TreeDevice& T, const DeviceProblem& P, const double* u,
                              double* out, hipStream_t s) {
  TreeFinishArgs f;
  f.u = u;
  f.S = T.S;
  f.rowS = T.rowS;
  f.colS = T.colS;
  f.perm = T.perm;
  f.istart = T.istart;
  f.prow = T.prow;
  f.inrow = T.inrow;
  f.incol = T.incol;
  f.crow = P.crow;
  f.ccol = P.ccol;
  f.blocks = P.blocks;
  f.M = P.M;
  f.lam1 = P.lam1;
  f.lam2 = P.lam2;
  f.scale = P.h * P.h * P.h / (4.0 * kPi);
  f.out = out;
  hipLaunchKernelGGL(tree_finish_kernel, dim3((unsigned)((P.M + 255) / 256)), dim3(256), 0, s, f);
  return hipGetLastError();
}

}  // namespace ibim
