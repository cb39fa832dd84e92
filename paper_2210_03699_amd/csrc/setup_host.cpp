// Host part of the problem setup: tube nodes, finite-difference geometry and
// the CTR2 correction sets N_h(y_k).
//
// Geometry follows Section 2.1: d > 0 inside, P(y) = y - d(y) g(y) with the
// normalised central-difference gradient g, outward normal n = -g, the
// level-set Jacobian J of eq. (jacobian) and w = J * delta_eps(d) with the
// cosine averaging kernel of Section 2.6.  Curvatures come from the Hessian
// taken as the central difference of the central gradient (+-2 nodes).
//
// Correction sets follow Section 2.4: for the target x* = P(y_k) with
// normal n, the dominant axis i = argmax |n_j| (ties: lowest j) fixes the
// family of grid planes t = origin_i + p h; in each plane the normal line
// meets the point L = x* + s n, s = (t - x*_i)/n_i; for |s| <= eps + h its
// nearest grid node (shift (alpha, beta) in [-1/2, 1/2)) is corrected when it
// lies in the tube.  eta = -s is the signed distance of L.
//
// HYB-IBIM (Section 3.2): a node is bad when its finite-difference geometry
// is unreliable (| |grad d| - 1 | > 0.05, |g.H g| > 0.1/h, or a corrected
// plane with 1 - |eta| max|kappa| < 0.2).  Bad rows take the K-reg rule of
// eq. (regularized-kernel) with tau = 2h over the tube nodes y with
// tangential distance |(I - n n^T)(y - x*)| < tau and normal distance
// |n.(y - x*)| <= eps + h; bad nodes carry J = 1 (eq. Jacobian-hybrid).
//
// The quantities that decide which node is corrected, regularised or bad
// (gradient, Hessian, P, n, the dominant axis, L, the nearest node, the
// tangential distance) are evaluated with plain IEEE operations in a fixed
// order and without contraction (this file is compiled with
// -ffp-contract=off), so the sets are reproducible exactly.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ibim.h"
#include "ibim_internal.h"

namespace ibim {
namespace {

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix.
// On return a[i][i] are eigenvalues, columns of v the eigenvectors.
void jacobi3(double a[3][3], double v[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) v[i][j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = std::fabs(a[0][1]) + std::fabs(a[0][2]) + std::fabs(a[1][2]);
    double diag = std::fabs(a[0][0]) + std::fabs(a[1][1]) + std::fabs(a[2][2]);
    if (off <= 1e-300 || off < 1e-18 * diag) break;
    for (int p = 0; p < 2; ++p) {
      for (int q = p + 1; q < 3; ++q) {
        if (a[p][q] == 0.0) continue;
        double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 3; ++k) {  // A <- A J
          double akp = a[k][p], akq = a[k][q];
          a[k][p] = c * akp - s * akq;
          a[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {  // A <- J^T A
          double apk = a[p][k], aqk = a[q][k];
          a[p][k] = c * apk - s * aqk;
          a[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          double vkp = v[k][p], vkq = v[k][q];
          v[k][p] = c * vkp - s * vkq;
          v[k][q] = s * vkp + c * vkq;
        }
      }
    }
  }
}

struct SdfView {
  const double* d;
  int n0, n1, n2;
  double operator()(int i, int j, int k) const {
    return d[((int64_t)i * n1 + j) * n2 + k];
  }
};

struct Candidate {
  int32_t col;
  int8_t axis;
  double alpha, beta, eta;
};

}  // namespace

void set_host_setup_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

int build_host_plan(const double* sdf, int nx, int ny, int nz, const double origin[3], double h,
                    double eps, int hybrid, HostPlan* plan, std::string* err) {
  if (!sdf || !origin || !plan || nx < 5 || ny < 5 || nz < 5) {
    *err = "null pointer or grid smaller than 5 nodes per axis";
    return IBIM_EINVAL;
  }
  if (!(h > 0.0) || !(eps > 0.0) || !std::isfinite(h) || !std::isfinite(eps)) {
    *err = "h and eps_tube must be positive and finite";
    return IBIM_EINVAL;
  }
  if (hybrid < 0 || hybrid > 2) {
    *err = "hybrid must be 0, 1 or 2";
    return IBIM_EINVAL;
  }
  const int64_t ngrid = (int64_t)nx * ny * nz;
  SdfView D{sdf, nx, ny, nz};
  plan->dims[0] = nx;
  plan->dims[1] = ny;
  plan->dims[2] = nz;
  for (int a = 0; a < 3; ++a) plan->origin[a] = origin[a];
  plan->h = h;
  plan->eps = eps;

  // Tube membership in grid scan order: nodes counted per chunk of the grid,
  // then numbered from each chunk's offset (the same numbering as one scan).
  const int64_t kChunk = 1 << 16;
  const int64_t nchunk = (ngrid + kChunk - 1) / kChunk;
  std::vector<int64_t> first(nchunk + 1, 0);
  int has_nan = 0;
#pragma omp parallel for schedule(static) reduction(| : has_nan)
  for (int64_t c = 0; c < nchunk; ++c) {
    const int64_t q1 = std::min(ngrid, (c + 1) * kChunk);
    int64_t n = 0;
    for (int64_t q = c * kChunk; q < q1; ++q) {
      const double v = sdf[q];
      has_nan |= std::isnan(v) ? 1 : 0;
      n += std::fabs(v) < eps ? 1 : 0;
    }
    first[c + 1] = n;
  }
  if (has_nan) {
    *err = "NaN in the signed distance";
    return IBIM_EGEOM;
  }
  for (int64_t c = 0; c < nchunk; ++c) first[c + 1] += first[c];
  const int64_t M = first[nchunk];
  if (M > INT32_MAX) {
    *err = "more than 2^31-1 tube nodes";
    return IBIM_EINVAL;
  }
  if (M == 0) {
    *err = "empty tube: no grid node with |d| < eps_tube";
    return IBIM_EGEOM;
  }
  plan->M = M;
  plan->grid_index.resize(M);
  std::vector<int32_t> node_of(ngrid);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nchunk; ++c) {
    const int64_t q1 = std::min(ngrid, (c + 1) * kChunk);
    int64_t m = first[c];
    for (int64_t q = c * kChunk; q < q1; ++q) {
      if (std::fabs(sdf[q]) < eps) {
        plan->grid_index[m] = q;
        node_of[q] = (int32_t)m++;
      } else {
        node_of[q] = -1;
      }
    }
  }

  auto& G = *plan;
  G.px.resize(M); G.py.resize(M); G.pz.resize(M);
  G.nx.resize(M); G.ny.resize(M); G.nz.resize(M);
  G.w.resize(M); G.kap1.resize(M); G.kap2.resize(M); G.tau.resize(6 * M);
  G.bad.assign(M, hybrid == 2 ? 1 : 0);
  G.ktau = 2.0 * h;
  std::vector<double> dval(M);
  std::vector<int32_t> ijk(3 * M);
  int edge = 0;
  for (int64_t m = 0; m < M; ++m) {
    int64_t q = G.grid_index[m];
    int i = (int)(q / ((int64_t)ny * nz));
    int j = (int)((q / nz) % ny);
    int k = (int)(q % nz);
    ijk[3 * m] = i; ijk[3 * m + 1] = j; ijk[3 * m + 2] = k;
    if (i < 2 || j < 2 || k < 2 || i + 2 >= nx || j + 2 >= ny || k + 2 >= nz) edge = 1;
  }
  if (edge) {
    *err = "the tube comes within two nodes of the grid edge";
    return IBIM_EGEOM;
  }

  int bad_grad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad_grad)
  for (int64_t m = 0; m < M; ++m) {
    const int i = ijk[3 * m], j = ijk[3 * m + 1], k = ijk[3 * m + 2];
    const double d0 = D(i, j, k);
    // central-difference gradient, normalised (decides P and n)
    const double gx = (D(i + 1, j, k) - D(i - 1, j, k)) / (2.0 * h);
    const double gy = (D(i, j + 1, k) - D(i, j - 1, k)) / (2.0 * h);
    const double gz = (D(i, j, k + 1) - D(i, j, k - 1)) / (2.0 * h);
    const double gn = std::sqrt(gx * gx + gy * gy + gz * gz);
    if (!(gn > 0.0)) {
      bad_grad = 1;
      continue;
    }
    const double g[3] = {gx / gn, gy / gn, gz / gn};
    const double y0 = origin[0] + (double)i * h;
    const double y1 = origin[1] + (double)j * h;
    const double y2 = origin[2] + (double)k * h;
    G.px[m] = y0 - d0 * g[0];
    G.py[m] = y1 - d0 * g[1];
    G.pz[m] = y2 - d0 * g[2];
    G.nx[m] = -g[0];
    G.ny[m] = -g[1];
    G.nz[m] = -g[2];

    // Hessian, central difference of the central gradient (each entry as
    // (sum of the stencil values in a fixed order) / (4 h^2))
    const double fh2 = 4.0 * h * h;
    double H[3][3];
    H[0][0] = (D(i + 2, j, k) - 2.0 * d0 + D(i - 2, j, k)) / fh2;
    H[1][1] = (D(i, j + 2, k) - 2.0 * d0 + D(i, j - 2, k)) / fh2;
    H[2][2] = (D(i, j, k + 2) - 2.0 * d0 + D(i, j, k - 2)) / fh2;
    H[0][1] = H[1][0] = (D(i + 1, j + 1, k) - D(i + 1, j - 1, k) - D(i - 1, j + 1, k) +
                         D(i - 1, j - 1, k)) / fh2;
    H[0][2] = H[2][0] = (D(i + 1, j, k + 1) - D(i + 1, j, k - 1) - D(i - 1, j, k + 1) +
                         D(i - 1, j, k - 1)) / fh2;
    H[1][2] = H[2][1] = (D(i, j + 1, k + 1) - D(i, j + 1, k - 1) - D(i, j - 1, k + 1) +
                         D(i, j - 1, k - 1)) / fh2;
    if (hybrid == 1) {
      double gHg = 0.0;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) gHg += g[a] * H[a][b] * g[b];
      if (std::fabs(gn - 1.0) > 0.05 || std::fabs(gHg) > 0.1 / h) G.bad[m] = 1;
    }
    dval[m] = d0;
    // Shape operator of the level set: tangential part of H.  Adding a large
    // multiple of g g^T isolates the normal direction as the top eigenvector,
    // so the other two eigenvectors span the tangent plane exactly even when
    // the tangential eigenvalues are degenerate.
    double Tm[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) Tm[a][b] = (a == b ? 1.0 : 0.0) - g[a] * g[b];
    double S[3][3];
    double hmax = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) hmax = std::max(hmax, std::fabs(H[a][b]));
    const double shift = 10.0 * hmax + 1.0 / h + 1.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double acc = 0.0;
        for (int c = 0; c < 3; ++c)
          for (int e = 0; e < 3; ++e) acc += Tm[a][c] * H[c][e] * Tm[e][b];
        S[a][b] = acc + shift * g[a] * g[b];
      }
    double V[3][3];
    jacobi3(S, V);
    int top = 0;
    for (int c = 1; c < 3; ++c)
      if (S[c][c] > S[top][top]) top = c;
    int t1 = (top + 1) % 3, t2 = (top + 2) % 3;
    // level-set curvatures (positive on a sphere): minus the Hessian eigenvalues
    const double ke1 = -S[t1][t1], ke2 = -S[t2][t2];
    const double J = (1.0 + d0 * ke1) * (1.0 + d0 * ke2);
    G.kap1[m] = ke1 / (1.0 + d0 * ke1);
    G.kap2[m] = ke2 / (1.0 + d0 * ke2);
    for (int a = 0; a < 3; ++a) {
      G.tau[6 * m + a] = V[a][t1];
      G.tau[6 * m + 3 + a] = V[a][t2];
    }
    const double xi = d0 / eps;
    const double phi = (std::fabs(xi) <= 1.0) ? 0.5 * (1.0 + std::cos(kPi * xi)) : 0.0;
    G.w[m] = J * phi / eps;
  }
  if (bad_grad) {
    *err = "zero finite-difference gradient at a tube node";
    return IBIM_EGEOM;
  }

  // Correction candidates, one per grid plane crossed by the normal line.
  const int cap = (int)std::ceil(2.0 * (eps + h) / h) + 6;
  std::vector<Candidate> cand((size_t)M * cap);
  std::vector<int32_t> count(M, 0);
  int64_t own_missing = -1;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < M; ++k) {
    const double xs[3] = {G.px[k], G.py[k], G.pz[k]};
    const double nv[3] = {G.nx[k], G.ny[k], G.nz[k]};
    int ia = 0;
    if (std::fabs(nv[1]) > std::fabs(nv[ia])) ia = 1;
    if (std::fabs(nv[2]) > std::fabs(nv[ia])) ia = 2;
    const int aa = (ia + 1) % 3, bb = (ia + 2) % 3;
    // Only line points with |s| <= eps + h can have their nearest node in the
    // tube around x*; crossings farther out (the far side of a thin body)
    // are not singular and are not corrected.
    const double reach = eps + h;
    const int plo = std::max(0, (int)std::floor((xs[ia] - reach - origin[ia]) / h) - 1);
    const int phi_ =
        std::min(plan->dims[ia] - 1, (int)std::ceil((xs[ia] + reach - origin[ia]) / h) + 1);
    Candidate* out = &cand[(size_t)k * cap];
    int cnt = 0;
    bool own = false;
    for (int p = plo; p <= phi_; ++p) {
      const double t = origin[ia] + (double)p * h;
      const double s = (t - xs[ia]) / nv[ia];
      if (!(std::fabs(s) <= reach)) continue;
      const double La = xs[aa] + s * nv[aa];
      const double Lb = xs[bb] + s * nv[bb];
      const double fa = (La - origin[aa]) / h;
      const double fb = (Lb - origin[bb]) / h;
      const double ja = std::floor(fa + 0.5);
      const double jb = std::floor(fb + 0.5);
      if (ja < 0.0 || jb < 0.0 || ja >= (double)plan->dims[aa] || jb >= (double)plan->dims[bb])
        continue;
      int gi[3];
      gi[ia] = p;
      gi[aa] = (int)ja;
      gi[bb] = (int)jb;
      const int32_t mcol = node_of[((int64_t)gi[0] * ny + gi[1]) * nz + gi[2]];
      if (mcol < 0) continue;
      if (cnt >= cap) break;
      if (mcol == (int32_t)k) own = true;
      out[cnt].col = mcol;
      out[cnt].axis = (int8_t)ia;
      out[cnt].alpha = fa - ja;
      out[cnt].beta = fb - jb;
      out[cnt].eta = -s;
      ++cnt;
    }
    std::sort(out, out + cnt, [](const Candidate& a, const Candidate& b) { return a.col < b.col; });
    count[k] = cnt;
    if (!own) {
#pragma omp critical
      own_missing = k;
    }
  }
  if (own_missing >= 0) {
    *err = "node " + std::to_string(own_missing) +
           " is not the nearest node of its own normal line (reach violated or degenerate normal)";
    return IBIM_EGEOM;
  }
  if (hybrid) {
    // bad rows by the plane margin, then J = 1 and the K-reg sets at bad nodes
    for (int64_t k = 0; k < M; ++k) {
      const double kmax = std::fmax(std::fabs(G.kap1[k]), std::fabs(G.kap2[k]));
      const Candidate* in = &cand[(size_t)k * cap];
      for (int c = 0; c < count[k]; ++c)
        if (1.0 - std::fabs(in[c].eta) * kmax < 0.2) G.bad[k] = 1;
    }
    for (int64_t m = 0; m < M; ++m)
      if (G.bad[m]) {
        const double xi = dval[m] / eps;
        const double phi = (std::fabs(xi) <= 1.0) ? 0.5 * (1.0 + std::cos(kPi * xi)) : 0.0;
        G.w[m] = phi / eps;
      }
  }
  std::vector<std::vector<Candidate>> kreg(M);
  if (hybrid) {
    const double tau = G.ktau, reach = eps + h;
    const double rb = std::sqrt(tau * tau + reach * reach) + eps;
    const int W = (int)std::ceil(rb / h);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < M; ++k) {
      if (!G.bad[k]) continue;
      const double xk[3] = {G.px[k], G.py[k], G.pz[k]};
      const double nk[3] = {G.nx[k], G.ny[k], G.nz[k]};
      const int i0 = ijk[3 * k], j0 = ijk[3 * k + 1], l0 = ijk[3 * k + 2];
      std::vector<Candidate>& out = kreg[k];
      for (int di = -W; di <= W; ++di)
        for (int dj = -W; dj <= W; ++dj)
          for (int dl = -W; dl <= W; ++dl) {
            const int i = i0 + di, j = j0 + dj, l = l0 + dl;
            if (i < 0 || j < 0 || l < 0 || i >= nx || j >= ny || l >= nz) continue;
            const int32_t mm = node_of[((int64_t)i * ny + j) * nz + l];
            if (mm < 0) continue;
            const double v0 = (origin[0] + (double)i * h) - xk[0];
            const double v1 = (origin[1] + (double)j * h) - xk[1];
            const double v2 = (origin[2] + (double)l * h) - xk[2];
            const double vn = v0 * nk[0] + v1 * nk[1] + v2 * nk[2];
            const double t0 = v0 - vn * nk[0], t1 = v1 - vn * nk[1], t2 = v2 - vn * nk[2];
            const double tt = t0 * t0 + t1 * t1 + t2 * t2;
            if (!(tt < tau * tau) || !(std::fabs(vn) <= reach)) continue;
            out.push_back(Candidate{mm, (int8_t)-1, 0.0, 0.0, vn});
          }
      std::sort(out.begin(), out.end(),
                [](const Candidate& a, const Candidate& b) { return a.col < b.col; });
    }
    for (int64_t k = 0; k < M; ++k) {
      if (!G.bad[k]) continue;
      count[k] = (int32_t)kreg[k].size();
      ++G.n_bad;
    }
  }
  G.crow.resize(M + 1);
  G.crow[0] = 0;
  for (int64_t k = 0; k < M; ++k) G.crow[k + 1] = G.crow[k] + count[k];
  const int64_t nnz = G.crow[M];
  if (nnz >= INT32_MAX) {
    *err = "too many correction entries";
    return IBIM_EINVAL;
  }
  G.ccol.resize(nnz); G.crowid.resize(nnz); G.caxis.resize(nnz);
  G.calpha.resize(nnz); G.cbeta.resize(nnz); G.ceta.resize(nnz);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < M; ++k) {
    const Candidate* in = G.bad[k] ? kreg[k].data() : &cand[(size_t)k * cap];
    for (int c = 0; c < count[k]; ++c) {
      const int64_t e = G.crow[k] + c;
      G.ccol[e] = in[c].col;
      G.crowid[e] = (int32_t)k;
      G.caxis[e] = in[c].axis;
      G.calpha[e] = in[c].alpha;
      G.cbeta[e] = in[c].beta;
      G.ceta[e] = in[c].eta;
    }
  }
  return IBIM_OK;
}

}  // namespace ibim
