/*
 * CTR-IBIM oracle: a plain, slow, FP64 CPU implementation of the discretised
 * linearised Poisson-Boltzmann system of Izzo, Zhong, Runborg and Tsai,
 * "Corrected trapezoidal rule-IBIM for linearized Poisson-Boltzmann equation"
 * (arXiv:2210.03699).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this file.  It shares no code with the
 * HIP library and must never be reached from the product path.
 *
 * Every function follows the paper's order of operations with no blocking,
 * fusion or reordering; OpenMP only distributes independent rows.
 *
 * Readings taken where the paper is silent or misprinted (each is also listed
 * in the design notes):
 *  - d > 0 inside, outward normal n = -grad d / |grad d| (Section 2.1).
 *  - psi_n is the interior normal derivative (Juffer BIE, eq. PB-BIE-1/2).
 *  - P(y) = y - d(y) g(y) with the *normalised* finite-difference gradient g.
 *  - Five-node stencils per direction (Section 3.3): gradient = central
 *    difference, Hessian = central difference of the central gradient.
 *  - Theorem 2.1 leading terms with the sign of s0^(11), s0^(22) flipped and
 *    the factor kappa^2 added to s0^(21) (derived from the kernels; pinned by
 *    the limit tests).
 *  - A plane is corrected iff its line point L = x* + s n has |s| <= eps + h
 *    and the nearest node of L lies in the tube; eta is the signed distance
 *    of the line point, -s along the outward normal.
 *  - Dominant axis ties go to the lowest axis; in-plane axes (i+1, i+2) mod 3.
 *  - Weights are evaluated exactly (Ewald form of the lattice sum that the
 *    limit definition eq. single_correction_weight reduces to), not from a
 *    table.
 *  - GMRES: x0 = 0, modified Gram-Schmidt, Givens rotations, stop when
 *    |g_{j+1}| <= tol ||b||_2; by default on the system with each block row
 *    divided by its free-term coefficient (D^-1 A x = D^-1 b, D = Lambda), the
 *    form whose iteration counts match the paper's; precond = 0 keeps A x = b.
 *  - HYB-IBIM (Section 3.2): the paper calls a node bad when its curvatures
 *    are away from the true ones, which needs the true surface.  From the
 *    signed distance alone a node is taken as bad when its finite-difference
 *    geometry is unreliable: | |grad_h d| - 1 | > 0.05, or the Hessian's
 *    normal component |g.H g| > 0.1/h, or a corrected plane has
 *    1 - |eta| max|kappa| < 0.2 (D0 near singular).  Bad rows use K-reg
 *    (eq. regularized-kernel) with tau = 2h; its regularised set is the tube
 *    nodes y with tangential distance |(I - n n^T)(y - P(y_k))| < tau and
 *    normal distance |n.(y - P(y_k))| <= eps + h (the same reach as the CTR2
 *    planes); bad nodes carry J = 1 (eq. Jacobian-hybrid).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OC_PI 3.14159265358979323846

/* Fourier modes kept for l(theta) (even modes 0..OC_KMAX), samples per 2 pi. */
#define OC_KMAX 80
#define OC_NMODE (OC_KMAX / 2 + 1)
#define OC_NTHETA 256
/* lattice half-width of both Ewald sums */
#define OC_NLAT 8

typedef struct {
  int64_t M;
  int dims[3];
  double origin[3];
  double h, eps, eps_in, eps_out, kappa;
  int64_t* grid_node; /* dims product; tube node index or -1 */
  int32_t* ijk;       /* 3M grid coordinates */
  double* y;          /* 3M node positions */
  double* d;          /* M signed distance */
  double* g;          /* 3M normalised gradient */
  double* nrm;        /* 3M outward normal */
  double* P;          /* 3M projection */
  double* J;          /* M Jacobian */
  double* w;          /* M J * delta_eps(d) */
  double* kap;        /* 2M surface principal curvatures */
  double* tau;        /* 6M principal directions (tau1, tau2) */
  /* correction sets N_k in CSR form */
  int64_t* crow;      /* M+1 */
  int64_t* ccol;
  int32_t* cplane;    /* dominant axis of the row, per entry */
  double* calpha;
  double* cbeta;
  double* ceta;
  double* om11;
  double* om21;
  int64_t nnz;
  /* HYB-IBIM (Section 3.2): node classification and K-reg parameter */
  int hybrid;         /* 0: CTR2 rows everywhere; 1: HYB; 2: every node bad (K-reg) */
  double ktau;        /* K-reg radius */
  double c12;         /* K-reg constant of K12 */
  unsigned char* bad; /* M: node in M_B */
} oc_ctx;

static char oc_err[512];
const char* oc_last_error(void) { return oc_err; }

static void* xmalloc(size_t n) {
  void* p = malloc(n ? n : 1);
  if (!p) {
    fprintf(stderr, "oracle: out of memory (%zu bytes)\n", n);
    abort();
  }
  return p;
}

void oc_free(oc_ctx* c) {
  if (!c) return;
  free(c->grid_node); free(c->ijk); free(c->y); free(c->d); free(c->g);
  free(c->nrm); free(c->P); free(c->J); free(c->w); free(c->kap); free(c->tau);
  free(c->crow); free(c->ccol); free(c->cplane); free(c->calpha); free(c->cbeta);
  free(c->ceta); free(c->om11); free(c->om21); free(c->bad);
  free(c);
}

/* ------------------------------------------------------------------------ */
/* K-reg constant of K12 (Section 2.3): the mean of K12 over the tangent disc
 * of radius tau, (e^{-k tau} - 1 + k tau) / (2 pi k tau^2); the constants of
 * K11, K21 and K22 are zero.  Small k tau by the series of the numerator. */
double oc_kreg_c12(double kappa, double tau) {
  if (kappa == 0.0) return 0.0;
  double x = kappa * tau, num;
  if (x < 1e-2)
    num = x * x * (0.5 - x * (1.0 / 6.0 - x * (1.0 / 24.0 - x / 120.0)));
  else
    num = expm1(-x) + x;
  return num / (2.0 * OC_PI * kappa * tau * tau);
}

/* ------------------------------------------------------------------------ */
/* Averaging kernel phi(x) = (1 + cos(pi x))/2 on |x| <= 1 (Section 2.6).    */
static double phi_cos(double x) {
  if (fabs(x) > 1.0) return 0.0;
  return 0.5 * (1.0 + cos(OC_PI * x));
}

/* ------------------------------------------------------------------------ */
/* Lattice sums behind the correction weights.                               */
/*
 * The weight omega[s; alpha, beta] of eq. (single_correction_weight) for
 * s(y) = |y|^-1 e^{ik psi(y)} is minus the regularised punctured lattice sum
 *     Z_k(a) = "sum"_{n in Z^2, n != 0} e^{ik psi(n-a)} / |n - a| ,
 * (the h -> 0 limit removes exactly the divergent integral).  Split with the
 * incomplete gamma function (Ewald) and Poisson-summed with the Hecke
 * identity for the harmonic polynomial (y1 + i y2)^k, this is
 *   Z_k(a) = sum_{n!=0} e^{ik psi(n-a)} Q(s, pi|n-a|^2)/|n-a|
 *          + (-i)^k sum_{m!=0} e^{ik psi(m)} e^{-2 pi i m.a} Q(s, pi|m|^2)/|m|
 *          - 2 [k = 0]
 *          - e^{ik psi(-a)} P(s, pi|a|^2)/|a|,            s = (k+1)/2,
 * with Q, P the regularised upper/lower incomplete gamma functions.  Only
 * even k are needed (l is pi-periodic).  zr[j] + i zi[j] = Z_{2j}.
 */
void oc_lattice_sums(double al, double be, int nmode, double* zr, double* zi) {
  for (int j = 0; j < nmode; ++j) zr[j] = zi[j] = 0.0;
  const double sqpi = sqrt(OC_PI);
  for (int pass = 0; pass < 2; ++pass) {
    for (int n1 = -OC_NLAT; n1 <= OC_NLAT; ++n1) {
      for (int n2 = -OC_NLAT; n2 <= OC_NLAT; ++n2) {
        if (n1 == 0 && n2 == 0) continue;
        double y1, y2, ph_r = 1.0, ph_i = 0.0;
        if (pass == 0) {
          y1 = n1 - al;
          y2 = n2 - be;
        } else {
          y1 = n1;
          y2 = n2;
          double arg = -2.0 * OC_PI * (n1 * al + n2 * be);
          ph_r = cos(arg);
          ph_i = sin(arg);
        }
        double r = sqrt(y1 * y1 + y2 * y2);
        double x = OC_PI * r * r;
        double Q = erfc(sqrt(x));                /* Q(1/2, x) */
        double term = sqrt(x) * exp(-x) / (0.5 * sqpi); /* x^s e^-x / Gamma(s+1), s=1/2 */
        double ur = y1 / r, ui = y2 / r;         /* e^{i psi} */
        double u2r = ur * ur - ui * ui, u2i = 2.0 * ur * ui;
        double zkr = 1.0, zki = 0.0;             /* e^{i k psi}, k = 0 */
        double s = 0.5;
        for (int j = 0; j < nmode; ++j) {
          double cr = zkr * Q / r, ci = zki * Q / r;
          if (pass == 1) {
            /* (-i)^k with k = 2j is (-1)^j; times the phase e^{-2 pi i m.a} */
            double sg = (j & 1) ? -1.0 : 1.0;
            double tr = cr * ph_r - ci * ph_i;
            double ti = cr * ph_i + ci * ph_r;
            cr = sg * tr;
            ci = sg * ti;
          }
          zr[j] += cr;
          zi[j] += ci;
          /* advance s -> s + 1 (two steps of k) */
          Q = Q + term;
          term = term * x / (s + 1.0);
          s += 1.0;
          double nr = zkr * u2r - zki * u2i;
          double ni = zkr * u2i + zki * u2r;
          zkr = nr;
          zki = ni;
        }
      }
    }
  }
  zr[0] += -2.0;
  double r0 = sqrt(al * al + be * be);
  if (r0 == 0.0) {
    zr[0] += -2.0; /* limit of -P(1/2, pi r^2)/r as r -> 0; zero for k > 0 */
    return;
  }
  double x0 = OC_PI * r0 * r0;
  double ur = -al / r0, ui = -be / r0;
  double u2r = ur * ur - ui * ui, u2i = 2.0 * ur * ui;
  double zkr = 1.0, zki = 0.0;
  double s = 0.5;
  /* pref = x^s e^-x / Gamma(s+1) */
  double pref = sqrt(x0) * exp(-x0) / (0.5 * sqpi);
  for (int j = 0; j < nmode; ++j) {
    /* P(s, x) = x^s e^-x / Gamma(s+1) * sum_l x^l / ((s+1)...(s+l)) */
    double sum = 0.0, t = 1.0;
    for (int l = 0; l < 200; ++l) {
      sum += t;
      t *= x0 / (s + 1.0 + l);
      if (t < 1e-18 * sum) break;
    }
    double Pv = pref * sum;
    zr[j] -= zkr * Pv / r0;
    zi[j] -= zki * Pv / r0;
    pref = pref * x0 / (s + 1.0);
    s += 1.0;
    double nr = zkr * u2r - zki * u2i;
    double ni = zkr * u2i + zki * u2r;
    zkr = nr;
    zki = ni;
  }
}

/* ------------------------------------------------------------------------ */
/* Leading terms l^(11), l^(21) of Theorem 2.1 (signs / kappa^2 corrected).  */
/*
 * A  = rows (tau1, tau2) restricted to the in-plane axes (a, b);
 * M  = diag(k1, k2); D0 = (I - eta M)^-1;  v = D0 A (cos t, sin t).
 * l11 = (eps_E/eps_I - 1) v^T M v / (8 pi |v|^3),  l21 = kappa^2 / (8 pi |v|).
 */
void oc_ell(const double* tau1, const double* tau2, double k1, double k2, double eta,
            int ax_a, int ax_b, double eps_in, double eps_out, double kappa, double theta,
            double* l11, double* l21) {
  double c = cos(theta), s = sin(theta);
  double A0 = tau1[ax_a] * c + tau1[ax_b] * s;
  double A1 = tau2[ax_a] * c + tau2[ax_b] * s;
  double v0 = A0 / (1.0 - eta * k1);
  double v1 = A1 / (1.0 - eta * k2);
  double vn = sqrt(v0 * v0 + v1 * v1);
  double qf = k1 * v0 * v0 + k2 * v1 * v1;
  *l11 = (eps_out / eps_in - 1.0) * qf / (8.0 * OC_PI * vn * vn * vn);
  *l21 = kappa * kappa / (8.0 * OC_PI * vn);
}

/* Fourier coefficients of l on [0, 2 pi) by the trapezoidal rule, combined
 * with the lattice sums: omega = sum_k a_k Wc_k + b_k Ws_k, W = -Z.  */
static void plane_weights(const double* tau1, const double* tau2, double k1, double k2,
                          double eta, int ax_a, int ax_b, double al, double be,
                          double eps_in, double eps_out, double kappa, double* om11,
                          double* om21) {
  double l11[OC_NTHETA], l21[OC_NTHETA];
  for (int p = 0; p < OC_NTHETA; ++p) {
    double th = 2.0 * OC_PI * p / OC_NTHETA;
    oc_ell(tau1, tau2, k1, k2, eta, ax_a, ax_b, eps_in, eps_out, kappa, th, &l11[p],
           &l21[p]);
  }
  double zr[OC_NMODE], zi[OC_NMODE];
  oc_lattice_sums(al, be, OC_NMODE, zr, zi);
  double o11 = 0.0, o21 = 0.0;
  for (int j = 0; j < OC_NMODE; ++j) {
    int k = 2 * j;
    double a11 = 0, b11 = 0, a21 = 0, b21 = 0;
    for (int p = 0; p < OC_NTHETA; ++p) {
      double th = 2.0 * OC_PI * p / OC_NTHETA;
      double ck = cos(k * th), sk = sin(k * th);
      a11 += l11[p] * ck;
      b11 += l11[p] * sk;
      a21 += l21[p] * ck;
      b21 += l21[p] * sk;
    }
    double f = (k == 0) ? 1.0 / OC_NTHETA : 2.0 / OC_NTHETA;
    a11 *= f; b11 *= f; a21 *= f; b21 *= f;
    o11 += -(a11 * zr[j] + b11 * zi[j]);
    o21 += -(a21 * zr[j] + b21 * zi[j]);
  }
  *om11 = o11;
  *om21 = o21;
}

/* exported for the tests: weights of one plane from its local geometry */
void oc_plane_weights(const double* tau1, const double* tau2, double k1, double k2,
                      double eta, int ax_a, int ax_b, double al, double be, double eps_in,
                      double eps_out, double kappa, double* om11, double* om21) {
  plane_weights(tau1, tau2, k1, k2, eta, ax_a, ax_b, al, be, eps_in, eps_out, kappa, om11,
                om21);
}

/* ------------------------------------------------------------------------ */
/* Symmetric 2x2 eigen-decomposition [[p, q], [q, r]].                       */
static void eig2(double p, double q, double r, double* mu, double* v /* 2x2 cols */) {
  double m = 0.5 * (p + r);
  double dd = sqrt(0.25 * (p - r) * (p - r) + q * q);
  mu[0] = m + dd;
  mu[1] = m - dd;
  if (dd == 0.0) {
    v[0] = 1; v[1] = 0; v[2] = 0; v[3] = 1;
    return;
  }
  /* eigenvector of mu0: (q, mu0 - p) or (mu0 - r, q), whichever is larger */
  double x1 = q, y1 = mu[0] - p;
  double x2 = mu[0] - r, y2 = q;
  double xa, ya;
  if (x1 * x1 + y1 * y1 >= x2 * x2 + y2 * y2) {
    xa = x1; ya = y1;
  } else {
    xa = x2; ya = y2;
  }
  double nn = sqrt(xa * xa + ya * ya);
  xa /= nn;
  ya /= nn;
  v[0] = xa; v[1] = ya;   /* column 0 */
  v[2] = -ya; v[3] = xa;  /* column 1, orthogonal */
}

/* ------------------------------------------------------------------------ */
/* Build: tube nodes, geometry, correction sets and weights.                 */
/* Returns NULL on error (message in oc_last_error()).                       */
/* Weights are computed for every row, or only for the rows listed in
 * weight_rows (other rows get NaN weights, so using them fails loudly). */
oc_ctx* oc_build_hyb(const double* sdf, int nx, int ny, int nz, const double* origin, double h,
                     double eps, double eps_in, double eps_out, double kappa, int hybrid,
                     const int64_t* weight_rows, int64_t n_weight_rows) {
  oc_err[0] = 0;
  if (!(h > 0) || !(eps > 0) || !(eps_in > 0) || !(eps_out > 0) || !(kappa >= 0) ||
      hybrid < 0 || hybrid > 2) {
    snprintf(oc_err, sizeof oc_err, "bad scalar parameter");
    return NULL;
  }
  oc_ctx* c = (oc_ctx*)calloc(1, sizeof(oc_ctx));
  c->hybrid = hybrid;
  c->ktau = 2.0 * h;
  c->c12 = oc_kreg_c12(kappa, c->ktau);
  c->dims[0] = nx; c->dims[1] = ny; c->dims[2] = nz;
  for (int a = 0; a < 3; ++a) c->origin[a] = origin[a];
  c->h = h; c->eps = eps; c->eps_in = eps_in; c->eps_out = eps_out; c->kappa = kappa;
  int64_t ng = (int64_t)nx * ny * nz;
  c->grid_node = (int64_t*)xmalloc(sizeof(int64_t) * ng);
  int64_t M = 0;
  for (int64_t q = 0; q < ng; ++q) {
    if (isnan(sdf[q])) {
      snprintf(oc_err, sizeof oc_err, "NaN in signed distance");
      oc_free(c);
      return NULL;
    }
    c->grid_node[q] = (fabs(sdf[q]) < eps) ? M++ : -1;
  }
  if (M == 0) {
    snprintf(oc_err, sizeof oc_err, "empty tube");
    oc_free(c);
    return NULL;
  }
  c->M = M;
  c->ijk = (int32_t*)xmalloc(sizeof(int32_t) * 3 * M);
  c->y = (double*)xmalloc(sizeof(double) * 3 * M);
  c->d = (double*)xmalloc(sizeof(double) * M);
  c->g = (double*)xmalloc(sizeof(double) * 3 * M);
  c->nrm = (double*)xmalloc(sizeof(double) * 3 * M);
  c->P = (double*)xmalloc(sizeof(double) * 3 * M);
  c->J = (double*)xmalloc(sizeof(double) * M);
  c->w = (double*)xmalloc(sizeof(double) * M);
  c->kap = (double*)xmalloc(sizeof(double) * 2 * M);
  c->tau = (double*)xmalloc(sizeof(double) * 6 * M);
  c->bad = (unsigned char*)calloc((size_t)M, 1);

#define SDF(i, j, k) sdf[((int64_t)(i) * ny + (j)) * nz + (k)]
  int bad = 0;
  for (int i = 0; i < nx; ++i)
    for (int j = 0; j < ny; ++j)
      for (int k = 0; k < nz; ++k) {
        int64_t m = c->grid_node[((int64_t)i * ny + j) * nz + k];
        if (m < 0) continue;
        if (i < 2 || j < 2 || k < 2 || i + 2 >= nx || j + 2 >= ny || k + 2 >= nz) bad = 1;
        c->ijk[3 * m] = i; c->ijk[3 * m + 1] = j; c->ijk[3 * m + 2] = k;
      }
  if (bad) {
    snprintf(oc_err, sizeof oc_err, "tube within two nodes of the grid edge");
    oc_free(c);
    return NULL;
  }

  for (int64_t m = 0; m < M; ++m) {
    int i = c->ijk[3 * m], j = c->ijk[3 * m + 1], k = c->ijk[3 * m + 2];
    double d0 = SDF(i, j, k);
    double y[3] = {origin[0] + (double)i * h, origin[1] + (double)j * h,
                   origin[2] + (double)k * h};
    /* central-difference gradient */
    double gx = (SDF(i + 1, j, k) - SDF(i - 1, j, k)) / (2.0 * h);
    double gy = (SDF(i, j + 1, k) - SDF(i, j - 1, k)) / (2.0 * h);
    double gz = (SDF(i, j, k + 1) - SDF(i, j, k - 1)) / (2.0 * h);
    /* Hessian: central difference of the central gradient (+-2 nodes) */
    double H[3][3];
    H[0][0] = (SDF(i + 2, j, k) - 2.0 * d0 + SDF(i - 2, j, k)) / (4.0 * h * h);
    H[1][1] = (SDF(i, j + 2, k) - 2.0 * d0 + SDF(i, j - 2, k)) / (4.0 * h * h);
    H[2][2] = (SDF(i, j, k + 2) - 2.0 * d0 + SDF(i, j, k - 2)) / (4.0 * h * h);
    H[0][1] = H[1][0] = (SDF(i + 1, j + 1, k) - SDF(i + 1, j - 1, k) - SDF(i - 1, j + 1, k) +
                         SDF(i - 1, j - 1, k)) / (4.0 * h * h);
    H[0][2] = H[2][0] = (SDF(i + 1, j, k + 1) - SDF(i + 1, j, k - 1) - SDF(i - 1, j, k + 1) +
                         SDF(i - 1, j, k - 1)) / (4.0 * h * h);
    H[1][2] = H[2][1] = (SDF(i, j + 1, k + 1) - SDF(i, j + 1, k - 1) - SDF(i, j - 1, k + 1) +
                         SDF(i, j - 1, k - 1)) / (4.0 * h * h);
    double gn = sqrt(gx * gx + gy * gy + gz * gz);
    double g[3] = {gx / gn, gy / gn, gz / gn};
    if (hybrid == 1) {
      /* unreliable finite-difference geometry: |grad| away from 1 or a large
       * Hessian component along the normal (a distance function has none) */
      double gHg = 0.0;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) gHg += g[a] * H[a][b] * g[b];
      if (fabs(gn - 1.0) > 0.05 || fabs(gHg) > 0.1 / h) c->bad[m] = 1;
    } else if (hybrid == 2) {
      c->bad[m] = 1;
    }
    for (int a = 0; a < 3; ++a) {
      c->y[3 * m + a] = y[a];
      c->g[3 * m + a] = g[a];
      c->nrm[3 * m + a] = -g[a];
      c->P[3 * m + a] = y[a] - d0 * g[a];
    }
    c->d[m] = d0;
    /* orthonormal tangent basis e1, e2 of the plane orthogonal to g */
    int sm = 0;
    if (fabs(g[1]) < fabs(g[sm])) sm = 1;
    if (fabs(g[2]) < fabs(g[sm])) sm = 2;
    double ax[3] = {0, 0, 0};
    ax[sm] = 1.0;
    double e1[3] = {g[1] * ax[2] - g[2] * ax[1], g[2] * ax[0] - g[0] * ax[2],
                    g[0] * ax[1] - g[1] * ax[0]};
    double e1n = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (int a = 0; a < 3; ++a) e1[a] /= e1n;
    double e2[3] = {g[1] * e1[2] - g[2] * e1[1], g[2] * e1[0] - g[0] * e1[2],
                    g[0] * e1[1] - g[1] * e1[0]};
    double B[2][2];
    const double* E[2] = {e1, e2};
    for (int p = 0; p < 2; ++p)
      for (int q = 0; q < 2; ++q) {
        double acc = 0.0;
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) acc += E[p][a] * H[a][b] * E[q][b];
        B[p][q] = acc;
      }
    double mu[2], V[4];
    eig2(B[0][0], 0.5 * (B[0][1] + B[1][0]), B[1][1], mu, V);
    /* level-set curvatures (positive on a sphere) and the Jacobian, eq. jacobian */
    double ke1 = -mu[0], ke2 = -mu[1];
    c->J[m] = 1.0 + d0 * (ke1 + ke2) + d0 * d0 * ke1 * ke2;
    /* principal curvatures of Gamma at P(y) */
    c->kap[2 * m] = ke1 / (1.0 + d0 * ke1);
    c->kap[2 * m + 1] = ke2 / (1.0 + d0 * ke2);
    for (int a = 0; a < 3; ++a) {
      c->tau[6 * m + a] = V[0] * e1[a] + V[1] * e2[a];
      c->tau[6 * m + 3 + a] = V[2] * e1[a] + V[3] * e2[a];
    }
    c->w[m] = c->J[m] * phi_cos(d0 / eps) / eps;
  }

  /* correction sets: one candidate node per grid plane along the dominant axis */
  int64_t cap = 16 * M + 16;
  c->crow = (int64_t*)xmalloc(sizeof(int64_t) * (M + 1));
  c->ccol = (int64_t*)xmalloc(sizeof(int64_t) * cap);
  c->cplane = (int32_t*)xmalloc(sizeof(int32_t) * cap);
  c->calpha = (double*)xmalloc(sizeof(double) * cap);
  c->cbeta = (double*)xmalloc(sizeof(double) * cap);
  c->ceta = (double*)xmalloc(sizeof(double) * cap);
  int64_t nnz = 0;
  for (int64_t k = 0; k < M; ++k) {
    c->crow[k] = nnz;
    const double* xs = &c->P[3 * k];
    const double* nv = &c->nrm[3 * k];
    int ia = 0;
    if (fabs(nv[1]) > fabs(nv[ia])) ia = 1;
    if (fabs(nv[2]) > fabs(nv[ia])) ia = 2;
    int aa = (ia + 1) % 3, bb = (ia + 2) % 3;
    /* Theorem 2.1 needs the line point in the tube around x*: only planes
     * whose line point has |s| <= eps + h can have their nearest node in the
     * tube (that node lies within h/sqrt(2) of the line point); farther
     * crossings of the normal line with the tube (the far side of a thin
     * body) are not singular and are not corrected. */
    double reach = eps + h;
    int lo = (int)floor((xs[ia] - reach - origin[ia]) / h) - 1;
    int hi = (int)ceil((xs[ia] + reach - origin[ia]) / h) + 1;
    int own = 0;
    for (int p = lo; p <= hi; ++p) {
      if (p < 0 || p >= c->dims[ia]) continue;
      double t = origin[ia] + (double)p * h;
      double s = (t - xs[ia]) / nv[ia];
      if (!(fabs(s) <= reach)) continue;
      double La = xs[aa] + s * nv[aa];
      double Lb = xs[bb] + s * nv[bb];
      double fa = (La - origin[aa]) / h;
      double fb = (Lb - origin[bb]) / h;
      double ja = floor(fa + 0.5), jb = floor(fb + 0.5);
      int g3[3];
      g3[ia] = p;
      g3[aa] = (int)ja;
      g3[bb] = (int)jb;
      if (g3[aa] < 0 || g3[aa] >= c->dims[aa] || g3[bb] < 0 || g3[bb] >= c->dims[bb]) continue;
      int64_t mm = c->grid_node[((int64_t)g3[0] * ny + g3[1]) * nz + g3[2]];
      if (mm < 0) continue;
      if (nnz >= cap) {
        snprintf(oc_err, sizeof oc_err, "correction capacity exceeded");
        oc_free(c);
        return NULL;
      }
      if (mm == k) own = 1;
      c->ccol[nnz] = mm;
      c->cplane[nnz] = ia;
      c->calpha[nnz] = fa - ja;
      c->cbeta[nnz] = fb - jb;
      c->ceta[nnz] = -s;
      ++nnz;
    }
    if (!own) {
      snprintf(oc_err, sizeof oc_err, "row %lld: own node not on its normal line",
               (long long)k);
      oc_free(c);
      return NULL;
    }
  }
  c->crow[M] = nnz;
  c->nnz = nnz;
  if (hybrid) {
    /* a corrected plane where 1 - |eta| max|kappa| < 0.2 makes D0 near singular */
    for (int64_t k = 0; k < M; ++k) {
      double kmax = fmax(fabs(c->kap[2 * k]), fabs(c->kap[2 * k + 1]));
      for (int64_t e = c->crow[k]; e < c->crow[k + 1]; ++e)
        if (1.0 - fabs(c->ceta[e]) * kmax < 0.2) c->bad[k] = 1;
    }
    /* eq. Jacobian-hybrid: J = 1 at bad nodes */
    for (int64_t m = 0; m < M; ++m)
      if (c->bad[m]) {
        c->J[m] = 1.0;
        c->w[m] = phi_cos(c->d[m] / eps) / eps;
      }
    /* bad rows: the regularised set of eq. (regularized-kernel) replaces N_k */
    const double tau = c->ktau, reach = eps + h;
    const double rb = sqrt(tau * tau + reach * reach) + eps;
    const int W = (int)ceil(rb / h);
    int64_t cap2 = nnz + 16;
    for (int64_t k = 0; k < M; ++k)
      if (c->bad[k]) cap2 += (int64_t)(2 * W + 1) * (2 * W + 1) * (2 * W + 1);
    int64_t* nrow = (int64_t*)xmalloc(sizeof(int64_t) * (M + 1));
    int64_t* ncol = (int64_t*)xmalloc(sizeof(int64_t) * cap2);
    int32_t* npl = (int32_t*)xmalloc(sizeof(int32_t) * cap2);
    double* nal = (double*)xmalloc(sizeof(double) * cap2);
    double* nbe = (double*)xmalloc(sizeof(double) * cap2);
    double* net = (double*)xmalloc(sizeof(double) * cap2);
    int64_t n2 = 0;
    for (int64_t k = 0; k < M; ++k) {
      nrow[k] = n2;
      if (!c->bad[k]) {
        for (int64_t e = c->crow[k]; e < c->crow[k + 1]; ++e) {
          ncol[n2] = c->ccol[e];
          npl[n2] = c->cplane[e];
          nal[n2] = c->calpha[e];
          nbe[n2] = c->cbeta[e];
          net[n2] = c->ceta[e];
          ++n2;
        }
        continue;
      }
      const double* xk = &c->P[3 * k];
      const double* nk = &c->nrm[3 * k];
      const int i0 = c->ijk[3 * k], j0 = c->ijk[3 * k + 1], l0 = c->ijk[3 * k + 2];
      int64_t start = n2;
      for (int di = -W; di <= W; ++di)
        for (int dj = -W; dj <= W; ++dj)
          for (int dl = -W; dl <= W; ++dl) {
            int i = i0 + di, j = j0 + dj, l = l0 + dl;
            if (i < 0 || j < 0 || l < 0 || i >= nx || j >= ny || l >= nz) continue;
            int64_t mm = c->grid_node[((int64_t)i * ny + j) * nz + l];
            if (mm < 0) continue;
            const double v0 = (origin[0] + (double)i * h) - xk[0];
            const double v1 = (origin[1] + (double)j * h) - xk[1];
            const double v2 = (origin[2] + (double)l * h) - xk[2];
            const double vn = v0 * nk[0] + v1 * nk[1] + v2 * nk[2];
            const double t0 = v0 - vn * nk[0], t1 = v1 - vn * nk[1], t2 = v2 - vn * nk[2];
            const double tt = t0 * t0 + t1 * t1 + t2 * t2;
            if (!(tt < tau * tau) || !(fabs(vn) <= reach)) continue;
            ncol[n2] = mm;
            npl[n2] = -1; /* K-reg entry */
            nal[n2] = 0.0;
            nbe[n2] = 0.0;
            net[n2] = vn;
            ++n2;
          }
      /* column order (insertion sort: short rows) */
      for (int64_t a = start + 1; a < n2; ++a)
        for (int64_t b = a; b > start && ncol[b - 1] > ncol[b]; --b) {
          int64_t tc = ncol[b]; ncol[b] = ncol[b - 1]; ncol[b - 1] = tc;
          double te = net[b]; net[b] = net[b - 1]; net[b - 1] = te;
        }
    }
    nrow[M] = n2;
    free(c->crow); free(c->ccol); free(c->cplane); free(c->calpha); free(c->cbeta);
    free(c->ceta);
    c->crow = nrow; c->ccol = ncol; c->cplane = npl; c->calpha = nal; c->cbeta = nbe;
    c->ceta = net;
    nnz = n2;
    c->nnz = nnz;
  }
  c->om11 = (double*)xmalloc(sizeof(double) * (nnz ? nnz : 1));
  c->om21 = (double*)xmalloc(sizeof(double) * (nnz ? nnz : 1));
  for (int64_t e = 0; e < nnz; ++e) c->om11[e] = c->om21[e] = NAN;
  int64_t nrows = weight_rows ? n_weight_rows : M;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < nrows; ++r) {
    int64_t k = weight_rows ? weight_rows[r] : r;
    if (k < 0 || k >= M) continue;
    for (int64_t e = c->crow[k]; e < c->crow[k + 1]; ++e) {
      int ia = c->cplane[e];
      if (ia < 0) { /* K-reg entry: its constants enter the apply directly */
        c->om11[e] = c->om21[e] = 0.0;
        continue;
      }
      plane_weights(&c->tau[6 * k], &c->tau[6 * k + 3], c->kap[2 * k], c->kap[2 * k + 1],
                    c->ceta[e], (ia + 1) % 3, (ia + 2) % 3, c->calpha[e], c->cbeta[e],
                    eps_in, eps_out, kappa, &c->om11[e], &c->om21[e]);
    }
  }
#undef SDF
  return c;
}

oc_ctx* oc_build_rows(const double* sdf, int nx, int ny, int nz, const double* origin, double h,
                      double eps, double eps_in, double eps_out, double kappa,
                      const int64_t* weight_rows, int64_t n_weight_rows) {
  return oc_build_hyb(sdf, nx, ny, nz, origin, h, eps, eps_in, eps_out, kappa, 0, weight_rows,
                      n_weight_rows);
}

oc_ctx* oc_build(const double* sdf, int nx, int ny, int nz, const double* origin, double h,
                 double eps, double eps_in, double eps_out, double kappa) {
  return oc_build_rows(sdf, nx, ny, nz, origin, h, eps, eps_in, eps_out, kappa, NULL, 0);
}

void oc_get_bad(const oc_ctx* c, unsigned char* bad) { memcpy(bad, c->bad, (size_t)c->M); }

/* ------------------------------------------------------------------------ */
/* Kernels K11, K12, K21, K22 of eq. (Kij-kernels) at target x (normal nx)   */
/* and source y (normal ny).                                                 */
/* phi2 = 1 - e^-x (1 + x), phi3 = 1 - e^-x (1 + x + x^2/3); e = e^-x.
 * Below x = 0.5 the Taylor series (no cancellation) is summed instead:
 *   phi2 = sum_{n>=2} (-1)^n (n-1) x^n / n!,
 *   phi3 = sum_{n>=2} (-1)^n (n-1)(3-n) x^n / (3 n!).                      */
static void phi23(double x, double e, double* p2, double* p3) {
  if (x < 0.5) {
    double s2 = 0.0, s3 = 0.0, t = x * x / 2.0; /* x^n / n!, n = 2 */
    for (int n = 2; n < 26; ++n) {
      double sg = (n & 1) ? -1.0 : 1.0;
      s2 += sg * (double)(n - 1) * t;
      s3 += sg * (double)(n - 1) * (double)(3 - n) / 3.0 * t;
      t *= x / (double)(n + 1);
    }
    *p2 = s2;
    *p3 = s3;
    return;
  }
  *p2 = 1.0 - e * (1.0 + x);
  *p3 = 1.0 - e * (1.0 + x + x * x / 3.0);
}

void oc_kernels(const double* x, const double* nx, const double* y, const double* ny,
                double eps_in, double eps_out, double kappa, double* K) {
  double r[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
  double R = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  double kr = kappa * R;
  double e = exp(-kr);
  double p2, p3;
  phi23(kr, e, &p2, &p3);
  double rny = r[0] * ny[0] + r[1] * ny[1] + r[2] * ny[2];
  double rnx = r[0] * nx[0] + r[1] * nx[1] + r[2] * nx[2];
  double nxny = nx[0] * ny[0] + nx[1] * ny[1] + nx[2] * ny[2];
  double fpi = 4.0 * OC_PI;
  double R3 = R * R * R;
  K[0] = rny / (fpi * R3) * (1.0 - (eps_out / eps_in) * e * (1.0 + kr));
  K[1] = -expm1(-kr) / (fpi * R);
  K[2] = nxny * p2 / (fpi * R3) - 3.0 * rnx * rny * p3 / (fpi * R3 * R * R);
  K[3] = -rnx / (fpi * R3) * (1.0 - (eps_in / eps_out) * e * (1.0 + kr));
}

/* ------------------------------------------------------------------------ */
/* One row of the operator, eq. (corr-trapz-rule-sys1/2).                    */
static void apply_row(const oc_ctx* c, const double* u, int64_t k, char* excl, double* o1,
                      double* o2) {
  const int64_t M = c->M;
  const double h = c->h, h2 = h * h, h3 = h * h * h;
  const double lam1 = 0.5 * (1.0 + c->eps_out / c->eps_in);
  const double lam2 = 0.5 * (1.0 + c->eps_in / c->eps_out);
  for (int64_t e = c->crow[k]; e < c->crow[k + 1]; ++e) excl[c->ccol[e]] = 1;
  const double* xk = &c->P[3 * k];
  const double* nk = &c->nrm[3 * k];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t m = 0; m < M; ++m) {
    if (excl[m]) continue;
    double K[4];
    oc_kernels(xk, nk, &c->P[3 * m], &c->nrm[3 * m], c->eps_in, c->eps_out, c->kappa, K);
    double a1 = u[m] * c->w[m], a2 = u[M + m] * c->w[m];
    s1 += K[0] * a1 - K[1] * a2;
    s2 += K[2] * a1 - K[3] * a2;
  }
  double c1 = 0.0, c2 = 0.0;
  const double w12 = c->kappa / (4.0 * OC_PI); /* omega^(12) = kappa/(4 pi) * omega[1] = kappa/(4 pi) */
  const double r22 = c->eps_in / c->eps_out;   /* omega^(22) = -(eps_I/eps_E) omega^(11) */
  for (int64_t e = c->crow[k]; e < c->crow[k + 1]; ++e) {
    int64_t m = c->ccol[e];
    double a1 = u[m] * c->w[m], a2 = u[M + m] * c->w[m];
    if (c->cplane[e] < 0) {
      /* K-reg: the regularised kernels are the constants 0, C12, 0, 0 */
      c1 += -h3 * c->c12 * a2;
    } else {
      c1 += h2 * c->om11[e] * a1 - h3 * w12 * a2;
      c2 += h2 * c->om21[e] * a1 - h2 * (-r22 * c->om11[e]) * a2;
    }
    excl[m] = 0;
  }
  *o1 = lam1 * u[k] + h3 * s1 + c1;
  *o2 = lam2 * u[M + k] + h3 * s2 + c2;
}

void oc_apply_rows(const oc_ctx* c, const double* u, const int64_t* rows, int64_t nrows,
                   double* out1, double* out2) {
#pragma omp parallel
  {
    char* excl = (char*)calloc((size_t)c->M, 1);
#pragma omp for schedule(dynamic, 4)
    for (int64_t r = 0; r < nrows; ++r) apply_row(c, u, rows[r], excl, &out1[r], &out2[r]);
    free(excl);
  }
}

void oc_apply(const oc_ctx* c, const double* u, double* out) {
  const int64_t M = c->M;
#pragma omp parallel
  {
    char* excl = (char*)calloc((size_t)M, 1);
#pragma omp for schedule(dynamic, 4)
    for (int64_t k = 0; k < M; ++k) apply_row(c, u, k, excl, &out[k], &out[M + k]);
    free(excl);
  }
}

/* ------------------------------------------------------------------------ */
/* Right-hand side g1, g2 of eq. (PB-lambda-g) at the projected nodes.        */
void oc_rhs(const oc_ctx* c, const double* zq, const double* q, int nc, double* g) {
  const int64_t M = c->M;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < M; ++k) {
    const double* x = &c->P[3 * k];
    const double* nk = &c->nrm[3 * k];
    double g1 = 0.0, g2 = 0.0;
    for (int j = 0; j < nc; ++j) {
      double r[3] = {x[0] - zq[3 * j], x[1] - zq[3 * j + 1], x[2] - zq[3 * j + 2]};
      double R = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
      double rn = r[0] * nk[0] + r[1] * nk[1] + r[2] * nk[2];
      g1 += q[j] / c->eps_in / (4.0 * OC_PI * R);
      g2 += q[j] / c->eps_in * (-rn / (4.0 * OC_PI * R * R * R));
    }
    g[k] = g1;
    g[M + k] = g2;
  }
}

/* ------------------------------------------------------------------------ */
/* Reaction potential (eq. psi-rxn, plain trapezoidal IBIM sum) and G_pol.   */
double oc_psi_rxn(const oc_ctx* c, const double* x, const double* z) {
  const int64_t M = c->M;
  const double h3 = c->h * c->h * c->h;
  double acc = 0.0;
  for (int64_t m = 0; m < M; ++m) {
    const double* y = &c->P[3 * m];
    const double* ny = &c->nrm[3 * m];
    double r[3] = {z[0] - y[0], z[1] - y[1], z[2] - y[2]};
    double R = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    double kr = c->kappa * R;
    double e = exp(-kr);
    double rn = r[0] * ny[0] + r[1] * ny[1] + r[2] * ny[2];
    double dG0 = rn / (4.0 * OC_PI * R * R * R);
    double dGk = dG0 * e * (1.0 + kr);
    double G0mGk = -expm1(-kr) / (4.0 * OC_PI * R);
    double f = ((c->eps_out / c->eps_in) * dGk - dG0) * x[m] + G0mGk * x[M + m];
    acc += f * c->w[m];
  }
  return h3 * acc;
}

double oc_energy(const oc_ctx* c, const double* x, const double* zq, const double* q, int nc) {
  double* psi = (double*)xmalloc(sizeof(double) * (nc ? nc : 1));
#pragma omp parallel for schedule(static)
  for (int j = 0; j < nc; ++j) psi[j] = oc_psi_rxn(c, x, &zq[3 * j]);
  double G = 0.0;
  for (int j = 0; j < nc; ++j) G += 0.5 * q[j] * psi[j];
  free(psi);
  return G;
}

double oc_area(const oc_ctx* c) {
  double s = 0.0;
  for (int64_t m = 0; m < c->M; ++m) s += c->w[m];
  return c->h * c->h * c->h * s;
}

/* ------------------------------------------------------------------------ */
/* Restarted GMRES(m): x0 = 0, modified Gram-Schmidt, Givens rotations.
 * precond = 1 solves D^-1 A x = D^-1 b with D = Lambda (lambda1 on the psi
 * rows, lambda2 on the psi_n rows): each block row divided by its free-term
 * coefficient; residuals and the stopping test are those of that system.    */
static void apply_op(const oc_ctx* c, int precond, const double* u, double* out) {
  oc_apply(c, u, out);
  if (!precond) return;
  const int64_t M = c->M;
  const double lam1 = 0.5 * (1.0 + c->eps_out / c->eps_in);
  const double lam2 = 0.5 * (1.0 + c->eps_in / c->eps_out);
  for (int64_t k = 0; k < M; ++k) {
    out[k] /= lam1;
    out[M + k] /= lam2;
  }
}

static double dot(const double* a, const double* b, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

int oc_gmres(const oc_ctx* c, const double* b_in, double tol, int restart, int maxit,
             int precond, double* x, int* iters, double* est_relres, double* true_relres) {
  const int64_t N = 2 * c->M;
  const int m = restart;
  double* b = (double*)xmalloc(sizeof(double) * N);
  memcpy(b, b_in, sizeof(double) * N);
  if (precond) {
    const double lam1 = 0.5 * (1.0 + c->eps_out / c->eps_in);
    const double lam2 = 0.5 * (1.0 + c->eps_in / c->eps_out);
    for (int64_t k = 0; k < c->M; ++k) {
      b[k] /= lam1;
      b[c->M + k] /= lam2;
    }
  }
  double* V = (double*)xmalloc(sizeof(double) * (size_t)N * (m + 1));
  double* H = (double*)calloc((size_t)(m + 1) * m, sizeof(double)); /* H[i*m + j] */
  double* cs = (double*)xmalloc(sizeof(double) * m);
  double* sn = (double*)xmalloc(sizeof(double) * m);
  double* gv = (double*)xmalloc(sizeof(double) * (m + 1));
  double* yv = (double*)xmalloc(sizeof(double) * m);
  double* r = (double*)xmalloc(sizeof(double) * N);
  for (int64_t i = 0; i < N; ++i) x[i] = 0.0;
  double bnorm = sqrt(dot(b, b, N));
  int total = 0, converged = 0;
  double resid = bnorm;
  if (bnorm == 0.0) {
    *iters = 0;
    *est_relres = 0.0;
    *true_relres = 0.0;
    free(V); free(H); free(cs); free(sn); free(gv); free(yv); free(r); free(b);
    return 0;
  }
  while (total < maxit && !converged) {
    /* r = b - A x */
    apply_op(c, precond, x, r);
    for (int64_t i = 0; i < N; ++i) r[i] = b[i] - r[i];
    double beta = sqrt(dot(r, r, N));
    if (beta <= tol * bnorm) {
      converged = 1;
      resid = beta;
      break;
    }
    for (int64_t i = 0; i < N; ++i) V[i] = r[i] / beta;
    for (int i = 0; i <= m; ++i) gv[i] = 0.0;
    gv[0] = beta;
    memset(H, 0, sizeof(double) * (size_t)(m + 1) * m);
    int jend = 0;
    for (int j = 0; j < m; ++j) {
      double* w = &V[(size_t)(j + 1) * N];
      apply_op(c, precond, &V[(size_t)j * N], w);
      ++total;
      for (int i = 0; i <= j; ++i) {
        double hij = dot(&V[(size_t)i * N], w, N);
        H[i * m + j] = hij;
        for (int64_t t = 0; t < N; ++t) w[t] -= hij * V[(size_t)i * N + t];
      }
      double hn = sqrt(dot(w, w, N));
      H[(j + 1) * m + j] = hn;
      if (hn > 0.0)
        for (int64_t t = 0; t < N; ++t) w[t] /= hn;
      for (int i = 0; i < j; ++i) {
        double t1 = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
        double t2 = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
        H[i * m + j] = t1;
        H[(i + 1) * m + j] = t2;
      }
      double den = hypot(H[j * m + j], H[(j + 1) * m + j]);
      cs[j] = H[j * m + j] / den;
      sn[j] = H[(j + 1) * m + j] / den;
      H[j * m + j] = den;
      H[(j + 1) * m + j] = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      jend = j + 1;
      resid = fabs(gv[j + 1]);
      if (resid <= tol * bnorm || hn == 0.0) {
        converged = 1;
        break;
      }
      if (total >= maxit) break;
    }
    /* back substitution H y = g and update x += V y */
    for (int i = jend - 1; i >= 0; --i) {
      double s = gv[i];
      for (int t = i + 1; t < jend; ++t) s -= H[i * m + t] * yv[t];
      yv[i] = s / H[i * m + i];
    }
    for (int i = 0; i < jend; ++i)
      for (int64_t t = 0; t < N; ++t) x[t] += yv[i] * V[(size_t)i * N + t];
  }
  apply_op(c, precond, x, r);
  for (int64_t i = 0; i < N; ++i) r[i] = b[i] - r[i];
  *true_relres = sqrt(dot(r, r, N)) / bnorm;
  *est_relres = resid / bnorm;
  *iters = total;
  free(V); free(H); free(cs); free(sn); free(gv); free(yv); free(r); free(b);
  return converged ? 0 : 1;
}

/* ------------------------------------------------------------------------ */
/* Accessors for the Python wrapper.                                         */
int64_t oc_num_nodes(const oc_ctx* c) { return c->M; }
int64_t oc_num_corrections(const oc_ctx* c) { return c->nnz; }

void oc_get_nodes(const oc_ctx* c, int32_t* ijk, double* y, double* d, double* P, double* nrm,
                  double* J, double* w, double* kap, double* tau) {
  const int64_t M = c->M;
  memcpy(ijk, c->ijk, sizeof(int32_t) * 3 * M);
  memcpy(y, c->y, sizeof(double) * 3 * M);
  memcpy(d, c->d, sizeof(double) * M);
  memcpy(P, c->P, sizeof(double) * 3 * M);
  memcpy(nrm, c->nrm, sizeof(double) * 3 * M);
  memcpy(J, c->J, sizeof(double) * M);
  memcpy(w, c->w, sizeof(double) * M);
  memcpy(kap, c->kap, sizeof(double) * 2 * M);
  memcpy(tau, c->tau, sizeof(double) * 6 * M);
}

void oc_get_corrections(const oc_ctx* c, int64_t* row, int64_t* col, int32_t* axis,
                        double* alpha, double* beta, double* eta, double* om11, double* om21) {
  memcpy(row, c->crow, sizeof(int64_t) * (c->M + 1));
  size_t n = (size_t)c->nnz;
  memcpy(col, c->ccol, sizeof(int64_t) * n);
  memcpy(axis, c->cplane, sizeof(int32_t) * n);
  memcpy(alpha, c->calpha, sizeof(double) * n);
  memcpy(beta, c->cbeta, sizeof(double) * n);
  memcpy(eta, c->ceta, sizeof(double) * n);
  memcpy(om11, c->om11, sizeof(double) * n);
  memcpy(om21, c->om21, sizeof(double) * n);
}

int oc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
