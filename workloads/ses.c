/*
 * Signed distance (positive inside) to the solvent-excluded surface of a set
 * of atoms, sampled on a uniform grid.  Input generation only.
 *
 * With R_i = r_i + r_p, let B = union of the balls B(c_i, R_i) and A the
 * complement of B (probe centres).  The solvent region is A dilated by r_p,
 * the molecule its complement, and near the surface
 *     d(x) = dist(x, boundary of A) - r_p.
 * The nearest boundary point of A lies on an exposed sphere patch (radial
 * projection of x onto a sphere), an exposed circle arc of two spheres
 * (nearest point of the circle) or an exposed vertex of three spheres; a
 * candidate counts only if no other ball contains it.  Enclosed cavities are
 * removed in a second pass: solvent bubbles (grid nodes with d < 0 that a
 * flood fill from the grid boundary does not reach) are at least a probe
 * ball across and so resolved by the grid; the second pass rejects every
 * candidate whose nearest grid node lies in a bubble (a probe centre's own
 * ball lies in its bubble) and treats bubble nodes as interior.  Points
 * farther than `band` from the surface get a cheap bound with the right sign
 * instead: only candidates within probe + band are examined, nearest first,
 * and a point with none exposed gets a lower bound of at least band.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  double c[3];
  double R;
} Ball;

typedef struct {
  double C[3], u[3], rho; /* centre, unit axis, radius */
  int i, j;
} Circle;

typedef struct {
  double p[3];
  int i, j, k;
} Vertex;

static double dist3(const double* a, const double* b) {
  double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  return sqrt(dx * dx + dy * dy + dz * dz);
}

/* cell list over atom centres */
typedef struct {
  double lo[3], cs;
  int n[3];
  int* start; /* ncell + 1 */
  int* idx;
} Cells;

static int cell_of(const Cells* cl, const double* p, int a) {
  int v = (int)floor((p[a] - cl->lo[a]) / cl->cs);
  if (v < 0) v = 0;
  if (v >= cl->n[a]) v = cl->n[a] - 1;
  return v;
}

static void cells_build(Cells* cl, const Ball* b, int n, double cs) {
  for (int a = 0; a < 3; ++a) {
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < n; ++i) {
      if (b[i].c[a] < lo) lo = b[i].c[a];
      if (b[i].c[a] > hi) hi = b[i].c[a];
    }
    cl->lo[a] = lo - cs;
    cl->n[a] = (int)((hi - lo) / cs) + 3;
  }
  cl->cs = cs;
  int nc = cl->n[0] * cl->n[1] * cl->n[2];
  int* cnt = (int*)calloc((size_t)nc + 1, sizeof(int));
  int* cid = (int*)malloc(sizeof(int) * (size_t)n);
  for (int i = 0; i < n; ++i) {
    int ci = (cell_of(cl, b[i].c, 0) * cl->n[1] + cell_of(cl, b[i].c, 1)) * cl->n[2] +
             cell_of(cl, b[i].c, 2);
    cid[i] = ci;
    cnt[ci + 1]++;
  }
  for (int q = 0; q < nc; ++q) cnt[q + 1] += cnt[q];
  cl->start = cnt;
  cl->idx = (int*)malloc(sizeof(int) * (size_t)n);
  int* fill = (int*)calloc((size_t)nc, sizeof(int));
  for (int i = 0; i < n; ++i) cl->idx[cnt[cid[i]] + fill[cid[i]]++] = i;
  free(fill);
  free(cid);
}

/* growable list of indices */
typedef struct {
  int* v;
  int n, cap;
} IntBuf;

static void ib_push(IntBuf* b, int i) {
  if (b->n == b->cap) {
    b->cap = b->cap ? 2 * b->cap : 1024;
    b->v = (int*)realloc(b->v, sizeof(int) * (size_t)b->cap);
  }
  b->v[b->n++] = i;
}

/* every point with centre within `rad` of p -> out (replaced), returns count */
static int cells_query(const Cells* cl, const Ball* b, const double* p, double rad, IntBuf* out) {
  int lo[3], hi[3];
  out->n = 0;
  for (int a = 0; a < 3; ++a) {
    lo[a] = (int)floor((p[a] - rad - cl->lo[a]) / cl->cs);
    hi[a] = (int)floor((p[a] + rad - cl->lo[a]) / cl->cs);
    if (lo[a] < 0) lo[a] = 0;
    if (hi[a] >= cl->n[a]) hi[a] = cl->n[a] - 1;
  }
  for (int x = lo[0]; x <= hi[0]; ++x)
    for (int y = lo[1]; y <= hi[1]; ++y)
      for (int z = lo[2]; z <= hi[2]; ++z) {
        int q = (x * cl->n[1] + y) * cl->n[2] + z;
        for (int t = cl->start[q]; t < cl->start[q + 1]; ++t) {
          int i = cl->idx[t];
          if (dist3(b[i].c, p) < rad) ib_push(out, i);
        }
      }
  return out->n;
}

typedef struct {
  const uint8_t* bubble; /* grid flag: enclosed solvent (NULL in the first pass) */
  const double* origin;
  int nx, ny, nz;
  double h;
} GridInfo;

/* a boundary candidate of A: point p at distance dd from the grid node;
 * e1, e2: balls it lies on (excluded from its burial test); vertices were
 * tested at construction */
typedef struct {
  double dd, p[3];
  int e1, e2, vertex;
} Cand;

static int cand_cmp(const void* a, const void* b) {
  double x = ((const Cand*)a)->dd, y = ((const Cand*)b)->dd;
  return (x > y) - (x < y);
}

static int buried(const Ball* b, const int* nb, int nn, const double* p, int e1, int e2, int e3) {
  for (int t = 0; t < nn; ++t) {
    int k = nb[t];
    if (k == e1 || k == e2 || k == e3) continue;
    if (dist3(b[k].c, p) < b[k].R * (1.0 - 1e-12)) return 1;
  }
  return 0;
}

/* 1 if the probe centre p belongs to an enclosed cavity: its nearest grid
 * node is a bubble node. */
static int in_bubble(const GridInfo* g, const double* p) {
  if (!g->bubble) return 0;
  int ii = (int)floor((p[0] - g->origin[0]) / g->h + 0.5);
  int jj = (int)floor((p[1] - g->origin[1]) / g->h + 0.5);
  int kk = (int)floor((p[2] - g->origin[2]) / g->h + 0.5);
  if (ii < 0 || jj < 0 || kk < 0 || ii >= g->nx || jj >= g->ny || kk >= g->nz) return 0;
  return g->bubble[((int64_t)ii * g->ny + jj) * g->nz + kk];
}

/*
 * xyz (3n), radii (n), probe; grid (nx, ny, nz) at origin + h*(i,j,k);
 * band: points with |d| below about band get the exact value.  Returns 0.
 */
int ses_sdf(const double* xyz, const double* radii, int n, double probe, const double* origin,
            int nx, int ny, int nz, double h, double band, double* out) {
  if (n <= 0) return -1;
  Ball* b = (Ball*)malloc(sizeof(Ball) * (size_t)n);
  double Rmax = 0.0;
  for (int i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a) b[i].c[a] = xyz[3 * i + a];
    b[i].R = radii[i] + probe;
    if (b[i].R > Rmax) Rmax = b[i].R;
  }
  Cells cl, fcl; /* coarse cells for the wide query of step 1, fine ones elsewhere */
  cells_build(&cl, b, n, 2.0 * Rmax);
  cells_build(&fcl, b, n, 0.5 * Rmax);
  /* overlapping balls of every ball: a point on sphere i can only lie inside
   * ball k if the two balls overlap */
  int* ov_start = (int*)calloc((size_t)n + 1, sizeof(int));
  int ov_cap = 32 * n + 32;
  int* ov = (int*)malloc(sizeof(int) * ov_cap);
  {
    IntBuf qb = {0};
    for (int i = 0; i < n; ++i) {
      const int m = cells_query(&cl, b, b[i].c, 2.0 * Rmax, &qb);
      for (int t = 0; t < m; ++t) {
        int k = qb.v[t];
        if (k == i || dist3(b[i].c, b[k].c) >= b[i].R + b[k].R) continue;
        if (ov_start[i + 1] + 1 > ov_cap) {
          ov_cap *= 2;
          ov = (int*)realloc(ov, sizeof(int) * ov_cap);
        }
        ov[ov_start[i + 1]++] = k;
      }
      if (i + 1 < n) ov_start[i + 2] = ov_start[i + 1];
    }
    free(qb.v);
  }
  const int64_t ng = (int64_t)nx * ny * nz;

  /* 1. s(x) = min_i |x - c_i| - R_i (>= 0 in A), inner(x) = max_i R_i - |x - c_i| */
  double* s = (double*)malloc(sizeof(double) * ng);
  double* inner = (double*)malloc(sizeof(double) * ng);
  int* deepest = (int*)malloc(sizeof(int) * ng); /* the ball of largest depth, -1 if none */
#pragma omp parallel for schedule(dynamic, 4)
  for (int i = 0; i < nx; ++i) {
    IntBuf qb = {0};
    for (int j = 0; j < ny; ++j)
      for (int k = 0; k < nz; ++k) {
        double x[3] = {origin[0] + i * h, origin[1] + j * h, origin[2] + k * h};
        const int m = cells_query(&cl, b, x, 2.0 * Rmax + band + probe, &qb);
        const int* nb = qb.v;
        double sm = 1e300, im = -1e300;
        int deep = -1;
        for (int t = 0; t < m; ++t) {
          double dd = dist3(x, b[nb[t]].c) - b[nb[t]].R;
          if (dd < sm) sm = dd;
          if (-dd > im) {
            im = -dd;
            deep = nb[t];
          }
        }
        if (m == 0) sm = 1e300;
        int64_t q = ((int64_t)i * ny + j) * nz + k;
        s[q] = sm;
        inner[q] = im;
        deepest[q] = deep;
      }
    free(qb.v);
  }

  /* 2. circles of intersecting sphere pairs */
  int ccap = 64 * n + 64, nc = 0;
  Circle* circ = (Circle*)malloc(sizeof(Circle) * ccap);
  {
    IntBuf qb = {0};
    for (int i = 0; i < n; ++i) {
      const int m = cells_query(&cl, b, b[i].c, 2.0 * Rmax, &qb);
      for (int t = 0; t < m; ++t) {
        int j = qb.v[t];
        if (j <= i) continue;
        double D = dist3(b[i].c, b[j].c);
        if (D >= b[i].R + b[j].R || D <= fabs(b[i].R - b[j].R) || D == 0.0) continue;
        double a = (D * D + b[i].R * b[i].R - b[j].R * b[j].R) / (2.0 * D);
        double rho2 = b[i].R * b[i].R - a * a;
        if (rho2 <= 0.0) continue;
        if (nc >= ccap) {
          ccap *= 2;
          circ = (Circle*)realloc(circ, sizeof(Circle) * ccap);
        }
        Circle* C = &circ[nc++];
        for (int q = 0; q < 3; ++q) {
          C->u[q] = (b[j].c[q] - b[i].c[q]) / D;
          C->C[q] = b[i].c[q] + a * C->u[q];
        }
        C->rho = sqrt(rho2);
        C->i = i;
        C->j = j;
      }
    }
    free(qb.v);
  }
  /* circles listed under their first sphere (i < j) */
  int* cstart = (int*)calloc((size_t)n + 1, sizeof(int));
  int* cidx = (int*)malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
  for (int q = 0; q < nc; ++q) cstart[circ[q].i + 1]++;
  for (int i = 0; i < n; ++i) cstart[i + 1] += cstart[i];
  {
    int* fill = (int*)calloc((size_t)n, sizeof(int));
    for (int q = 0; q < nc; ++q) cidx[cstart[circ[q].i] + fill[circ[q].i]++] = q;
    free(fill);
  }
  /* 3. exposed vertices of sphere triples */
  int vcap = 64 * n + 64, nv = 0;
  Vertex* vert = (Vertex*)malloc(sizeof(Vertex) * vcap);
  {
    IntBuf qb = {0}, qb2 = {0};
    for (int ci = 0; ci < nc; ++ci) {
      const Circle* C = &circ[ci];
      const int m = cells_query(&cl, b, C->C, C->rho + Rmax, &qb);
      for (int t = 0; t < m; ++t) {
        int k = qb.v[t];
        if (k <= C->j) continue; /* i < j < k once */
        /* intersect circle with sphere k: points p = C + rho (cos t e1 + sin t e2) */
        double w[3] = {b[k].c[0] - C->C[0], b[k].c[1] - C->C[1], b[k].c[2] - C->C[2]};
        double wu = w[0] * C->u[0] + w[1] * C->u[1] + w[2] * C->u[2];
        double wp[3] = {w[0] - wu * C->u[0], w[1] - wu * C->u[1], w[2] - wu * C->u[2]};
        double L = sqrt(wp[0] * wp[0] + wp[1] * wp[1] + wp[2] * wp[2]);
        if (L == 0.0) continue;
        /* |p - c_k|^2 = rho^2 + |w|^2 - 2 rho L cos(phi) = R_k^2 */
        double ww = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
        double cph = (C->rho * C->rho + ww - b[k].R * b[k].R) / (2.0 * C->rho * L);
        if (cph <= -1.0 || cph >= 1.0) continue;
        double sph = sqrt(1.0 - cph * cph);
        double e1[3] = {wp[0] / L, wp[1] / L, wp[2] / L};
        double e2[3] = {C->u[1] * e1[2] - C->u[2] * e1[1], C->u[2] * e1[0] - C->u[0] * e1[2],
                        C->u[0] * e1[1] - C->u[1] * e1[0]};
        for (int sg = -1; sg <= 1; sg += 2) {
          double p[3];
          for (int q = 0; q < 3; ++q) p[q] = C->C[q] + C->rho * (cph * e1[q] + sg * sph * e2[q]);
          const int m2 = cells_query(&fcl, b, p, Rmax, &qb2);
          if (buried(b, qb2.v, m2, p, C->i, C->j, k)) continue;
          if (nv >= vcap) {
            vcap *= 2;
            vert = (Vertex*)realloc(vert, sizeof(Vertex) * vcap);
          }
          Vertex* V = &vert[nv++];
          for (int q = 0; q < 3; ++q) V->p[q] = p[q];
          V->i = C->i;
          V->j = C->j;
          V->k = k;
        }
      }
    }
    free(qb.v);
    free(qb2.v);
  }
  /* cell list over the vertices (reuse the Ball layout) */
  Ball* vb = (Ball*)malloc(sizeof(Ball) * (nv > 0 ? nv : 1));
  for (int q = 0; q < nv; ++q) {
    for (int a = 0; a < 3; ++a) vb[q].c[a] = vert[q].p[a];
    vb[q].R = 0.0;
  }
  /* cells of edge Rmax for the sphere queries of step 4 (radius at most
   * Rmax + reach_d), half that for the vertex queries */
  Cells acl, vcl;
  cells_build(&acl, b, n, Rmax);
  if (nv > 0) cells_build(&vcl, vb, nv, 0.5 * Rmax);

  /* 4. distances: pass 0 keeps every exposed candidate, pass 1 drops the
   * candidates of enclosed solvent bubbles found after pass 0.  Two exact
   * prunings keep the candidate lists short.  (a) A point inside ball k at
   * depth D = R_k - |x - c_k| has every point within D of it inside that
   * ball, so a candidate nearer than the deepest ball's depth (inner[q]),
   * less a slack far above rounding and the 1e-12 burial margin, is buried
   * and skipped untested; so is a candidate that the burial test of that
   * ball alone finds inside it (buried() would find that ball: the point lies
   * on a sphere that the ball overlaps).  (b) Vertices are stored only when
   * exposed, so the nearest vertex bounds the answer and farther candidates
   * are skipped.
   * Pass 1 recomputes only bubble nodes and nodes whose pass-0 candidate lies
   * in a bubble: elsewhere the candidates before the chosen one were buried
   * and stay so, and the chosen one stays valid. */
  const double reach_d = probe + band; /* candidates farther than this do not matter */
  const double slack = 1e-12 * Rmax + 1e-9;
  uint8_t* bubble = NULL;
  int64_t* chosen = (int64_t*)malloc(sizeof(int64_t) * ng); /* nearest node of the chosen candidate */
  for (int pass = 0; pass < 2; ++pass) {
  GridInfo gi = {bubble, origin, nx, ny, nz, h};
#pragma omp parallel for schedule(dynamic, 2)
  for (int i = 0; i < nx; ++i) {
    IntBuf qb = {0};
    Cand* cand = NULL;
    int cand_cap = 0;
    int64_t* stamp = (int64_t*)malloc(sizeof(int64_t) * (size_t)n); /* last node each sphere passed */
    double* sdist = (double*)malloc(sizeof(double) * (size_t)n);
    for (int a = 0; a < n; ++a) stamp[a] = -1;
    for (int j = 0; j < ny; ++j) {
      /* signed distance to the boundary of B (positive inside) at the
       * previous node of this line when it is exact; it is 1-Lipschitz, so
       * the answer here lies within h of it (pass 0 only) */
      int prev_exact = 0;
      double Dprev = 0.0;
      for (int k = 0; k < nz; ++k) {
        int64_t q = ((int64_t)i * ny + j) * nz + k;
        const int nb_ok = pass == 0 && prev_exact;
        prev_exact = 0;
        if (pass == 1 && !bubble[q] && (chosen[q] < 0 || !bubble[chosen[q]])) continue;
        chosen[q] = -1;
        double x[3] = {origin[0] + i * h, origin[1] + j * h, origin[2] + k * h};
        if (s[q] >= 0.0 && !(bubble && bubble[q])) {
          /* probe centre: at least r_p from the molecule */
          out[q] = -(probe + (s[q] < 1e3 ? s[q] : 1e3));
          /* s is the exact distance to B when the nearest ball's centre lay
           * within the radius of step 1 */
          if (s[q] <= Rmax + band + probe) {
            prev_exact = 1;
            Dprev = -s[q];
          }
          continue;
        }
        if (inner[q] - probe > band) {
          out[q] = inner[q] - probe; /* deep inside: a lower bound is enough */
          continue;
        }
        double lower = inner[q] - slack;
        double upper = 1e300;
        if (nb_ok) {
          if (Dprev - h - slack > lower) lower = Dprev - h - slack;
          upper = Dprev + h + slack;
        }
        const int kd = deepest[q];
        /* exposed vertices within reach_d (outside bubbles in pass 1) */
        int nk = 0;
        if (nv > 0) {
          const double vrad = upper < reach_d ? upper : reach_d;
          const int mv = cells_query(&vcl, vb, x, vrad, &qb);
          if (mv > cand_cap) {
            cand_cap = 2 * mv;
            cand = (Cand*)realloc(cand, sizeof(Cand) * (size_t)cand_cap);
          }
          for (int t = 0; t < mv; ++t) {
            const Vertex* V = &vert[qb.v[t]];
            if (in_bubble(&gi, V->p)) continue;
            Cand* K = &cand[nk++];
            for (int a = 0; a < 3; ++a) K->p[a] = V->p[a];
            K->dd = dist3(x, V->p);
            K->e1 = K->e2 = -1;
            K->vertex = 1;
            if (K->dd < upper) upper = K->dd;
          }
        }
        /* sphere patches and circle arcs within reach_d, between the bounds.
         * A patch or arc point within bnd of x lies on a sphere within bnd
         * of x (|R_i - |x - c_i|| <= bnd), whose centre is within Rmax + bnd;
         * an arc is examined only when both of its spheres are. */
        const double bnd = upper < reach_d ? upper : reach_d;
        const int m = cells_query(&acl, b, x, Rmax + bnd + slack, &qb);
        int nsel = 0;
        for (int t = 0; t < m; ++t) {
          const int ib = qb.v[t];
          const double dxc = dist3(x, b[ib].c);
          if (fabs(b[ib].R - dxc) > bnd + slack) continue;
          stamp[ib] = q;  /* sphere ib passes within bnd of x */
          qb.v[nsel] = ib;
          sdist[nsel++] = dxc;
        }
        for (int t = 0; t < nsel; ++t) {
          const int ib = qb.v[t];
          const Ball* B = &b[ib];
          const double dxc = sdist[t];
          const double sd = fabs(B->R - dxc);
          if (nk + 1 + (cstart[ib + 1] - cstart[ib]) > cand_cap) {
            cand_cap = 2 * (nk + 1 + (cstart[ib + 1] - cstart[ib]));
            cand = (Cand*)realloc(cand, sizeof(Cand) * (size_t)cand_cap);
          }
          if (dxc != 0.0 && sd <= reach_d && sd >= lower && sd <= upper) {
            Cand* K = &cand[nk];
            K->dd = sd;
            for (int a = 0; a < 3; ++a) K->p[a] = B->c[a] + B->R * ((x[a] - B->c[a]) / dxc);
            if (!(kd >= 0 && kd != ib && dist3(b[kd].c, K->p) < b[kd].R * (1.0 - 1e-12))) {
              ++nk;
              K->e1 = ib;
              K->e2 = -1;
              K->vertex = 0;
            }
          }
          /* circles on this sphere and a later one */
          for (int u = cstart[ib]; u < cstart[ib + 1]; ++u) {
            const Circle* C = &circ[cidx[u]];
            if (stamp[C->j] != q) continue;
            double w[3] = {x[0] - C->C[0], x[1] - C->C[1], x[2] - C->C[2]};
            /* every point of the circle is at least |x - C| - rho away */
            if (sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]) - C->rho > reach_d) continue;
            double wu = w[0] * C->u[0] + w[1] * C->u[1] + w[2] * C->u[2];
            double wp[3] = {w[0] - wu * C->u[0], w[1] - wu * C->u[1], w[2] - wu * C->u[2]};
            double L = sqrt(wp[0] * wp[0] + wp[1] * wp[1] + wp[2] * wp[2]);
            if (L == 0.0) continue;
            Cand* K = &cand[nk];
            for (int a = 0; a < 3; ++a) K->p[a] = C->C[a] + C->rho * wp[a] / L;
            K->dd = dist3(x, K->p);
            if (K->dd > reach_d || K->dd < lower || K->dd > upper) continue;
            if (kd >= 0 && kd != C->i && kd != C->j &&
                dist3(b[kd].c, K->p) < b[kd].R * (1.0 - 1e-12))
              continue;
            ++nk;
            K->e1 = C->i;
            K->e2 = C->j;
            K->vertex = 0;
          }
        }
        qsort(cand, (size_t)nk, sizeof(Cand), cand_cmp);
        double best = 1e300;
        for (int t = 0; t < nk; ++t) {
          const Cand* K = &cand[t];
          if (!K->vertex) {
            const int o0 = ov_start[K->e1], o1 = ov_start[K->e1 + 1];
            if (buried(b, ov + o0, o1 - o0, K->p, K->e1, K->e2, -1)) continue;
            if (in_bubble(&gi, K->p)) continue;
          }
          best = K->dd;
          /* the nearest grid node of the chosen point (as in_bubble rounds it) */
          const int ii = (int)floor((K->p[0] - origin[0]) / h + 0.5);
          const int jj = (int)floor((K->p[1] - origin[1]) / h + 0.5);
          const int kk = (int)floor((K->p[2] - origin[2]) / h + 0.5);
          if (ii >= 0 && jj >= 0 && kk >= 0 && ii < nx && jj < ny && kk < nz)
            chosen[q] = ((int64_t)ii * ny + jj) * nz + kk;
          break;
        }
        /* no exposed boundary point within reach_d: the distance is at least
         * reach_d (and at least the ball depth) */
        if (best > 1e299) best = inner[q] > reach_d ? inner[q] : reach_d;
        out[q] = best - probe;
        if (best < 1e299) {
          prev_exact = 1;
          Dprev = best;
        }
      }
    }
    free(qb.v);
    free(cand);
    free(stamp);
    free(sdist);
  }
  if (pass == 0) {
    /* flood fill the solvent (d < 0) from the grid boundary */
    uint8_t* reach = (uint8_t*)calloc(ng, 1);
    int64_t* stack = (int64_t*)malloc(sizeof(int64_t) * ng);
    int64_t top = 0;
    for (int i = 0; i < nx; ++i)
      for (int j = 0; j < ny; ++j)
        for (int k = 0; k < nz; ++k) {
          if (i == 0 || j == 0 || k == 0 || i == nx - 1 || j == ny - 1 || k == nz - 1) {
            int64_t q = ((int64_t)i * ny + j) * nz + k;
            if (out[q] < 0.0 && !reach[q]) {
              reach[q] = 1;
              stack[top++] = q;
            }
          }
        }
    while (top > 0) {
      int64_t q = stack[--top];
      int i = (int)(q / ((int64_t)ny * nz)), j = (int)((q / nz) % ny), k = (int)(q % nz);
      int nbr[6][3] = {{i - 1, j, k}, {i + 1, j, k}, {i, j - 1, k},
                       {i, j + 1, k}, {i, j, k - 1}, {i, j, k + 1}};
      for (int t = 0; t < 6; ++t) {
        int a = nbr[t][0], c = nbr[t][1], e = nbr[t][2];
        if (a < 0 || c < 0 || e < 0 || a >= nx || c >= ny || e >= nz) continue;
        int64_t r = ((int64_t)a * ny + c) * nz + e;
        if (out[r] < 0.0 && !reach[r]) {
          reach[r] = 1;
          stack[top++] = r;
        }
      }
    }
    free(stack);
    bubble = (uint8_t*)calloc(ng, 1);
    int64_t nb_bubble = 0;
    for (int64_t q = 0; q < ng; ++q) {
      bubble[q] = (out[q] < 0.0 && !reach[q]) ? 1 : 0;
      nb_bubble += bubble[q];
    }
    free(reach);
    if (nb_bubble == 0) break; /* no enclosed cavity: pass 0 is final */
  }
  }
  free(bubble);
  free(chosen);
  free(b);
  free(s);
  free(inner);
  free(deepest);
  free(circ);
  free(vert);
  free(vb);
  free(cl.start);
  free(cl.idx);
  free(fcl.start);
  free(fcl.idx);
  free(acl.start);
  free(acl.idx);
  free(ov_start);
  free(ov);
  free(cstart);
  free(cidx);
  if (nv > 0) {
    free(vcl.start);
    free(vcl.idx);
  }
  return 0;
}
