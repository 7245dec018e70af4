/*
 * oracle.c -- plain, slow, CPU-only FP64 reference for the short-range
 * Lennard-Jones molecular-dynamics hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  It is called by the test suite, by the smoke
 * check and by the benchmark's CPU-baseline leg, never by the product path.
 * It shares no code, header, table or helper with the HIP library.
 *
 * What it computes follows the paper's statement of the short-range MD
 * timestep (Introduction: neighbor list from a distance criterion, forces per
 * particle, propagation, re-sort; Cabana "Neighbor List Creation" and
 * "CabanaMD" subsections: Verlet lists by binning, Lennard-Jones force kernel
 * plus position integration).  The paper prints no formula for any of these,
 * so the textbook definitions are written out here, O(N^2) over all pairs:
 *
 *   minimum image (single shift):  d = x_i - x_j; if d > L/2: d -= L;
 *                                  else if d < -L/2: d += L   (per component)
 *   r^2 = (d0*d0 + d1*d1) + d2*d2, evaluated in that order, no contraction
 *   neighbor relation:  j != i and r^2 < rlist*rlist (strict)
 *   12-6 pair energy:   u(r) = 4 eps [ (sigma/r)^12 - (sigma/r)^6 ] for r^2 < rc^2
 *   pair scalar:        s(r) = -u'(r)/r,  F_i = sum_j s_ij d_ij
 *   per-atom energy:    e_i = 1/2 sum_j u_ij,  E = sum_i e_i
 *   virial:             W_ab = 1/2 sum_i sum_j d_ij,a s_ij d_ij,b
 *   velocity Verlet (m): v += dt/2 F/m; x += dt v; wrap; F(x); v += dt/2 F/m
 *
 * Parameters are per type pair, packed as the upper triangle of the
 * symmetric T x T table: entry (a,b), a <= b, sits at a*T - a*(a-1)/2 + (b-a).
 *
 * Adjoint (vector-Jacobian product of the forces).  For a cotangent g on the
 * forces, the gradient of L = sum_i g_i . F_i is, with K_ij the 3x3 Jacobian
 * d(s_ij d_ij)/d(d_ij) = s I + 2 s' d d^T (s' = ds/d(r^2)), and K_ij = K_ji:
 *   dL/dx_k      = sum_{j in N(k), r<rc} K_kj (g_k - g_j)
 *   dL/dtheta_p  = sum_i sum_{j : pair type p} g_i . d_ij  ds_ij/dtheta
 * with ds/deps = s/eps and ds/dsigma from differentiating s in sigma.
 * The pair set (r < rc) is held fixed: the truncation step is not
 * differentiated.
 *
 * Built with -O2 -fno-fast-math -ffp-contract=off; OpenMP over atoms i.
 * Every reduction over atoms is done serially over per-atom partials, so the
 * results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads an OpenMP parallel region of the oracle uses (1 without OpenMP). */
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Sets the thread count of later parallel regions (no effect without OpenMP). */
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

static int packed_index(int a, int b, int T) {
  if (a > b) { int t = a; a = b; b = t; }
  return a * T - a * (a - 1) / 2 + (b - a);
}

static double min_image(double d, double L) {
  if (d > 0.5 * L) d -= L;
  else if (d < -0.5 * L) d += L;
  return d;
}

/* d = minimum-image x_i - x_j; returns r^2 in the fixed evaluation order */
static double displacement(const double *xi, const double *xj, const double L[3], double d[3]) {
  d[0] = min_image(xi[0] - xj[0], L[0]);
  d[1] = min_image(xi[1] - xj[1], L[1]);
  d[2] = min_image(xi[2] - xj[2], L[2]);
  return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

/* 12-6 pair quantities, written from u(r) = 4 eps ((sigma/r)^12 - (sigma/r)^6). */
typedef struct {
  double u;        /* pair energy */
  double s;        /* -u'(r)/r */
  double ds_dr2;   /* d s / d(r^2) */
  double ds_deps;  /* d s / d eps */
  double ds_dsig;  /* d s / d sigma */
} pair_t;

static pair_t lj_pair(double r2, double eps, double sig) {
  pair_t p;
  double r = sqrt(r2);
  double sr = sig / r;
  double sr6 = pow(sr, 6.0);
  double sr12 = sr6 * sr6;
  p.u = 4.0 * eps * (sr12 - sr6);
  /* u'(r) = 4 eps (-12 sr^12 + 6 sr^6) / r, so s = -u'/r */
  p.s = 4.0 * eps * (12.0 * sr12 - 6.0 * sr6) / r2;
  /* s = 4 eps (12 sig^12 r^-14 - 6 sig^6 r^-8); d/d(r^2) of r^-2k is -k r^-2k-2 */
  p.ds_dr2 = 4.0 * eps * (-7.0 * 12.0 * sr12 + 4.0 * 6.0 * sr6) / (r2 * r2);
  p.ds_deps = p.s / eps;
  /* d/dsigma of sig^12 is 12 sig^11, of sig^6 is 6 sig^5 */
  p.ds_dsig = 4.0 * eps * (12.0 * 12.0 * sr12 - 6.0 * 6.0 * sr6) / (sig * r2);
  return p;
}

/* ---------------------------------------------------------------- grid --- */

/* Cell grid used by the binned counting sort: nc = floor(L/rlist) cells per
 * dimension (at least 1), reduced by one while the edge L/nc is not above
 * rlist by a relative margin of 1e-10, so that every pair within rlist sits in
 * adjacent cells whatever the rounding of x/h. */
void orc_grid(const double L[3], double rlist, int32_t nc[3]) {
  for (int k = 0; k < 3; ++k) {
    int64_t c = (int64_t)floor(L[k] / rlist);
    while (c > 1 && L[k] / (double)c < rlist * (1.0 + 1e-10)) --c;
    if (c < 1) c = 1;
    nc[k] = (int32_t)c;
  }
}

/* cell = min(floor(x/h), nc-1) per dimension with h = L/nc; x fastest. */
void orc_cell_index(int64_t n, const double *x, const double L[3], const int32_t nc[3],
                    int64_t *cell) {
  for (int64_t i = 0; i < n; ++i) {
    int64_t c[3];
    for (int k = 0; k < 3; ++k) {
      double h = L[k] / (double)nc[k];
      int64_t ck = (int64_t)floor(x[3 * i + k] / h);
      if (ck > nc[k] - 1) ck = nc[k] - 1;
      if (ck < 0) ck = 0;
      c[k] = ck;
    }
    cell[i] = (c[2] * nc[1] + c[1]) * nc[0] + c[0];
  }
}

/* ----------------------------------------------------------- neighbors --- */

/* Full Verlet list by brute force.  sel == NULL means every atom; otherwise
 * the rows are the atoms sel[0..nsel).  counts[k] = |N(sel[k])|. */
int64_t orc_neighbor_count(int64_t n, const double *x, const double L[3], double rlist,
                           int64_t nsel, const int64_t *sel, int32_t *counts) {
  double rl2 = rlist * rlist;
  int64_t rows = sel ? nsel : n;
  int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
  for (int64_t k = 0; k < rows; ++k) {
    int64_t i = sel ? sel[k] : k;
    int32_t c = 0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double d[3];
      if (displacement(x + 3 * i, x + 3 * j, L, d) < rl2) ++c;
    }
    counts[k] = c;
    total += c;
  }
  return total;
}

/* Fill the rows counted above, j ascending, into nbr[offsets[k] ..]. */
void orc_neighbor_fill(int64_t n, const double *x, const double L[3], double rlist,
                       int64_t nsel, const int64_t *sel, const int64_t *offsets,
                       int32_t *nbr) {
  double rl2 = rlist * rlist;
  int64_t rows = sel ? nsel : n;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < rows; ++k) {
    int64_t i = sel ? sel[k] : k;
    int64_t w = offsets[k];
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double d[3];
      if (displacement(x + 3 * i, x + 3 * j, L, d) < rl2) nbr[w++] = (int32_t)j;
    }
  }
}

/* The same relation as unordered pairs, each once: for every atom i the j > i
 * with r^2 < rlist^2, in ascending j, one pass over j > i (half the pair tests
 * of the two passes above).  Row i goes to upper[i*cap ..]; len[i] is its true
 * length, which may exceed cap (then the row is cut and the caller retries with
 * a larger cap). */
void orc_neighbor_upper(int64_t n, const double *x, const double L[3], double rlist, int32_t cap,
                        int32_t *upper, int32_t *len) {
  double rl2 = rlist * rlist;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    int32_t c = 0;
    int32_t *row = upper + (int64_t)cap * i;
    for (int64_t j = i + 1; j < n; ++j) {
      double d[3];
      if (displacement(x + 3 * i, x + 3 * j, L, d) < rl2) {
        if (c < cap) row[c] = (int32_t)j;
        ++c;
      }
    }
    len[i] = c;
  }
}

/* -------------------------------------------------------------- forces --- */

/* One row of the force sum.  js == NULL: all j != i; else the listed j. */
static void force_row(int64_t i, int64_t n, const double *x, const int32_t *type, int T,
                      const double *eps, const double *sig, const double L[3], double rc,
                      const int32_t *js, int64_t nj, double F[3], double *e, double W[6],
                      int64_t *npairs) {
  double rc2 = rc * rc;
  F[0] = F[1] = F[2] = 0.0;
  *e = 0.0;
  for (int q = 0; q < 6; ++q) W[q] = 0.0;
  int64_t cnt = js ? nj : n;
  for (int64_t q = 0; q < cnt; ++q) {
    int64_t j = js ? js[q] : q;
    if (j == i) continue;
    double d[3];
    double r2 = displacement(x + 3 * i, x + 3 * j, L, d);
    if (!(r2 < rc2)) continue;
    int p = packed_index(type ? type[i] : 0, type ? type[j] : 0, T);
    pair_t pr = lj_pair(r2, eps[p], sig[p]);
    double f[3] = {pr.s * d[0], pr.s * d[1], pr.s * d[2]};
    F[0] += f[0];
    F[1] += f[1];
    F[2] += f[2];
    *e += 0.5 * pr.u;
    W[0] += 0.5 * d[0] * f[0];
    W[1] += 0.5 * d[1] * f[1];
    W[2] += 0.5 * d[2] * f[2];
    W[3] += 0.5 * d[0] * f[1];
    W[4] += 0.5 * d[0] * f[2];
    W[5] += 0.5 * d[1] * f[2];
    if (npairs && j > i) npairs[p] += 1;
  }
}

/* All-pairs forces, per-atom energy and virial for rows sel (or all atoms).
 * F, e are per row; W[6] (xx, yy, zz, xy, xz, yz) and npairs[P] (unordered
 * pairs within rc with j > i, per packed type pair; only meaningful for
 * sel == NULL) are totals over the rows. */
void orc_forces(int64_t n, const double *x, const int32_t *type, int T, const double *eps,
                const double *sig, const double L[3], double rc, int64_t nsel,
                const int64_t *sel, double *F, double *e, double *W, int64_t *npairs) {
  int64_t rows = sel ? nsel : n;
  int P = T * (T + 1) / 2;
  double *Wrow = (double *)calloc((size_t)rows * 6, sizeof(double));
  int64_t *prow = npairs ? (int64_t *)calloc((size_t)rows * P, sizeof(int64_t)) : NULL;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < rows; ++k) {
    int64_t i = sel ? sel[k] : k;
    force_row(i, n, x, type, T, eps, sig, L, rc, NULL, 0, F + 3 * k, e + k, Wrow + 6 * k,
              prow ? prow + (int64_t)P * k : NULL);
  }
  if (W) {
    for (int q = 0; q < 6; ++q) W[q] = 0.0;
    for (int64_t k = 0; k < rows; ++k)
      for (int q = 0; q < 6; ++q) W[q] += Wrow[6 * k + q];
  }
  if (npairs) {
    for (int p = 0; p < P; ++p) npairs[p] = 0;
    for (int64_t k = 0; k < rows; ++k)
      for (int p = 0; p < P; ++p) npairs[p] += prow[(int64_t)P * k + p];
  }
  free(Wrow);
  free(prow);
}

/* Forces over a given CSR full list (offsets[n+1], nbr): the Verlet-list
 * mirror of the same definitions, used to follow a trajectory whose list is
 * rebuilt only every few steps.  npairs (may be NULL): unordered pairs of the
 * list within rc, per packed type pair. */
void orc_forces_list(int64_t n, const double *x, const int32_t *type, int T,
                     const double *eps, const double *sig, const double L[3], double rc,
                     const int64_t *offsets, const int32_t *nbr, double *F, double *e,
                     double *W, int64_t *npairs) {
  int P = T * (T + 1) / 2;
  double *Wrow = (double *)calloc((size_t)n * 6, sizeof(double));
  int64_t *prow = npairs ? (int64_t *)calloc((size_t)n * P, sizeof(int64_t)) : NULL;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    force_row(i, n, x, type, T, eps, sig, L, rc, nbr + offsets[i], offsets[i + 1] - offsets[i],
              F + 3 * i, e + i, Wrow + 6 * i, prow ? prow + (int64_t)P * i : NULL);
  }
  if (W) {
    for (int q = 0; q < 6; ++q) W[q] = 0.0;
    for (int64_t i = 0; i < n; ++i)
      for (int q = 0; q < 6; ++q) W[q] += Wrow[6 * i + q];
  }
  if (npairs) {
    for (int p = 0; p < P; ++p) npairs[p] = 0;
    for (int64_t i = 0; i < n; ++i)
      for (int p = 0; p < P; ++p) npairs[p] += prow[(int64_t)P * i + p];
  }
  free(Wrow);
  free(prow);
}

/* ------------------------------------------------------------- adjoint --- */

/* VJP of the forces for cotangent g [n][3]: gx [n][3], geps[P], gsig[P].
 * offsets == NULL: all pairs; else over the given CSR full list. */
void orc_force_vjp(int64_t n, const double *x, const int32_t *type, int T, const double *eps,
                   const double *sig, const double L[3], double rc, const int64_t *offsets,
                   const int32_t *nbr, const double *g, double *gx, double *geps,
                   double *gsig) {
  double rc2 = rc * rc;
  int P = T * (T + 1) / 2;
  double *prow = (double *)calloc((size_t)n * 2 * P, sizeof(double));
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    double acc[3] = {0.0, 0.0, 0.0};
    double *pe = prow + (int64_t)2 * P * i;
    double *ps = pe + P;
    int64_t cnt = offsets ? offsets[i + 1] - offsets[i] : n;
    for (int64_t q = 0; q < cnt; ++q) {
      int64_t j = offsets ? nbr[offsets[i] + q] : q;
      if (j == i) continue;
      double d[3];
      double r2 = displacement(x + 3 * i, x + 3 * j, L, d);
      if (!(r2 < rc2)) continue;
      int p = packed_index(type ? type[i] : 0, type ? type[j] : 0, T);
      pair_t pr = lj_pair(r2, eps[p], sig[p]);
      double dg[3] = {g[3 * i] - g[3 * j], g[3 * i + 1] - g[3 * j + 1],
                      g[3 * i + 2] - g[3 * j + 2]};
      double ddg = d[0] * dg[0] + d[1] * dg[1] + d[2] * dg[2];
      /* K (g_i - g_j) with K = s I + 2 s' d d^T */
      for (int a = 0; a < 3; ++a) acc[a] += pr.s * dg[a] + 2.0 * pr.ds_dr2 * d[a] * ddg;
      double gid = g[3 * i] * d[0] + g[3 * i + 1] * d[1] + g[3 * i + 2] * d[2];
      pe[p] += gid * pr.ds_deps;
      ps[p] += gid * pr.ds_dsig;
    }
    gx[3 * i] = acc[0];
    gx[3 * i + 1] = acc[1];
    gx[3 * i + 2] = acc[2];
  }
  for (int p = 0; p < P; ++p) geps[p] = gsig[p] = 0.0;
  for (int64_t i = 0; i < n; ++i)
    for (int p = 0; p < P; ++p) {
      geps[p] += prow[(int64_t)2 * P * i + p];
      gsig[p] += prow[(int64_t)2 * P * i + P + p];
    }
  free(prow);
}

/* ---------------------------------------------------------- integrator --- */

/* Half kick, drift and wrap of velocity Verlet.  img (may be NULL) counts box
 * crossings so that unwrapped positions are x + img*L. */
void orc_kick_drift(int64_t n, double *x, double *v, const double *F, double dt,
                    double mass, const double L[3], int32_t *img) {
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < 3; ++k) {
      int64_t q = 3 * i + k;
      v[q] += 0.5 * dt * F[q] / mass;
      x[q] += dt * v[q];
      if (x[q] >= L[k]) { x[q] -= L[k]; if (img) img[q] += 1; }
      else if (x[q] < 0.0) { x[q] += L[k]; if (img) img[q] -= 1; }
      if (x[q] >= L[k]) { x[q] -= L[k]; if (img) img[q] += 1; }
    }
}

/* Second half kick of velocity Verlet. */
void orc_kick(int64_t n, double *v, const double *F, double dt, double mass) {
  for (int64_t q = 0; q < 3 * n; ++q) v[q] += 0.5 * dt * F[q] / mass;
}
