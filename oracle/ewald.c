/*
 * ewald.c -- plain, slow, CPU-only FP64 reference for the Ewald sum of point
 * charges in a periodic orthorhombic box (test infrastructure only, under the
 * same rules as oracle.c).
 *
 * The paper's CabanaMD subsection composes the short-range path with smooth
 * particle-mesh Ewald (real space over the neighbor loops; spline spreading of
 * charge to a grid, 3-D FFTs and a gradient gather for reciprocal space; see
 * also Cabana "Long Range Solvers" and "Particle-Grid Interpolation") without
 * printing its equations.  SPME approximates the Ewald sum; the textbook Ewald sum
 * (Gaussian units, charges q_i, splitting parameter alpha, volume V, neutral
 * system, conducting boundary) is written out here:
 *
 *   E      = E_dir + E_rec + E_self
 *   E_dir  = 1/2 sum_i sum_{j != i, r_ij < rc} q_i q_j erfc(alpha r_ij) / r_ij
 *            (minimum image; rc <= L/2, so one image per pair)
 *   E_rec  = 1/(2 pi V) sum_{m != 0, |n_a| <= nmax} exp(-pi^2 |m|^2 / alpha^2) / |m|^2 |S(m)|^2
 *            m = (n_0/L_0, n_1/L_1, n_2/L_2),  S(m) = sum_j q_j exp(2 pi i m . x_j)
 *   E_self = -alpha / sqrt(pi) sum_i q_i^2
 *   F_i    = -dE/dx_i:
 *     direct:     sum_j q_i q_j [erfc(alpha r)/r + 2 alpha/sqrt(pi) exp(-alpha^2 r^2)] d_ij / r^2
 *     reciprocal: (2 q_i / V) sum_m exp(-pi^2 |m|^2/alpha^2)/|m|^2 m Im(conj(S(m)) exp(2 pi i m . x_i))
 *
 * Built with -O2 -fno-fast-math -ffp-contract=off; OpenMP over rows or k-vectors.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static const double kPiE = 3.14159265358979323846;

static double ew_min_image(double d, double L) {
  if (d > 0.5 * L) d -= L;
  else if (d < -0.5 * L) d += L;
  return d;
}

/* Direct-space part for rows sel[0..nsel) (all rows when sel is NULL; then
 * nsel = n): per-particle energy halves e_dir[k] (their sum over all rows is
 * E_dir) and forces F_dir[3k..3k+2] of particle sel[k]; all pairs with r < rc. */
void orc_ewald_direct(int64_t n, const double *x, const double *q, const double L[3],
                      double alpha, double rc, int64_t nsel, const int64_t *sel, double *e_dir,
                      double *F_dir) {
  const double c = 2.0 * alpha / sqrt(kPiE);
  const double rc2 = rc * rc;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < nsel; ++k) {
    const int64_t i = sel ? sel[k] : k;
    double e = 0.0, f[3] = {0.0, 0.0, 0.0};
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double d[3];
      d[0] = ew_min_image(x[3 * i] - x[3 * j], L[0]);
      d[1] = ew_min_image(x[3 * i + 1] - x[3 * j + 1], L[1]);
      d[2] = ew_min_image(x[3 * i + 2] - x[3 * j + 2], L[2]);
      double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
      if (!(r2 < rc2)) continue;
      double r = sqrt(r2);
      double qq = q[i] * q[j];
      double er = erfc(alpha * r) / r;
      e += 0.5 * qq * er;
      double s = qq * (er + c * exp(-alpha * alpha * r2)) / r2;
      f[0] += s * d[0];
      f[1] += s * d[1];
      f[2] += s * d[2];
    }
    e_dir[k] = e;
    F_dir[3 * k] = f[0];
    F_dir[3 * k + 1] = f[1];
    F_dir[3 * k + 2] = f[2];
  }
}

/* Reciprocal part over every m with |n_a| <= nmax, m != 0: returns E_rec and
 * writes F_rec [n][3]. */
double orc_ewald_recip(int64_t n, const double *x, const double *q, const double L[3],
                       double alpha, int nmax, double *F_rec) {
  const double V = L[0] * L[1] * L[2];
  const int side = 2 * nmax + 1;
  const int64_t nk = (int64_t)side * side * side;
  double *Sre = (double *)calloc((size_t)nk, sizeof(double));
  double *Sim = (double *)calloc((size_t)nk, sizeof(double));
  double *fac = (double *)calloc((size_t)nk, sizeof(double));
  double E = 0.0;
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t k = 0; k < nk; ++k) {
    int n0 = (int)(k % side) - nmax, n1 = (int)((k / side) % side) - nmax,
        n2 = (int)(k / ((int64_t)side * side)) - nmax;
    if (n0 == 0 && n1 == 0 && n2 == 0) continue;
    double m0 = n0 / L[0], m1 = n1 / L[1], m2 = n2 / L[2];
    double m2s = (m0 * m0 + m1 * m1) + m2 * m2;
    fac[k] = exp(-kPiE * kPiE * m2s / (alpha * alpha)) / m2s;
    double sr = 0.0, si = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      double ph = 2.0 * kPiE * ((m0 * x[3 * j] + m1 * x[3 * j + 1]) + m2 * x[3 * j + 2]);
      sr += q[j] * cos(ph);
      si += q[j] * sin(ph);
    }
    Sre[k] = sr;
    Sim[k] = si;
  }
  for (int64_t k = 0; k < nk; ++k) E += fac[k] * (Sre[k] * Sre[k] + Sim[k] * Sim[k]);
  E /= 2.0 * kPiE * V;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    double f[3] = {0.0, 0.0, 0.0};
    for (int64_t k = 0; k < nk; ++k) {
      if (fac[k] == 0.0) continue;
      int n0 = (int)(k % side) - nmax, n1 = (int)((k / side) % side) - nmax,
          n2 = (int)(k / ((int64_t)side * side)) - nmax;
      double m0 = n0 / L[0], m1 = n1 / L[1], m2 = n2 / L[2];
      double ph = 2.0 * kPiE * ((m0 * x[3 * i] + m1 * x[3 * i + 1]) + m2 * x[3 * i + 2]);
      /* Im(conj(S) e^{i ph}) = Sre sin(ph) - Sim cos(ph) */
      double im = Sre[k] * sin(ph) - Sim[k] * cos(ph);
      double w = fac[k] * im;
      f[0] += w * m0;
      f[1] += w * m1;
      f[2] += w * m2;
    }
    double s = 2.0 * q[i] / V;
    F_rec[3 * i] = s * f[0];
    F_rec[3 * i + 1] = s * f[1];
    F_rec[3 * i + 2] = s * f[2];
  }
  free(Sre);
  free(Sim);
  free(fac);
  return E;
}
