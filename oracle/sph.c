/*
 * sph.c -- plain, slow, CPU-only FP64 reference for a smoothed-particle
 * hydrodynamics (SPH) density and pressure-force pass.
 *
 * TEST INFRASTRUCTURE ONLY, under the same rules as oracle.c: called by the
 * test suite, the smoke check and the benchmark's CPU-baseline leg, never by
 * the product path; it shares no code, header, table or helper with the HIP
 * library.
 *
 * The paper names SPH beside MD as a user of the short-range particle-particle
 * sub-motif (Introduction) and of the same binned Verlet lists (Cabana
 * "Neighbor List Creation"), but prints none of its equations.  The textbook
 * forms are written out here, O(N^2) over all pairs:
 *
 *   cubic-spline kernel (Monaghan & Lattanzio 1985), support 2h, in 3D:
 *     W(r, h) = w(r/h) / (pi h^3)
 *     w(q) = 1 - 3/2 q^2 + 3/4 q^3     0 <= q < 1
 *          = 1/4 (2 - q)^3             1 <= q < 2
 *          = 0                         q >= 2
 *   its radial derivative over r, G(r, h) = (1/r) dW/dr = g(r/h) / (pi h^5):
 *     g(q) = -3 + 9/4 q                q < 1
 *          = -3/4 (2 - q)^2 / q        1 <= q < 2,   0 beyond
 *   neighbor relation: j != i and r^2 < (2h)^2 (strict), minimum image with
 *     the single shift of oracle.c, r^2 = (d0*d0 + d1*d1) + d2*d2
 *   density by summation, self term included:
 *     rho_i = m W(0, h) + sum_j m W(r_ij, h)
 *   weakly compressible equation of state:  p = c0^2 (rho - rho0)
 *   symmetric pressure acceleration, no artificial viscosity (Monaghan 1992,
 *   "Smoothed particle hydrodynamics", Annu. Rev. Astron. Astrophys. 30):
 *     a_i = - sum_j m (p_i / rho_i^2 + p_j / rho_j^2) G(r_ij, h) d_ij,
 *     d_ij = x_i - x_j
 *
 * That acceleration is minus the gradient, over m, of the internal energy
 * U = sum_i m u(rho_i) with du/drho = p/rho^2, i.e.
 *     u(rho) = c0^2 (ln(rho/rho0) + rho0/rho - 1),
 * which the tests use to pin the pass by finite differences.
 *
 * Built with -O2 -fno-fast-math -ffp-contract=off; OpenMP over rows.
 */
#include <math.h>
#include <stdint.h>

static const double kPi = 3.14159265358979323846;

static double sph_min_image(double d, double L) {
  if (d > 0.5 * L) d -= L;
  else if (d < -0.5 * L) d += L;
  return d;
}

static double sph_disp(const double *xi, const double *xj, const double L[3], double d[3]) {
  d[0] = sph_min_image(xi[0] - xj[0], L[0]);
  d[1] = sph_min_image(xi[1] - xj[1], L[1]);
  d[2] = sph_min_image(xi[2] - xj[2], L[2]);
  return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

/* w(q) and g(q) of the cubic spline (dimensionless parts, see the header) */
static double spline_w(double q) {
  if (q < 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
  if (q < 2.0) {
    double t = 2.0 - q;
    return 0.25 * t * t * t;
  }
  return 0.0;
}

static double spline_g(double q) {
  if (q < 1.0) return -3.0 + 2.25 * q;
  if (q < 2.0) {
    double t = 2.0 - q;
    return -0.75 * t * t / q;
  }
  return 0.0;
}

/* W(r, h) and G(r, h) for each of n distances r >= 0 */
void orc_sph_kernel(int64_t n, const double *r, double h, double *W, double *G) {
  double h3 = h * h * h;
  for (int64_t k = 0; k < n; ++k) {
    double q = r[k] / h;
    if (W) W[k] = spline_w(q) / (kPi * h3);
    if (G) G[k] = spline_g(q) / (kPi * h3 * h * h);
  }
}

/* rho for rows sel[0..nsel) (all rows 0..n-1 when sel is NULL; then nsel = n):
 * rho_out[k] is the density of particle sel[k]. */
void orc_sph_density(int64_t n, const double *x, const double L[3], double h, double mass,
                     int64_t nsel, const int64_t *sel, double *rho_out) {
  double h3 = h * h * h;
  double sup2 = (2.0 * h) * (2.0 * h);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < nsel; ++k) {
    int64_t i = sel ? sel[k] : k;
    double s = mass * spline_w(0.0) / (kPi * h3);
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double d[3];
      double r2 = sph_disp(x + 3 * i, x + 3 * j, L, d);
      if (r2 < sup2) s += mass * spline_w(sqrt(r2) / h) / (kPi * h3);
    }
    rho_out[k] = s;
  }
}

/* Pressure acceleration for rows sel (as above), from the densities rho[0..n)
 * of all particles: acc_out[3k..3k+2] belongs to particle sel[k]. */
void orc_sph_accel(int64_t n, const double *x, const double L[3], double h, double mass,
                   double c0, double rho0, const double *rho, int64_t nsel, const int64_t *sel,
                   double *acc_out) {
  double h5 = h * h * h * h * h;
  double sup2 = (2.0 * h) * (2.0 * h);
  double c2 = c0 * c0;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < nsel; ++k) {
    int64_t i = sel ? sel[k] : k;
    double pi_ = c2 * (rho[i] - rho0);
    double ti = pi_ / (rho[i] * rho[i]);
    double a[3] = {0.0, 0.0, 0.0};
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double d[3];
      double r2 = sph_disp(x + 3 * i, x + 3 * j, L, d);
      if (!(r2 < sup2)) continue;
      double pj = c2 * (rho[j] - rho0);
      double tj = pj / (rho[j] * rho[j]);
      double G = spline_g(sqrt(r2) / h) / (kPi * h5);
      double c = -mass * (ti + tj) * G;
      a[0] += c * d[0];
      a[1] += c * d[1];
      a[2] += c * d[2];
    }
    acc_out[3 * k] = a[0];
    acc_out[3 * k + 1] = a[1];
    acc_out[3 * k + 2] = a[2];
  }
}
