// Velocity-Verlet integration and the elementwise steps of its discrete
// adjoint, gfx950.  Paper: CabanaMD keeps position integration in the
// application (CabanaMD subsection); the timestep propagates particles with
// the forces (Introduction).
//
// All kernels are streaming: one thread per scalar component, coalesced
// FP64 loads/stores; reductions (kinetic energy, trajectory loss) write
// per-block partials summed by one fixed-order column-sum launch.
#include "common.h"

namespace ljmd {

namespace {

constexpr int kThreads = 256;

// v += (dt/2 F)/m; x += dt v; wrap (x >= L: x -= L, else x < 0: x += L; then x >= L: x -= L)
__global__ __launch_bounds__(kThreads) void k_kick_drift(int64_t m3, double hdt, double dt,
                                                         double mass, int unit_mass, BoxK b,
                                                         double *__restrict__ x,
                                                         double *__restrict__ v,
                                                         const double *__restrict__ F) {
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (q >= m3) return;
  const int k = (int)(q % 3);
  const double L = k == 0 ? b.L[0] : (k == 1 ? b.L[1] : b.L[2]);
  double kick = hdt * F[q];
  if (!unit_mass) kick = kick / mass;
  const double vq = v[q] + kick;
  double xq = x[q] + dt * vq;
  if (xq >= L) xq -= L;
  else if (xq < 0.0) xq += L;
  if (xq >= L) xq -= L;
  v[q] = vq;
  x[q] = xq;
}

// End-of-step half kick, kinetic energy, then the next step's half kick,
// drift and wrap: the same operations as k_kick followed by k_kick_drift.
template <bool KE>
__global__ __launch_bounds__(kThreads) void k_kick_kick_drift(int64_t m3, double hdt, double dt,
                                                              double mass, int unit_mass, BoxK b,
                                                              double *__restrict__ x,
                                                              double *__restrict__ v,
                                                              const double *__restrict__ F,
                                                              double *__restrict__ partial) {
  __shared__ double red[kThreads / kWave];
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  double vv = 0.0;
  if (q < m3) {
    const int k = (int)(q % 3);
    const double L = k == 0 ? b.L[0] : (k == 1 ? b.L[1] : b.L[2]);
    double kick = hdt * F[q];
    if (!unit_mass) kick = kick / mass;
    const double vn = v[q] + kick;
    vv = vn * vn;
    const double vh = vn + kick;
    double xq = x[q] + dt * vh;
    if (xq >= L) xq -= L;
    else if (xq < 0.0) xq += L;
    if (xq >= L) xq -= L;
    v[q] = vh;
    x[q] = xq;
  }
  if constexpr (KE) {
    const double s[1] = {vv};
    block_sum<kThreads / kWave, 1>(s, red, partial + blockIdx.x);
  }
}

template <bool KE>
__global__ __launch_bounds__(kThreads) void k_kick(int64_t m3, double hdt, double mass,
                                                   int unit_mass, double *__restrict__ v,
                                                   const double *__restrict__ F,
                                                   double *__restrict__ partial) {
  __shared__ double red[kThreads / kWave];
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  double vv = 0.0;
  if (q < m3) {
    double kick = hdt * F[q];
    if (!unit_mass) kick = kick / mass;
    const double vq = v[q] + kick;
    v[q] = vq;
    vv = vq * vq;
  }
  if constexpr (KE) {
    const double s[1] = {vv};
    block_sum<kThreads / kWave, 1>(s, red, partial + blockIdx.x);
  }
}

__global__ __launch_bounds__(kThreads) void k_sumsq_v(int64_t m3, const double *__restrict__ v,
                                                      double *__restrict__ partial) {
  __shared__ double red[kThreads / kWave];
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const double vq = q < m3 ? v[q] : 0.0;
  const double s[1] = {vq * vq};
  block_sum<kThreads / kWave, 1>(s, red, partial + blockIdx.x);
}

__global__ __launch_bounds__(kThreads) void k_adjoint_kick(int64_t m3, double dt, double wdt,
                                                           const double *__restrict__ xbar,
                                                           double *__restrict__ vbar,
                                                           double *__restrict__ g) {
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (q >= m3) return;
  const double vb = vbar[q] + dt * xbar[q];
  vbar[q] = vb;
  g[q] = wdt * vb;
}

__global__ __launch_bounds__(kThreads) void k_loss(int64_t m3, BoxK b, const double *__restrict__ x,
                                                   const double *__restrict__ xref,
                                                   double *__restrict__ xbar,
                                                   double *__restrict__ partial) {
  __shared__ double red[kThreads / kWave];
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  double d = 0.0;
  if (q < m3) {
    const int k = (int)(q % 3);
    const double L = k == 0 ? b.L[0] : (k == 1 ? b.L[1] : b.L[2]);
    const double iL = k == 0 ? b.invL[0] : (k == 1 ? b.invL[1] : b.invL[2]);
    d = min_image(x[q] - xref[q], L, iL);
    xbar[q] = d;
  }
  const double s[1] = {d * d};
  block_sum<kThreads / kWave, 1>(s, red, partial + blockIdx.x);
}

__global__ __launch_bounds__(kThreads) void k_scatter_rows(int64_t n, int32_t width,
                                                           const int64_t *__restrict__ id,
                                                           const double *__restrict__ src,
                                                           double *__restrict__ dst) {
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (q >= n * width) return;
  const int64_t r = q / width;
  const int64_t c = q - r * width;
  const int64_t t = id[r];
  if (t >= 0 && t < n) dst[t * width + c] = src[q];  // ids outside [0, n) are skipped
}

__global__ __launch_bounds__(kThreads) void k_gather_rows(int64_t n, int32_t width,
                                                          const int64_t *__restrict__ id,
                                                          const double *__restrict__ src,
                                                          double *__restrict__ dst) {
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (q >= n * width) return;
  const int64_t r = q / width;
  const int64_t c = q - r * width;
  const int64_t t = id[r];
  if (t >= 0 && t < n) dst[q] = src[t * width + c];
}

__device__ __forceinline__ double wave_max_f64(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

// Largest value over the block's threads into out (every thread calls it).
__device__ __forceinline__ void block_max(double v, double *red, double *out) {
  v = wave_max_f64(v);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int k = 1; k < (int)(blockDim.x / kWave); ++k) m = fmax(m, red[k]);
    *out = m;
  }
}

// Squared minimum-image displacement |x_i - xref_i|^2 of each atom (one thread per
// atom), the block's largest into partial[block].
__global__ __launch_bounds__(kThreads) void k_disp2_max(int64_t n, BoxK b,
                                                        const double *__restrict__ x,
                                                        const double *__restrict__ xref,
                                                        double *__restrict__ partial) {
  __shared__ double red[kThreads / kWave];
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  double d2 = 0.0;
  if (i < n) {
    const double dx = min_image(x[3 * i] - xref[3 * i], b.L[0], b.invL[0]);
    const double dy = min_image(x[3 * i + 1] - xref[3 * i + 1], b.L[1], b.invL[1]);
    const double dz = min_image(x[3 * i + 2] - xref[3 * i + 2], b.L[2], b.invL[2]);
    d2 = dist2(dx, dy, dz);
  }
  block_max(d2, red, partial + blockIdx.x);
}

// Largest of m partial values (one block).
__global__ __launch_bounds__(1024) void k_max_rows(int64_t m, const double *__restrict__ p,
                                                   double *__restrict__ out) {
  __shared__ double red[1024 / kWave];
  double v = 0.0;
  for (int64_t q = threadIdx.x; q < m; q += 1024) v = fmax(v, p[q]);
  block_max(v, red, out);
}

inline unsigned nblocks(int64_t m) {
  const int64_t b = (m + kThreads - 1) / kThreads;
  return (unsigned)(b > 0 ? b : 1);
}

}  // namespace

size_t stream_workspace(int64_t n) { return ((size_t)nblocks(3 * n) + 1) * sizeof(double); }

int launch_integrate(int stage, double dt, double mass, const BoxK &b, int64_t n, double *x,
                     double *v, const double *F, double *ke, void *ws, hipStream_t st) {
  const int64_t m3 = 3 * n;
  const unsigned nb = nblocks(m3);
  const double hdt = 0.5 * dt;
  const int unit = mass == 1.0;
  double *partial = (double *)ws;
  if (stage == LJMD_KINETIC) {
    k_sumsq_v<<<nb, kThreads, 0, st>>>(m3, v, partial);
  } else if (stage == LJMD_KICK_KICK_DRIFT) {
    if (ke)
      k_kick_kick_drift<true><<<nb, kThreads, 0, st>>>(m3, hdt, dt, mass, unit, b, x, v, F,
                                                       partial);
    else if (n > 0)
      k_kick_kick_drift<false><<<nb, kThreads, 0, st>>>(m3, hdt, dt, mass, unit, b, x, v, F,
                                                        partial);
  } else if (stage == LJMD_KICK_DRIFT) {
    if (n > 0) k_kick_drift<<<nb, kThreads, 0, st>>>(m3, hdt, dt, mass, unit, b, x, v, F);
    if (ke) k_sumsq_v<<<nb, kThreads, 0, st>>>(m3, v, partial);
  } else {
    if (ke)
      k_kick<true><<<nb, kThreads, 0, st>>>(m3, hdt, mass, unit, v, F, partial);
    else if (n > 0)
      k_kick<false><<<nb, kThreads, 0, st>>>(m3, hdt, mass, unit, v, F, partial);
  }
  if (ke) k_colsum<1024><<<1, 1024, 0, st>>>(nb, 1, 1, partial, ke, 0.5 * mass, 0);
  return check_launch("ljmd_integrate");
}

int launch_adjoint_kick(int64_t n, double dt, double w, const double *xbar, double *vbar,
                        double *g, hipStream_t st) {
  if (n > 0)
    k_adjoint_kick<<<nblocks(3 * n), kThreads, 0, st>>>(3 * n, dt, w * dt, xbar, vbar, g);
  return check_launch("ljmd_adjoint_kick");
}

int launch_max_displacement(const BoxK &b, int64_t n, const double *x, const double *xref,
                            double *max_d2, void *ws, hipStream_t st) {
  const unsigned nb = nblocks(n);
  double *partial = (double *)ws;
  if (n > 0) k_disp2_max<<<nb, kThreads, 0, st>>>(n, b, x, xref, partial);
  k_max_rows<<<1, 1024, 0, st>>>(n > 0 ? nb : 0, partial, max_d2);
  return check_launch("ljmd_max_displacement");
}

int launch_loss(const BoxK &b, int64_t n, const double *x, const double *xref, double *xbar,
                double *loss, void *ws, hipStream_t st) {
  const unsigned nb = nblocks(3 * n);
  double *partial = (double *)ws;
  k_loss<<<nb, kThreads, 0, st>>>(3 * n, b, x, xref, xbar, partial);
  k_colsum<1024><<<1, 1024, 0, st>>>(nb, 1, 1, partial, loss, 0.5, 0);
  return check_launch("ljmd_traj_loss");
}

int launch_scatter_rows(int64_t n, int32_t width, const int64_t *id, const double *src,
                        double *dst, hipStream_t st) {
  if (n > 0)
    k_scatter_rows<<<nblocks(n * width), kThreads, 0, st>>>(n, width, id, src, dst);
  return check_launch("ljmd_scatter_rows");
}

int launch_gather_rows(int64_t n, int32_t width, const int64_t *id, const double *src,
                       double *dst, hipStream_t st) {
  if (n > 0)
    k_gather_rows<<<nblocks(n * width), kThreads, 0, st>>>(n, width, id, src, dst);
  return check_launch("ljmd_gather_rows");
}

}  // namespace ljmd
