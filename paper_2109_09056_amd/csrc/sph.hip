// SPH density summation and symmetric pressure acceleration over the tiled-ELL
// full neighbor list, gfx950.  Paper: SPH is the other short-range
// particle-particle user of binned Verlet lists beside MD (Introduction;
// Cabana "Neighbor List Creation"); the paper prints no SPH equations, so the
// textbook forms are used.
//
//   cubic spline (Monaghan & Lattanzio 1985), support 2h, q = r/h:
//     W = w(q) / (pi h^3),  w = 1 - 3/2 q^2 + 3/4 q^3 (q < 1), 1/4 (2 - q)^3 (q < 2)
//     G = W'(r)/r = g(q) / (pi h^5),  g = -3 + 9/4 q (q < 1), -3/4 (2 - q)^2 / q (q < 2)
//   density:       rho_i = m W(0) + sum_j m W(r_ij)
//   state:         p = c0^2 (rho - rho0),  P = p / rho^2
//   acceleration:  a_i = -sum_j m (P_i + P_j) G(r_ij) d_ij,  d_ij = x_i - x_j
//                  (Monaghan 1992, no artificial viscosity)
//
// Traversal as in the LJ force kernel: two lanes per particle over its row of
// the 64-particle tile (entries t, t + 2, ...), six gathers in flight per
// lane, a butterfly to combine the team, 128 particles per block, blocks
// renumbered per XCD; no atomics, so results are bitwise reproducible.  The
// acceleration pass first packs (x, y, z, P) per particle into 32-byte
// records in the workspace: a neighbour then costs two 16-byte gathers
// instead of three loads, and no division per pair for P_j.
#include "common.h"

namespace ljmd {

namespace {

constexpr int kSphAtoms = 128;  // particles per block
constexpr int kSphTeam = 2;     // lanes per particle
constexpr int kSphThreads = kSphAtoms * kSphTeam;
constexpr int kSphWaves = kSphThreads / kWave;
constexpr int kSphUnroll = 6;   // gathers in flight per lane
constexpr double kPi = 3.14159265358979323846;

struct SphArgs {
  BoxK b;
  double sup2;    // (2h)^2
  double margin;  // 2h: particles this far from every face need no minimum image
  double inv_h;
  double wnorm;   // m / (pi h^3)
  double gnorm;   // m / (pi h^5)
  double mass, c0sq, rho0;
  int32_t n;
  const double *x;
  const int32_t *nbr;
  const int32_t *nnbr;
  int32_t maxn;
  double *rho;             // density pass: output
  double *partial;         // density pass: per-block internal energy
  const double4 *xp;       // acceleration pass: packed (x, y, z, P)
  double *acc;
  // acceleration pass with the integration step (k_sph_accel<..., true>)
  double *v, *x_out;
  double dt, hdt;
};

template <bool WIDE>
__device__ __forceinline__ const double4 *rec_of(const double4 *xp, int32_t j) {
  if constexpr (WIDE)
    return xp + j;
  else
    return (const double4 *)((const char *)xp + ((uint32_t)j << 5));
}

// q = r/h and 1/q (only used where q >= 1).  Measured against r^-1 from the
// hardware reciprocal square root with Newton steps, this form was as fast for
// the density pass and faster for the acceleration pass.
__device__ __forceinline__ void q_of(double r2, const SphArgs &a, double &q, double &hq) {
  q = __builtin_sqrt(r2) * a.inv_h;
  hq = recip64(q);
}

// w(q) inside the support, 0 outside or on padding slots
__device__ __forceinline__ double spline_w(double r2, bool ok, const SphArgs &a) {
  double q, hq;
  q_of(r2, a, q, hq);
  const double t = 2.0 - q;
  const double wi = __builtin_fma(q * q, __builtin_fma(0.75, q, -1.5), 1.0);
  const double wo = 0.25 * (t * t) * t;
  const double w = q < 1.0 ? wi : wo;
  return ok && r2 < a.sup2 ? w : 0.0;
}

// g(q) inside the support, 0 outside or on padding slots
__device__ __forceinline__ double spline_g(double r2, bool ok, const SphArgs &a) {
  double q, hq;
  q_of(r2, a, q, hq);
  const double t = 2.0 - q;
  const double gi = __builtin_fma(2.25, q, -3.0);
  const double go = -0.75 * (t * t) * hq;
  const double g = q < 1.0 ? gi : go;
  return ok && r2 < a.sup2 ? g : 0.0;
}

template <bool WRAP>
__device__ __forceinline__ void disp(const SphArgs &a, double xi, double yi, double zi,
                                     double xj, double yj, double zj, double &dx, double &dy,
                                     double &dz) {
  dx = xi - xj;
  dy = yi - yj;
  dz = zi - zj;
  if constexpr (WRAP) {
    dx = min_image(dx, a.b.L[0], a.b.invL[0]);
    dy = min_image(dy, a.b.L[1], a.b.invL[1]);
    dz = min_image(dz, a.b.L[2], a.b.invL[2]);
  }
}

// Sum of w over lane t's entries of the row (cnt of them, kStep ints apart):
// whole groups of U without masks, then one masked group.
template <bool WRAP, bool WIDE>
__device__ __forceinline__ double density_row(const SphArgs &a, const int32_t *row, int32_t cnt,
                                              double xi, double yi, double zi) {
  constexpr int U = kSphUnroll;
  constexpr int kStep = kSphTeam * kWave;
  double s = 0.0;
  const int32_t whole = cnt - cnt % U;
  int32_t k = 0;
  for (; k < whole; k += U, row += U * kStep) {
    int32_t j[U];
#pragma unroll
    for (int u = 0; u < U; ++u) j[u] = row[u * kStep];
    double xj[U], yj[U], zj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double *p = pos_of<WIDE>(a.x, j[u]);
      xj[u] = p[0];
      yj[u] = p[1];
      zj[u] = p[2];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      double dx, dy, dz;
      disp<WRAP>(a, xi, yi, zi, xj[u], yj[u], zj[u], dx, dy, dz);
      s += spline_w(dist2(dx, dy, dz), true, a);
    }
  }
  if (k < cnt) {
    int32_t j[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ok[u] = k + u < cnt;
      j[u] = row[(ok[u] ? u : 0) * kStep];
    }
    double xj[U], yj[U], zj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      xj[u] = xi;
      yj[u] = yi;
      zj[u] = zi;
      if (ok[u]) {  // no gathers for the padding slots
        const double *p = pos_of<WIDE>(a.x, j[u]);
        xj[u] = p[0];
        yj[u] = p[1];
        zj[u] = p[2];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      double dx, dy, dz;
      disp<WRAP>(a, xi, yi, zi, xj[u], yj[u], zj[u], dx, dy, dz);
      s += spline_w(dist2(dx, dy, dz), ok[u], a);
    }
  }
  return s;
}

template <bool WIDE, bool WANT_U>
__global__ __launch_bounds__(kSphThreads) void k_sph_density(SphArgs a) {
  __shared__ double red[kSphWaves];
  const int t = (int)threadIdx.x % kSphTeam;
  const int32_t i = xcd_block(blockIdx.x, gridDim.x) * kSphAtoms + (int)threadIdx.x / kSphTeam;
  const bool live = i < a.n;
  double xi = 0.0, yi = 0.0, zi = 0.0;
  if (live) {
    xi = a.x[3 * (int64_t)i];
    yi = a.x[3 * (int64_t)i + 1];
    zi = a.x[3 * (int64_t)i + 2];
  }
  const double m = a.margin;
  const bool in = !live || (xi >= m && xi <= a.b.L[0] - m && yi >= m && yi <= a.b.L[1] - m &&
                            zi >= m && zi <= a.b.L[2] - m);
  const bool interior = __ballot(!in) == 0;  // wavefront-uniform
  double s = 0.0;
  if (live) {
    const int32_t ctot = a.nnbr[i];
    const int32_t cnt = ctot > t ? (ctot - t + kSphTeam - 1) / kSphTeam : 0;
    const int32_t *row =
        a.nbr + (int64_t)(i >> 6) * a.maxn * kWave + (i & (kWave - 1)) + (int64_t)t * kWave;
    s = interior ? density_row<false, WIDE>(a, row, cnt, xi, yi, zi)
                 : density_row<true, WIDE>(a, row, cnt, xi, yi, zi);
  }
  s += __shfl_xor(s, 1, kWave);  // both lanes of the team end with the same sum
  double rho = 0.0;
  if (live) {
    rho = a.wnorm * (1.0 + s);  // self term: w(0) = 1
    if (t == 0) a.rho[i] = rho;
  }
  if constexpr (WANT_U) {
    double u[1] = {0.0};
    if (live && t == 0)
      u[0] = a.mass * a.c0sq * (log(rho / a.rho0) + a.rho0 / rho - 1.0);
    block_sum<kSphWaves, 1>(u, red, a.partial + blockIdx.x);
  }
}

// xp[i] = (x_i, y_i, z_i, P_i), P = c0^2 (rho - rho0) / rho^2
__global__ __launch_bounds__(256) void k_sph_pack(SphArgs a, double4 *xp) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const double r = a.rho[i];
  double4 v;
  v.x = a.x[3 * i];
  v.y = a.x[3 * i + 1];
  v.z = a.x[3 * i + 2];
  v.w = a.c0sq * (r - a.rho0) / (r * r);
  xp[i] = v;
}

template <bool WRAP, bool WIDE>
__device__ __forceinline__ void accel_pair(const SphArgs &a, const double4 &me, const double4 &o,
                                           bool ok, double &ax, double &ay, double &az) {
  double dx, dy, dz;
  disp<WRAP>(a, me.x, me.y, me.z, o.x, o.y, o.z, dx, dy, dz);
  const double c = (me.w + o.w) * spline_g(dist2(dx, dy, dz), ok, a);
  ax = __builtin_fma(c, dx, ax);
  ay = __builtin_fma(c, dy, ay);
  az = __builtin_fma(c, dz, az);
}

// Lane t's entries of the row: whole groups of U without masks, then one masked group.
template <bool WRAP, bool WIDE>
__device__ __forceinline__ void accel_row(const SphArgs &a, const int32_t *row, int32_t cnt,
                                          const double4 &me, double &ax, double &ay,
                                          double &az) {
  constexpr int U = kSphUnroll;
  constexpr int kStep = kSphTeam * kWave;
  const int32_t whole = cnt - cnt % U;
  int32_t k = 0;
  for (; k < whole; k += U, row += U * kStep) {
    int32_t j[U];
#pragma unroll
    for (int u = 0; u < U; ++u) j[u] = row[u * kStep];
    double4 o[U];
#pragma unroll
    for (int u = 0; u < U; ++u) o[u] = *rec_of<WIDE>(a.xp, j[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) accel_pair<WRAP, WIDE>(a, me, o[u], true, ax, ay, az);
  }
  if (k < cnt) {
    int32_t j[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ok[u] = k + u < cnt;
      j[u] = row[(ok[u] ? u : 0) * kStep];
    }
    double4 o[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      o[u] = me;
      if (ok[u]) o[u] = *rec_of<WIDE>(a.xp, j[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) accel_pair<WRAP, WIDE>(a, me, o[u], ok[u], ax, ay, az);
  }
}

// STEP: after the acceleration, the closing half kick of this step and the next
// step's opening half kick and drift with wrap, per component exactly as the
// integrator's fused kick-kick-drift (unit mass: the acceleration is F/m).
template <bool WIDE, bool STEP>
__global__ __launch_bounds__(kSphThreads) void k_sph_accel(SphArgs a) {
  const int t = (int)threadIdx.x % kSphTeam;
  const int32_t i = xcd_block(blockIdx.x, gridDim.x) * kSphAtoms + (int)threadIdx.x / kSphTeam;
  const bool live = i < a.n;
  double4 me = make_double4(0.0, 0.0, 0.0, 0.0);
  if (live) me = a.xp[i];
  const double m = a.margin;
  const bool in = !live || (me.x >= m && me.x <= a.b.L[0] - m && me.y >= m &&
                            me.y <= a.b.L[1] - m && me.z >= m && me.z <= a.b.L[2] - m);
  const bool interior = __ballot(!in) == 0;
  double ax = 0.0, ay = 0.0, az = 0.0;
  if (live) {
    const int32_t ctot = a.nnbr[i];
    const int32_t cnt = ctot > t ? (ctot - t + kSphTeam - 1) / kSphTeam : 0;
    const int32_t *row =
        a.nbr + (int64_t)(i >> 6) * a.maxn * kWave + (i & (kWave - 1)) + (int64_t)t * kWave;
    if (interior)
      accel_row<false, WIDE>(a, row, cnt, me, ax, ay, az);
    else
      accel_row<true, WIDE>(a, row, cnt, me, ax, ay, az);
  }
  ax += __shfl_xor(ax, 1, kWave);
  ay += __shfl_xor(ay, 1, kWave);
  az += __shfl_xor(az, 1, kWave);
  if (live && t == 0) {
    const double f[3] = {-a.gnorm * ax, -a.gnorm * ay, -a.gnorm * az};
    if (!STEP || a.acc) {
      a.acc[3 * (int64_t)i] = f[0];
      a.acc[3 * (int64_t)i + 1] = f[1];
      a.acc[3 * (int64_t)i + 2] = f[2];
    }
    if constexpr (STEP) {
      const double xo[3] = {me.x, me.y, me.z};  // the packed copy of x_i
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int64_t q = 3 * (int64_t)i + k;
        const double L = a.b.L[k];
        const double kick = a.hdt * f[k];
        const double vh = (a.v[q] + kick) + kick;
        double xq = xo[k] + a.dt * vh;
        if (xq >= L) xq -= L;
        else if (xq < 0.0) xq += L;
        if (xq >= L) xq -= L;
        a.v[q] = vh;
        a.x_out[q] = xq;
      }
    }
  }
}

unsigned sph_blocks(int64_t n) {
  const int64_t b = (n + kSphAtoms - 1) / kSphAtoms;
  return (unsigned)(b > 0 ? b : 1);
}

SphArgs make_args(const BoxK &b, double h, double mass, double c0, double rho0, int64_t n,
                  const double *x, const int32_t *nbr, const int32_t *nnbr, int32_t maxn) {
  SphArgs a{};
  a.b = b;
  a.sup2 = (2.0 * h) * (2.0 * h);
  a.margin = 2.0 * h;
  a.inv_h = 1.0 / h;
  a.wnorm = mass / (kPi * h * h * h);
  a.gnorm = mass / (kPi * h * h * h * h * h);
  a.mass = mass;
  a.c0sq = c0 * c0;
  a.rho0 = rho0;
  a.n = (int32_t)n;
  a.x = x;
  a.nbr = nbr;
  a.nnbr = nnbr;
  a.maxn = maxn;
  return a;
}

}  // namespace

size_t sph_workspace(int64_t n) {
  const size_t rec = (size_t)(n > 0 ? n : 0) * sizeof(double4);
  const size_t part = (size_t)sph_blocks(n) * sizeof(double);
  return rec > part ? rec : part;
}

int launch_sph_density(const BoxK &b, double h, double mass, double c0, double rho0, int64_t n,
                       const double *x, const int32_t *nbr, const int32_t *nnbr, int32_t maxn,
                       double *rho, double *u_total, void *ws, hipStream_t st) {
  SphArgs a = make_args(b, h, mass, c0, rho0, n, x, nbr, nnbr, maxn);
  a.rho = rho;
  a.partial = (double *)ws;
  const unsigned nblk = sph_blocks(n);
  const bool wide = n > kNarrowAtoms;
  if (n > 0) {
    if (u_total) {
      if (wide) k_sph_density<true, true><<<nblk, kSphThreads, 0, st>>>(a);
      else k_sph_density<false, true><<<nblk, kSphThreads, 0, st>>>(a);
    } else {
      if (wide) k_sph_density<true, false><<<nblk, kSphThreads, 0, st>>>(a);
      else k_sph_density<false, false><<<nblk, kSphThreads, 0, st>>>(a);
    }
  }
  if (u_total)
    k_colsum<1024><<<1, 1024, 0, st>>>(n > 0 ? nblk : 0, 1, 1, a.partial, u_total, 1.0, 0);
  return check_launch("ljmd_sph_density");
}

// v == NULL: the acceleration pass alone; otherwise also the kick-kick-drift of
// the particles into x_out (= x: the pass reads positions from the packed copy).
int launch_sph_accel(const BoxK &b, double h, double mass, double c0, double rho0, int64_t n,
                     const double *x, const double *rho, const int32_t *nbr,
                     const int32_t *nnbr, int32_t maxn, double *acc, double dt, double *v,
                     double *x_out, void *ws, hipStream_t st) {
  SphArgs a = make_args(b, h, mass, c0, rho0, n, x, nbr, nnbr, maxn);
  a.rho = const_cast<double *>(rho);  // read only in this pass
  a.xp = (const double4 *)ws;
  a.acc = acc;
  a.v = v;
  a.x_out = x_out;
  a.dt = dt;
  a.hdt = 0.5 * dt;
  if (n > 0) {
    k_sph_pack<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(a, (double4 *)ws);
    const unsigned nblk = sph_blocks(n);
    const bool wide = n > kNarrowAtoms;
    if (v) {
      if (wide) k_sph_accel<true, true><<<nblk, kSphThreads, 0, st>>>(a);
      else k_sph_accel<false, true><<<nblk, kSphThreads, 0, st>>>(a);
    } else {
      if (wide) k_sph_accel<true, false><<<nblk, kSphThreads, 0, st>>>(a);
      else k_sph_accel<false, false><<<nblk, kSphThreads, 0, st>>>(a);
    }
  }
  return check_launch(v ? "ljmd_sph_accel_step" : "ljmd_sph_accel");
}

}  // namespace ljmd
