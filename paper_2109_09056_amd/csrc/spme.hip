// Smooth particle-mesh Ewald for point charges, gfx950.  Paper: CabanaMD's
// long-range path -- real-space energies and forces through the neighbor
// parallel loops, and for reciprocal space spline spreading of charge onto a
// uniform grid, 3-D FFTs and a gradient gather back to the particles
// (CabanaMD subsection; Cabana "Long Range Solvers", "Particle-Grid
// Interpolation").  The paper prints no equation; the method is SPME as
// defined by Essmann et al. (1995, J. Chem. Phys. 103, 8577), Gaussian units:
//
//   real space:  E_dir = 1/2 sum_i sum_{j, r < rc} q_i q_j erfc(alpha r)/r
//                F_i   = sum_j q_i q_j [erfc(alpha r)/r + 2 alpha/sqrt(pi) e^{-alpha^2 r^2}] d_ij / r^2
//   reciprocal:  u_a = K_a x_a / L_a; cardinal B-splines M_n of even order n
//                Q(k) = sum_i q_i prod_a M_n(u_ai - k_a)   (k_a = floor(u_ai) - j mod K_a)
//                E_rec = 1/2 sum_m B(m) C(m) |F(Q)(m)|^2,
//                B = prod_a |sum_{k<n-1} M_n(k+1) e^{2 pi i m_a k/K_a}|^-2,
//                C = e^{-pi^2 |m'|^2/alpha^2} / (pi V |m'|^2), C(0) = 0
//                phi = unnormalised inverse transform of B C F(Q);
//                F_i = -q_i sum_k grad_i[prod_a M_n(u_ai - k_a)] phi(k)
//   self:        E_self = -alpha/sqrt(pi) sum_i q_i^2
//
// Kernels: the real-space pair loop walks the tiled full list with two lanes
// per particle over packed (x, y, z, q) records (the SPH and LJ traversal),
// with erfc taken as e^{-x^2} times a tabulated polynomial for erfcx;
// charge is spread onto a real grid (LDS-privatised per wavefront, then FP64
// atomics); the 3-D transform is real-to-complex: the x pass turns each row of
// K0 reals into K0/2 + 1 coefficients through one complex FFT of length K0/2
// plus a split step, and the y and z passes run on that half grid, each pass
// a set of radix-2 FFTs over rows staged in LDS (rows along y and z loaded
// with consecutive x across lanes, so every pass reads and writes whole cache
// lines); the influence function B C is applied on the half grid, each
// coefficient with 0 < m_0 < K0/2 counted twice in the energy (Hermitian
// symmetry of a real input); the inverse mirrors it and leaves phi real; the
// gather is one thread per particle.
#include "common.h"

namespace ljmd {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxGrid = 256;  // points per edge
constexpr int kThreads = 256;
constexpr int kEwAtoms = 128;  // real space: particles per block
constexpr int kEwTeam = 2;
constexpr int kEwThreads = kEwAtoms * kEwTeam;
constexpr int kEwUnroll = 6;
// erfc(x) = e^{-x^2} erfcx(x) on [0, alpha rc]: erfcx by degree-10 Taylor polynomials
// about the centres of 32 equal intervals (relative error ~1e-15); e^{-x^2} is
// needed for the force anyway, so a pair costs ten FMAs instead of a library erfc.
constexpr int kErfcIntervals = 32;
constexpr int kErfcDegree = 10;
constexpr int kErfcStride = 12;  // coefficients per interval, padded
constexpr int kErfcTable = kErfcIntervals * kErfcStride;

// ------------------------------------------------------------ real space --

struct RealArgs {
  BoxK b;
  double alpha, a2, c2a;  // alpha, alpha^2, 2 alpha / sqrt(pi)
  double rc2, margin;
  int32_t n;
  const int32_t *nbr;
  const int32_t *nnbr;
  int32_t maxn;
  const double4 *xq;  // packed (x, y, z, q)
  double *F;
  int accumulate;
  double *partial;  // per-block E_dir, or null
  const double *erfcx_tab;  // [kErfcIntervals][kErfcStride] Taylor coefficients
  double inv_dx, half_dx;   // intervals of width dx = alpha rc / kErfcIntervals
};

// Packs (x, y, z, q) records; block 0 also writes the erfcx table: about each
// interval centre c, a_n = erfcx^(n)(c) / n! from erfcx(c) = e^{c^2} erfc(c) and
// the recurrence y' = 2 x y - 2/sqrt(pi), y^(n+1) = 2 x y^(n) + 2 n y^(n-1).
__global__ __launch_bounds__(kThreads) void k_pack_xq(int32_t n, const double *x, const double *q,
                                                      double4 *xq, double half_dx,
                                                      double *erfcx_tab) {
  if (blockIdx.x == 0 && threadIdx.x < kErfcIntervals) {
    const double c = (2 * threadIdx.x + 1) * half_dx;
    double *a = erfcx_tab + threadIdx.x * kErfcStride;
    double ym1 = exp(c * c) * erfc(c);
    double y = 2.0 * c * ym1 - 2.0 / sqrt(kPi);
    double fact = 1.0;
    a[0] = ym1;
    a[1] = y;
    for (int k = 1; k < kErfcDegree; ++k) {
      const double yn = 2.0 * c * y + 2.0 * k * ym1;
      fact *= (k + 1);
      a[k + 1] = yn / fact;
      ym1 = y;
      y = yn;
    }
    for (int k = kErfcDegree + 1; k < kErfcStride; ++k) a[k] = 0.0;
  }
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  xq[i] = make_double4(x[3 * i], x[3 * i + 1], x[3 * i + 2], q[i]);
}

template <bool WIDE>
__device__ __forceinline__ const double4 *xq_of(const double4 *p, int32_t j) {
  if constexpr (WIDE)
    return p + j;
  else
    return (const double4 *)((const char *)p + ((uint32_t)j << 5));
}

// One pair: adds q_j-weighted force scalar times d and the energy kernel.
template <bool WRAP>
__device__ __forceinline__ void real_pair(const RealArgs &a, const double *tab, const double4 &me,
                                          const double4 &o, bool ok, double &fx, double &fy,
                                          double &fz, double &e) {
  double dx = me.x - o.x, dy = me.y - o.y, dz = me.z - o.z;
  if constexpr (WRAP) {
    dx = min_image(dx, a.b.L[0], a.b.invL[0]);
    dy = min_image(dy, a.b.L[1], a.b.invL[1]);
    dz = min_image(dz, a.b.L[2], a.b.invL[2]);
  }
  const double r2 = dist2(dx, dy, dz);
  const bool in = ok && r2 < a.rc2;
  const double rr2 = in ? r2 : 1.0;  // keeps padding and far pairs finite
  // 1/r from one refined reciprocal square root of r^2 and r = r^2 / r: about
  // 9 % faster at 500k atoms than a square root followed by a reciprocal
  const double ir = rsqrt64(rr2);
  const double r = rr2 * ir;
  const double xa = a.alpha * r;
  int it = (int)(xa * a.inv_dx);
  it = it < kErfcIntervals - 1 ? it : kErfcIntervals - 1;
  const double t = xa - (2 * it + 1) * a.half_dx;
  const double *cf = tab + it * kErfcStride;
  double p = cf[kErfcDegree];
#pragma unroll
  for (int k = kErfcDegree - 1; k >= 0; --k) p = __builtin_fma(p, t, cf[k]);
  const double ex = exp(-a.a2 * rr2);
  const double er = ex * p * ir;  // erfc(alpha r) / r
  const double s = (er + a.c2a * ex) * (ir * ir);
  const double qs = in ? o.w * s : 0.0;
  fx = __builtin_fma(qs, dx, fx);
  fy = __builtin_fma(qs, dy, fy);
  fz = __builtin_fma(qs, dz, fz);
  e += in ? o.w * er : 0.0;
}

template <bool WRAP, bool WIDE>
__device__ __forceinline__ void real_row(const RealArgs &a, const double *tab, const int32_t *row,
                                         int32_t cnt, const double4 &me, double &fx, double &fy,
                                         double &fz, double &e) {
  constexpr int U = kEwUnroll;
  constexpr int kStep = kEwTeam * kWave;
  const int32_t whole = cnt - cnt % U;
  int32_t k = 0;
  for (; k < whole; k += U, row += U * kStep) {
    int32_t j[U];
#pragma unroll
    for (int u = 0; u < U; ++u) j[u] = row[u * kStep];
    double4 o[U];
#pragma unroll
    for (int u = 0; u < U; ++u) o[u] = *xq_of<WIDE>(a.xq, j[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) real_pair<WRAP>(a, tab, me, o[u], true, fx, fy, fz, e);
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
      if (ok[u]) o[u] = *xq_of<WIDE>(a.xq, j[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) real_pair<WRAP>(a, tab, me, o[u], ok[u], fx, fy, fz, e);
  }
}

template <bool WIDE, bool EV>
__global__ __launch_bounds__(kEwThreads) void k_ewald_real(RealArgs a) {
  __shared__ double red[kEwThreads / kWave];
  __shared__ double tab[kErfcTable];
  for (int k = threadIdx.x; k < kErfcTable; k += kEwThreads) tab[k] = a.erfcx_tab[k];
  __syncthreads();
  const int t = (int)threadIdx.x % kEwTeam;
  const int32_t i = xcd_block(blockIdx.x, gridDim.x) * kEwAtoms + (int)threadIdx.x / kEwTeam;
  const bool live = i < a.n;
  double4 me = make_double4(0.0, 0.0, 0.0, 0.0);
  if (live) me = a.xq[i];
  const double m = a.margin;
  const bool inside = !live || (me.x >= m && me.x <= a.b.L[0] - m && me.y >= m &&
                                me.y <= a.b.L[1] - m && me.z >= m && me.z <= a.b.L[2] - m);
  const bool interior = __ballot(!inside) == 0;
  double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0;
  if (live) {
    const int32_t ctot = a.nnbr[i];
    const int32_t cnt = ctot > t ? (ctot - t + kEwTeam - 1) / kEwTeam : 0;
    const int32_t *row =
        a.nbr + (int64_t)(i >> 6) * a.maxn * kWave + (i & (kWave - 1)) + (int64_t)t * kWave;
    if (interior)
      real_row<false, WIDE>(a, tab, row, cnt, me, fx, fy, fz, e);
    else
      real_row<true, WIDE>(a, tab, row, cnt, me, fx, fy, fz, e);
  }
  fx += __shfl_xor(fx, 1, kWave);
  fy += __shfl_xor(fy, 1, kWave);
  fz += __shfl_xor(fz, 1, kWave);
  if (live && t == 0) {
    double *F = a.F + 3 * (int64_t)i;
    const double q = me.w;
    if (a.accumulate) {
      F[0] += q * fx;
      F[1] += q * fy;
      F[2] += q * fz;
    } else {
      F[0] = q * fx;
      F[1] = q * fy;
      F[2] = q * fz;
    }
  }
  if constexpr (EV) {
    double v[1] = {live ? 0.5 * me.w * e : 0.0};  // per lane: the team's lanes add up
    block_sum<kEwThreads / kWave, 1>(v, red, a.partial + blockIdx.x);
  }
}

// ------------------------------------------------------------- B-splines --

// M_n(w + j) for j = 0..n-1 (w in [0, 1)) by the recursion
//   M_k(v) = (v M_{k-1}(v) + (k - v) M_{k-1}(v - 1)) / (k - 1),  M_2(w) = w, M_2(w+1) = 1 - w;
// dm receives dM_n(w + j)/dv = M_{n-1}(w + j) - M_{n-1}(w + j - 1) when requested.
template <int N, bool DERIV>
__device__ __forceinline__ void spline_weights(double w, double (&m)[N], double (&dm)[N]) {
  double a[N];
  a[0] = w;
  a[1] = 1.0 - w;
#pragma unroll
  for (int j = 2; j < N; ++j) a[j] = 0.0;
#pragma unroll
  for (int k = 3; k <= N; ++k) {
    if (DERIV && k == N) {
#pragma unroll
      for (int j = 0; j < N; ++j) dm[j] = a[j] - (j > 0 ? a[j - 1] : 0.0);
    }
    const double inv = 1.0 / (k - 1);
#pragma unroll
    for (int j = k - 1; j >= 0; --j) {
      const double v = w + j;
      const double lo = j > 0 ? a[j - 1] : 0.0;
      a[j] = (v * a[j] + (k - v) * lo) * inv;
    }
  }
#pragma unroll
  for (int j = 0; j < N; ++j) m[j] = a[j];
}

struct RecArgs {
  BoxK b;
  int32_t K[3];
  double scale[3];  // K_a / L_a
  double alpha;
  int32_t n;
  const double *x;
  const double *q;
  double *grid;        // [K2][K1][K0] real: Q, later phi; x fastest
  double2 *half;       // [K2][K1][K0/2 + 1] complex transform of the grid
  double *bmod;        // |b_a(m)|^2 tables at bmod + a * kMaxGrid
  double *partial;     // influence blocks, then gather blocks
  double *F;
  int accumulate;
};

__device__ __forceinline__ int wrapi(int k, int K) {
  k %= K;
  return k < 0 ? k + K : k;
}

// |b_a(m)|^2 = |sum_{k=0}^{n-2} M_n(k+1) e^{2 pi i m k / K_a}|^-2 for every axis a, m < K_a.
template <int N>
__global__ __launch_bounds__(kThreads) void k_bmod(RecArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int ax = t / kMaxGrid, m = t % kMaxGrid;
  if (ax >= 3 || m >= a.K[ax]) return;
  double mk[N], dk[N];
  spline_weights<N, false>(0.0, mk, dk);  // mk[j] = M_n(j): M_n(k+1) = mk[k+1]
  double re = 0.0, im = 0.0;
  for (int k = 0; k <= N - 2; ++k) {
    double s, c;
    sincospi(2.0 * (double)((int64_t)m * k % a.K[ax]) / a.K[ax], &s, &c);
    re += mk[k + 1] * c;
    im += mk[k + 1] * s;
  }
  a.bmod[ax * kMaxGrid + m] = 1.0 / (re * re + im * im);
}

__global__ __launch_bounds__(kThreads) void k_zero_grid(double *g, int64_t npts) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < npts) g[i] = 0.0;
}

// Charge spreading, one wavefront of 64 consecutive (cell-sorted, hence
// nearby) particles per block.  The wavefront first adds its n^3 weights per
// particle into a private box of grid points in LDS (LDS atomics), then adds
// every non-zero point of that box to the grid with one global FP64 atomic:
// ~4x fewer global atomics than adding each weight directly, which is what
// bounds this kernel.  Per axis the box is taken in whichever of two cyclic
// frames (indices as they are, or shifted by K/2) gives the smaller extent,
// so groups that straddle a periodic face stay compact.  A group whose box
// exceeds the LDS capacity adds its weights straight to the grid.
constexpr int kSpreadCap = 2048;  // grid points (doubles) in the LDS box

__device__ __forceinline__ int wave_min_i(int v) { return -wave_max(-v); }

template <int N>
__global__ __launch_bounds__(kWave) void k_spread(RecArgs a) {
  __shared__ double box[kSpreadCap];
  const int lane = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * kWave + lane;
  const bool live = i < a.n;
  double w[3][N], dw[N];
  int b[3] = {0, 0, 0};
  double qi = 0.0;
  if (live) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double u = a.x[3 * i + d] * a.scale[d];
      const double fl = floor(u);
      b[d] = wrapi((int)fl, a.K[d]);
      spline_weights<N, false>(u - fl, w[d], dw);
    }
    qi = a.q[i];
  }
  int lo[3], ext[3], sh[3], sb[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int K = a.K[d];
    const int s0 = b[d], s1 = (b[d] + K / 2) % K;
    const int mn0 = wave_min_i(live ? s0 : 1 << 30), mx0 = wave_max(live ? s0 : -(1 << 30));
    const int mn1 = wave_min_i(live ? s1 : 1 << 30), mx1 = wave_max(live ? s1 : -(1 << 30));
    const bool shift = mx1 - mn1 < mx0 - mn0;
    sh[d] = shift ? K / 2 : 0;
    lo[d] = shift ? mn1 : mn0;
    ext[d] = (shift ? mx1 - mn1 : mx0 - mn0) + N;
    sb[d] = shift ? s1 : s0;
  }
  const int64_t vol = (int64_t)ext[0] * ext[1] * ext[2];
  if (vol > kSpreadCap) {  // wavefront-uniform
    if (!live) return;
    for (int jz = 0; jz < N; ++jz) {
      const int kz = wrapi(b[2] - jz, a.K[2]);
      for (int jy = 0; jy < N; ++jy) {
        const int ky = wrapi(b[1] - jy, a.K[1]);
        const double wyz = qi * w[2][jz] * w[1][jy];
        double *line = a.grid + ((int64_t)kz * a.K[1] + ky) * a.K[0];
#pragma unroll
        for (int jx = 0; jx < N; ++jx)
          unsafeAtomicAdd(&line[wrapi(b[0] - jx, a.K[0])], wyz * w[0][jx]);
      }
    }
    return;
  }
  for (int p = lane; p < vol; p += kWave) box[p] = 0.0;
  __syncthreads();
  if (live) {
    const int c0 = sb[0] - lo[0] + N - 1, c1 = sb[1] - lo[1] + N - 1, c2 = sb[2] - lo[2] + N - 1;
    for (int jz = 0; jz < N; ++jz) {
      for (int jy = 0; jy < N; ++jy) {
        const double wyz = qi * w[2][jz] * w[1][jy];
        double *row = box + ((int64_t)(c2 - jz) * ext[1] + (c1 - jy)) * ext[0] + c0;
#pragma unroll
        for (int jx = 0; jx < N; ++jx) unsafeAtomicAdd(row - jx, wyz * w[0][jx]);
      }
    }
  }
  __syncthreads();
  for (int p = lane; p < vol; p += kWave) {
    const double v = box[p];
    if (v == 0.0) continue;
    const int l0 = p % ext[0], l1 = (p / ext[0]) % ext[1], l2 = p / (ext[0] * ext[1]);
    const int k0 = wrapi(lo[0] + l0 - (N - 1) - sh[0], a.K[0]);
    const int k1 = wrapi(lo[1] + l1 - (N - 1) - sh[1], a.K[1]);
    const int k2 = wrapi(lo[2] + l2 - (N - 1) - sh[2], a.K[2]);
    unsafeAtomicAdd(&a.grid[((int64_t)k2 * a.K[1] + k1) * a.K[0] + k0], v);
  }
}

// Radix-2 transforms of rows of length NP, R rows per block staged in LDS:
// bit-reversed load, log2(NP) butterfly stages, natural-order result.
// sign = -1: sum_k v_k e^{-2 pi i m k / NP}; +1: the unnormalised inverse.
// Rows per block: 1024 points, at most 64 rows.
template <int NP>
constexpr int fft_rows() {
  return 1024 / NP < 64 ? 1024 / NP : 64;
}

template <int NP>
__device__ __forceinline__ int bitrev(int k) {
  return (int)(__builtin_bitreverse32((uint32_t)k) >> (32 - __builtin_ctz(NP)));
}

// Twiddle table in LDS: tw[j] = e^{sign 2 pi i j / (TS NP)}, j <= TS NP / 2.
template <int NP, int TS>
__device__ __forceinline__ void fill_twiddles(double2 *tw, double sign) {
  for (int j = threadIdx.x; j <= TS * NP / 2; j += kThreads) {
    double s, c;
    sincospi(sign * 2.0 * (double)j / (double)(TS * NP), &s, &c);
    tw[j] = make_double2(c, s);
  }
}

// The butterfly stages over R rows of NP points in buf (bit-reversed order in,
// natural order out); the twiddle of stage h, position pos, e^{sign i pi pos/h},
// is tw[TS pos NP / (2h)].  Every thread of the block calls it.
template <int NP, int R, int TS>
__device__ __forceinline__ void fft_stages(double2 *buf, const double2 *tw) {
  for (int h = 1; h < NP; h <<= 1) {
    const int step = TS * NP / (2 * h);
    for (int b = threadIdx.x; b < R * NP / 2; b += kThreads) {
      const int m = b / (NP / 2), bb = b % (NP / 2);
      const int pos = bb % h, grp = bb / h;
      const int i0 = m * NP + grp * 2 * h + pos, i1 = i0 + h;
      const double2 w = tw[pos * step];
      const double c = w.x, s = w.y;
      const double2 u = buf[i0], v = buf[i1];
      const double tr = c * v.x - s * v.y, ti = c * v.y + s * v.x;
      buf[i0] = make_double2(u.x + tr, u.y + ti);
      buf[i1] = make_double2(u.x - tr, u.y - ti);
    }
    __syncthreads();
  }
}

// y (axis 1) or z (axis 2) pass over the half grid of width W = K0/2 + 1:
// rows r < rows, element k of row r at (r % W) + (r / W) W K1 + k W (axis 1)
// or r + k W K1 (axis 2); consecutive rows are consecutive x.
template <int NP>
__global__ __launch_bounds__(kThreads) void k_fft_yz(double2 *g, int axis, int W, int K1,
                                                     int64_t rows, double sign) {
  constexpr int R = fft_rows<NP>();
  __shared__ double2 buf[R * NP];
  __shared__ double2 tw[NP / 2 + 1];
  fill_twiddles<NP, 1>(tw, sign);
  const int64_t r0 = (int64_t)blockIdx.x * R;
  const int64_t plane = (int64_t)W * K1;
  for (int idx = threadIdx.x; idx < R * NP; idx += kThreads) {
    const int m = idx % R, k = idx / R;
    const int64_t r = r0 + m;
    if (r >= rows) continue;
    const int64_t at = axis == 1 ? (r % W) + (r / W) * plane + (int64_t)k * W : r + k * plane;
    buf[m * NP + bitrev<NP>(k)] = g[at];
  }
  __syncthreads();
  fft_stages<NP, R, 1>(buf, tw);
  for (int idx = threadIdx.x; idx < R * NP; idx += kThreads) {
    const int m = idx % R, k = idx / R;
    const int64_t r = r0 + m;
    if (r >= rows) continue;
    const int64_t at = axis == 1 ? (r % W) + (r / W) * plane + (int64_t)k * W : r + k * plane;
    g[at] = buf[m * NP + k];
  }
}

// x pass, real to complex: row r of NP reals -> NP/2 + 1 coefficients X_m =
// sum_k v_k e^{-2 pi i m k / NP}.  With z_k = v_2k + i v_2k+1 and Z its
// transform of length NH = NP/2: X_m = E_m + e^{-2 pi i m/NP} O_m, where
// E_m = (Z_m + conj Z_{NH-m}) / 2 and O_m = (Z_m - conj Z_{NH-m}) / (2i) are the
// transforms of the even and odd samples (indices of Z mod NH).
template <int NP>
__global__ __launch_bounds__(kThreads) void k_fft_x_r2c(const double *rg, double2 *h,
                                                        int64_t rows) {
  constexpr int NH = NP / 2;
  constexpr int R = fft_rows<NH>();
  __shared__ double2 buf[R * NH];
  __shared__ double2 tw[NP / 2 + 1];  // e^{-2 pi i j / NP}
  fill_twiddles<NH, 2>(tw, -1.0);
  const int64_t r0 = (int64_t)blockIdx.x * R;
  for (int idx = threadIdx.x; idx < R * NH; idx += kThreads) {
    const int m = idx / NH, k = idx % NH;
    const int64_t r = r0 + m;
    if (r >= rows) continue;
    buf[m * NH + bitrev<NH>(k)] = *(const double2 *)(rg + r * NP + 2 * k);
  }
  __syncthreads();
  fft_stages<NH, R, 2>(buf, tw);
  for (int idx = threadIdx.x; idx < R * (NH + 1); idx += kThreads) {
    const int m = idx / (NH + 1), k = idx % (NH + 1);
    const int64_t r = r0 + m;
    if (r >= rows) continue;
    const double2 zm = buf[m * NH + (k % NH)], zc = buf[m * NH + ((NH - k) % NH)];
    const double er = 0.5 * (zm.x + zc.x), ei = 0.5 * (zm.y - zc.y);
    const double orr = 0.5 * (zm.y + zc.y), oi = -0.5 * (zm.x - zc.x);
    const double c = tw[k].x, s = tw[k].y;
    h[r * (NH + 1) + k] = make_double2(er + (c * orr - s * oi), ei + (c * oi + s * orr));
  }
}

// x pass, complex to real: the NP/2 + 1 coefficients X_m of a Hermitian row
// -> v_k = sum_{m<NP} X_m e^{+2 pi i m k / NP}.  With A_m = X_m + conj X_{NH-m},
// B_m = (X_m - conj X_{NH-m}) e^{+2 pi i m/NP} for m < NH, the inverse transform
// of length NH of A + iB is z_k = v_2k + i v_2k+1.
template <int NP>
__global__ __launch_bounds__(kThreads) void k_fft_x_c2r(const double2 *h, double *rg,
                                                        int64_t rows) {
  constexpr int NH = NP / 2;
  constexpr int R = fft_rows<NH>();
  __shared__ double2 xin[R * (NH + 1)];
  __shared__ double2 buf[R * NH];
  __shared__ double2 tw[NP / 2 + 1];  // e^{+2 pi i j / NP}
  fill_twiddles<NH, 2>(tw, 1.0);
  const int64_t r0 = (int64_t)blockIdx.x * R;
  for (int idx = threadIdx.x; idx < R * (NH + 1); idx += kThreads) {
    const int m = idx / (NH + 1), k = idx % (NH + 1);
    const int64_t r = r0 + m;
    if (r < rows) xin[idx] = h[r * (NH + 1) + k];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < R * NH; idx += kThreads) {
    const int m = idx / NH, k = idx % NH;
    const double2 x1 = xin[m * (NH + 1) + k], x2 = xin[m * (NH + 1) + NH - k];
    const double ar = x1.x + x2.x, ai = x1.y - x2.y;  // X_m + conj X_{NH-m}
    const double dr = x1.x - x2.x, di = x1.y + x2.y;  // X_m - conj X_{NH-m}
    const double c = tw[k].x, s = tw[k].y;
    const double br = c * dr - s * di, bi = c * di + s * dr;
    buf[m * NH + bitrev<NH>(k)] = make_double2(ar - bi, ai + br);
  }
  __syncthreads();
  fft_stages<NH, R, 2>(buf, tw);
  for (int idx = threadIdx.x; idx < R * NH; idx += kThreads) {
    const int m = idx / NH, k = idx % NH;
    const int64_t r = r0 + m;
    if (r < rows) *(double2 *)(rg + r * NP + 2 * k) = buf[m * NH + k];
  }
}

// z pass with the influence function between its two transforms: the rows of
// the z pass of k_fft_yz (row r = m0 + W m1, element m2 at r + m2 W K1) are
// transformed forward, multiplied by G(m) = B(m) C(m), transformed back, all in
// LDS, so the half grid makes one round trip instead of three.  Per block the
// reciprocal energy 1/2 sum G |F(Q)|^2 (fixed order).
template <int NP>
__global__ __launch_bounds__(kThreads) void k_fft_z_influence(RecArgs a, int64_t rows) {
  constexpr int R = fft_rows<NP>();
  __shared__ double2 buf[R * NP];
  __shared__ double2 inv[R * NP];
  __shared__ double2 twf[NP / 2 + 1];
  __shared__ double2 twi[NP / 2 + 1];
  __shared__ double red[kThreads / kWave];
  fill_twiddles<NP, 1>(twf, -1.0);
  fill_twiddles<NP, 1>(twi, 1.0);
  const int W = a.K[0] / 2 + 1;
  const int64_t r0 = (int64_t)blockIdx.x * R;
  const int64_t plane = (int64_t)W * a.K[1];
  double2 *g = a.half;
  for (int idx = threadIdx.x; idx < R * NP; idx += kThreads) {
    const int m = idx % R, k = idx / R;
    const int64_t r = r0 + m;
    buf[m * NP + bitrev<NP>(k)] = r < rows ? g[r + k * plane] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  fft_stages<NP, R, 1>(buf, twf);
  const double V = a.b.L[0] * a.b.L[1] * a.b.L[2];
  double v[1] = {0.0};
  for (int idx = threadIdx.x; idx < R * NP; idx += kThreads) {
    const int m = idx / NP, m2 = idx % NP;
    const int64_t r = r0 + m;
    double2 out = make_double2(0.0, 0.0);
    if (r < rows) {
      const int m0 = (int)(r % W);
      const int m1 = (int)(r / W);
      const double f0 = m0 * a.b.invL[0];
      const double f1 = (m1 <= a.K[1] / 2 ? m1 : m1 - a.K[1]) * a.b.invL[1];
      const double f2 = (m2 <= a.K[2] / 2 ? m2 : m2 - a.K[2]) * a.b.invL[2];
      const double msq = (f0 * f0 + f1 * f1) + f2 * f2;
      double G = 0.0;
      if (r != 0 || m2 != 0) {
        const double C = exp(-kPi * kPi * msq / (a.alpha * a.alpha)) / (kPi * V * msq);
        G = C * a.bmod[m0] * a.bmod[kMaxGrid + m1] * a.bmod[2 * kMaxGrid + m2];
      }
      const double2 z = buf[m * NP + m2];
      // 1/2 G |F|^2, doubled for the columns 0 < m0 < K0/2 whose mirror -m0 is not stored
      const double mult = (m0 == 0 || 2 * m0 == a.K[0]) ? 0.5 : 1.0;
      v[0] += mult * G * (z.x * z.x + z.y * z.y);
      out = make_double2(G * z.x, G * z.y);
    }
    inv[m * NP + bitrev<NP>(m2)] = out;
  }
  __syncthreads();
  fft_stages<NP, R, 1>(inv, twi);
  for (int idx = threadIdx.x; idx < R * NP; idx += kThreads) {
    const int m = idx % R, k = idx / R;
    const int64_t r = r0 + m;
    if (r < rows) g[r + k * plane] = inv[m * NP + k];
  }
  block_sum<kThreads / kWave, 1>(v, red, a.partial + blockIdx.x);
}

// Blocks of k_fft_z_influence (one energy partial each) for grid K.
unsigned z_influence_blocks(const int32_t K[3]) {
  const int R = 1024 / K[2] < 64 ? 1024 / K[2] : 64;  // fft_rows<K[2]>()
  const int64_t rows = (int64_t)(K[0] / 2 + 1) * K[1];
  return (unsigned)((rows + R - 1) / R);
}

// F_i = -q_i grad sum_k theta_i(k) phi(k); per block the self energy -alpha/sqrt(pi) q_i^2
template <int N>
__global__ __launch_bounds__(kThreads) void k_gather(RecArgs a, double *self_partial) {
  __shared__ double red[kThreads / kWave];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double v[1] = {0.0};
  if (i < a.n) {
    double w[3][N], dw[3][N];
    int base[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double u = a.x[3 * i + d] * a.scale[d];
      const double fl = floor(u);
      base[d] = (int)fl;
      spline_weights<N, true>(u - fl, w[d], dw[d]);
    }
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    for (int jz = 0; jz < N; ++jz) {
      const int kz = wrapi(base[2] - jz, a.K[2]);
      for (int jy = 0; jy < N; ++jy) {
        const int ky = wrapi(base[1] - jy, a.K[1]);
        const double *line = a.grid + ((int64_t)kz * a.K[1] + ky) * a.K[0];
        double sx = 0.0, sdx = 0.0;
#pragma unroll
        for (int jx = 0; jx < N; ++jx) {
          const double ph = line[wrapi(base[0] - jx, a.K[0])];
          sx = __builtin_fma(w[0][jx], ph, sx);
          sdx = __builtin_fma(dw[0][jx], ph, sdx);
        }
        g0 = __builtin_fma(sdx * w[1][jy], w[2][jz], g0);
        g1 = __builtin_fma(sx * dw[1][jy], w[2][jz], g1);
        g2 = __builtin_fma(sx * w[1][jy], dw[2][jz], g2);
      }
    }
    const double qi = a.q[i];
    double *F = a.F + 3 * i;
    const double f0 = -qi * g0 * a.scale[0], f1 = -qi * g1 * a.scale[1],
                 f2 = -qi * g2 * a.scale[2];
    if (a.accumulate) {
      F[0] += f0;
      F[1] += f1;
      F[2] += f2;
    } else {
      F[0] = f0;
      F[1] = f1;
      F[2] = f2;
    }
    v[0] = -a.alpha / __builtin_sqrt(kPi) * qi * qi;
  }
  if (self_partial) block_sum<kThreads / kWave, 1>(v, red, self_partial + blockIdx.x);
}

template <int NP>
void yz_pass(double2 *h, int axis, const int32_t K[3], double sign, hipStream_t st) {
  constexpr int R = fft_rows<NP>();
  const int W = K[0] / 2 + 1;
  const int64_t rows = (int64_t)W * (axis == 1 ? K[2] : K[1]);
  k_fft_yz<NP><<<(unsigned)((rows + R - 1) / R), kThreads, 0, st>>>(h, axis, W, K[1], rows, sign);
}

template <int NP>
void z_influence_pass(const RecArgs &a, hipStream_t st) {
  const int64_t rows = (int64_t)(a.K[0] / 2 + 1) * a.K[1];
  k_fft_z_influence<NP><<<z_influence_blocks(a.K), kThreads, 0, st>>>(a, rows);
}

void fft_z_influence(const RecArgs &a, hipStream_t st) {
  switch (a.K[2]) {
    case 8: z_influence_pass<8>(a, st); break;
    case 16: z_influence_pass<16>(a, st); break;
    case 32: z_influence_pass<32>(a, st); break;
    case 64: z_influence_pass<64>(a, st); break;
    case 128: z_influence_pass<128>(a, st); break;
    default: z_influence_pass<256>(a, st); break;
  }
}

void fft_yz(double2 *h, int axis, const int32_t K[3], double sign, hipStream_t st) {
  switch (K[axis]) {
    case 8: yz_pass<8>(h, axis, K, sign, st); break;
    case 16: yz_pass<16>(h, axis, K, sign, st); break;
    case 32: yz_pass<32>(h, axis, K, sign, st); break;
    case 64: yz_pass<64>(h, axis, K, sign, st); break;
    case 128: yz_pass<128>(h, axis, K, sign, st); break;
    default: yz_pass<256>(h, axis, K, sign, st); break;
  }
}

template <int NP>
void x_pass(double *g, double2 *h, const int32_t K[3], bool forward, hipStream_t st) {
  constexpr int R = fft_rows<NP / 2>();
  const int64_t rows = (int64_t)K[1] * K[2];
  const unsigned nb = (unsigned)((rows + R - 1) / R);
  if (forward)
    k_fft_x_r2c<NP><<<nb, kThreads, 0, st>>>(g, h, rows);
  else
    k_fft_x_c2r<NP><<<nb, kThreads, 0, st>>>(h, g, rows);
}

void fft_x(double *g, double2 *h, const int32_t K[3], bool forward, hipStream_t st) {
  switch (K[0]) {
    case 8: x_pass<8>(g, h, K, forward, st); break;
    case 16: x_pass<16>(g, h, K, forward, st); break;
    case 32: x_pass<32>(g, h, K, forward, st); break;
    case 64: x_pass<64>(g, h, K, forward, st); break;
    case 128: x_pass<128>(g, h, K, forward, st); break;
    default: x_pass<256>(g, h, K, forward, st); break;
  }
}

int64_t grid_points(const int32_t K[3]) { return (int64_t)K[0] * K[1] * K[2]; }
unsigned blocks_of(int64_t n, int per) { return (unsigned)((n + per - 1) / per > 0 ? (n + per - 1) / per : 1); }

template <int N>
void launch_rec_order(const RecArgs &a, double *self_partial, hipStream_t st) {
  const int64_t npts = grid_points(a.K);
  k_bmod<N><<<blocks_of(3 * kMaxGrid, kThreads), kThreads, 0, st>>>(a);
  k_zero_grid<<<blocks_of(npts, kThreads), kThreads, 0, st>>>(a.grid, npts);
  if (a.n > 0) k_spread<N><<<blocks_of(a.n, kWave), kWave, 0, st>>>(a);
  fft_x(a.grid, a.half, a.K, true, st);
  fft_yz(a.half, 1, a.K, -1.0, st);
  fft_z_influence(a, st);
  fft_yz(a.half, 1, a.K, 1.0, st);
  fft_x(a.grid, a.half, a.K, false, st);
  if (a.n > 0) k_gather<N><<<blocks_of(a.n, kThreads), kThreads, 0, st>>>(a, self_partial);
}

}  // namespace

size_t ewald_real_workspace(int64_t n) {
  return (size_t)(n > 0 ? n : 0) * sizeof(double4) +
         (size_t)blocks_of(n, kEwAtoms) * sizeof(double) + kErfcTable * sizeof(double) + 256;
}

// real grid, half grid (at most npts/2 + npts/8 complex points: K0 >= 8), tables,
// partials (the z/influence pass keeps at least 512 half-grid points per block)
size_t spme_workspace(int64_t n, int64_t npts) {
  const int64_t half = npts / 2 + npts / 8;
  return (size_t)npts * sizeof(double) + (size_t)half * sizeof(double2) +
         3 * kMaxGrid * sizeof(double) +
         ((size_t)blocks_of(half, 512) + blocks_of(n, kThreads)) * sizeof(double) + 256;
}

int launch_ewald_real(const BoxK &b, double alpha, double rc, int64_t n, const double *x,
                      const double *q, const int32_t *nbr, const int32_t *nnbr, int32_t maxn,
                      double *F, double *e_total, int accumulate, void *ws, hipStream_t st) {
  RealArgs a{};
  a.b = b;
  a.alpha = alpha;
  a.a2 = alpha * alpha;
  a.c2a = 2.0 * alpha / sqrt(kPi);
  a.rc2 = rc * rc;
  a.margin = rc;
  a.n = (int32_t)n;
  a.nbr = nbr;
  a.nnbr = nnbr;
  a.maxn = maxn;
  a.xq = (const double4 *)ws;
  a.F = F;
  a.accumulate = accumulate;
  const unsigned nblk = blocks_of(n, kEwAtoms);
  a.partial = (double *)((char *)ws + (size_t)(n > 0 ? n : 0) * sizeof(double4));
  double *tab = a.partial + nblk;
  a.erfcx_tab = tab;
  const double dx = alpha * rc / kErfcIntervals;
  a.inv_dx = 1.0 / dx;
  a.half_dx = 0.5 * dx;
  if (n > 0) {
    k_pack_xq<<<blocks_of(n, kThreads), kThreads, 0, st>>>((int32_t)n, x, q, (double4 *)ws,
                                                           a.half_dx, tab);
    const bool wide = n > kNarrowAtoms;
    if (e_total) {
      if (wide) k_ewald_real<true, true><<<nblk, kEwThreads, 0, st>>>(a);
      else k_ewald_real<false, true><<<nblk, kEwThreads, 0, st>>>(a);
    } else {
      if (wide) k_ewald_real<true, false><<<nblk, kEwThreads, 0, st>>>(a);
      else k_ewald_real<false, false><<<nblk, kEwThreads, 0, st>>>(a);
    }
  }
  if (e_total)
    k_colsum<1024><<<1, 1024, 0, st>>>(n > 0 ? nblk : 0, 1, 1, a.partial, e_total, 1.0, 0);
  return check_launch("ljmd_ewald_real");
}

int launch_spme_recip(const BoxK &b, double alpha, int32_t order, const int32_t K[3], int64_t n,
                      const double *x, const double *q, double *F, double *e_total,
                      int accumulate, void *ws, hipStream_t st) {
  RecArgs a{};
  a.b = b;
  for (int d = 0; d < 3; ++d) {
    a.K[d] = K[d];
    a.scale[d] = (double)K[d] / b.L[d];
  }
  a.alpha = alpha;
  a.n = (int32_t)n;
  a.x = x;
  a.q = q;
  a.F = F;
  a.accumulate = accumulate;
  const int64_t npts = grid_points(K);
  char *p = (char *)ws;
  a.grid = (double *)p;
  p += (size_t)npts * sizeof(double);
  a.half = (double2 *)p;
  p += (size_t)(npts / 2 + npts / 8) * sizeof(double2);
  a.bmod = (double *)p;
  p += 3 * kMaxGrid * sizeof(double);
  a.partial = (double *)p;
  const unsigned ninf = z_influence_blocks(K);
  const unsigned ngat = blocks_of(n, kThreads);
  double *self_partial = n > 0 ? a.partial + ninf : nullptr;
  switch (order) {
    case 4: launch_rec_order<4>(a, self_partial, st); break;
    case 6: launch_rec_order<6>(a, self_partial, st); break;
    default: launch_rec_order<8>(a, self_partial, st); break;
  }
  if (e_total)
    k_colsum<1024><<<1, 1024, 0, st>>>((int64_t)ninf + (n > 0 ? ngat : 0), 1, 1, a.partial, e_total,
                                     1.0, 0);
  return check_launch("ljmd_spme_recip");
}

}  // namespace ljmd
