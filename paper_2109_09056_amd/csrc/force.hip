// 12-6 Lennard-Jones forces, per-atom energy, energy and virial over the
// tiled-ELL neighbor list, gfx950.  Paper: CabanaMD's Lennard-Jones
// short-range force kernel expressed as a neighbor parallel loop (Cabana
// "Parallel Loops", "CabanaMD").
//
// Pair arithmetic, from u = 4 eps [(sigma/r)^12 - (sigma/r)^6]:
//   ri2 = 1/r^2, sr6 = (sigma^2 ri2)^3
//   s   = -u'(r)/r = ri2 sr6 (48 eps sr6 - 24 eps)
//   u   = sr6 (4 eps sr6 - 4 eps)
// FP64 form: all of it in FP64 (reciprocal = hardware estimate + two Newton
// steps).  Mixed form: displacement, r^2 and the cutoff test in FP64 (so the
// pair set is the FP64 one), then ri2, sr6 and the force scalar s in FP32; s
// is promoted once, and the pair force s*d (with the FP64 d) and the
// accumulation of F, e, E and W are FP64.  The pair energy u is taken in
// FP64 from the FP32 reciprocal refined by one FP64 Newton step.
//
// FULL list: a team of lanes (two; four for grids of at most one block per
// compute unit) owns atom i and walks its row of the tile (row k of lane l of
// tile t at nbr[(t*maxn + k)*64 + l]; lane t of the team takes entries t,
// t + team, ...); no atomics, fixed summation order, so the result is bitwise
// reproducible.  HALF list: the owner adds s*d to F_i in
// registers and subtracts it from F_j with FP64 hardware atomics.
// Energy and virial: per-block partial sums in a fixed tree order, then one
// column-sum launch (deterministic); in chained steps the first workgroup of
// the next step's launch sums them instead.  Full lists take the virial as
// sum_i x_i (x) F_i plus the pairs that cross a box face (add_pair).
#include <type_traits>

#include "common.h"

namespace ljmd {

constexpr int kForceThreads = 128;  // atoms per block of the tiled kernels
constexpr int kForceWaves = kForceThreads / kWave;
constexpr int kCsrThreads = 256;    // threads per block of the CSR kernel (256 / team atoms)
constexpr int kCsrWaves = kCsrThreads / kWave;
constexpr int kEvStride = 8;  // partial row: E, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz, pad

struct ForceArgs {
  BoxK b;
  double rc;
  double rc2;
  int32_t ntypes;
  const double *eps;
  const double *sig;
  int32_t n;
  const double *x;
  const int32_t *type;
  const int32_t *nbr;
  const int32_t *nnbr;
  int32_t maxn;
  double *F;
  double *e_atom;
  double *partial;
  // fused velocity-Verlet step (k_force_full<..., STEP = true> only)
  double *v;
  double *x_next;
  double dt, hdt, mass;
  int unit_mass, open_next;
  // chained steps: block 0 also sums the previous step's partial rows into prev_ev
  const double *prev_partial;
  double *prev_ev;
  int64_t prev_rows;
};

namespace {

// Coefficients of one type pair: sigma^2, 48 eps, 24 eps, 4 eps.
struct Coef {
  double sig2, c12, c6, e4;
};

__device__ __forceinline__ Coef coef_of(const double *eps, const double *sig, int p) {
  Coef c;
  const double e = eps[p], s = sig[p];
  c.sig2 = s * s;
  c.c12 = 48.0 * e;
  c.c6 = 24.0 * e;
  c.e4 = 4.0 * e;
  return c;
}

// Full T x T table in LDS (T > 1): entry (a, b) at 4*(a*T + b).
__device__ __forceinline__ void load_table(const ForceArgs &a, double *tab) {
  const int T = a.ntypes;
  for (int q = threadIdx.x; q < T * T; q += blockDim.x) {
    const Coef c = coef_of(a.eps, a.sig, packed_index(q / T, q % T, T));
    tab[4 * q] = c.sig2;
    tab[4 * q + 1] = c.c12;
    tab[4 * q + 2] = c.c6;
    tab[4 * q + 3] = c.e4;
  }
  __syncthreads();
}

struct PairOut {
  double fx, fy, fz, u;
};

// Pair force components s*d and energy u for r2 < rc2.
template <bool MIXED, bool EV>
__device__ __forceinline__ PairOut lj_pair(double dx, double dy, double dz, double r2,
                                           const Coef &c) {
  PairOut o;
  if constexpr (MIXED) {
    const float ri2 = recip32((float)r2);
    const float sr2 = (float)c.sig2 * ri2;
    const float sr6 = sr2 * sr2 * sr2;
    const double s = (double)(ri2 * sr6 * __builtin_fmaf((float)c.c12, sr6, -(float)c.c6));
    o.fx = s * dx;
    o.fy = s * dy;
    o.fz = s * dz;
    if constexpr (EV) {
      // The pair energy changes sign at r = sigma, and a per-atom energy can
      // nearly cancel; an FP32 u would leave such atoms with relative errors
      // far above the FP32 rounding.  u is formed in FP64 from the FP32
      // reciprocal after one FP64 Newton step (relative error ~1e-13).
      const double y0 = (double)ri2;
      const double y = __builtin_fma(y0, __builtin_fma(-r2, y0, 1.0), y0);
      const double s2 = c.sig2 * y;
      const double s6 = s2 * s2 * s2;
      o.u = s6 * __builtin_fma(c.e4, s6, -c.e4);
    }
  } else {
    const double ri2 = recip64(r2);
    const double sr2 = c.sig2 * ri2;
    const double sr6 = sr2 * sr2 * sr2;
    const double s = ri2 * sr6 * __builtin_fma(c.c12, sr6, -c.c6);
    o.fx = s * dx;
    o.fy = s * dy;
    o.fz = s * dz;
    if constexpr (EV) o.u = sr6 * __builtin_fma(c.e4, sr6, -c.e4);
  }
  return o;
}

// Accumulators of one atom's row.
struct Acc {
  double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0;
  double wxx = 0.0, wyy = 0.0, wzz = 0.0, wxy = 0.0, wxz = 0.0, wyz = 0.0;
};

// One neighbor j of atom i: minimum image (WRAP), cutoff test, pair force and
// the row's accumulators.  `valid` is false for padding slots of a short group.
//
// Virial of the full list, W = 1/2 sum_i sum_j d_ij (x) f_ij with
// d_ij = x_i - x_j + S_ij (S_ij = -k L, the minimum-image shift):
//   W = sum_i x_i (x) F_i + 1/2 sum_i sum_j S_ij (x) f_ij,
// exactly, component by component (sum_i f_ij = -F_j for the symmetric pair
// set).  So a pair adds to W only when it crosses a box face (WRAP path,
// S != 0), and every lane adds 2 x_i (x) (its part of F_i) once (add_xf).
template <bool MIXED, bool T1, bool EV, bool WRAP>
__device__ __forceinline__ void add_pair(const ForceArgs &a, double xi, double yi, double zi,
                                         double xj, double yj, double zj, int32_t j, bool valid,
                                         int ti, const Coef &c1, const double *tab, Acc &s) {
  double dx = xi - xj, dy = yi - yj, dz = zi - zj;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  if constexpr (WRAP) {  // min_image, keeping the shift
    const double kx = __builtin_rint(dx * a.b.invL[0]);
    const double ky = __builtin_rint(dy * a.b.invL[1]);
    const double kz = __builtin_rint(dz * a.b.invL[2]);
    dx = __builtin_fma(-kx, a.b.L[0], dx);
    dy = __builtin_fma(-ky, a.b.L[1], dy);
    dz = __builtin_fma(-kz, a.b.L[2], dz);
    sx = -kx * a.b.L[0];
    sy = -ky * a.b.L[1];
    sz = -kz * a.b.L[2];
  }
  const double r2 = dist2(dx, dy, dz);
  if (valid && r2 < a.rc2) {
    Coef c;
    if constexpr (T1) {
      c = c1;
    } else {
      const double *t = tab + 4 * (ti * a.ntypes + a.type[j]);
      c = Coef{t[0], t[1], t[2], t[3]};
    }
    const PairOut p = lj_pair<MIXED, EV>(dx, dy, dz, r2, c);
    s.fx += p.fx;
    s.fy += p.fy;
    s.fz += p.fz;
    if constexpr (EV) {
      s.e += p.u;
      if constexpr (WRAP) {
        s.wxx = __builtin_fma(sx, p.fx, s.wxx);
        s.wyy = __builtin_fma(sy, p.fy, s.wyy);
        s.wzz = __builtin_fma(sz, p.fz, s.wzz);
        s.wxy = __builtin_fma(sx, p.fy, s.wxy);
        s.wxz = __builtin_fma(sx, p.fz, s.wxz);
        s.wyz = __builtin_fma(sy, p.fz, s.wyz);
      }
    }
  }
}

// The per-lane x_i (x) F term of the virial (see add_pair), with the lane's
// part of F_i; called once per lane after its row, before any team sums.
__device__ __forceinline__ void add_xf(double xi, double yi, double zi, Acc &s) {
  const double x2 = 2.0 * xi, y2 = 2.0 * yi, z2 = 2.0 * zi;
  s.wxx = __builtin_fma(x2, s.fx, s.wxx);
  s.wyy = __builtin_fma(y2, s.fy, s.wyy);
  s.wzz = __builtin_fma(z2, s.fz, s.wzz);
  s.wxy = __builtin_fma(x2, s.fy, s.wxy);
  s.wxz = __builtin_fma(x2, s.fz, s.wxz);
  s.wyz = __builtin_fma(y2, s.fz, s.wyz);
}

// Positions and forces in an AoSoA(V) layout (Cabana's array of structs of
// arrays): chunks of V consecutive atoms, each chunk holding its x's, then its
// y's, then its z's; the last chunk holds the m = n mod V remaining atoms (when
// nonzero) in the same way, so the array is exactly 3n long.  V = 1 is [n][3];
// V = 0 stands for plain SoA (three arrays of n).  Component k of atom i sits
// at aos_index<V>(i, k, n).
template <int V>
__device__ __forceinline__ int64_t aos_width(int64_t c, int64_t n) {  // atoms in chunk c
  const int64_t left = n - c * V;
  return left < V ? left : V;
}

template <int V>
__device__ __forceinline__ int64_t aos_index(int64_t i, int k, int64_t n) {
  if constexpr (V == 0) {
    return k * n + i;
  } else if constexpr (V == 1) {
    return 3 * i + k;
  } else {
    const int64_t c = i / V;
    return c * (3 * V) + k * aos_width<V>(c, n) + (i - c * V);
  }
}

// Atom j's position: V = 1 as a 16-byte and an 8-byte load (pos_of); other
// layouts as three 8-byte loads.
template <int V, bool WIDE>
__device__ __forceinline__ void load_pos(const double *x, int32_t j, int64_t n, double &xj,
                                         double &yj, double &zj) {
  if constexpr (V == 1) {
    const double *p = pos_of<WIDE>(x, j);
    xj = p[0];
    yj = p[1];
    zj = p[2];
  } else if constexpr (V == 0) {
    const double *p = x + j;
    xj = p[0];
    yj = p[n];
    zj = p[2 * n];
  } else {
    const int64_t c = j / V;
    const int64_t m = aos_width<V>(c, n);
    const double *p = x + c * (3 * V) + (j - c * V);
    xj = p[0];
    yj = p[m];
    zj = p[2 * m];
  }
}

// Walk atom i's row in groups of U slots: the U index loads, then the U
// position gathers, then the U pair evaluations, so several loads are in
// flight per lane.  Whole groups read their indices at fixed offsets from one
// row pointer (no per-slot address arithmetic); the last, partial group loads
// indices and positions only for slots below cnt.
// Slots are visited in row order, so the sums are the same as one slot at a
// time.  STRIDE > 1: the lane owns every STRIDE-th entry of the row (row points
// at its first one).  WRAP = false skips the minimum image; the caller only takes that
// path when every atom of the wavefront is at least rc from all box faces,
// where any pair closer than rc has the same raw and minimum-image
// displacement, and any other pair has some |raw component| above L/2 > rc
// and is rejected by the cutoff test either way.
template <bool MIXED, bool T1, bool EV, int U, bool WRAP, bool WIDE, int STRIDE = 1, int V = 1>
__device__ __forceinline__ void walk_row(const ForceArgs &a, const int32_t *row, int32_t cnt,
                                         double xi, double yi, double zi, int ti,
                                         const Coef &c1, const double *tab, Acc &s) {
  constexpr int kStep = STRIDE * kWave;  // ints between this lane's consecutive entries
  const int32_t whole = cnt - cnt % U;
  int32_t k = 0;
  for (; k < whole; k += U, row += U * kStep) {
    int32_t j[U];
#pragma unroll
    for (int u = 0; u < U; ++u) j[u] = row[u * kStep];
    double xj[U], yj[U], zj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      load_pos<V, WIDE>(a.x, j[u], a.n, xj[u], yj[u], zj[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      add_pair<MIXED, T1, EV, WRAP>(a, xi, yi, zi, xj[u], yj[u], zj[u], j[u], true, ti, c1, tab,
                                    s);
  }
  if (k < cnt) {
    int32_t j[U];
#pragma unroll
    for (int u = 0; u < U; ++u) j[u] = row[(k + u < cnt ? u : 0) * kStep];
    double xj[U], yj[U], zj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      xj[u] = xi;
      yj[u] = yi;
      zj[u] = zi;
      if (k + u < cnt) {  // no gathers for the padding slots
        load_pos<V, WIDE>(a.x, j[u], a.n, xj[u], yj[u], zj[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      add_pair<MIXED, T1, EV, WRAP>(a, xi, yi, zi, xj[u], yj[u], zj[u], j[u], k + u < cnt, ti, c1,
                                    tab, s);
  }
}

// TEAM lanes per atom: lane t of an atom's team walks the row entries t,
// t + TEAM, ...; neighbouring entries of one row are mostly nearby atoms, so
// the lanes of a team gather from nearby addresses and each gather instruction
// touches fewer cache lines than with one lane per atom.  The team's force
// and per-atom energy are combined by a butterfly over the team (both lanes
// of every exchange add the same two numbers: every lane ends with the same,
// order-fixed sum); energy and virial partials enter the block sum per lane.
//
// STEP: after the row, the team also finishes its atom's velocity-Verlet
// step -- closing half kick (kinetic energy taken there), and when open_next
// the next step's half kick, drift and wrap into x_next -- with exactly the
// operations of ljmd_integrate, so the trajectory is bitwise the same as the
// unfused calls; lane t handles components t, t + TEAM, ...  Partial rows
// then carry the kinetic energy in column 7.
// Column sums of `rows` partial rows of kEvStride doubles by the THREADS threads
// of one block, out[q] = sum_r p[r*kEvStride + q] for q < kEvStride: thread t
// reads the flat array at t, t + THREADS, ... (column t % kEvStride), the lanes
// of one column meet by shuffles, the waves in LDS (`lds`: THREADS/64*kEvStride
// doubles).  Fixed order; every thread of the block calls it.
template <int THREADS>
__device__ void block_colsum(const double *__restrict__ p, int64_t rows, double *__restrict__ out,
                             double *lds) {
  static_assert(THREADS % kWave == 0 && kWave % kEvStride == 0, "column per lane");
  const int t = threadIdx.x;
  const int64_t total = rows * kEvStride;
  double s = 0.0;
  constexpr int B = 8;  // loads in flight per thread
  for (int64_t f0 = t; f0 < total; f0 += (int64_t)B * THREADS) {
    double v[B];
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const int64_t f = f0 + (int64_t)k * THREADS;
      v[k] = f < total ? p[f] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < B; ++k) s += v[k];
  }
#pragma unroll
  for (int mask = kWave / 2; mask >= kEvStride; mask >>= 1) s += __shfl_xor(s, mask, kWave);
  const int w = t / kWave, l = t % kWave;
  if (l < kEvStride) lds[w * kEvStride + l] = s;
  __syncthreads();
  if (t < kEvStride) {
    double r = 0.0;
#pragma unroll
    for (int q = 0; q < THREADS / kWave; ++q) r += lds[q * kEvStride + t];
    out[t] = r;
  }
}

template <bool MIXED, bool T1, bool EV, int U, bool SKIP, bool STEP, bool WIDE, int TEAM,
          int V = 1>
__global__ __launch_bounds__(kForceThreads * TEAM) void k_force_full(ForceArgs a) {
  static_assert(!STEP || V == 1, "the fused step works on [n][3] arrays");
  __shared__ double tab[T1 ? 4 : 4 * LJMD_MAX_TYPES * LJMD_MAX_TYPES];
  __shared__ double red[kForceWaves * TEAM * 8];
  if constexpr (STEP) {
    // chained steps: the previous launch's partial rows are complete (stream
    // order); block 0 is dispatched first, so its extra pass is off the tail
    if (a.prev_ev && blockIdx.x == 0) {  // block-uniform
      block_colsum<kForceThreads * TEAM>(a.prev_partial, a.prev_rows, a.prev_ev, red);
      __syncthreads();  // `red` is read above and written again by block_sum
    }
  }
  Coef c1{};
  if constexpr (T1) {
    c1 = coef_of(a.eps, a.sig, 0);
  } else {
    load_table(a, tab);
  }
  const int t = (int)threadIdx.x % TEAM;
  const int32_t i = xcd_block(blockIdx.x, gridDim.x) * kForceThreads + (int)threadIdx.x / TEAM;
  Acc s;
  double ke = 0.0;
  const bool live = i < a.n;
  double xi = 0.0, yi = 0.0, zi = 0.0;
  if (live) {
    xi = a.x[aos_index<V>(i, 0, a.n)];
    yi = a.x[aos_index<V>(i, 1, a.n)];
    zi = a.x[aos_index<V>(i, 2, a.n)];
  }
  bool interior = false;
  if constexpr (SKIP) {
    const double m = a.rc;
    const bool in = !live || (xi >= m && xi <= a.b.L[0] - m && yi >= m && yi <= a.b.L[1] - m &&
                              zi >= m && zi <= a.b.L[2] - m);
    interior = __ballot(!in) == 0;  // wavefront-uniform
  }
  if (live) {
    const int ti = T1 ? 0 : a.type[i];
    const int32_t ctot = a.nnbr[i];
    const int32_t cnt = ctot > t ? (ctot - t + TEAM - 1) / TEAM : 0;
    const int32_t *row =
        a.nbr + (int64_t)(i >> 6) * a.maxn * kWave + (i & (kWave - 1)) + (int64_t)t * kWave;
    if (SKIP && interior)
      walk_row<MIXED, T1, EV, U, false, WIDE, TEAM, V>(a, row, cnt, xi, yi, zi, ti, c1, tab, s);
    else
      walk_row<MIXED, T1, EV, U, true, WIDE, TEAM, V>(a, row, cnt, xi, yi, zi, ti, c1, tab, s);
    if constexpr (EV) add_xf(xi, yi, zi, s);
  }
  const double e_lane = s.e;
  if constexpr (TEAM > 1) {
#pragma unroll
    for (int mask = TEAM / 2; mask > 0; mask >>= 1) {
      s.fx += __shfl_xor(s.fx, mask, kWave);
      s.fy += __shfl_xor(s.fy, mask, kWave);
      s.fz += __shfl_xor(s.fz, mask, kWave);
      if constexpr (EV) s.e += __shfl_xor(s.e, mask, kWave);
    }
  }
  if (live) {
    if (t == 0) {
      if (!STEP || a.F) {
        a.F[aos_index<V>(i, 0, a.n)] = s.fx;
        a.F[aos_index<V>(i, 1, a.n)] = s.fy;
        a.F[aos_index<V>(i, 2, a.n)] = s.fz;
      }
      if (a.e_atom) a.e_atom[i] = 0.5 * s.e;
    }
    if constexpr (STEP) {
      const double f[3] = {s.fx, s.fy, s.fz};
      const double xo[3] = {xi, yi, zi};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (k % TEAM != t) continue;
        const int64_t q = 3 * (int64_t)i + k;
        double kick = a.hdt * f[k];
        if (!a.unit_mass) kick = kick / a.mass;
        const double vn = a.v[q] + kick;
        ke = __builtin_fma(vn, vn, ke);
        if (a.open_next) {
          const double L = a.b.L[k];
          const double vh = vn + kick;
          double xq = xo[k] + a.dt * vh;
          if (xq >= L) xq -= L;
          else if (xq < 0.0) xq += L;
          if (xq >= L) xq -= L;
          a.v[q] = vh;
          a.x_next[q] = xq;
        } else {
          a.v[q] = vn;
        }
      }
    }
  }
  if constexpr (EV) {
    const double v[8] = {0.5 * e_lane, 0.5 * s.wxx, 0.5 * s.wyy, 0.5 * s.wzz,
                         0.5 * s.wxy,  0.5 * s.wxz, 0.5 * s.wyz, 0.5 * a.mass * ke};
    block_sum<kForceWaves * TEAM, 8>(v, red, a.partial + (int64_t)blockIdx.x * kEvStride);
  }
}

__global__ void k_zero_f64(double *p, int64_t m) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) p[q] = 0.0;
}

// p[0..m) = 0 and, when r is given, r[0..k) = 0, in one launch (k <= m).
__global__ void k_zero2_f64(double *p, int64_t m, double *r, int64_t k) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) p[q] = 0.0;
  if (r && q < k) r[q] = 0.0;
}

// Half list (HALF): blocks of ATOMS consecutive sorted atoms, TEAM lanes per
// atom (lane t takes the row entries t, t + TEAM, ...).  The owner of
// pair (i, j), j > i, keeps +s*d for F_i in registers and hands -s*d (and u/2
// for e_j) to j through LDS: the block's j-side sums are kept per 64-atom tile
// of sorted atoms, in SLOTS slots assigned at a tile's first touch by a small
// open-addressing table keyed by the tile; after the rows, each slot is added
// to F (and e_atom) with coalesced FP64 atomics, one per touched atom and
// component.  A pair whose tile finds no slot (more tiles than slots, or a slot
// another wave has claimed but not yet published) adds its j-side through
// direct global atomics.  Summation order is not fixed: HALF results are
// reproducible to rounding, not bitwise.
constexpr int kHalfTeam = 2;  // lanes per home atom (large grids)
constexpr int kHalfTabBits = 7;
constexpr int kHalfTab = 1 << kHalfTabBits;  // table entries

template <int NV, int SLOTS>
struct HalfLds {
  double acc[SLOTS][NV][kWave];  // per slot: Fx, Fy, Fz (, e) of the tile's 64 atoms
  int32_t key[kHalfTab];          // tile, or -1
  int32_t slot[kHalfTab];         // its slot, or -1 (none, or not yet published)
  int32_t tile_of[SLOTS];
  int32_t count;                  // slots claimed (may exceed SLOTS)
};

// Slot of `tile` in the block's table, claiming one at its first touch; -1 when
// there is none to use (table or slots full, or claimed by another lane whose
// publication this lane does not see yet).
template <int NV, int SLOTS>
__device__ __forceinline__ int32_t half_slot(HalfLds<NV, SLOTS> &s, int32_t tile) {
  uint32_t h = ((uint32_t)tile * 2654435761u) >> (32 - kHalfTabBits);
  for (int p = 0; p < kHalfTab; ++p) {
    const int32_t k = __atomic_load_n(&s.key[h], __ATOMIC_RELAXED);
    if (k == tile) return __atomic_load_n(&s.slot[h], __ATOMIC_RELAXED);
    if (k < 0) {
      const int32_t old = atomicCAS(&s.key[h], -1, tile);
      if (old < 0) {
        const int32_t q = atomicAdd(&s.count, 1);
        const int32_t v = q < SLOTS ? q : -1;
        if (v >= 0) s.tile_of[v] = tile;
        __atomic_store_n(&s.slot[h], v, __ATOMIC_RELAXED);
        return v;
      }
      if (old == tile) return __atomic_load_n(&s.slot[h], __ATOMIC_RELAXED);
    }
    h = (h + 1) & (kHalfTab - 1);
  }
  return -1;
}

// Row accumulators of the half-list kernel (per-pair virial, as the pair is seen once).
struct HalfAcc {
  double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0;
  double wxx = 0.0, wyy = 0.0, wzz = 0.0, wxy = 0.0, wxz = 0.0, wyz = 0.0;
};

// EV: energy and virial sums; EATOM: per-atom energies (j-side halves through LDS).
template <bool MIXED, bool T1, bool EV, bool EATOM, bool WRAP, int NV, int SLOTS>
__device__ __forceinline__ void half_pair(const ForceArgs &a, HalfLds<NV, SLOTS> &s,
                                          double xi, double yi, double zi, double xj, double yj,
                                          double zj, int32_t j, bool valid, int ti,
                                          const Coef &c1, const double *tab, HalfAcc &r,
                                          int32_t &ltile, int32_t &lslot) {
  double dx = xi - xj, dy = yi - yj, dz = zi - zj;
  if constexpr (WRAP) {
    dx = min_image(dx, a.b.L[0], a.b.invL[0]);
    dy = min_image(dy, a.b.L[1], a.b.invL[1]);
    dz = min_image(dz, a.b.L[2], a.b.invL[2]);
  }
  const double r2 = dist2(dx, dy, dz);
  if (valid && r2 < a.rc2) {
    Coef c;
    if constexpr (T1) {
      c = c1;
    } else {
      const double *t = tab + 4 * (ti * a.ntypes + a.type[j]);
      c = Coef{t[0], t[1], t[2], t[3]};
    }
    const PairOut p = lj_pair<MIXED, EV || EATOM>(dx, dy, dz, r2, c);
    r.fx += p.fx;
    r.fy += p.fy;
    r.fz += p.fz;
    if constexpr (EV || EATOM) r.e += p.u;
    if constexpr (EV) {
      r.wxx = __builtin_fma(dx, p.fx, r.wxx);
      r.wyy = __builtin_fma(dy, p.fy, r.wyy);
      r.wzz = __builtin_fma(dz, p.fz, r.wzz);
      r.wxy = __builtin_fma(dx, p.fy, r.wxy);
      r.wxz = __builtin_fma(dx, p.fz, r.wxz);
      r.wyz = __builtin_fma(dy, p.fz, r.wyz);
    }
    const int32_t tile = j >> 6;
    if (tile != ltile || lslot < 0) {
      lslot = half_slot(s, tile);
      ltile = tile;
    }
    if (lslot >= 0) {
      const int l = j & (kWave - 1);
      unsafeAtomicAdd(&s.acc[lslot][0][l], -p.fx);
      unsafeAtomicAdd(&s.acc[lslot][1][l], -p.fy);
      unsafeAtomicAdd(&s.acc[lslot][2][l], -p.fz);
      if constexpr (EATOM) unsafeAtomicAdd(&s.acc[lslot][NV - 1][l], 0.5 * p.u);
    } else {
      unsafeAtomicAdd(&a.F[3 * (int64_t)j], -p.fx);
      unsafeAtomicAdd(&a.F[3 * (int64_t)j + 1], -p.fy);
      unsafeAtomicAdd(&a.F[3 * (int64_t)j + 2], -p.fz);
      if constexpr (EATOM) unsafeAtomicAdd(&a.e_atom[j], 0.5 * p.u);
    }
  }
}

// One lane's share of a half row: every TEAM-th entry from `row`, in groups of
// U (indices, then gathers, then pairs, as walk_row).
template <bool MIXED, bool T1, bool EV, bool EATOM, bool WRAP, bool WIDE, int U, int TEAM,
          int NV, int SLOTS>
__device__ __forceinline__ void half_row(const ForceArgs &a, HalfLds<NV, SLOTS> &s,
                                         const int32_t *row, int32_t cnt, double xi, double yi,
                                         double zi, int ti, const Coef &c1, const double *tab,
                                         HalfAcc &r) {
  constexpr int kStep = TEAM * kWave;
  int32_t ltile = -1, lslot = -1;
  for (int32_t k = 0; k < cnt; k += U, row += U * kStep) {
    int32_t j[U];
#pragma unroll
    for (int u = 0; u < U; ++u) j[u] = row[(k + u < cnt ? u : 0) * kStep];
    double xj[U], yj[U], zj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      xj[u] = xi;
      yj[u] = yi;
      zj[u] = zi;
      if (k + u < cnt) {
        const double *q = pos_of<WIDE>(a.x, j[u]);
        xj[u] = q[0];
        yj[u] = q[1];
        zj[u] = q[2];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      half_pair<MIXED, T1, EV, EATOM, WRAP>(a, s, xi, yi, zi, xj[u], yj[u], zj[u], j[u],
                                            k + u < cnt, ti, c1, tab, r, ltile, lslot);
  }
}

template <bool MIXED, bool T1, bool EV, bool EATOM, bool WIDE, int ATOMS, int SLOTS, int U,
          int TEAM = kHalfTeam>
__global__ __launch_bounds__(ATOMS * TEAM) void k_force_half(ForceArgs a) {
  constexpr int NV = EATOM ? 4 : 3;
  constexpr int kThreads = ATOMS * TEAM;
  constexpr int kWaves = kThreads / kWave;
  __shared__ HalfLds<NV, SLOTS> s;
  __shared__ double tab[T1 ? 4 : 4 * LJMD_MAX_TYPES * LJMD_MAX_TYPES];
  __shared__ double red[kWaves * 7];
  for (int q = threadIdx.x; q < SLOTS * NV * kWave; q += kThreads) (&s.acc[0][0][0])[q] = 0.0;
  for (int q = threadIdx.x; q < kHalfTab; q += kThreads) {
    s.key[q] = -1;
    s.slot[q] = -1;
  }
  if (threadIdx.x == 0) s.count = 0;
  Coef c1{};
  if constexpr (T1) {
    c1 = coef_of(a.eps, a.sig, 0);
  } else {
    load_table(a, tab);  // ends with a barrier
  }
  __syncthreads();
  const int t = (int)threadIdx.x % TEAM;
  const int32_t i = xcd_block(blockIdx.x, gridDim.x) * ATOMS + (int)threadIdx.x / TEAM;
  const bool live = i < a.n;
  double xi = 0.0, yi = 0.0, zi = 0.0;
  if (live) {
    xi = a.x[3 * (int64_t)i];
    yi = a.x[3 * (int64_t)i + 1];
    zi = a.x[3 * (int64_t)i + 2];
  }
  const double m = a.rc;
  const bool in = !live || (xi >= m && xi <= a.b.L[0] - m && yi >= m && yi <= a.b.L[1] - m &&
                            zi >= m && zi <= a.b.L[2] - m);
  const bool interior = __ballot(!in) == 0;  // wavefront-uniform
  HalfAcc r;
  if (live) {
    const int ti = T1 ? 0 : a.type[i];
    const int32_t ctot = a.nnbr[i];
    const int32_t cnt = ctot > t ? (ctot - t + TEAM - 1) / TEAM : 0;
    const int32_t *row =
        a.nbr + (int64_t)(i >> 6) * a.maxn * kWave + (i & (kWave - 1)) + (int64_t)t * kWave;
    if (interior)
      half_row<MIXED, T1, EV, EATOM, false, WIDE, U, TEAM>(a, s, row, cnt, xi, yi, zi, ti, c1,
                                                           tab, r);
    else
      half_row<MIXED, T1, EV, EATOM, true, WIDE, U, TEAM>(a, s, row, cnt, xi, yi, zi, ti, c1,
                                                          tab, r);
  }
  const double e_lane = r.e;
#pragma unroll
  for (int mask = TEAM / 2; mask > 0; mask >>= 1) {
    r.fx += __shfl_xor(r.fx, mask, kWave);
    r.fy += __shfl_xor(r.fy, mask, kWave);
    r.fz += __shfl_xor(r.fz, mask, kWave);
    if constexpr (EATOM) r.e += __shfl_xor(r.e, mask, kWave);
  }
  if (live && t == 0) {  // the owner's side of its pairs joins the j-side sums of its tile
    const int32_t sl = half_slot(s, i >> 6);
    const int l = i & (kWave - 1);
    if (sl >= 0) {
      unsafeAtomicAdd(&s.acc[sl][0][l], r.fx);
      unsafeAtomicAdd(&s.acc[sl][1][l], r.fy);
      unsafeAtomicAdd(&s.acc[sl][2][l], r.fz);
      if constexpr (EATOM) unsafeAtomicAdd(&s.acc[sl][NV - 1][l], 0.5 * r.e);
    } else {
      unsafeAtomicAdd(&a.F[3 * (int64_t)i], r.fx);
      unsafeAtomicAdd(&a.F[3 * (int64_t)i + 1], r.fy);
      unsafeAtomicAdd(&a.F[3 * (int64_t)i + 2], r.fz);
      if constexpr (EATOM) unsafeAtomicAdd(&a.e_atom[i], 0.5 * r.e);
    }
  }
  __syncthreads();
  // flush: slot sl's F block is the 3*64 consecutive doubles of its tile; wave w
  // adds rows (sl, q) = w, w + kWaves, ..., 64 consecutive doubles per row
  const int nsl = s.count < SLOTS ? s.count : SLOTS;
  constexpr int kRows = NV;  // F in three rows of 64 doubles (+ e_atom)
  const int lane = (int)threadIdx.x & (kWave - 1);
  for (int q = (int)threadIdx.x / kWave; q < nsl * kRows; q += kWaves) {
    const int sl = q / kRows, part = q % kRows;
    const int64_t base = (int64_t)s.tile_of[sl] * kWave;
    if (part < 3) {
      const int e = part * kWave + lane;  // element of the tile's F block
      const int atom = e / 3, comp = e % 3;
      const double v = s.acc[sl][comp][atom];
      if (base + atom < a.n && v != 0.0) unsafeAtomicAdd(&a.F[3 * base + e], v);
    } else {
      const double v = s.acc[sl][NV - 1][lane];
      if (base + lane < a.n && v != 0.0) unsafeAtomicAdd(&a.e_atom[base + lane], v);
    }
  }
  if constexpr (EV) {
    const double v[7] = {e_lane, r.wxx, r.wyy, r.wzz, r.wxy, r.wxz, r.wyz};
    block_sum<kWaves, 7>(v, red, a.partial + (int64_t)blockIdx.x * kEvStride);
  }
}

// CSR list, `TEAM` lanes per atom (hierarchical traversal): lane t of an
// atom's team takes the row entries t, t + TEAM, ... in groups of U (whole
// groups first, the partial group gathers only live slots), then the team's
// sums are combined by a butterfly over the team (both lanes of every exchange
// add the same two numbers, so every lane ends with the same, order-fixed sum).
// Each lane walks its entries in row order, as k_force_full does: with the
// same team size the two kernels give bitwise the same forces and per-atom
// energies.
template <bool MIXED, bool T1, bool EV, int TEAM, int U, bool WIDE>
__global__ __launch_bounds__(kCsrThreads) void k_force_csr(ForceArgs a,
                                                            const int64_t *__restrict__ off,
                                                            const int32_t *__restrict__ csr) {
  __shared__ double tab[T1 ? 4 : 4 * LJMD_MAX_TYPES * LJMD_MAX_TYPES];
  __shared__ double red[kCsrWaves * 8];
  Coef c1{};
  if constexpr (T1) {
    c1 = coef_of(a.eps, a.sig, 0);
  } else {
    load_table(a, tab);
  }
  constexpr int kAtoms = kCsrThreads / TEAM;  // atoms per block
  const int t = threadIdx.x % TEAM;
  const int64_t i64 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kAtoms + threadIdx.x / TEAM;
  const bool live = i64 < a.n;
  const int32_t i = live ? (int32_t)i64 : 0;
  double xi = 0.0, yi = 0.0, zi = 0.0;
  if (live) {
    xi = a.x[3 * (int64_t)i];
    yi = a.x[3 * (int64_t)i + 1];
    zi = a.x[3 * (int64_t)i + 2];
  }
  const double m = a.rc;
  const bool in = !live || (xi >= m && xi <= a.b.L[0] - m && yi >= m && yi <= a.b.L[1] - m &&
                            zi >= m && zi <= a.b.L[2] - m);
  const bool interior = __ballot(!in) == 0;  // wavefront-uniform
  Acc s;
  if (live) {
    const int ti = T1 ? 0 : a.type[i];
    const int64_t r0 = off[i], r1 = off[i + 1];
    const int32_t cnt = r1 - r0 > t ? (int32_t)((r1 - r0 - t + TEAM - 1) / TEAM) : 0;
    const int32_t *row = csr + r0 + t;
    auto walk = [&](auto wrap) {
      constexpr bool W = decltype(wrap)::value;
      const int32_t whole = cnt - cnt % U;
      const int32_t *rp = row;
      int32_t k = 0;
      for (; k < whole; k += U, rp += U * TEAM) {
        int32_t j[U];
#pragma unroll
        for (int u = 0; u < U; ++u) j[u] = rp[u * TEAM];
        double xj[U], yj[U], zj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const double *p = pos_of<WIDE>(a.x, j[u]);
          xj[u] = p[0];
          yj[u] = p[1];
          zj[u] = p[2];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
          add_pair<MIXED, T1, EV, W>(a, xi, yi, zi, xj[u], yj[u], zj[u], j[u], true, ti, c1, tab, s);
      }
      if (k < cnt) {
        int32_t j[U];
#pragma unroll
        for (int u = 0; u < U; ++u) j[u] = rp[(k + u < cnt ? u : 0) * TEAM];
        double xj[U], yj[U], zj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          xj[u] = xi;
          yj[u] = yi;
          zj[u] = zi;
          if (k + u < cnt) {
            const double *p = pos_of<WIDE>(a.x, j[u]);
            xj[u] = p[0];
            yj[u] = p[1];
            zj[u] = p[2];
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
          add_pair<MIXED, T1, EV, W>(a, xi, yi, zi, xj[u], yj[u], zj[u], j[u], k + u < cnt, ti, c1,
                                     tab, s);
      }
    };
    if (interior)
      walk(std::false_type{});
    else
      walk(std::true_type{});
    if constexpr (EV) add_xf(xi, yi, zi, s);
  }
  if constexpr (TEAM > 1) {
#pragma unroll
    for (int mask = TEAM / 2; mask > 0; mask >>= 1) {
      s.fx += __shfl_xor(s.fx, mask, kWave);
      s.fy += __shfl_xor(s.fy, mask, kWave);
      s.fz += __shfl_xor(s.fz, mask, kWave);
      if constexpr (EV) {
        s.e += __shfl_xor(s.e, mask, kWave);
        s.wxx += __shfl_xor(s.wxx, mask, kWave);
        s.wyy += __shfl_xor(s.wyy, mask, kWave);
        s.wzz += __shfl_xor(s.wzz, mask, kWave);
        s.wxy += __shfl_xor(s.wxy, mask, kWave);
        s.wxz += __shfl_xor(s.wxz, mask, kWave);
        s.wyz += __shfl_xor(s.wyz, mask, kWave);
      }
    }
  }
  const bool lead = live && t == 0;
  if (lead) {
    a.F[3 * (int64_t)i] = s.fx;
    a.F[3 * (int64_t)i + 1] = s.fy;
    a.F[3 * (int64_t)i + 2] = s.fz;
    if (a.e_atom) a.e_atom[i] = 0.5 * s.e;
  }
  if constexpr (EV) {
    const double z = 0.0;
    const double v[7] = {lead ? 0.5 * s.e : z,   lead ? 0.5 * s.wxx : z, lead ? 0.5 * s.wyy : z,
                         lead ? 0.5 * s.wzz : z, lead ? 0.5 * s.wxy : z, lead ? 0.5 * s.wxz : z,
                         lead ? 0.5 * s.wyz : z};
    block_sum<kCsrWaves, 7>(v, red, a.partial + (int64_t)blockIdx.x * kEvStride);
  }
}

// Loop shapes, measured on MI355X.  One lane per atom (the CSR kernel with
// team 1): 8 slots per group, against 1, 2 and 4.  Tiled full list: two lanes
// per atom with 6 slots per group each, against one lane with 8 slots and
// teams of 4 (fewer cache lines per gather instruction); 128 atoms (256
// threads) per block, against 64 and 256 atoms (more resident blocks per CU
// hide more gather latency; 64 pays for its extra energy/virial partial rows).
constexpr int kUnroll = 8;
constexpr int kTeam = 2;
constexpr int kTeamUnroll = 6;
// Up to LJMD_SMALL_GRID_ATOMS atoms (at most one 128-atom block per compute
// unit) the tiled full-list kernels take four lanes per atom with 3 slots per
// group: twice the waves in flight on a chip the grid leaves mostly idle.
// Measured at 32,000 atoms: fused step 12.5 -> 11.6 us (FP64 12.1 -> 11.5),
// forces with energy/virial 11.1 -> 10.1 us; from about 42,000 atoms (two
// blocks per compute unit) on, four lanes gain nothing on the step, and at
// 500,000 atoms the step takes 110 against 90 us.
constexpr int64_t kSmallGridAtoms = LJMD_SMALL_GRID_ATOMS;
constexpr int kSmallTeam = 4;
constexpr int kSmallTeamUnroll = 3;
static_assert(kSmallGridAtoms == 256 * kForceThreads, "one block per compute unit");

// Half-list blocks: 256 home atoms with two lanes each (512 threads), 32 tile
// slots, 4 entries per group.  Up to kHalfSmallAtoms atoms: blocks of 128 home
// atoms with four lanes each (more blocks and more waves for grids that do not
// fill the chip); up to LJMD_SMALL_GRID_ATOMS atoms (one block per compute
// unit): eight lanes each and 48 slots.  Measured with per-atom energies and
// virial (us): 32,000 atoms 38.0 (128 x 2) -> 28.0 (128 x 4) -> 23.2 (128 x 8,
// 48 slots); 108,000 atoms 77.5 -> 61.7 (128 x 4; 256 x 2: 64.9); 256,000
// atoms 153.4 -> 127.9 (256 x 2: 141.0); 500,000 atoms 256 x 2 234.2, 128 x 4
// 236.3, 128 x 8 373.
constexpr int kHalfAtoms = 256;
constexpr int kHalfSmallBlock = 128;
constexpr int64_t kHalfSmallAtoms = 262144;
constexpr int kHalfSlots = 32;
constexpr int kHalfUnroll = 4;
constexpr int kHalfSmallTeam = 4;
constexpr int kHalfTinyTeam = 8;
constexpr int kHalfTinySlots = 48;

int half_block_atoms(int64_t n) { return n <= kHalfSmallAtoms ? kHalfSmallBlock : kHalfAtoms; }

unsigned half_blocks(int64_t n) {
  const int64_t per = half_block_atoms(n);
  const int64_t b = (n + per - 1) / per;
  return (unsigned)(b > 0 ? b : 1);
}

template <bool MIXED, bool T1, bool EV, bool EATOM>
void launch_half(const ForceArgs &a, hipStream_t st) {
  const unsigned nb = half_blocks(a.n);
  if (a.n <= kSmallGridAtoms)
    k_force_half<MIXED, T1, EV, EATOM, false, kHalfSmallBlock, kHalfTinySlots, kHalfUnroll,
                 kHalfTinyTeam><<<nb, kHalfSmallBlock * kHalfTinyTeam, 0, st>>>(a);
  else if (a.n <= kHalfSmallAtoms)
    k_force_half<MIXED, T1, EV, EATOM, false, kHalfSmallBlock, kHalfSlots, kHalfUnroll,
                 kHalfSmallTeam><<<nb, kHalfSmallBlock * kHalfSmallTeam, 0, st>>>(a);
  else if (a.n <= kNarrowAtoms)
    k_force_half<MIXED, T1, EV, EATOM, false, kHalfAtoms, kHalfSlots, kHalfUnroll>
        <<<nb, kHalfAtoms * kHalfTeam, 0, st>>>(a);
  else
    k_force_half<MIXED, T1, EV, EATOM, true, kHalfAtoms, kHalfSlots, kHalfUnroll>
        <<<nb, kHalfAtoms * kHalfTeam, 0, st>>>(a);
}

// The tiled full-list kernel in the team shape for a.n atoms (every caller --
// forces, AoSoA forces, fused step -- takes the same shape, so their sums agree
// bitwise); nblk = force_blocks(a.n).
template <bool MIXED, bool T1, bool EV, bool STEP, int V = 1>
void launch_full(const ForceArgs &a, unsigned nblk, hipStream_t st) {
  if (a.n <= kSmallGridAtoms)
    k_force_full<MIXED, T1, EV, kSmallTeamUnroll, true, STEP, false, kSmallTeam, V>
        <<<nblk, kForceThreads * kSmallTeam, 0, st>>>(a);
  else if (V != 1 || a.n <= kNarrowAtoms)
    k_force_full<MIXED, T1, EV, kTeamUnroll, true, STEP, false, kTeam, V>
        <<<nblk, kForceThreads * kTeam, 0, st>>>(a);
  else if constexpr (V == 1)
    k_force_full<MIXED, T1, EV, kTeamUnroll, true, STEP, true, kTeam>
        <<<nblk, kForceThreads * kTeam, 0, st>>>(a);
}

template <bool MIXED, bool T1, bool EV>
void launch_one(const ForceArgs &a, int kind, unsigned nblk, hipStream_t st) {
  if (kind == LJMD_HALF) {
    if (a.e_atom)
      launch_half<MIXED, T1, EV, true>(a, st);
    else
      launch_half<MIXED, T1, EV, false>(a, st);
  } else {
    launch_full<MIXED, T1, EV, false>(a, nblk, st);
  }
}

template <bool MIXED>
void launch_prec(const ForceArgs &a, int kind, bool ev, unsigned nblk, hipStream_t st) {
  const bool t1 = a.ntypes == 1;
  if (t1 && ev) launch_one<MIXED, true, true>(a, kind, nblk, st);
  else if (t1) launch_one<MIXED, true, false>(a, kind, nblk, st);
  else if (ev) launch_one<MIXED, false, true>(a, kind, nblk, st);
  else launch_one<MIXED, false, false>(a, kind, nblk, st);
}

}  // namespace

unsigned force_blocks(int64_t n) {
  const int64_t b = (n + kForceThreads - 1) / kForceThreads;
  return (unsigned)(b > 0 ? b : 1);
}

size_t force_workspace(int64_t n) { return (size_t)force_blocks(n) * kEvStride * sizeof(double); }

// Atoms whose partial rows share one row of the force workspace (one block's).
int64_t force_workspace_atoms() { return kForceThreads; }

int launch_forces(const BoxK &b, int precision, int kind, double rc, int32_t ntypes,
                  const double *eps, const double *sig, int64_t n, const double *x,
                  const int32_t *type, const int32_t *nbr, const int32_t *nnbr, int32_t maxn,
                  double *F, double *e_atom, double *ev, void *ws, hipStream_t st) {
  ForceArgs a{};
  a.b = b;
  a.rc = rc;
  a.rc2 = rc * rc;
  a.ntypes = ntypes;
  a.eps = eps;
  a.sig = sig;
  a.n = (int32_t)n;
  a.x = x;
  a.type = type;
  a.nbr = nbr;
  a.nnbr = nnbr;
  a.maxn = maxn;
  a.F = F;
  a.e_atom = e_atom;
  a.partial = (double *)ws;
  const unsigned nblk = force_blocks(n);
  const bool want_ev = ev != nullptr || e_atom != nullptr;
  if (kind == LJMD_HALF) {
    k_zero2_f64<<<(unsigned)((3 * n + 255) / 256 + 1), 256, 0, st>>>(F, 3 * n, e_atom, n);
  }
  if (n > 0) {
    if (precision == LJMD_MIXED)
      launch_prec<true>(a, kind, want_ev, nblk, st);
    else
      launch_prec<false>(a, kind, want_ev, nblk, st);
  } else if (ev) {
    k_zero_f64<<<1, 256, 0, st>>>(a.partial, kEvStride);
  }
  const unsigned rows = n == 0 ? 1 : (kind == LJMD_HALF ? half_blocks(n) : nblk);
  if (ev) k_colsum<1024><<<1, 1024, 0, st>>>(rows, kEvStride, 7, a.partial, ev, 1.0, 0);
  return check_launch("ljmd_compute_forces");
}

// CSR forces: blocks of kCsrThreads / team atoms.
unsigned csr_force_blocks(int64_t n, int team) {
  const int64_t apb = kCsrThreads / team;
  const int64_t b = (n + apb - 1) / apb;
  return (unsigned)(b > 0 ? b : 1);
}

size_t csr_force_workspace(int64_t n) {
  return (size_t)csr_force_blocks(n, LJMD_MAX_TEAM) * kEvStride * sizeof(double);
}

namespace {
template <bool MIXED, bool T1, bool EV, int TEAM>
void launch_csr_team(const ForceArgs &a, const int64_t *off, const int32_t *csr, hipStream_t st) {
  constexpr int U = TEAM == 1 ? kUnroll : 4;
  const unsigned nblk = csr_force_blocks(a.n, TEAM);
  if (a.n <= kNarrowAtoms)
    k_force_csr<MIXED, T1, EV, TEAM, U, false><<<nblk, kCsrThreads, 0, st>>>(a, off, csr);
  else
    k_force_csr<MIXED, T1, EV, TEAM, U, true><<<nblk, kCsrThreads, 0, st>>>(a, off, csr);
}

template <bool MIXED, bool T1, bool EV>
void launch_csr_kind(const ForceArgs &a, int team, const int64_t *off, const int32_t *csr,
                     hipStream_t st) {
  switch (team) {
    case 1: launch_csr_team<MIXED, T1, EV, 1>(a, off, csr, st); break;
    case 2: launch_csr_team<MIXED, T1, EV, 2>(a, off, csr, st); break;
    case 4: launch_csr_team<MIXED, T1, EV, 4>(a, off, csr, st); break;
    case 8: launch_csr_team<MIXED, T1, EV, 8>(a, off, csr, st); break;
    default: launch_csr_team<MIXED, T1, EV, 16>(a, off, csr, st); break;
  }
}

template <bool MIXED>
void launch_csr_prec(const ForceArgs &a, int team, bool ev, const int64_t *off,
                     const int32_t *csr, hipStream_t st) {
  const bool t1 = a.ntypes == 1;
  if (t1 && ev) launch_csr_kind<MIXED, true, true>(a, team, off, csr, st);
  else if (t1) launch_csr_kind<MIXED, true, false>(a, team, off, csr, st);
  else if (ev) launch_csr_kind<MIXED, false, true>(a, team, off, csr, st);
  else launch_csr_kind<MIXED, false, false>(a, team, off, csr, st);
}
}  // namespace

int launch_forces_csr(const BoxK &b, int precision, double rc, int32_t ntypes, const double *eps,
                      const double *sig, int64_t n, const double *x, const int32_t *type,
                      const int64_t *offsets, const int32_t *csr, int team, double *F,
                      double *e_atom, double *ev, void *ws, hipStream_t st) {
  ForceArgs a{};
  a.b = b;
  a.rc = rc;
  a.rc2 = rc * rc;
  a.ntypes = ntypes;
  a.eps = eps;
  a.sig = sig;
  a.n = (int32_t)n;
  a.x = x;
  a.type = type;
  a.F = F;
  a.e_atom = e_atom;
  a.partial = (double *)ws;
  const bool want_ev = ev != nullptr || e_atom != nullptr;
  const unsigned nblk = csr_force_blocks(n, team);
  if (n > 0) {
    if (precision == LJMD_MIXED)
      launch_csr_prec<true>(a, team, want_ev, offsets, csr, st);
    else
      launch_csr_prec<false>(a, team, want_ev, offsets, csr, st);
  } else if (ev) {
    k_zero_f64<<<1, 256, 0, st>>>(a.partial, kEvStride);
  }
  if (ev)
    k_colsum<1024><<<1, 1024, 0, st>>>(n > 0 ? nblk : 1, kEvStride, 7, a.partial, ev, 1.0, 0);
  return check_launch("ljmd_compute_forces_csr");
}

namespace {
template <bool MIXED, bool T1, bool EV, int V>
void launch_aosoa_one(const ForceArgs &a, unsigned nblk, hipStream_t st) {
  launch_full<MIXED, T1, EV, false, V>(a, nblk, st);
}

template <bool MIXED, int V>
void launch_aosoa_v(const ForceArgs &a, bool ev, unsigned nblk, hipStream_t st) {
  const bool t1 = a.ntypes == 1;
  if (t1 && ev) launch_aosoa_one<MIXED, true, true, V>(a, nblk, st);
  else if (t1) launch_aosoa_one<MIXED, true, false, V>(a, nblk, st);
  else if (ev) launch_aosoa_one<MIXED, false, true, V>(a, nblk, st);
  else launch_aosoa_one<MIXED, false, false, V>(a, nblk, st);
}

template <bool MIXED>
void launch_aosoa_prec(const ForceArgs &a, int vlen, bool ev, unsigned nblk, hipStream_t st) {
  if (vlen == 0) launch_aosoa_v<MIXED, 0>(a, ev, nblk, st);
  else if (vlen == 8) launch_aosoa_v<MIXED, 8>(a, ev, nblk, st);
  else launch_aosoa_v<MIXED, 64>(a, ev, nblk, st);
}

// One thread per element: [n][3] <-> AoSoA(V).
template <int V, bool TO_AOSOA>
__global__ __launch_bounds__(256) void k_aosoa_convert(int64_t n, const double *__restrict__ src,
                                                        double *__restrict__ dst) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= 3 * n) return;
  const int64_t i = q / 3;
  const int k = (int)(q - 3 * i);
  if constexpr (TO_AOSOA)
    dst[aos_index<V>(i, k, n)] = src[q];
  else
    dst[q] = src[aos_index<V>(i, k, n)];
}

template <int V>
void launch_convert_v(int64_t n, int to_aosoa, const double *src, double *dst, hipStream_t st) {
  const unsigned nb = (unsigned)((3 * n + 255) / 256);
  if (to_aosoa)
    k_aosoa_convert<V, true><<<nb, 256, 0, st>>>(n, src, dst);
  else
    k_aosoa_convert<V, false><<<nb, 256, 0, st>>>(n, src, dst);
}
}  // namespace

// Full-list forces over AoSoA(vlen) positions and forces (vlen 0: SoA; 1: the
// [n][3] arrays of launch_forces; 8 or 64).  Same traversal and summation order
// as the full-list kernel, so the same bits in any layout.
int launch_forces_aosoa(const BoxK &b, int precision, double rc, int32_t ntypes, const double *eps,
                        const double *sig, int64_t n, int vlen, const double *x,
                        const int32_t *type, const int32_t *nbr, const int32_t *nnbr,
                        int32_t maxn, double *F, double *e_atom, double *ev, void *ws,
                        hipStream_t st) {
  if (vlen == 1)
    return launch_forces(b, precision, LJMD_FULL, rc, ntypes, eps, sig, n, x, type, nbr, nnbr,
                         maxn, F, e_atom, ev, ws, st);
  ForceArgs a{};
  a.b = b;
  a.rc = rc;
  a.rc2 = rc * rc;
  a.ntypes = ntypes;
  a.eps = eps;
  a.sig = sig;
  a.n = (int32_t)n;
  a.x = x;
  a.type = type;
  a.nbr = nbr;
  a.nnbr = nnbr;
  a.maxn = maxn;
  a.F = F;
  a.e_atom = e_atom;
  a.partial = (double *)ws;
  const unsigned nblk = force_blocks(n);
  const bool want_ev = ev != nullptr || e_atom != nullptr;
  if (n > 0) {
    if (precision == LJMD_MIXED)
      launch_aosoa_prec<true>(a, vlen, want_ev, nblk, st);
    else
      launch_aosoa_prec<false>(a, vlen, want_ev, nblk, st);
  } else if (ev) {
    k_zero_f64<<<1, 256, 0, st>>>(a.partial, kEvStride);
  }
  if (ev)
    k_colsum<1024><<<1, 1024, 0, st>>>(n > 0 ? nblk : 1, kEvStride, 7, a.partial, ev, 1.0, 0);
  return check_launch("ljmd_compute_forces_aosoa");
}

int launch_aosoa_convert(int64_t n, int vlen, int to_aosoa, const double *src, double *dst,
                         hipStream_t st) {
  if (n > 0) {
    if (vlen == 0) launch_convert_v<0>(n, to_aosoa, src, dst, st);
    else if (vlen == 1) launch_convert_v<1>(n, to_aosoa, src, dst, st);
    else if (vlen == 8) launch_convert_v<8>(n, to_aosoa, src, dst, st);
    else launch_convert_v<64>(n, to_aosoa, src, dst, st);
  }
  return check_launch("ljmd_aosoa_convert");
}

// partial: this step's partial rows; ev: their sums, or NULL to leave them in
// `partial`; prev_partial/prev_ev: the rows a previous step left and the output of
// their sums (NULL: none).
int launch_md_step(const BoxK &b, int precision, double rc, int32_t ntypes, const double *eps,
                   const double *sig, int64_t n, const double *x, const int32_t *type,
                   const int32_t *nbr, const int32_t *nnbr, int32_t maxn, double dt, double mass,
                   double *v, double *x_next, int open_next, double *F, double *e_atom, double *ev,
                   double *partial, const double *prev_partial, double *prev_ev, hipStream_t st) {
  ForceArgs a{};
  a.b = b;
  a.rc = rc;
  a.rc2 = rc * rc;
  a.ntypes = ntypes;
  a.eps = eps;
  a.sig = sig;
  a.n = (int32_t)n;
  a.x = x;
  a.type = type;
  a.nbr = nbr;
  a.nnbr = nnbr;
  a.maxn = maxn;
  a.F = F;
  a.e_atom = e_atom;
  a.partial = partial;
  a.v = v;
  a.x_next = x_next;
  a.dt = dt;
  a.hdt = 0.5 * dt;
  a.mass = mass;
  a.unit_mass = mass == 1.0;
  a.open_next = open_next;
  const unsigned nblk = force_blocks(n);
  a.prev_partial = prev_partial;
  a.prev_ev = prev_ev;
  a.prev_rows = nblk;
  const bool mixed = precision == LJMD_MIXED;
  const bool t1 = ntypes == 1;
  if (n > 0) {
    if (mixed) {
      if (t1) launch_full<true, true, true, true>(a, nblk, st);
      else launch_full<true, false, true, true>(a, nblk, st);
    } else {
      if (t1) launch_full<false, true, true, true>(a, nblk, st);
      else launch_full<false, false, true, true>(a, nblk, st);
    }
  } else {
    k_zero_f64<<<1, 256, 0, st>>>(a.partial, kEvStride);
    if (prev_ev) k_colsum<1024><<<1, 1024, 0, st>>>(1, kEvStride, 8, prev_partial, prev_ev, 1.0, 0);
  }
  if (ev) k_colsum<1024><<<1, 1024, 0, st>>>(nblk, kEvStride, 8, a.partial, ev, 1.0, 0);
  return check_launch("ljmd_md_step");
}

// The sums of the partial rows one md_step launch left (same form as its own).
int launch_md_step_sums(int64_t n, const double *partial, double *ev, hipStream_t st) {
  k_colsum<1024><<<1, 1024, 0, st>>>(force_blocks(n), kEvStride, 8, partial, ev, 1.0, 0);
  return check_launch("ljmd_md_step_sums");
}

}  // namespace ljmd
