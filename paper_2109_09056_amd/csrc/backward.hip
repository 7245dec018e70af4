// Adjoint (vector-Jacobian product) of the Lennard-Jones forces over the FULL
// tiled-ELL list, gfx950.
//
// With F_i = sum_j s(r^2_ij) d_ij, a cotangent g on the forces and the pair
// set held fixed:
//   dL/dx_i = sum_j K_ij (g_i - g_j),   K_ij = s I + 2 s' d d^T,  s' = ds/d(r^2)
//   dL/dp   = sum_i sum_j g_i . d_ij ds_ij/dp      (p = eps or sigma of the type pair)
// Expanding s = ri2 sr6 (48 eps sr6 - 24 eps) with t = ri2 sr6 = sigma^6 r^-8:
//   s'       = t ri2 (-336 eps sr6 + 96 eps)
//   ds/deps  = t (48 sr6 - 24)
//   ds/dsig  = t (576 eps/sigma sr6 - 144 eps/sigma)
// K_ij is symmetric in (i, j), so the position gradient is a gather over the
// row of atom i -- one lane per atom, no atomics.  Parameter gradients are
// accumulated per lane by the neighbor's type, reduced per block by the
// lane's own type in a fixed order, and summed over blocks by one column-sum
// launch: the whole adjoint is bitwise reproducible.
#include <type_traits>

#include "common.h"

namespace ljmd {

namespace {

constexpr int kThreads = 128;  // atoms per block
constexpr int kWaves = kThreads / kWave;
constexpr int kTeam = 2;       // lanes per atom for one or two types
// Up to this many atoms (at most 512 blocks, two per compute unit at kTeam
// lanes) one or two types take four lanes per atom: more waves in flight for a
// grid that would leave the chip half idle (32k atoms: 26.6 -> 22.1 us; at
// 256k atoms the four-lane form is 5 % slower).
constexpr int64_t kSmallVjp = 65536;

struct BwdArgs {
  BoxK b;
  double rc, rc2;
  int32_t ntypes;
  const double *eps;
  const double *sig;
  int32_t n;
  const double *x;
  const int32_t *type;
  const int32_t *nbr;
  const int32_t *nnbr;
  int32_t maxn;
  const double *g;
  double *gx;
  int accumulate;
  int stride;       // partial row length: 2 T T rounded up to a power of two
  double *partial;  // [nblk][stride]: (eps | sigma) x (type of i) x (type of j), then padding
};

// sigma^2, 48 eps, 24 eps, -336 eps, 96 eps, 576 eps/sigma, 144 eps/sigma
struct BCoef {
  double sig2, c12, c6, d12, d6, q12, q6;
};

__device__ __forceinline__ BCoef bcoef(const double *eps, const double *sig, int p) {
  const double e = eps[p], s = sig[p];
  return BCoef{s * s, 48.0 * e, 24.0 * e, -336.0 * e, 96.0 * e, 576.0 * e / s, 144.0 * e / s};
}

struct PairB {
  double s, sp, dse, dss;
};

template <bool MIXED>
__device__ __forceinline__ PairB pair_b(double r2, const BCoef &c) {
  PairB o;
  if constexpr (MIXED) {
    const float ri2 = recip32((float)r2);
    const float sr2 = (float)c.sig2 * ri2;
    const float sr6 = sr2 * sr2 * sr2;
    const float t = ri2 * sr6;
    o.s = (double)(t * __builtin_fmaf((float)c.c12, sr6, -(float)c.c6));
    o.sp = (double)(t * ri2 * __builtin_fmaf((float)c.d12, sr6, (float)c.d6));
    o.dse = (double)(t * __builtin_fmaf(48.0f, sr6, -24.0f));
    o.dss = (double)(t * __builtin_fmaf((float)c.q12, sr6, -(float)c.q6));
  } else {
    const double ri2 = recip64(r2);
    const double sr2 = c.sig2 * ri2;
    const double sr6 = sr2 * sr2 * sr2;
    const double t = ri2 * sr6;
    o.s = t * __builtin_fma(c.c12, sr6, -c.c6);
    o.sp = t * ri2 * __builtin_fma(c.d12, sr6, c.d6);
    o.dse = t * __builtin_fma(48.0, sr6, -24.0);
    o.dss = t * __builtin_fma(c.q12, sr6, -c.q6);
  }
  return o;
}

// TT: 1 or 2 types with register accumulators; 0: any T <= LJMD_MAX_TYPES with
// lane-private LDS columns.  TEAM lanes per atom (TEAM > 1 only with TT > 0):
// lane t of the team walks the row entries t, t + TEAM, ... (neighbouring
// entries are mostly nearby atoms, so a gather instruction touches fewer
// cache lines); gx is combined by a butterfly over the team (every lane ends
// with the same, order-fixed sum) and the parameter-gradient partials enter
// the block sums per lane.  A block always covers kThreads atoms.
template <bool MIXED, int TT, bool WIDE, int TEAM>
__global__ __launch_bounds__(kThreads * TEAM) void k_vjp(BwdArgs a) {
  static_assert(TEAM == 1 || TT != 0, "lane-private LDS columns are sized for one lane per atom");
  constexpr int MT = LJMD_MAX_TYPES;
  constexpr int NW = kWaves * TEAM;  // wavefronts per block
  __shared__ double tab[(TT == 1 ? 1 : MT * MT) * 7];
  __shared__ double red[NW * (TT == 0 ? 1 : 2 * TT * TT)];
  __shared__ double acc[TT == 0 ? kThreads * 2 * MT : 1];
  __shared__ int32_t tid_type[TT == 0 ? kThreads : 1];
  const int T = TT == 0 ? a.ntypes : TT;
  if constexpr (TT != 1) {
    for (int q = threadIdx.x; q < T * T; q += kThreads * TEAM) {
      const BCoef c = bcoef(a.eps, a.sig, packed_index(q / T, q % T, T));
      double *t = tab + 7 * q;
      t[0] = c.sig2; t[1] = c.c12; t[2] = c.c6; t[3] = c.d12; t[4] = c.d6; t[5] = c.q12; t[6] = c.q6;
    }
  }
  if constexpr (TT == 0) {
    for (int q = 0; q < 2 * MT; ++q) acc[threadIdx.x * 2 * MT + q] = 0.0;
  }
  if constexpr (TT != 1) __syncthreads();
  BCoef c1{};
  if constexpr (TT == 1) c1 = bcoef(a.eps, a.sig, 0);

  const int tm = (int)threadIdx.x % TEAM;
  const int32_t i = xcd_block(blockIdx.x, gridDim.x) * kThreads + (int)threadIdx.x / TEAM;
  double ge[TT == 0 ? 1 : TT], gs[TT == 0 ? 1 : TT];
#pragma unroll
  for (int q = 0; q < (TT == 0 ? 1 : TT); ++q) ge[q] = gs[q] = 0.0;
  int ti = 0;
  const bool live = i < a.n;
  double xi = 0.0, yi = 0.0, zi = 0.0;
  if (live) {
    xi = a.x[3 * (int64_t)i];
    yi = a.x[3 * (int64_t)i + 1];
    zi = a.x[3 * (int64_t)i + 2];
  }
  // wavefront-uniform: every atom of the wavefront at least rc from all faces
  // (then the raw displacement is the minimum image for every pair inside rc)
  const bool in = !live || (xi >= a.rc && xi <= a.b.L[0] - a.rc && yi >= a.rc &&
                            yi <= a.b.L[1] - a.rc && zi >= a.rc && zi <= a.b.L[2] - a.rc);
  const bool interior = __ballot(!in) == 0;
  if (live) {
    const double gxi = a.g[3 * (int64_t)i], gyi = a.g[3 * (int64_t)i + 1],
                 gzi = a.g[3 * (int64_t)i + 2];
    ti = TT == 1 ? 0 : a.type[i];
    const int32_t ctot = a.nnbr[i];
    const int32_t cnt = ctot > tm ? (ctot - tm + TEAM - 1) / TEAM : 0;
    const int32_t *row =
        a.nbr + (int64_t)(i >> 6) * a.maxn * kWave + (i & (kWave - 1)) + (int64_t)tm * kWave;
    double ax = 0.0, ay = 0.0, az = 0.0;
    // one list entry: j with its position and cotangent
    auto entry = [&](auto wrap, int32_t j, const double *xj, const double *gj, bool valid) {
      double dx = xi - xj[0], dy = yi - xj[1], dz = zi - xj[2];
      if constexpr (decltype(wrap)::value) {
        dx = min_image(dx, a.b.L[0], a.b.invL[0]);
        dy = min_image(dy, a.b.L[1], a.b.invL[1]);
        dz = min_image(dz, a.b.L[2], a.b.invL[2]);
      }
      const double r2 = dist2(dx, dy, dz);
      if (valid && r2 < a.rc2) {
        int tj = 0;
        BCoef c;
        if constexpr (TT == 1) {
          c = c1;
        } else {
          tj = a.type[j];
          const double *t = tab + 7 * (ti * T + tj);
          c = BCoef{t[0], t[1], t[2], t[3], t[4], t[5], t[6]};
        }
        const PairB p = pair_b<MIXED>(r2, c);
        const double dgx = gxi - gj[0];
        const double dgy = gyi - gj[1];
        const double dgz = gzi - gj[2];
        const double ddg = __builtin_fma(dx, dgx, __builtin_fma(dy, dgy, dz * dgz));
        const double q = 2.0 * p.sp * ddg;
        ax = __builtin_fma(p.s, dgx, __builtin_fma(q, dx, ax));
        ay = __builtin_fma(p.s, dgy, __builtin_fma(q, dy, ay));
        az = __builtin_fma(p.s, dgz, __builtin_fma(q, dz, az));
        const double gid = __builtin_fma(gxi, dx, __builtin_fma(gyi, dy, gzi * dz));
        if constexpr (TT == 1) {
          ge[0] = __builtin_fma(gid, p.dse, ge[0]);
          gs[0] = __builtin_fma(gid, p.dss, gs[0]);
        } else if constexpr (TT == 2) {
          const double ve = gid * p.dse, vs = gid * p.dss;
          if (tj == 0) {
            ge[0] += ve;
            gs[0] += vs;
          } else {
            ge[1] += ve;
            gs[1] += vs;
          }
        } else {
          double *col = acc + threadIdx.x * 2 * MT;
          col[tj] = __builtin_fma(gid, p.dse, col[tj]);
          col[MT + tj] = __builtin_fma(gid, p.dss, col[MT + tj]);
        }
      }
    };
    // Groups of U slots: the U index loads, then the gathers of x_j and g_j, then
    // the U entries.  Whole groups read indices at fixed offsets from one row
    // pointer; the last, partial group gathers only slots below cnt.  Row order
    // throughout, so the sums match one slot at a time.
    auto walk = [&](auto wrap) {
      // 3 slots per group: 99 VGPRs against 112-118 with 4, and at 256,000 atoms
      // (two types) 96.2 -> 92.4 us mixed, 95.3 -> 92.1 us FP64; 2 slots or
      // occupancy hints (5-6 waves per SIMD) gained nothing or spilled.
      constexpr int U = 3;
      const int32_t whole = cnt - cnt % U;
      const int32_t *rp = row;
      int32_t k = 0;
      constexpr int kStep = TEAM * kWave;  // ints between this lane's consecutive entries
      for (; k < whole; k += U, rp += U * kStep) {
        int32_t jj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) jj[u] = rp[u * kStep];
        double xj[U][3], gj[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const double *px = pos_of<WIDE>(a.x, jj[u]);
          const double *pg = pos_of<WIDE>(a.g, jj[u]);
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            xj[u][q] = px[q];
            gj[u][q] = pg[q];
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) entry(wrap, jj[u], xj[u], gj[u], true);
      }
      if (k < cnt) {
        int32_t jj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) jj[u] = rp[(k + u < cnt ? u : 0) * kStep];
        double xj[U][3], gj[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
          for (int q = 0; q < 3; ++q) xj[u][q] = gj[u][q] = 0.0;
          if (k + u < cnt) {
            const double *px = pos_of<WIDE>(a.x, jj[u]);
            const double *pg = pos_of<WIDE>(a.g, jj[u]);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              xj[u][q] = px[q];
              gj[u][q] = pg[q];
            }
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) entry(wrap, jj[u], xj[u], gj[u], k + u < cnt);
      }
    };
    if (interior)
      walk(std::false_type{});
    else
      walk(std::true_type{});
    if constexpr (TEAM > 1) {
#pragma unroll
      for (int mask = TEAM / 2; mask > 0; mask >>= 1) {
        ax += __shfl_xor(ax, mask, kWave);
        ay += __shfl_xor(ay, mask, kWave);
        az += __shfl_xor(az, mask, kWave);
      }
    }
    double *o = a.gx + 3 * (int64_t)i;
    if (tm != 0) {
      // the team's lead lane writes gx
    } else if (a.accumulate) {
      o[0] += ax;
      o[1] += ay;
      o[2] += az;
    } else {
      o[0] = ax;
      o[1] = ay;
      o[2] = az;
    }
  }
  // per-block sums G[which][ti][tj] in a fixed order
  double *out = a.partial + (int64_t)blockIdx.x * a.stride;
  if constexpr (TT == 1) {
    const double v[2] = {ge[0], gs[0]};
    block_sum<NW, 2>(v, red, out);
  } else if constexpr (TT == 2) {
    // layout: [which][a][b] -> which*4 + a*2 + b
    double v[8];
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
      for (int aa = 0; aa < 2; ++aa)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
          v[w * 4 + aa * 2 + bb] = (ti == aa) ? (w == 0 ? ge[bb] : gs[bb]) : 0.0;
    block_sum<NW, 8>(v, red, out);
  } else {
    tid_type[threadIdx.x] = (i < a.n) ? ti : -1;
    __syncthreads();
    for (int q = threadIdx.x; q < 2 * T * T; q += kThreads) {
      const int w = q / (T * T), aa = (q / T) % T, bb = q % T;
      double s = 0.0;
      for (int l = 0; l < kThreads; ++l)
        if (tid_type[l] == aa) s += acc[l * 2 * MT + w * MT + bb];
      out[q] = s;
    }
  }
}

// The parameter gradients from the VJP's partial rows, in one launch: the
// column sums G[w][a][b] (w = 0: eps, 1: sigma) of the rows, then
// geps[p] (+)= G[0][a][b] + G[0][b][a] (a != b) or G[0][a][a]; gsig likewise.
template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_param_grad(int64_t rows, int stride, int32_t T,
                                                       const double *__restrict__ partial,
                                                       double *__restrict__ geps,
                                                       double *__restrict__ gsig,
                                                       int accumulate) {
  __shared__ double part[THREADS];
  colsum_lds<THREADS>(rows, stride, partial, part);
  const int P = T * (T + 1) / 2;
  const int q = threadIdx.x;
  if (q >= 2 * P) return;
  const int w = q / P, p = q % P;
  int aa = 0, rem = p;
  while (rem >= T - aa) {
    rem -= T - aa;
    ++aa;
  }
  const int bb = aa + rem;
  double v = part[w * T * T + aa * T + bb];
  if (aa != bb) v += part[w * T * T + bb * T + aa];
  double *o = w == 0 ? geps : gsig;
  o[p] = accumulate ? o[p] + v : v;
}

}  // namespace

unsigned bwd_blocks(int64_t n) {
  const int64_t b = (n + kThreads - 1) / kThreads;
  return (unsigned)(b > 0 ? b : 1);
}

static int partial_stride(int32_t ntypes) {
  int s = 1;
  while (s < 2 * ntypes * ntypes) s <<= 1;
  return s;
}

size_t bwd_workspace(int64_t n, int32_t ntypes) {
  return (size_t)bwd_blocks(n) * partial_stride(ntypes) * sizeof(double);
}

int launch_backward(const BoxK &b, int precision, double rc, int32_t ntypes, const double *eps,
                    const double *sig, int64_t n, const double *x, const int32_t *type,
                    const int32_t *nbr, const int32_t *nnbr, int32_t maxn, const double *g,
                    double *gx, double *geps, double *gsig, int accumulate, void *ws,
                    hipStream_t st) {
  BwdArgs a;
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
  a.g = g;
  a.gx = gx;
  a.accumulate = accumulate;
  a.stride = partial_stride(ntypes);
  a.partial = (double *)ws;
  const unsigned nblk = bwd_blocks(n);
  const int stride = a.stride;
  const bool mixed = precision == LJMD_MIXED;
#define LJMD_VJP(M, TT, TEAM)                                                \
  do {                                                                       \
    if (n <= kNarrowAtoms)                                                   \
      k_vjp<M, TT, false, TEAM><<<nblk, kThreads * TEAM, 0, st>>>(a);       \
    else                                                                     \
      k_vjp<M, TT, true, TEAM><<<nblk, kThreads * TEAM, 0, st>>>(a);        \
  } while (0)
  const bool small = n <= kSmallVjp;
  if (ntypes == 1) {
    if (small) {
      if (mixed) LJMD_VJP(true, 1, 4); else LJMD_VJP(false, 1, 4);
    } else {
      if (mixed) LJMD_VJP(true, 1, kTeam); else LJMD_VJP(false, 1, kTeam);
    }
  } else if (ntypes == 2) {
    if (small) {
      if (mixed) LJMD_VJP(true, 2, 4); else LJMD_VJP(false, 2, 4);
    } else {
      if (mixed) LJMD_VJP(true, 2, kTeam); else LJMD_VJP(false, 2, kTeam);
    }
  } else {
    if (mixed) LJMD_VJP(true, 0, 1); else LJMD_VJP(false, 0, 1);
  }
#undef LJMD_VJP
  k_param_grad<1024><<<1, 1024, 0, st>>>(nblk, stride, ntypes, a.partial, geps, gsig, accumulate);
  return check_launch("ljmd_force_backward");
}

}  // namespace ljmd
