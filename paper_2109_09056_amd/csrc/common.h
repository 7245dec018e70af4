// Internal helpers shared by the gfx950 kernels of libljmd (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ljmd.h"

namespace ljmd {

constexpr int kWave = 64;

// Box constants handed to kernels by value.
struct BoxK {
  double L[3];
  double invL[3];
};

// Binning grid: nc cells per dimension, edge h = L/nc.
struct GridK {
  int32_t nc[3];
  double h[3];
  int32_t ncells;
};

// Representative of d modulo L nearest zero.  For |d| < L this equals the
// single shift "d > L/2: d - L; d < -L/2: d + L" bit for bit except when
// |d| is within rounding of L/2, where both representatives lie at ~L/2,
// beyond any list cutoff the ABI accepts.
__device__ __forceinline__ double min_image(double d, double L, double invL) {
  double k = __builtin_rint(d * invL);
  return __builtin_fma(-k, L, d);
}

// Atom j's 3-vector in an [n][3] FP64 array.  Narrow form (every index below
// kNarrowAtoms): a 32-bit byte offset from the array base, formed with the
// full-rate 24-bit multiply; wide form: 64-bit index arithmetic.
constexpr int64_t kNarrowAtoms = int64_t(1) << 24;
template <bool WIDE>
__device__ __forceinline__ const double *pos_of(const double *x, int32_t j) {
  if constexpr (WIDE)
    return x + 3 * (int64_t)j;
  else
    return (const double *)((const char *)x + __umul24((uint32_t)j, 24u));
}

// r^2 in the fixed order (dx*dx + dy*dy) + dz*dz; the library is compiled
// with -ffp-contract=off so no FMA is formed here.
__device__ __forceinline__ double dist2(double dx, double dy, double dz) {
  return (dx * dx + dy * dy) + dz * dz;
}

// Reciprocal by the hardware estimate refined with Newton-Raphson steps
// y <- y + y (1 - a y), each of which squares the relative error.
__device__ __forceinline__ double recip64(double a) {
  double y = __builtin_amdgcn_rcp(a);
  double e = __builtin_fma(-a, y, 1.0);
  y = __builtin_fma(y, e, y);
  e = __builtin_fma(-a, y, 1.0);
  return __builtin_fma(y, e, y);
}

// a^(-1/2) by the hardware estimate refined with Newton-Raphson steps
// y <- y (3/2 - (a/2) y^2), each of which squares the relative error.
__device__ __forceinline__ double rsqrt64(double a) {
  const double h = 0.5 * a;
  double y = __builtin_amdgcn_rsq(a);
  y = __builtin_fma(y, __builtin_fma(-h * y, y, 0.5), y);
  return __builtin_fma(y, __builtin_fma(-h * y, y, 0.5), y);
}

__device__ __forceinline__ float recip32(float a) {
  float y = __builtin_amdgcn_rcpf(a);
  float e = __builtin_fmaf(-a, y, 1.0f);
  return __builtin_fmaf(y, e, y);
}

// Value of v in lane `src` (wavefront-uniform src), through two scalar readlanes.
__device__ __forceinline__ double readlane_f64(double v, int src) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), src);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    int o = __shfl_xor(v, off, kWave);
    v = o > v ? o : v;
  }
  return v;
}

// Block of `NW` waves: sums NV values per thread into out[0..NV) for the
// block, in a fixed order (wave tree, then waves 0..NW-1).  Every thread of
// the block must call it.  `red` is __shared__ storage of NW*NV doubles.
template <int NW, int NV>
__device__ __forceinline__ void block_sum(const double (&v)[NV], double *red, double *out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = wave_sum(v[q]);
    if (lane == 0) red[w * NV + q] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NW; ++k) s += red[k * NV + threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// Column sums over `rows` partial rows of `stride` doubles (stride a power of
// two dividing THREADS) by one block of THREADS threads, left in LDS:
// part[q] = sum_r p[r*stride + q] for q < stride.  Thread t reads the flat
// array at t, t + THREADS, ... (coalesced), so it always sees column
// t % stride; the THREADS/stride threads of a column are then added by a tree
// in `part` (THREADS doubles of LDS).  Fixed order throughout; every thread of
// the block calls it and part[0..stride) is visible to all of them on return.
template <int THREADS>
__device__ __forceinline__ void colsum_lds(int64_t rows, int stride, const double *__restrict__ p,
                                           double *part) {
  const int t = threadIdx.x;
  double s = 0.0;
  const int64_t total = rows * stride;
  constexpr int B = 16;  // loads in flight per thread
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
  part[t] = s;
  __syncthreads();
  for (int off = THREADS / 2; off >= stride; off >>= 1) {
    if (t < off) part[t] += part[t + off];
    __syncthreads();
  }
}

// One launch of colsum_lds: out[q] = scale * column q for q < ncols (+= when
// accumulate).
template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_colsum(int64_t rows, int stride, int ncols,
                                                   const double *__restrict__ p,
                                                   double *__restrict__ out, double scale,
                                                   int accumulate) {
  __shared__ double part[THREADS];
  colsum_lds<THREADS>(rows, stride, p, part);
  const int t = threadIdx.x;
  if (t < ncols) out[t] = accumulate ? out[t] + scale * part[t] : scale * part[t];
}

// Workgroups are handed to the 8 XCDs round-robin (block b runs on XCD b % 8),
// and each XCD has its own L2.  Renumbering so that XCD x gets one contiguous
// run of logical blocks keeps spatially adjacent tiles -- and the neighbor
// positions they gather -- inside one L2.  A bijection on [0, nblk).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int nblk) {
  const int q = nblk / kXcds, r = nblk % kXcds;
  const int x = b % kXcds, k = b / kXcds;
  return x * q + (x < r ? x : r) + k;
}

// Packed upper-triangle index of the type pair (a, b).
__host__ __device__ __forceinline__ int packed_index(int a, int b, int T) {
  if (a > b) {
    int t = a;
    a = b;
    b = t;
  }
  return a * T - a * (a - 1) / 2 + (b - a);
}

// ---- host side ----
int set_error(int code, const char *fmt, ...);
int check_launch(const char *what);
BoxK make_box(const ljmd_box *b);
int make_grid(const ljmd_box *b, double rlist, GridK *g);

}  // namespace ljmd
