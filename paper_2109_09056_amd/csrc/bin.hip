// Counting sort of atoms into binning cells (cell-major, ascending id inside a
// cell), gfx950.  Paper: Cabana "Particle Sorting" (geometric binning) and the
// re-sort that begins each MD timestep (Introduction).
//
// Four launches:
//   1. cell id + histogram   one thread per atom; lanes of a wavefront in the
//                            same cell share one atomic add and get ranks
//   2. exclusive scan        one 1024-thread block over all cells, in chunks
//                            (wavefront shuffle scans)
//   3. scatter               one thread per atom to slot start[cell] + rank
//   4. in-cell rank + permute  one wavefront per cell: ids of the cell are
//                            staged in LDS, each lane ranks its atom among
//                            them, then copies x, v, type, id to the ranked slot.
// The rank order of step 1 depends on atomic timing; step 4 replaces it by
// the id order, so the output permutation is deterministic.
#include "common.h"

namespace ljmd {

namespace {

constexpr int kScanThreads = 1024;
constexpr int kPermWaves = 4;
constexpr int kStage = 256;  // ids per wavefront staged in LDS

__device__ __forceinline__ int32_t cell_of(const double *xi, const GridK &g) {
  int32_t c[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int32_t ck = (int32_t)floor(xi[k] / g.h[k]);
    ck = ck > g.nc[k] - 1 ? g.nc[k] - 1 : ck;
    c[k] = ck < 0 ? 0 : ck;
  }
  return (c[2] * g.nc[1] + c[1]) * g.nc[0] + c[0];
}

__global__ void k_fill_i32(int32_t *p, int64_t m, int32_t val) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) p[i] = val;
}

// Cell of every atom and its rank among the atoms of its cell that were
// counted before it.  Lanes of a wavefront that fall in the same cell (the
// common case: the input is usually the previous sorted order) are grouped by
// a ballot loop, and each group's leader makes one atomic add for the group.
__global__ void k_count(int64_t n, const double *__restrict__ x, GridK g,
                        int32_t *__restrict__ cell, int32_t *__restrict__ rank,
                        int32_t *__restrict__ counts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < n;
  const int32_t c = live ? cell_of(x + 3 * i, g) : -1;
  const int lane = threadIdx.x & (kWave - 1);
  bool pending = live;
  int32_t r = 0;
  while (__ballot(pending) != 0) {
    const uint64_t act = __ballot(pending);
    const int leader = __builtin_ctzll(act);
    const int32_t lc = __shfl(c, leader, kWave);
    const bool mine = pending && c == lc;
    const uint64_t grp = __ballot(mine);
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(&counts[lc], (int32_t)__popcll(grp));
    base = __shfl(base, leader, kWave);
    if (mine) {
      r = base + (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(grp >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)grp, 0u));
      pending = false;
    }
  }
  if (live) {
    cell[i] = c;
    rank[i] = r;
  }
}

// Inclusive prefix sum of v over the lanes of the wavefront (shuffles only).
__device__ __forceinline__ int32_t wave_inclusive_scan(int32_t v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int32_t o = __shfl_up(v, off, kWave);
    if (lane >= off) v += o;
  }
  return v;
}

// Exclusive scan of counts[0..m) into start[0..m] (start[m] = total).  One
// block walks the cells in chunks of 4 * kScanThreads, kScanAhead chunks loaded
// at once (one load latency per group of chunks): in a chunk each thread holds
// four consecutive counts, the waves scan their threads' sums with shuffles,
// and the wave totals meet in LDS (two barriers per chunk); a running carry
// joins the chunks.
constexpr int kScanAhead = 8;

__global__ __launch_bounds__(kScanThreads) void k_scan(int32_t m, const int32_t *__restrict__ counts,
                                                     int32_t *__restrict__ start) {
  constexpr int kWaves = kScanThreads / kWave;
  constexpr int32_t kChunk = 4 * kScanThreads;
  __shared__ int32_t wsum[kWaves];
  const int t = threadIdx.x;
  const int lane = t & (kWave - 1), w = t / kWave;
  int32_t carry = 0;  // the same in every thread
  for (int32_t g0 = 0; g0 < m; g0 += kScanAhead * kChunk) {
    int32_t v[kScanAhead][4];
#pragma unroll
    for (int p = 0; p < kScanAhead; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int32_t c = g0 + p * kChunk + 4 * t + q;
        v[p][q] = c < m ? counts[c] : 0;
      }
#pragma unroll
    for (int p = 0; p < kScanAhead; ++p) {
      const int32_t c0 = g0 + p * kChunk;
      if (c0 >= m) break;  // block-uniform
      const int32_t s = v[p][0] + v[p][1] + v[p][2] + v[p][3];
      const int32_t inc = wave_inclusive_scan(s);
      if (lane == kWave - 1) wsum[w] = inc;
      __syncthreads();
      int32_t before = 0, total = 0;
#pragma unroll
      for (int k = 0; k < kWaves; ++k) {
        const int32_t ws = wsum[k];
        before += k < w ? ws : 0;
        total += ws;
      }
      int32_t run = carry + before + inc - s;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int32_t c = c0 + 4 * t + q;
        if (c < m) start[c] = run;
        run += v[p][q];
      }
      carry += total;
      __syncthreads();  // wsum is written again by the next chunk
    }
  }
  if (t == 0) start[m] = carry;
}

// Slot of atom i: start of its cell plus its rank (no atomics).
__global__ void k_scatter(int64_t n, const int32_t *__restrict__ cell,
                          const int32_t *__restrict__ rank, const int32_t *__restrict__ start,
                          int32_t *__restrict__ src) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  src[start[cell[i]] + rank[i]] = (int32_t)i;
}

__device__ __forceinline__ int64_t id_at(const int64_t *id_in, int32_t s) {
  return id_in ? id_in[s] : (int64_t)s;
}

__global__ __launch_bounds__(kPermWaves *kWave) void k_permute(
    int32_t ncells, const int32_t *__restrict__ start, const int32_t *__restrict__ src,
    const double *__restrict__ x_in, const double *__restrict__ v_in,
    const int32_t *__restrict__ type_in, const int64_t *__restrict__ id_in,
    double *__restrict__ x_out, double *__restrict__ v_out, int32_t *__restrict__ type_out,
    int64_t *__restrict__ id_out) {
  __shared__ int64_t ids[kPermWaves][kStage];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int32_t c = blockIdx.x * kPermWaves + w;
  if (c >= ncells) return;  // whole wavefront leaves together; no block barrier below
  const int32_t s0 = start[c];
  const int32_t m = start[c + 1] - s0;
  const bool staged = m <= kStage;
  if (staged) {
    for (int32_t k = lane; k < m; k += kWave) ids[w][k] = id_at(id_in, src[s0 + k]);
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  for (int32_t k0 = 0; k0 < m; k0 += kWave) {
    const int32_t k = k0 + lane;
    if (k < m) {
      const int32_t s = src[s0 + k];
      const int64_t my = id_at(id_in, s);
      int32_t rank = 0;
      if (staged) {
        for (int32_t q = 0; q < m; ++q) rank += ids[w][q] < my;
      } else {
        for (int32_t q = 0; q < m; ++q) rank += id_at(id_in, src[s0 + q]) < my;
      }
      const int64_t o = (int64_t)s0 + rank;
      x_out[3 * o] = x_in[3 * (int64_t)s];
      x_out[3 * o + 1] = x_in[3 * (int64_t)s + 1];
      x_out[3 * o + 2] = x_in[3 * (int64_t)s + 2];
      if (v_in) {
        v_out[3 * o] = v_in[3 * (int64_t)s];
        v_out[3 * o + 1] = v_in[3 * (int64_t)s + 1];
        v_out[3 * o + 2] = v_in[3 * (int64_t)s + 2];
      }
      if (type_in) type_out[o] = type_in[s];
      id_out[o] = my;
    }
  }
}

inline unsigned blocks_for(int64_t n, int threads) {
  return (unsigned)((n + threads - 1) / threads);
}

}  // namespace

size_t bin_workspace(int64_t n, int64_t ncells) {
  // counts[ncells] + cell[n] + rank[n] + src[n], int32, 256-byte aligned
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  return al((size_t)ncells * 4) + 3 * al((size_t)n * 4);
}

int launch_bin(const GridK &g, int64_t n, const double *x_in, const double *v_in,
               const int32_t *type_in, const int64_t *id_in, double *x_out, double *v_out,
               int32_t *type_out, int64_t *id_out, int32_t *cell_start, void *ws,
               hipStream_t st) {
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  char *p = (char *)ws;
  int32_t *counts = (int32_t *)p;
  p += al((size_t)g.ncells * 4);
  int32_t *cell = (int32_t *)p;
  p += al((size_t)n * 4);
  int32_t *rank = (int32_t *)p;
  p += al((size_t)n * 4);
  int32_t *src = (int32_t *)p;

  k_fill_i32<<<blocks_for(g.ncells, 256), 256, 0, st>>>(counts, g.ncells, 0);
  if (n > 0) k_count<<<blocks_for(n, 256), 256, 0, st>>>(n, x_in, g, cell, rank, counts);
  k_scan<<<1, kScanThreads, 0, st>>>(g.ncells, counts, cell_start);
  if (n > 0) {
    k_scatter<<<blocks_for(n, 256), 256, 0, st>>>(n, cell, rank, cell_start, src);
    k_permute<<<blocks_for(g.ncells, kPermWaves), kPermWaves * kWave, 0, st>>>(
        g.ncells, cell_start, src, x_in, v_in, type_in, id_in, x_out, v_out, type_out, id_out);
  }
  return check_launch("ljmd_bin");
}

}  // namespace ljmd
