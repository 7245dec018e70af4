// Verlet neighbor lists over the 27-cell stencil, gfx950.  Paper: Cabana
// "Neighbor List Creation" (distance-criterion lists built by binning, dense
// storage, thread-parallel creation).
//
// One wavefront per home cell (on grids of fewer than 2,048 cells, per part of
// a cell's home atoms: a 32,000-atom liquid has 1,331 cells, one wavefront per
// SIMD or fewer).  The candidates -- every atom of the stencil
// cells (offsets -1, 0, +1 per dimension modulo nc, with repeats removed when
// nc < 3) -- are loaded once into registers, 64 per register slot (lane t of
// slot r holds candidate 64 r + t).  The wavefront then walks the home atoms
// one at a time: every lane tests its candidates against the (uniform) home
// atom, a ballot + mbcnt prefix compacts the hits, and each hit is stored in
// the home atom's row of the tiled-ELL list:
//   nbr[((i / 64) * maxn + k) * 64 + (i % 64)].
// Cells with more candidates than the register slots hold fall back to
// reading candidates from global memory per home atom.
#include "common.h"

namespace ljmd {

namespace {

// Two shapes of the build kernel.  Standard: 12 register slots (up to 768
// candidates staged) and rows of up to 128 entries buffered in LDS.  Dense
// (chosen when maxn > 128, i.e. long rows and so crowded stencils): 16 slots
// (1024 candidates) and rows of up to 256 entries, at twice the LDS.
constexpr int kSlots = 12;
constexpr int kRowCap = 128;
constexpr int kDenseSlots = 16;
constexpr int kDenseRowCap = 256;
constexpr int kBatch = 16;  // home atoms whose rows are buffered in LDS at once
constexpr int kFlushRows = kWave / kBatch;  // list rows of a batch written per store instruction
// LDS row stride ROWCAP + 1 (odd): lanes reading entry k of different rows hit distinct banks

__global__ void k_fill_scalar(int32_t *p, int32_t val) { *p = val; }

// What a build pass writes: the tiled list (rows cut at maxn, counts in nnbr),
// only the true row lengths (into nnbr), or compressed rows at csr[offsets[i]..]
// (entries at or beyond cap dropped).
enum BuildMode { kTiled = 0, kCount = 1, kCsr = 2 };

// Output of a build pass.
struct BuildOut {
  int32_t *nbr;            // tiled list (kTiled)
  int32_t *nnbr;           // row lengths (kTiled: cut at maxn; kCount: true)
  int32_t maxn;
  const int64_t *offsets;  // kCsr: row starts
  int32_t *csr;            // kCsr: rows
  int64_t cap;             // kCsr: capacity of csr
};

// Stencil of cell c: its candidate ranges [rs[s], rs[s] + len) in sorted order
// and the prefix pre[s] of their lengths.  Returns the number of ranges.
__device__ __forceinline__ int stencil_ranges(const GridK &g, int32_t c, const int32_t *cell_start,
                                              int32_t *rs, int32_t *pre) {
  const int lane = threadIdx.x & (kWave - 1);
  int32_t cc[3] = {c % g.nc[0], (c / g.nc[0]) % g.nc[1], c / (g.nc[0] * g.nc[1])};
  // y and z: the distinct cells among c-1, c, c+1 (mod nc)
  int32_t cells[2][3];
  int cnt[2];
#pragma unroll
  for (int k = 1; k < 3; ++k) {
    const int32_t m = g.nc[k];
    if (m >= 3) {
      cells[k - 1][0] = cc[k] == 0 ? m - 1 : cc[k] - 1;
      cells[k - 1][1] = cc[k];
      cells[k - 1][2] = cc[k] == m - 1 ? 0 : cc[k] + 1;
      cnt[k - 1] = 3;
    } else {
      cells[k - 1][0] = 0;
      cells[k - 1][1] = 1;
      cells[k - 1][2] = 0;
      cnt[k - 1] = m;
    }
  }
  // x: runs of consecutive cells, which are consecutive in sorted order too
  const int32_t mx = g.nc[0];
  int32_t run0[2], runlen[2];
  int nrun;
  if (mx < 3) {
    run0[0] = 0, runlen[0] = mx, nrun = 1;
  } else if (cc[0] == 0) {
    run0[0] = 0, runlen[0] = 2, run0[1] = mx - 1, runlen[1] = 1, nrun = 2;
  } else if (cc[0] == mx - 1) {
    run0[0] = mx - 2, runlen[0] = 2, run0[1] = 0, runlen[1] = 1, nrun = 2;
  } else {
    run0[0] = cc[0] - 1, runlen[0] = 3, nrun = 1;
  }
  const int S = nrun * cnt[0] * cnt[1];
  int32_t len = 0;
  if (lane < S) {
    const int ir = lane % nrun;
    const int iy = (lane / nrun) % cnt[0];
    const int iz = lane / (nrun * cnt[0]);
    const int32_t row = (cells[1][iz] * g.nc[1] + cells[0][iy]) * mx;
    const int32_t a = cell_start[row + run0[ir]];
    rs[lane] = a;
    len = cell_start[row + run0[ir] + runlen[ir]] - a;
  }
  // inclusive prefix of len over the first S lanes (S <= 18 < 32)
  int32_t inc = len;
#pragma unroll
  for (int off = 1; off < 32; off <<= 1) {
    int32_t o = __shfl_up(inc, off, kWave);
    if (lane >= off) inc += o;
  }
  if (lane < S) pre[lane + 1] = inc;
  if (lane == 0) pre[0] = 0;
  __syncthreads();  // the block is this one wavefront
  return S;
}

// Sorted index of candidate t (t < pre[S]).
__device__ __forceinline__ int32_t locate(int32_t t, const int32_t *rs, const int32_t *pre) {
  int r = 0;
  while (t >= pre[r + 1]) ++r;
  return rs[r] + (t - pre[r]);
}

// Register-staged build of one cell's rows (candidates <= SLOTS * 64).  BUF:
// rows are compacted in LDS (maxn <= ROWCAP) rather than stored directly.
template <bool HALF, bool WRAP, bool BUF, int SLOTS, int ROWCAP, int MODE>
__device__ __forceinline__ void build_staged(const BoxK &b, double rl2, const double *__restrict__ x,
                                             int32_t h0, int32_t h1, int32_t total, int nslot,
                                             const int32_t *rs, const int32_t *pre,
                                             const BuildOut &o, int32_t *rowbuf, int32_t *rowcnt,
                                             int32_t &maxc) {
  const int32_t maxn = o.maxn;
  int32_t *__restrict__ nbr = o.nbr;
  int32_t *__restrict__ nnbr = o.nnbr;
  static_assert(!BUF || MODE == kTiled, "rows are buffered only for the tiled list");
  const int lane = threadIdx.x & (kWave - 1);
  const double L0 = b.L[0], L1 = b.L[1], L2 = b.L[2];
  const double iL0 = b.invL[0], iL1 = b.invL[1], iL2 = b.invL[2];
  constexpr int kRowStride = ROWCAP + 1;
  double qx[SLOTS], qy[SLOTS], qz[SLOTS];
  int32_t qj[SLOTS];
#pragma unroll
  for (int r = 0; r < SLOTS; ++r) {
    const int32_t t = r * kWave + lane;
    qj[r] = -1;
    qx[r] = qy[r] = qz[r] = 0.0;
    if (r < nslot && t < total) {
      const int32_t j = locate(t, rs, pre);
      qj[r] = j;
      qx[r] = x[3 * (int64_t)j];
      qy[r] = x[3 * (int64_t)j + 1];
      qz[r] = x[3 * (int64_t)j + 2];
    }
  }
  // Rows of up to kBatch home atoms are compacted into LDS first (when they fit)
  // and then written out k by k: the atoms of a batch are consecutive, so each
  // store instruction covers one contiguous run of a tile row instead of
  // scattering 4-byte entries 256 bytes apart.
  constexpr bool buffered = BUF;
  // home positions: lane l holds atom c0 + l of the current chunk of 64, read
  // back by every lane with a scalar readlane (no load latency per home atom)
  double hx = 0.0, hy = 0.0, hz = 0.0;
  for (int32_t b0 = h0; b0 < h1; b0 += kBatch) {
    const int nb = h1 - b0 < kBatch ? h1 - b0 : kBatch;
    if ((b0 - h0) % kWave == 0) {
      const int32_t ih = b0 + lane;
      if (ih < h1) {
        hx = x[3 * (int64_t)ih];
        hy = x[3 * (int64_t)ih + 1];
        hz = x[3 * (int64_t)ih + 2];
      }
    }
    for (int bi = 0; bi < nb; ++bi) {
      const int32_t i = b0 + bi;
      const int src = (b0 - h0) % kWave + bi;
      const double xi = readlane_f64(hx, src), yi = readlane_f64(hy, src),
                   zi = readlane_f64(hz, src);
      int32_t *row = MODE == kTiled ? nbr + (int64_t)(i >> 6) * maxn * kWave + (i & (kWave - 1))
                                    : nullptr;
      const int64_t off = MODE == kCsr ? o.offsets[i] : 0;
      int32_t base = 0;
#pragma unroll
      for (int r = 0; r < SLOTS; ++r) {
        if (r < nslot) {
          double dx = xi - qx[r], dy = yi - qy[r], dz = zi - qz[r];
          if constexpr (WRAP) {
            dx = min_image(dx, L0, iL0);
            dy = min_image(dy, L1, iL1);
            dz = min_image(dz, L2, iL2);
          }
          const double r2 = dist2(dx, dy, dz);
          const bool ok = qj[r] >= 0 && r2 < rl2 && (HALF ? qj[r] > i : qj[r] != i);
          const uint64_t m = __builtin_amdgcn_ballot_w64(ok);
          if (MODE != kCount && ok) {
            const int32_t k = base + (int32_t)__builtin_amdgcn_mbcnt_hi(
                                         (uint32_t)(m >> 32),
                                         __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            if constexpr (MODE == kCsr) {
              if (off + k < o.cap) o.csr[off + k] = qj[r];
            } else if (k < maxn) {
              if (buffered)
                rowbuf[bi * kRowStride + k] = qj[r];
              else
                row[(int64_t)k * kWave] = qj[r];
            }
          }
          base += (int32_t)__popcll(m);
        }
      }
      if (lane == 0) rowcnt[bi] = MODE == kTiled ? (base < maxn ? base : maxn) : base;
      maxc = base > maxc ? base : maxc;
    }
    __syncthreads();  // rowbuf / rowcnt written by other lanes of this one-wavefront block
    if (MODE != kCsr && lane < nb) nnbr[b0 + lane] = rowcnt[lane];
    if (buffered) {
      // lane (a, h) = (lane % kBatch, lane / kBatch) stores rows k = h, h + kFlushRows,
      // ... of batch atom a: every store instruction covers kFlushRows list rows of
      // the whole batch
      const int a = lane % kBatch;
      const int32_t mine = a < nb ? rowcnt[a] : 0;
      const int32_t kmax = wave_max(mine);
      const int32_t i = b0 + a;
      int32_t *row = nbr + (int64_t)(i >> 6) * maxn * kWave + (i & (kWave - 1));
      for (int32_t k = lane / kBatch; k < kmax; k += kFlushRows)
        if (k < mine) row[(int64_t)k * kWave] = rowbuf[a * kRowStride + k];
    }
    __syncthreads();  // before the next batch overwrites rowbuf / rowcnt
  }
}

// Block -> (home cell, part): part p of nsplit takes the cell's home atoms
// [len p / nsplit, len (p + 1) / nsplit) (each part stages the whole stencil).
// The standard shape asks for 4 resident wavefronts per SIMD (at most 128
// VGPRs: the full-list build needs 131 and keeps 3 otherwise; 2 registers
// spill): 500k 299.5 -> 259.6 us, 256k 171.3 -> 153.4 us, 32k unchanged.
// Fewer register slots reach the same occupancy without spills (11: 258.6 us)
// but send more crowded cells to the unstaged path (10 slots: 32k 43 -> 148 us).
// The dense shape asks for 3 (the full list needs 179 VGPRs, 2 per SIMD
// otherwise; no spills at 166): the 512,000-particle SPH build 528.7 -> 496.7 us.
template <int SLOTS>
constexpr int build_occupancy() { return SLOTS <= kSlots ? 4 : 3; }

template <bool HALF, int SLOTS, int ROWCAP, int MODE = kTiled>
__global__ __launch_bounds__(kWave, build_occupancy<SLOTS>())
void k_build(GridK g, BoxK b, double rl2, const double *__restrict__ x,
             const int32_t *__restrict__ cell_start, BuildOut o, int32_t *__restrict__ max_count,
             int nsplit) {
  const int32_t maxn = o.maxn;
  __shared__ int32_t rs[27];
  __shared__ int32_t pre[28];
  __shared__ int32_t rowbuf[kBatch * (ROWCAP + 1)];
  __shared__ int32_t rowcnt[kBatch];
  const int lane = threadIdx.x;
  const int32_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int32_t c = blk / nsplit;
  const int part = blk - c * nsplit;
  const int32_t c0 = cell_start[c], clen = cell_start[c + 1] - c0;
  const int32_t h0 = c0 + (int32_t)(((int64_t)clen * part) / nsplit);
  const int32_t h1 = c0 + (int32_t)(((int64_t)clen * (part + 1)) / nsplit);
  if (h0 == h1) return;
  const int S = stencil_ranges(g, c, cell_start, rs, pre);
  const int32_t total = pre[S];
  const int nslot = (total + kWave - 1) / kWave;
  int32_t maxc = 0;
  // A home cell whose stencil does not wrap (nc >= 4 and the cell is not on a
  // face) pairs atoms at most two cell edges = L/2 apart per dimension: the raw
  // displacement is then the minimum image for every pair that can be inside
  // rlist, and any pair at ~L/2 is beyond rlist whichever image is taken.
  bool wrap = false;
  {
    const int32_t cc[3] = {c % g.nc[0], (c / g.nc[0]) % g.nc[1], c / (g.nc[0] * g.nc[1])};
    for (int k = 0; k < 3; ++k)
      wrap |= g.nc[k] < 4 || cc[k] == 0 || cc[k] == g.nc[k] - 1;
  }
  if (nslot <= SLOTS) {
#define LJMD_STAGED(W, B)                                                                     \
  build_staged<HALF, W, B, SLOTS, ROWCAP, MODE>(b, rl2, x, h0, h1, total, nslot, rs, pre, o, \
                                                rowbuf, rowcnt, maxc)
    if constexpr (MODE == kTiled) {
      if (maxn <= ROWCAP) {
        if (wrap) LJMD_STAGED(true, true); else LJMD_STAGED(false, true);
      } else {
        if (wrap) LJMD_STAGED(true, false); else LJMD_STAGED(false, false);
      }
    } else {
      if (wrap) LJMD_STAGED(true, false); else LJMD_STAGED(false, false);
    }
#undef LJMD_STAGED
  } else {
    const double L0 = b.L[0], L1 = b.L[1], L2 = b.L[2];
    const double iL0 = b.invL[0], iL1 = b.invL[1], iL2 = b.invL[2];
    for (int32_t i = h0; i < h1; ++i) {
      const double xi = x[3 * (int64_t)i], yi = x[3 * (int64_t)i + 1], zi = x[3 * (int64_t)i + 2];
      int32_t *row = MODE == kTiled
                         ? o.nbr + (int64_t)(i >> 6) * maxn * kWave + (i & (kWave - 1))
                         : nullptr;
      const int64_t off = MODE == kCsr ? o.offsets[i] : 0;
      int32_t base = 0;
      for (int r = 0; r < nslot; ++r) {
        const int32_t t = r * kWave + lane;
        bool ok = false;
        int32_t j = -1;
        if (t < total) {
          j = locate(t, rs, pre);
          const double dx = min_image(xi - x[3 * (int64_t)j], L0, iL0);
          const double dy = min_image(yi - x[3 * (int64_t)j + 1], L1, iL1);
          const double dz = min_image(zi - x[3 * (int64_t)j + 2], L2, iL2);
          ok = dist2(dx, dy, dz) < rl2 && (HALF ? j > i : j != i);
        }
        const uint64_t m = __ballot(ok);
        if (MODE != kCount && ok) {
          const int32_t k = base + (int32_t)__builtin_amdgcn_mbcnt_hi(
                                       (uint32_t)(m >> 32),
                                       __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
          if constexpr (MODE == kCsr) {
            if (off + k < o.cap) o.csr[off + k] = j;
          } else if (k < maxn) {
            row[(int64_t)k * kWave] = j;
          }
        }
        base += (int32_t)__popcll(m);
      }
      if (MODE != kCsr && lane == 0) o.nnbr[i] = MODE == kTiled ? (base < maxn ? base : maxn) : base;
      maxc = base > maxc ? base : maxc;
    }
  }
  // Every wavefront's atomic on the one max_count word is serialised (≈ 11 ns
  // each, 24,389 of them at 500,000 atoms): add only a maximum above the one
  // already there (the value only grows, so a skipped one is never the largest).
  if (lane == 0 && max_count) {
    const int32_t seen = __hip_atomic_load(max_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (maxc > seen) atomicMax(max_count, maxc);
  }
}

// Parts per home cell: grids of fewer than 2,048 cells (two wavefronts per
// SIMD) split each cell's home atoms over up to 8 wavefronts.  Measured (us):
// 32,000 atoms (1,331 cells) 60.9 -> 43.4 with 2 parts (3: 48.5); 256 atoms
// (8 cells) 32.0 -> 11.0 with 8; at 256,000 and 500,000 atoms (12,167 and
// 24,389 cells) 2 parts cost 10-14 %.
constexpr int64_t kSplitCells = 2048;
constexpr int kMaxSplit = 8;

int build_split(int64_t ncells) {
  if (ncells >= kSplitCells) return 1;
  const int64_t s = (kSplitCells + ncells - 1) / ncells;
  return (int)(s < kMaxSplit ? s : kMaxSplit);
}

template <int MODE>
void launch_mode(const GridK &g, const BoxK &b, double rl2, bool half, const double *x,
                 const int32_t *cell_start, const BuildOut &o, int32_t *max_count,
                 hipStream_t st) {
  const int ns = build_split(g.ncells);
  if (MODE != kTiled || o.maxn <= kRowCap) {
    if (half)
      k_build<true, kSlots, kRowCap, MODE><<<g.ncells * ns, kWave, 0, st>>>(g, b, rl2, x, cell_start, o,
                                                                      max_count, ns);
    else
      k_build<false, kSlots, kRowCap, MODE><<<g.ncells * ns, kWave, 0, st>>>(g, b, rl2, x, cell_start,
                                                                       o, max_count, ns);
  } else {
    if (half)
      k_build<true, kDenseSlots, kDenseRowCap, MODE><<<g.ncells * ns, kWave, 0, st>>>(
          g, b, rl2, x, cell_start, o, max_count, ns);
    else
      k_build<false, kDenseSlots, kDenseRowCap, MODE><<<g.ncells * ns, kWave, 0, st>>>(
          g, b, rl2, x, cell_start, o, max_count, ns);
  }
}

}  // namespace

int launch_offsets(int64_t n, const int32_t *counts, int64_t *offsets, void *ws, hipStream_t st);
size_t csr_workspace(int64_t n);

// Compressed rows straight from the cells: a counting pass (true row lengths),
// their exclusive scan into offsets (offsets[n] = total), then a filling pass
// that writes row i at csr[offsets[i] ..] (entries at or beyond cap dropped:
// the caller compares offsets[n] with cap and builds again with more room).
size_t build_csr_workspace(int64_t n) {
  return (((size_t)(n > 0 ? n : 1) * sizeof(int32_t) + 255) / 256) * 256 + csr_workspace(n);
}

int launch_build_csr(const GridK &g, const BoxK &b, double rlist, int kind, int64_t n,
                     const double *x, const int32_t *cell_start, int64_t *offsets, int32_t *csr,
                     int64_t cap, void *ws, hipStream_t st) {
  int32_t *counts = (int32_t *)ws;
  void *scan_ws = (char *)ws + (((size_t)(n > 0 ? n : 1) * sizeof(int32_t) + 255) / 256) * 256;
  const double rl2 = rlist * rlist;
  const bool half = kind == LJMD_HALF;
  BuildOut o{};
  o.nnbr = counts;
  o.maxn = 1;
  if (n > 0) launch_mode<kCount>(g, b, rl2, half, x, cell_start, o, nullptr, st);
  const int rc = launch_offsets(n, counts, offsets, scan_ws, st);
  if (rc != LJMD_OK) return rc;
  if (n > 0) {
    o.offsets = offsets;
    o.csr = csr;
    o.cap = cap;
    launch_mode<kCsr>(g, b, rl2, half, x, cell_start, o, nullptr, st);
  }
  return check_launch("ljmd_build_neighbors_csr");
}

int launch_build(const GridK &g, const BoxK &b, double rlist, int kind, int64_t n, const double *x,
                 const int32_t *cell_start, int32_t maxn, int32_t *nbr, int32_t *nnbr,
                 int32_t *max_count, hipStream_t st) {
  k_fill_scalar<<<1, 1, 0, st>>>(max_count, 0);
  if (n > 0) {
    BuildOut o{};
    o.nbr = nbr;
    o.nnbr = nnbr;
    o.maxn = maxn;
    launch_mode<kTiled>(g, b, rlist * rlist, kind == LJMD_HALF, x, cell_start, o, max_count, st);
  }
  return check_launch("ljmd_build_neighbors");
}

}  // namespace ljmd
