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
// On grids of 3 or more cells per dimension the candidates are staged as
// 16-bit lattice coordinates and tested with packed integer arithmetic
// (QuantK below); only pairs within the lattice's error band of rlist take the
// FP64 test, so the lists are exactly those of the FP64 test everywhere.
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
// Home atoms whose rows are buffered in LDS at once.  8 rather than 16 halves
// the one-wavefront block's LDS, so more blocks fit on a compute unit: the
// integer-tested build at 500,000 atoms went 230.5 -> 207.0 us (full list),
// 200.9 -> 173.3 (half), 388.9 -> 240.2 (dense shape); 4 gave 213.7 / 178.4 /
// 231.6.
constexpr int kBatch = 8;
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

// Integer pre-test of the candidate distances (grids of at least 3 cells per
// dimension).  Each staged position is taken relative to the home cell's
// centre, minimum-imaged there and rounded to a lattice of spacing q: u =
// rint(min_image(x - centre) / q), |u| <= kQuantMax (the 27 stencil cells lie
// within 1.5 cell edges of the centre).  A pair's lattice displacement then
// differs from the true one by at most q per axis, so its length by at most
// sqrt(3) q, and with R = rlist / q the integer r2q = |u_i - u_j|^2 decides
//   r2q < t_in  = floor((R - 1.75)^2): inside rlist,
//   r2q > t_out = ceil((R + 1.75)^2):  outside rlist,
// and only the pairs between (about 0.15 per atom in the dense liquid) take
// the FP64 test with the minimum image.  The image of a candidate nearest the
// centre is the one nearest the home atom for every pair within rlist when
// the home atom lies within L/2 - rlist of the centre per axis (the pair is
// then within L/2 of the centre); atoms inside their cell always do (cell
// edges exceed rlist and nc >= 3), and a wavefront whose home atoms do not
// (positions outside the box) takes the unstaged FP64 path.  So the lists are
// exactly those of the FP64 test.
struct QuantK {
  double invq;     // 1 / q
  int32_t t_in;    // r2q below: inside rlist
  int32_t t_out;   // r2q above: outside rlist
  double home[3];  // bound on |home atom - centre| per axis: L/2 - rlist, rounded down
};
constexpr double kQuantSpan = 8000.0;  // lattice steps per 1.5 cell edges
constexpr int32_t kQuantMax = 8190;    // |u| of a staged coordinate
// z of an empty slot: |dz| <= 33,190, so r2q stays below 2^31 and above t_out
constexpr int32_t kQuantEmpty = 25000;

typedef short short2v __attribute__((ext_vector_type(2)));

// Lattice coordinates of x relative to the centre cc; false when a coordinate
// is out of range (or not finite).
__device__ __forceinline__ bool quantize(const double *p, const double *cc, const BoxK &b,
                                         double invq, int32_t &uxy, int32_t &uz) {
  int32_t u[3];
  bool in = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double d = min_image(p[k] - cc[k], b.L[k], b.invL[k]) * invq;
    in = in && __builtin_fabs(d) <= (double)kQuantMax;
    u[k] = in ? (int32_t)__builtin_rint(d) : 0;
  }
  uxy = (int32_t)((uint32_t)(uint16_t)u[0] | ((uint32_t)u[1] << 16));
  uz = u[2];
  return in;
}

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

// Store a hit of the lanes' ballot m: entry base + (hits in lower lanes) of the
// home atom's row (LDS buffer, tiled row or compressed row).
// room: base + popcount(m) <= maxn (uniform), so no lane needs its own test.
template <bool BUF, int ROWCAP, int MODE>
__device__ __forceinline__ void store_hit(const BuildOut &o, int32_t *row, int32_t *rowbuf, int bi,
                                          int64_t off, int32_t base, uint64_t m, bool room,
                                          int32_t j, int32_t maxn) {
  const int32_t k = (int32_t)__builtin_amdgcn_mbcnt_hi(
      (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, (uint32_t)base));
  if constexpr (MODE == kCsr) {
    if (off + k < o.cap) o.csr[off + k] = j;
  } else if (room) {
    if (BUF)
      rowbuf[bi * (ROWCAP + 1) + k] = j;
    else
      row[(int64_t)k * kWave] = j;
  } else if (k < maxn) {
    if (BUF)
      rowbuf[bi * (ROWCAP + 1) + k] = j;
    else
      row[(int64_t)k * kWave] = j;
  }
}

// Register-staged build with the integer pre-test (QuantK): three registers
// per slot (packed x/y lattice coordinates, z, index) instead of seven.  Same
// rows in the same order as build_staged.  Returns false, having written
// nothing, when a staged coordinate or a home atom is outside the bounds the
// pre-test needs (positions outside the box); the caller then takes the
// unstaged path.
template <bool HALF, bool BUF, int SLOTS, int ROWCAP, int MODE>
__device__ __forceinline__ bool build_quant(const BoxK &b, const QuantK &q, const double *cc,
                                            double rl2, const double *__restrict__ x, int32_t h0,
                                            int32_t h1, int32_t total, int nslot,
                                            const int32_t *rs, const int32_t *pre,
                                            const BuildOut &o, int32_t *rowbuf, int32_t *rowcnt,
                                            int32_t &maxc) {
  const int32_t maxn = o.maxn;
  int32_t *__restrict__ nbr = o.nbr;
  int32_t *__restrict__ nnbr = o.nnbr;
  static_assert(!BUF || MODE == kTiled, "rows are buffered only for the tiled list");
  const int lane = threadIdx.x & (kWave - 1);
  constexpr int kRowStride = ROWCAP + 1;
  int32_t qxy[SLOTS], qz[SLOTS], qj[SLOTS];
  bool good = true;
#pragma unroll
  for (int r = 0; r < SLOTS; ++r) {
    const int32_t t = r * kWave + lane;
    qj[r] = -1;
    qxy[r] = 0;
    qz[r] = kQuantEmpty;
    if (r < nslot && t < total) {
      const int32_t j = locate(t, rs, pre);
      qj[r] = j;
      good = quantize(x + 3 * (int64_t)j, cc, b, q.invq, qxy[r], qz[r]) && good;
    }
  }
  for (int32_t c0 = h0; c0 < h1; c0 += kWave) {
    const int32_t ih = c0 + lane;
    if (ih < h1) {
      const double *p = x + 3 * (int64_t)ih;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        good = good && __builtin_fabs(min_image(p[k] - cc[k], b.L[k], b.invL[k])) <= q.home[k];
    }
  }
  if (__builtin_amdgcn_ballot_w64(!good) != 0) return false;
  // candidate number of home atom h0: the home cell lies in one stencil range
  // (ranges are disjoint on grids of 3 or more cells per dimension)
  int32_t tc = 0;
  for (int sr = 0; pre[sr] < total; ++sr)
    if (rs[sr] <= h0 && h0 < rs[sr] + (pre[sr + 1] - pre[sr])) tc = pre[sr] + (h0 - rs[sr]);
  double hx = 0.0, hy = 0.0, hz = 0.0;
  int32_t hxy = 0, huz = 0;
  for (int32_t b0 = h0; b0 < h1; b0 += kBatch) {
    const int nb = h1 - b0 < kBatch ? h1 - b0 : kBatch;
    if ((b0 - h0) % kWave == 0) {
      const int32_t ih = b0 + lane;
      if (ih < h1) {
        const double *p = x + 3 * (int64_t)ih;
        hx = p[0];
        hy = p[1];
        hz = p[2];
        quantize(p, cc, b, q.invq, hxy, huz);  // a staged candidate: in range
      }
    }
    for (int bi = 0; bi < nb; ++bi) {
      const int32_t i = b0 + bi;
      const int src = (b0 - h0) % kWave + bi;
      const short2v ui = __builtin_bit_cast(short2v, __builtin_amdgcn_readlane(hxy, src));
      const int32_t uzi = __builtin_amdgcn_readlane(huz, src);
      int32_t *row = MODE == kTiled ? nbr + (int64_t)(i >> 6) * maxn * kWave + (i & (kWave - 1))
                                    : nullptr;
      const int64_t off = MODE == kCsr ? o.offsets[i] : 0;
      const int32_t tself = tc + (i - h0);  // candidate number of atom i
      int32_t base = 0;
#pragma unroll
      for (int r = 0; r < SLOTS; ++r) {
        if (r < nslot) {
          const short2v d = __builtin_bit_cast(short2v, qxy[r]) - ui;
          const int32_t dz = qz[r] - uzi;
          const int32_t r2q = __builtin_amdgcn_sdot2(d, d, __mul24(dz, dz), false);
          // lane masks of single compares (one v_cmp each) combined in scalar
          // registers; the full list drops atom i itself by its lane bit
          uint64_t keep;
          if constexpr (HALF)
            keep = __builtin_amdgcn_ballot_w64(qj[r] > i);
          else
            keep = r == (tself >> 6) ? ~(1ull << (tself & (kWave - 1))) : ~0ull;
          uint64_t m = __builtin_amdgcn_ballot_w64(r2q < q.t_in) & keep;
          const uint64_t m_near = __builtin_amdgcn_ballot_w64(r2q <= q.t_out) & keep & ~m;
          if (m_near != 0) {
            // the FP64 test with the minimum image for the pairs near rlist, on
            // every lane (lanes not near read atom i)
            const bool near = __builtin_amdgcn_inverse_ballot_w64(m_near);
            const double xi = readlane_f64(hx, src), yi = readlane_f64(hy, src),
                         zi = readlane_f64(hz, src);
            const double *p = x + 3 * (int64_t)(near ? qj[r] : i);
            const double dx = min_image(xi - p[0], b.L[0], b.invL[0]);
            const double dy = min_image(yi - p[1], b.L[1], b.invL[1]);
            const double dzz = min_image(zi - p[2], b.L[2], b.invL[2]);
            m |= __builtin_amdgcn_ballot_w64(dist2(dx, dy, dzz) < rl2) & m_near;
          }
          const int32_t k0 = base;  // row entries before this slot's hits
          base += (int32_t)__popcll(m);
          const bool room = base <= maxn;
          if (MODE != kCount && __builtin_amdgcn_inverse_ballot_w64(m))
            store_hit<BUF, ROWCAP, MODE>(o, row, rowbuf, bi, off, k0, m, room, qj[r], maxn);
        }
      }
      if (lane == 0) rowcnt[bi] = MODE == kTiled ? (base < maxn ? base : maxn) : base;
      maxc = base > maxc ? base : maxc;
    }
    __syncthreads();  // rowbuf / rowcnt written by other lanes of this one-wavefront block
    if (MODE != kCsr && lane < nb) nnbr[b0 + lane] = rowcnt[lane];
    if (BUF) {
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
  return true;
}

// Block -> (home cell, part): part p of nsplit takes the cell's home atoms
// [len p / nsplit, len (p + 1) / nsplit) (each part stages the whole stencil).
// QUANT: integer pre-test (grids of 3 or more cells per dimension); 76-93
// VGPRs, so residency is set by the LDS row buffer.  Against the FP64-staged
// kernel on the same lists at 500,000 atoms: 259 -> 207 us (full), 243 -> 173
// us (half), 390 -> 240 us (dense shape).
// FP64-staged kernel (smaller grids): the standard shape asks for 4 resident
// wavefronts per SIMD (at most 128 VGPRs: the full-list build needs 131 and
// keeps 3 otherwise; 2 registers spill), which took the 500k build from 299.5
// to 259.6 us when this kernel served every grid; the dense shape asks for 3
// (179 VGPRs otherwise, no spills at 166).
template <int SLOTS>
constexpr int build_occupancy() { return SLOTS <= kSlots ? 4 : 3; }

template <bool HALF, int SLOTS, int ROWCAP, int MODE = kTiled, bool QUANT = false>
__global__ __launch_bounds__(kWave, QUANT ? 1 : build_occupancy<SLOTS>())
void k_build(GridK g, BoxK b, double rl2, const double *__restrict__ x,
             const int32_t *__restrict__ cell_start, BuildOut o, int32_t *__restrict__ max_count,
             int nsplit, QuantK q) {
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
  bool staged = false;
  if constexpr (QUANT) {
    if (nslot <= SLOTS) {
      const int32_t cc3[3] = {c % g.nc[0], (c / g.nc[0]) % g.nc[1], c / (g.nc[0] * g.nc[1])};
      const double cc[3] = {(cc3[0] + 0.5) * g.h[0], (cc3[1] + 0.5) * g.h[1],
                            (cc3[2] + 0.5) * g.h[2]};
#define LJMD_QUANT(B)                                                                            \
  build_quant<HALF, B, SLOTS, ROWCAP, MODE>(b, q, cc, rl2, x, h0, h1, total, nslot, rs, pre, o, \
                                            rowbuf, rowcnt, maxc)
      if constexpr (MODE == kTiled)
        staged = maxn <= ROWCAP ? LJMD_QUANT(true) : LJMD_QUANT(false);
      else
        staged = LJMD_QUANT(false);
#undef LJMD_QUANT
    }
  } else if (nslot <= SLOTS) {
    staged = true;
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
  }
  if (!staged) {
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

// Lattice and thresholds of the integer pre-test for this grid and cutoff.
QuantK make_quant(const GridK &g, const BoxK &b, double rl2) {
  const double h = fmax(g.h[0], fmax(g.h[1], g.h[2]));
  QuantK q;
  q.invq = kQuantSpan / (1.5 * h);
  const double R = sqrt(rl2) * q.invq;  // <= kQuantSpan / 1.5: cell edges exceed rlist
  q.t_in = (int32_t)floor((R - 1.75) * (R - 1.75));
  q.t_out = (int32_t)ceil((R + 1.75) * (R + 1.75));
  for (int k = 0; k < 3; ++k) q.home[k] = (0.5 * b.L[k] - sqrt(rl2)) * (1.0 - 1e-12);
  return q;
}

template <bool HALF, int SLOTS, int ROWCAP, int MODE>
void launch_shape(const GridK &g, const BoxK &b, double rl2, const double *x,
                  const int32_t *cell_start, const BuildOut &o, int32_t *max_count, int ns,
                  hipStream_t st) {
  const unsigned nblk = (unsigned)(g.ncells * ns);
  if (g.nc[0] >= 3 && g.nc[1] >= 3 && g.nc[2] >= 3)
    k_build<HALF, SLOTS, ROWCAP, MODE, true><<<nblk, kWave, 0, st>>>(
        g, b, rl2, x, cell_start, o, max_count, ns, make_quant(g, b, rl2));
  else
    k_build<HALF, SLOTS, ROWCAP, MODE, false><<<nblk, kWave, 0, st>>>(
        g, b, rl2, x, cell_start, o, max_count, ns, QuantK{});
}

template <int MODE>
void launch_mode(const GridK &g, const BoxK &b, double rl2, bool half, const double *x,
                 const int32_t *cell_start, const BuildOut &o, int32_t *max_count,
                 hipStream_t st) {
  const int ns = build_split(g.ncells);
  if (MODE != kTiled || o.maxn <= kRowCap) {
    if (half)
      launch_shape<true, kSlots, kRowCap, MODE>(g, b, rl2, x, cell_start, o, max_count, ns, st);
    else
      launch_shape<false, kSlots, kRowCap, MODE>(g, b, rl2, x, cell_start, o, max_count, ns, st);
  } else {
    if (half)
      launch_shape<true, kDenseSlots, kDenseRowCap, MODE>(g, b, rl2, x, cell_start, o, max_count,
                                                          ns, st);
    else
      launch_shape<false, kDenseSlots, kDenseRowCap, MODE>(g, b, rl2, x, cell_start, o, max_count,
                                                           ns, st);
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
