// Compressed (CSR) copy of a tiled neighbor list, gfx950.  Paper: Cabana
// "Neighbor List Creation" -- lists are stored either compressed (row offsets
// plus one flat array of neighbor indices) or dense (fixed row capacity).
//
// Three launches: per-chunk sums of the row counts, one scan of the chunk sums,
// then per chunk a local scan that yields offsets[i] and copies every row from
// its tile (entry k of atom i at nbr[((i/64) maxn + k) 64 + i%64]) to
// csr[offsets[i] + k].  Integer sums: the result does not depend on the order.
#include "common.h"

namespace ljmd {

namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 4;
constexpr int kChunk = kThreads * kPerThread;  // atoms per chunk (one block)

// chunk_sum[c] = sum of min(nnbr, maxn) over atoms [c kChunk, (c+1) kChunk)
__global__ __launch_bounds__(kThreads) void k_chunk_sums(int64_t n, const int32_t *__restrict__ nnbr,
                                                         int32_t maxn,
                                                         int64_t *__restrict__ chunk_sum) {
  __shared__ int64_t red[kThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  int64_t s = 0;
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int64_t i = base + (int64_t)q * kThreads + threadIdx.x;
    if (i < n) s += nnbr[i] < maxn ? nnbr[i] : maxn;
  }
  for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < kThreads / kWave; ++w) t += red[w];
    chunk_sum[blockIdx.x] = t;
  }
}

// In place: chunk_sum[c] <- sum of chunk_sum[0 .. c) (exclusive), one block,
// kThreads values per pass with a running carry; total[0] = sum of all.
__global__ __launch_bounds__(kThreads) void k_scan_chunks(int64_t nchunks, int64_t *__restrict__ cs,
                                                          int64_t *__restrict__ total) {
  __shared__ int64_t buf[kThreads];
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < nchunks; c0 += kThreads) {
    const int64_t c = c0 + threadIdx.x;
    const int64_t v = c < nchunks ? cs[c] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {  // inclusive Hillis-Steele scan
      const int64_t o = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
      __syncthreads();
      buf[threadIdx.x] += o;
      __syncthreads();
    }
    if (c < nchunks) cs[c] = carry + buf[threadIdx.x] - v;
    carry += buf[kThreads - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

// offsets[i] for the chunk's atoms (local exclusive scan + chunk prefix), then
// each thread copies its atoms' rows.
__global__ __launch_bounds__(kThreads) void k_fill(int64_t n, const int32_t *__restrict__ nbr,
                                                   const int32_t *__restrict__ nnbr, int32_t maxn,
                                                   const int64_t *__restrict__ chunk_prefix,
                                                   int64_t *__restrict__ offsets,
                                                   int32_t *__restrict__ csr, int64_t cap) {
  __shared__ int64_t buf[kThreads];
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  // thread t owns atoms base + t kPerThread .. + kPerThread - 1 (contiguous)
  int32_t cnt[kPerThread];
  int64_t own = 0;
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int64_t i = base + (int64_t)threadIdx.x * kPerThread + q;
    cnt[q] = i < n ? (nnbr[i] < maxn ? nnbr[i] : maxn) : 0;
    own += cnt[q];
  }
  buf[threadIdx.x] = own;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    const int64_t o = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
    __syncthreads();
    buf[threadIdx.x] += o;
    __syncthreads();
  }
  int64_t pos = chunk_prefix[blockIdx.x] + buf[threadIdx.x] - own;
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int64_t i = base + (int64_t)threadIdx.x * kPerThread + q;
    if (i < n) {
      offsets[i] = pos;
      const int32_t *row = nbr + (i >> 6) * (int64_t)maxn * kWave + (i & (kWave - 1));
      for (int32_t k = 0; k < cnt[q]; ++k)
        if (pos + k < cap) csr[pos + k] = row[(int64_t)k * kWave];
      pos += cnt[q];
    }
  }
}

// offsets[i] = sum of counts over atoms before i, per chunk (local exclusive scan
// plus the chunk's prefix).
__global__ __launch_bounds__(kThreads) void k_offsets(int64_t n, const int32_t *__restrict__ cnt,
                                                      const int64_t *__restrict__ chunk_prefix,
                                                      int64_t *__restrict__ offsets) {
  __shared__ int64_t buf[kThreads];
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  int32_t c[kPerThread];
  int64_t own = 0;
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int64_t i = base + (int64_t)threadIdx.x * kPerThread + q;
    c[q] = i < n ? cnt[i] : 0;
    own += c[q];
  }
  buf[threadIdx.x] = own;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    const int64_t o = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
    __syncthreads();
    buf[threadIdx.x] += o;
    __syncthreads();
  }
  int64_t pos = chunk_prefix[blockIdx.x] + buf[threadIdx.x] - own;
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int64_t i = base + (int64_t)threadIdx.x * kPerThread + q;
    if (i < n) offsets[i] = pos;
    pos += c[q];
  }
}

int64_t nchunks(int64_t n) { return n > 0 ? (n + kChunk - 1) / kChunk : 1; }

}  // namespace

// Exclusive scan of row lengths: offsets[i] (i < n) and offsets[n] = the total.
int launch_offsets(int64_t n, const int32_t *counts, int64_t *offsets, void *ws, hipStream_t st) {
  const int64_t nc = nchunks(n);
  int64_t *chunk = (int64_t *)ws;
  if (n > 0) {
    k_chunk_sums<<<(unsigned)nc, kThreads, 0, st>>>(n, counts, INT32_MAX, chunk);
    k_scan_chunks<<<1, kThreads, 0, st>>>(nc, chunk, offsets + n);
    k_offsets<<<(unsigned)nc, kThreads, 0, st>>>(n, counts, chunk, offsets);
  } else {
    k_scan_chunks<<<1, kThreads, 0, st>>>(0, chunk, offsets);
  }
  return check_launch("row offsets");
}

size_t csr_workspace(int64_t n) { return (size_t)(nchunks(n) + 1) * sizeof(int64_t); }

int launch_list_to_csr(int64_t n, const int32_t *nbr, const int32_t *nnbr, int32_t maxn,
                       int64_t *offsets, int32_t *csr, int64_t cap, void *ws, hipStream_t st) {
  const int64_t nc = nchunks(n);
  int64_t *chunk = (int64_t *)ws;
  if (n > 0) {
    k_chunk_sums<<<(unsigned)nc, kThreads, 0, st>>>(n, nnbr, maxn, chunk);
    k_scan_chunks<<<1, kThreads, 0, st>>>(nc, chunk, offsets + n);
    k_fill<<<(unsigned)nc, kThreads, 0, st>>>(n, nbr, nnbr, maxn, chunk, offsets, csr, cap);
  } else {
    k_scan_chunks<<<1, kThreads, 0, st>>>(0, chunk, offsets);
  }
  return check_launch("ljmd_list_to_csr");
}

}  // namespace ljmd
