// Marker binning: the partition of markers among grid cells (Sec. 3.3).
//
// The paper partitions fluid and material grids so that no two processors
// touch the same data.  Here the partition is a cell key per marker,
// key = (c3*n + c2)*n + c1 with c = floor(X/h) wrapped into [0, n), and a
// stable LSD radix sort of marker ids by key.  Sorting makes the markers of
// one grid row (fixed c2, c3) contiguous and ordered by c1, so the spreading
// kernel can gather a tile's markers row by row with two binary searches per
// row (row_start gives each row's range).  Everything here is integer work
// and bit-exact.
#include "dev_common.h"
#include "ib_internal.h"

namespace ib {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortChunk = kSortThreads * kSortItems;

__global__ __launch_bounds__(256) void k_keys(const double *__restrict__ X, int64_t M, double h,
                                              int n, int log2n, uint32_t *__restrict__ keys,
                                              int32_t *__restrict__ vals) {
  const int64_t q = gtid();
  if (q >= M) return;
  uint32_t key = 0;
  for (int d = 2; d >= 0; d--) {
    const double s = X[d * M + q] / h;
    int64_t c = isfinite(s) ? (int64_t)floor(s) : 0;
    c &= (int64_t)(n - 1);                 // periodic wrap (n is a power of two)
    key = (key << log2n) | (uint32_t)c;
  }
  keys[q] = key;
  vals[q] = (int32_t)q;
}

// Per-block digit histogram, layout hist[digit * nblk + block].
__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t *__restrict__ keys, int64_t M,
                                                    int shift, int radix, uint32_t *__restrict__ hist,
                                                    int nblk) {
  __shared__ uint32_t cnt[256];
  for (int i = threadIdx.x; i < 256; i += kSortThreads) cnt[i] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortChunk;
  for (int it = 0; it < kSortItems; it++) {
    const int64_t i = base + (int64_t)it * kSortThreads + threadIdx.x;
    if (i < M) atomicAdd(&cnt[(keys[i] >> shift) & (uint32_t)(radix - 1)], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < radix; d += kSortThreads) hist[(int64_t)d * nblk + blockIdx.x] = cnt[d];
}

// Block-wide exclusive scan of one value per thread (256 threads); returns the
// exclusive prefix and writes the block total to *total.
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t v, uint32_t *sh, uint32_t *total) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  uint32_t incl = v;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) sh[w] = incl;
  __syncthreads();
  uint32_t wbase = 0, tot = 0;
  for (int i = 0; i < 4; i++) {
    if (i < w) wbase += sh[i];
    tot += sh[i];
  }
  __syncthreads();
  *total = tot;
  return wbase + incl - v;
}

// One block per digit: exclusive scan of that digit's per-block counts (in
// place) and the digit's total.
__global__ __launch_bounds__(256) void k_radix_scan_digit(uint32_t *__restrict__ hist, int nblk,
                                                          uint32_t *__restrict__ dtot) {
  __shared__ uint32_t sh[4];
  uint32_t *row = hist + (int64_t)blockIdx.x * nblk;
  uint32_t carry = 0;
  for (int base = 0; base < nblk; base += kSortThreads) {
    const int i = base + threadIdx.x;
    const uint32_t v = i < nblk ? row[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan256(v, sh, &tot);
    if (i < nblk) row[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) dtot[blockIdx.x] = carry;
}

// Stable scatter: items are ranked in their original order (round, wave, lane)
// using wave ballots to find lanes holding the same digit.
__global__ __launch_bounds__(256) void k_radix_scatter(const uint32_t *__restrict__ kin,
                                                       const int32_t *__restrict__ vin,
                                                       uint32_t *__restrict__ kout,
                                                       int32_t *__restrict__ vout, int64_t M, int shift,
                                                       int bits, const uint32_t *__restrict__ hist,
                                                       const uint32_t *__restrict__ dtot, int nblk) {
  const int R = 1 << bits;
  __shared__ uint32_t dbase[256];
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[4][256];
  __shared__ uint32_t sh[4];
  const int tid = threadIdx.x, w = tid >> 6;
  {
    const uint32_t v = tid < R ? dtot[tid] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan256(v, sh, &tot);
    dbase[tid] = tid < R ? ex + hist[(int64_t)tid * nblk + blockIdx.x] : 0u;
    run[tid] = 0;
    for (int i = 0; i < 4; i++) wcnt[i][tid] = 0;
  }
  __syncthreads();
  const uint64_t lt = lanemask_lt();
  const int64_t base = (int64_t)blockIdx.x * kSortChunk;
  for (int it = 0; it < kSortItems; it++) {
    const int64_t i = base + (int64_t)it * kSortThreads + tid;
    const bool valid = i < M;
    const uint32_t key = valid ? kin[i] : 0u;
    const int32_t val = valid ? vin[i] : 0;
    const uint32_t d = (key >> shift) & (uint32_t)(R - 1);
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; b++) {
      const uint64_t bb = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? bb : ~bb;
    }
    const uint32_t rank = __popcll(peers & lt);
    if (valid && (peers & lt) == 0) wcnt[w][d] = __popcll(peers);
    __syncthreads();
    uint32_t pos = 0;
    if (valid) {
      uint32_t off = run[d];
      for (int ww = 0; ww < w; ww++) off += wcnt[ww][d];
      pos = dbase[d] + off + rank;
    }
    __syncthreads();
    if (tid < R) {
      run[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
      wcnt[0][tid] = wcnt[1][tid] = wcnt[2][tid] = wcnt[3][tid] = 0;
    }
    __syncthreads();
    if (valid) {
      kout[pos] = key;
      vout[pos] = val;
    }
  }
}

// row_start[r] = first sorted position whose key is >= r * n, r in [0, n^2].
__global__ __launch_bounds__(256) void k_row_start(const uint32_t *__restrict__ keys, int64_t M,
                                                   int log2n, int64_t nrows, int32_t *__restrict__ row_start) {
  const int64_t r = gtid();
  if (r > nrows) return;
  const uint64_t target = (uint64_t)r << log2n;
  int64_t lo = 0, hi = M;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((uint64_t)keys[mid] < target) lo = mid + 1;
    else hi = mid;
  }
  row_start[r] = (int32_t)lo;
}

hipError_t launch_bin(ib_ctx *c, const double *X) {
  PhaseScope ps(c, PH_BIN);
  const int64_t M = c->M;
  Workspace &ws = c->ws;
  const int nrows = c->n * c->n;
  if (M > 0) {
    const int gb = (int)((M + 255) / 256);
    hipLaunchKernelGGL(k_keys, dim3(gb), dim3(256), 0, c->stream, X, M, c->h, c->n, c->log2n,
                       ws.keys[0], ws.vals[0]);
    int cur = 0;
    const int bits = c->digit_bits, R = 1 << bits;
    const int nblk = (int)((M + kSortChunk - 1) / kSortChunk);
    for (int pass = 0; pass < c->sort_passes; pass++) {
      const int shift = pass * bits;
      hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kSortThreads), 0, c->stream, ws.keys[cur], M,
                         shift, R, ws.hist, nblk);
      hipLaunchKernelGGL(k_radix_scan_digit, dim3(R), dim3(kSortThreads), 0, c->stream, ws.hist, nblk,
                         ws.hist + (int64_t)R * nblk);
      hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(kSortThreads), 0, c->stream, ws.keys[cur],
                         ws.vals[cur], ws.keys[cur ^ 1], ws.vals[cur ^ 1], M, shift, bits, ws.hist,
                         ws.hist + (int64_t)R * nblk, nblk);
      cur ^= 1;
    }
    c->sorted_buf = cur;
  } else {
    c->sorted_buf = 0;
  }
  hipLaunchKernelGGL(k_row_start, dim3((nrows + 1 + 255) / 256), dim3(256), 0, c->stream,
                     ws.keys[c->sorted_buf], M, c->log2n, (int64_t)nrows, ws.row_start);
  return hipGetLastError();
}

int sort_hist_words(int64_t M, int digit_bits) {
  const int64_t nblk = (M + kSortChunk - 1) / kSortChunk;
  return (int)((int64_t)(1 << digit_bits) * (nblk + 1));
}

}  // namespace ib
