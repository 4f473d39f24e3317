// Marker binning: the partition of markers among grid cells (Sec. 3.3).
//
// The paper partitions fluid and material grids so that no two processors
// touch the same data.  Here the partition is a cell key per marker: cells
// are grouped in 8^3 tiles and key = tile * 512 + cell within the tile, with
// c = floor(X/h) wrapped into [0, n); a stable LSD radix sort orders marker
// ids by key.  Sorting makes the markers of one tile a contiguous run of the
// sorted order (tile_start gives each tile's range), ordered by cell.  The
// runs are then cut into work items (see item_range), which the spreading
// and interpolation kernels take.  Everything here is
// integer work and bit-exact.
#include "dev_common.h"
#include "ib_internal.h"

namespace ib {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;    // 2048 keys per block: several blocks per CU hide the scatter's latency
constexpr int kSortChunk = kSortThreads * kSortItems;

// A block owns a contiguous chunk of kSortChunk keys; within it each wave owns
// a contiguous quarter (kSortItems rounds of 64).  Digit counts per block,
// layout hist[digit * nblk + block].
constexpr int kWaveKeys = 64 * kSortItems;

// Keys of the sort blocks' markers, with the first pass's digit counts of
// each block (the counts of the later passes depend on the order the earlier
// passes produce).
__global__ __launch_bounds__(256) void k_keys_hist(const double *__restrict__ X, const double *__restrict__ Y,
                                                   int64_t M, double h, int n,
                                                   int nz, int log2nt, int radix, uint32_t *__restrict__ keys,
                                                   int32_t *__restrict__ vals, uint32_t *__restrict__ hist,
                                                   int nblk) {
  __shared__ uint32_t cnt[256];
  for (int i = threadIdx.x; i < 256; i += kSortThreads) cnt[i] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortChunk;
  for (int it = 0; it < kSortItems; it++) {
    const int64_t q = base + (int64_t)it * kSortThreads + threadIdx.x;
    if (q < M) {
      int c[3];
      for (int d = 0; d < 3; d++) {
        // the position: X, or Y + D with displacements as the state
        const double s = (Y ? Y[d * M + q] + X[d * M + q] : X[d * M + q]) / h;
        int64_t cd = isfinite(s) ? (int64_t)floor(s) : 0;
        c[d] = d == 2 ? wrap_cell(cd, nz) : (int)(cd & (int64_t)(n - 1));   // periodic wrap (n a power of two)
      }
      const uint32_t k = cell_key(c[0], c[1], c[2], log2nt);
      keys[q] = k;
      vals[q] = (int32_t)q;
      atomicAdd(&cnt[k & (uint32_t)(radix - 1)], 1u);
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < radix; d += kSortThreads) hist[(int64_t)d * nblk + blockIdx.x] = cnt[d];
}

__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t *__restrict__ keys, int64_t M,
                                                    int shift, int radix, uint32_t *__restrict__ hist, int nblk) {
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

__device__ __forceinline__ void wave_sync_b() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Stable scatter with a block-local reorder.  Each wave ranks its quarter
// round by round (in key order) with ballots that find the lanes holding the
// same digit, keeping a running count per digit in its own LDS row; the
// block then places its keys in LDS in (digit, original order) and writes
// each digit's run contiguously to its global position.  The last pass also
// records each marker's sorted position (inv).
__global__ __launch_bounds__(256) void k_radix_scatter(const uint32_t *__restrict__ kin,
                                                       const int32_t *__restrict__ vin,
                                                       uint32_t *__restrict__ kout,
                                                       int32_t *__restrict__ vout, int64_t M, int shift,
                                                       int bits, const uint32_t *__restrict__ hist,
                                                       const uint32_t *__restrict__ dtot, int nblk,
                                                       int32_t *__restrict__ inv) {
  const int R = 1 << bits;
  __shared__ uint32_t run[4][256];     // per wave: running count, then the wave's offset within the digit
  __shared__ uint32_t lstart[256];     // block-local start of each digit
  __shared__ uint32_t gstart[256];     // global start of each digit's run of this block
  __shared__ uint32_t sk[kSortChunk];
  __shared__ int32_t sv[kSortChunk];
  __shared__ uint32_t sh[4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int d = lane; d < 256; d += 64) run[w][d] = 0;
  wave_sync_b();
  const uint64_t lt = lanemask_lt();
  const int64_t base = (int64_t)blockIdx.x * kSortChunk + (int64_t)w * kWaveKeys;
  uint32_t key[kSortItems], rk[kSortItems];
  int32_t val[kSortItems];
#pragma unroll
  for (int it = 0; it < kSortItems; it++) {
    const int64_t i = base + (int64_t)it * 64 + lane;
    key[it] = i < M ? kin[i] : 0xFFFFFFFFu;
    val[it] = i < M ? vin[i] : 0;
  }
#pragma unroll
  for (int it = 0; it < kSortItems; it++) {
    const bool valid = base + (int64_t)it * 64 + lane < M;
    const uint32_t d = (key[it] >> shift) & (uint32_t)(R - 1);
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; b++) {
      const uint64_t bb = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? bb : ~bb;
    }
    rk[it] = valid ? run[w][d] + (uint32_t)__popcll(peers & lt) : 0u;
    wave_sync_b();
    // the last lane of each digit group advances that digit's count
    if (valid && (peers >> lane) == 1ull) run[w][d] += (uint32_t)__popcll(peers);
    wave_sync_b();
  }
  __syncthreads();
  // per digit: block count, offsets of the waves, block-local and global starts
  {
    const int d = tid;
    uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    if (d < R) {
      c0 = run[0][d];
      c1 = run[1][d];
      c2 = run[2][d];
      c3 = run[3][d];
    }
    uint32_t tot;
    const uint32_t ls = block_excl_scan256(c0 + c1 + c2 + c3, sh, &tot);
    uint32_t db;
    const uint32_t dex = block_excl_scan256(d < R ? dtot[d] : 0u, sh, &tot);
    db = dex + (d < R ? hist[(int64_t)d * nblk + blockIdx.x] : 0u);
    lstart[d] = ls;
    gstart[d] = db;
    run[0][d] = ls;
    run[1][d] = ls + c0;
    run[2][d] = ls + c0 + c1;
    run[3][d] = ls + c0 + c1 + c2;
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kSortItems; it++) {
    const bool valid = base + (int64_t)it * 64 + lane < M;
    if (valid) {
      const uint32_t d = (key[it] >> shift) & (uint32_t)(R - 1);
      const uint32_t lp = run[w][d] + rk[it];
      sk[lp] = key[it];
      sv[lp] = val[it];
    }
  }
  __syncthreads();
  const int64_t cnt = min((int64_t)kSortChunk, M - (int64_t)blockIdx.x * kSortChunk);
  for (int i = tid; i < cnt; i += kSortThreads) {
    const uint32_t k = sk[i];
    const uint32_t d = (k >> shift) & (uint32_t)(R - 1);
    const uint32_t pos = gstart[d] + (uint32_t)i - lstart[d];
    kout[pos] = k;
    vout[pos] = sv[i];
    if (inv) inv[sv[i]] = (int32_t)pos;
  }
}

// tile_start[t] = first sorted position whose key is >= t * 512, t in [0, ntiles].
__global__ __launch_bounds__(256) void k_tile_start(const uint32_t *__restrict__ keys, int64_t M, int64_t ntiles,
                                                    int32_t *__restrict__ tile_start) {
  const int64_t t = gtid();
  if (t > ntiles) return;
  const uint64_t target = (uint64_t)t << 9;
  int64_t lo = 0, hi = M;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((uint64_t)keys[mid] < target) lo = mid + 1;
    else hi = mid;
  }
  tile_start[t] = (int32_t)lo;
}

// ---------------------------------------------------------- work list ----
// Items per tile: one per chunk that its markers [ts, te) meet (see
// item_range).  Tiles with more
// than one item ("split") are listed for the reduction of their halos, and
// tiles that the spread force reaches (some tile among the 3^3 around them,
// itself included, has markers: "touched") for the gather.  All three are
// numbered by exclusive scans over the tiles in three launches: per-block
// scans of 1024 tiles, a scan of the block totals, and the writes (tile_nit,
// tile_item0, item_tile, split_list, touch_list, tile_touch).
__device__ __forceinline__ int3 tile_items(const int32_t *tile_start, int64_t t, int64_t ntiles, int log2nt,
                                           int ntz, int chunk) {
  if (t >= ntiles) return make_int3(0, 0, 0);
  const int ts = tile_start[t], te = tile_start[t + 1];
  const int it = te > ts ? (te - 1) / chunk - ts / chunk + 1 : 0;
  const int tmask = (1 << log2nt) - 1;
  const int T1 = (int)(t & tmask), T2 = (int)((t >> log2nt) & tmask), T3 = (int)(t >> (2 * log2nt));
  int touched = 0;
#pragma unroll
  for (int d = 0; d < 27; d++) {     // all 54 loads independent
    const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
    const int t2 = (((((T3 + dz + ntz) % ntz) << log2nt) | ((T2 + dy) & tmask)) << log2nt) | ((T1 + dx) & tmask);
    touched |= tile_start[t2 + 1] > tile_start[t2];
  }
  return make_int3(it, it > 1 ? 1 : 0, touched);
}

// Exclusive scan of three values per thread over a 1024-thread block.
__device__ __forceinline__ int3 scan1024(int3 v, int3 *wsum, int3 *total) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int3 incl = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int x = __shfl_up(incl.x, o, 64), y = __shfl_up(incl.y, o, 64), z = __shfl_up(incl.z, o, 64);
    if (lane >= o) {
      incl.x += x;
      incl.y += y;
      incl.z += z;
    }
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int3 wb = make_int3(0, 0, 0), tot = make_int3(0, 0, 0);
  for (int i = 0; i < 16; i++) {
    if (i < w) {
      wb.x += wsum[i].x;
      wb.y += wsum[i].y;
      wb.z += wsum[i].z;
    }
    tot.x += wsum[i].x;
    tot.y += wsum[i].y;
    tot.z += wsum[i].z;
  }
  __syncthreads();
  *total = tot;
  return make_int3(wb.x + incl.x - v.x, wb.y + incl.y - v.y, wb.z + incl.z - v.z);
}

// Also stores each tile's item count and touched flag for the write pass.
__global__ __launch_bounds__(1024) void k_item_scan_blocks(const int32_t *__restrict__ tile_start, int64_t ntiles,
                                                           int log2nt, int ntz, int chunk,
                                                           int3 *__restrict__ block_tot,
                                                           int32_t *__restrict__ tile_nit,
                                                           int32_t *__restrict__ tile_touch,
                                                           uint32_t *__restrict__ touch_bits) {
  __shared__ int3 wsum[16];
  const int64_t t = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  const int3 v = tile_items(tile_start, t, ntiles, log2nt, ntz, chunk);
  if (t < ntiles) {
    tile_nit[t] = v.x;
    tile_touch[t] = v.z;
  }
  // the same flags as bits: a wave's 64 consecutive tiles are two words
  const uint64_t bits = __ballot(t < ntiles && v.z != 0);
  if ((threadIdx.x & 63) == 0) {
    const int64_t w0 = t >> 5, nw = (ntiles + 31) >> 5;
    if (w0 < nw) touch_bits[w0] = (uint32_t)bits;
    if (w0 + 1 < nw) touch_bits[w0 + 1] = (uint32_t)(bits >> 32);
  }
  int3 tot;
  (void)scan1024(v, wsum, &tot);
  if (threadIdx.x == 0) block_tot[blockIdx.x] = tot;
}

// counts[0] = work items, counts[1] = split tiles, counts[2] = touched tiles;
// chunk_item0[nchunks] = work items
__global__ __launch_bounds__(1024) void k_item_scan_top(int3 *__restrict__ block_tot, int nblk,
                                                        int32_t *__restrict__ counts, int nchunks,
                                                        int32_t *__restrict__ chunk_item0) {
  __shared__ int3 wsum[16];
  int3 carry = make_int3(0, 0, 0);
  for (int base = 0; base < nblk; base += 1024) {
    const int b = base + threadIdx.x;
    int3 tot;
    const int3 off = scan1024(b < nblk ? block_tot[b] : make_int3(0, 0, 0), wsum, &tot);
    if (b < nblk) block_tot[b] = make_int3(carry.x + off.x, carry.y + off.y, carry.z + off.z);
    carry.x += tot.x;
    carry.y += tot.y;
    carry.z += tot.z;
  }
  if (threadIdx.x == 0) {
    counts[0] = carry.x;
    counts[1] = carry.y;
    counts[2] = carry.z;
    chunk_item0[nchunks] = carry.x;
  }
}

__global__ __launch_bounds__(1024) void k_item_scan_write(const int32_t *__restrict__ tile_nit, int64_t ntiles,
                                                          const int32_t *__restrict__ tile_touch,
                                                          const int32_t *__restrict__ tile_start, int chunk,
                                                          const int3 *__restrict__ block_off,
                                                          int32_t *__restrict__ tile_item0,
                                                          int32_t *__restrict__ item_tile,
                                                          int32_t *__restrict__ split_list,
                                                          int32_t *__restrict__ touch_list,
                                                          int32_t *__restrict__ chunk_item0) {
  __shared__ int3 wsum[16];
  const int64_t t = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  int3 v = make_int3(0, 0, 0);
  if (t < ntiles) {
    v.x = tile_nit[t];
    v.y = v.x > 1 ? 1 : 0;
    v.z = tile_touch[t];
  }
  int3 tot;
  const int3 off = scan1024(v, wsum, &tot);
  if (t < ntiles) {
    const int3 bo = block_off[blockIdx.x];
    const int i0 = bo.x + off.x;
    tile_item0[t] = i0;
    const int ts = tile_start[t], c0 = ts / chunk;
    for (int j = 0; j < v.x; j++) {
      item_tile[i0 + j] = (int32_t)t;
      if (j > 0 || ts == c0 * chunk) chunk_item0[c0 + j] = i0 + j;   // the item starts chunk c0 + j
    }
    if (v.y) split_list[bo.y + off.y] = (int32_t)t;
    if (v.z) touch_list[bo.z + off.z] = (int32_t)t;
  }
}

hipError_t launch_bin(ib_ctx *c, const double *X) {
  PhaseScope ps(c, PH_BIN);
  const int64_t M = c->M;
  Workspace &ws = c->ws;
  if (M > 0) {
    int cur = 0;
    const int bits = c->digit_bits, R = 1 << bits;
    const int nblk = (int)((M + kSortChunk - 1) / kSortChunk);
    hipLaunchKernelGGL(k_keys_hist, dim3(nblk), dim3(kSortThreads), 0, c->stream, X,
                       c->mat.disp ? c->mat.X_ref : nullptr, M, c->h, c->n, c->nz, c->log2nt, R,
                       ws.keys[0], ws.vals[0], ws.hist, nblk);
    for (int pass = 0; pass < c->sort_passes; pass++) {
      const int shift = pass * bits;
      if (pass > 0)
        hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kSortThreads), 0, c->stream, ws.keys[cur], M,
                           shift, R, ws.hist, nblk);
      hipLaunchKernelGGL(k_radix_scan_digit, dim3(R), dim3(kSortThreads), 0, c->stream, ws.hist, nblk,
                         ws.hist + (int64_t)R * nblk);
      hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(kSortThreads), 0, c->stream, ws.keys[cur],
                         ws.vals[cur], ws.keys[cur ^ 1], ws.vals[cur ^ 1], M, shift, bits, ws.hist,
                         ws.hist + (int64_t)R * nblk, nblk, pass == c->sort_passes - 1 ? ws.inv : nullptr);
      cur ^= 1;
    }
    c->sorted_buf = cur;
  } else {
    c->sorted_buf = 0;
  }
  const int64_t nt = c->ntiles;
  hipLaunchKernelGGL(k_tile_start, dim3((unsigned)((nt + 1 + 255) / 256)), dim3(256), 0, c->stream,
                     ws.keys[c->sorted_buf], M, nt, ws.tile_start);
  const int nsb = (int)((nt + 1023) / 1024);
  int3 *tmp = (int3 *)ws.scan_tmp;
  hipLaunchKernelGGL(k_item_scan_blocks, dim3(nsb), dim3(1024), 0, c->stream, ws.tile_start, nt, c->log2nt,
                     c->ntz, c->chunk, tmp, ws.tile_nit, ws.tile_touch, ws.touch_bits);
  hipLaunchKernelGGL(k_item_scan_top, dim3(1), dim3(1024), 0, c->stream, tmp, nsb, ws.nitems, c->nchunks,
                     ws.chunk_item0);
  hipLaunchKernelGGL(k_item_scan_write, dim3(nsb), dim3(1024), 0, c->stream, ws.tile_nit, nt, ws.tile_touch,
                     ws.tile_start, c->chunk, tmp, ws.tile_item0, ws.item_tile, ws.split_list, ws.touch_list,
                     ws.chunk_item0);
  return hipGetLastError();
}

int sort_hist_words(int64_t M, int digit_bits) {
  const int64_t nblk = (M + kSortChunk - 1) / kSortChunk;
  return (int)((int64_t)(1 << digit_bits) * (nblk + 1));
}

}  // namespace ib
