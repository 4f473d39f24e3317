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
//
// Update of the last partition.  keys_id holds each marker's cell key from
// the last binning.  The keys pass compares every new key with the stored one
// and lists the markers whose cell changed ("movers"; markers of the method
// move a small fraction of a cell per step, so there are few).  With no
// movers the sorted order, tile ranges and work list of the last binning are
// exactly those of the new keys and stay in place.  With up to kMoverCap
// movers the new order is the merge of the markers that stayed (in their old
// order) with the movers sorted by (new key, id): one block sorts the movers
// and finds where each lands, and a pass over the range of sorted positions
// between the first and last place a mover leaves or takes rewrites that
// range; the work list is rebuilt only if some mover changed tile.  Both
// orders are sorted by (key, id), so the result is bitwise that of the full
// sort, which runs instead on the first binning, with more movers, or on
// request.  The choice is made on the device (bin_state), so no call waits
// for the host: kernels of the path not taken return at once.
#include <algorithm>

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

// A plain load: the words are written by earlier kernels on the stream (or,
// for BS_FULL, BS_NMOV and BS_TILES, only raised within k_keys, which reads
// BS_FULL once at the start), so a uniform scalar load suffices and lets a
// kernel of the path not taken exit early.
__device__ __forceinline__ uint32_t bs_word(const uint32_t *st, int i) { return st[i]; }
// the full sort is off this call
__device__ __forceinline__ bool full_off(const uint32_t *st) { return bs_word(st, BS_FULL) == 0u; }
// the tile ranges and work list stand
__device__ __forceinline__ bool worklist_off(const uint32_t *st) {
  return (bs_word(st, BS_FULL) | bs_word(st, BS_TILES)) == 0u;
}
// no incremental update this call (full sort, or no movers)
__device__ __forceinline__ bool update_off(const uint32_t *st) {
  return bs_word(st, BS_FULL) != 0u || bs_word(st, BS_NMOV) == 0u;
}

// Cell keys by marker id, compared with the stored ones: movers are listed
// with their new key and old sorted position (block-wide counts, one global
// atomic per block; their order in the list is irrelevant, the list is
// sorted later), a mover that changed tile sets BS_TILES, more than
// kMoverCap movers or rebuild set BS_FULL.  With BS_FULL already set (the
// first binning) nothing is listed.
__global__ __launch_bounds__(256) void k_keys(const double *__restrict__ X, const double *__restrict__ Y, int64_t M,
                                              double h, int n, int nz, int log2nt, uint32_t *__restrict__ keys_id,
                                              const int32_t *__restrict__ inv, int rebuild,
                                              uint32_t *__restrict__ st, int32_t *__restrict__ mov) {
  __shared__ uint32_t nloc, base;
  if (threadIdx.x == 0) nloc = 0;
  __syncthreads();
  const bool listing = !rebuild && full_off(st);
  const int64_t b0 = (int64_t)blockIdx.x * kSortChunk;
  int slot[kSortItems];
  uint32_t knew[kSortItems];
  bool tile_moved = false;
#pragma unroll
  for (int it = 0; it < kSortItems; it++) {
    const int64_t q = b0 + (int64_t)it * kSortThreads + threadIdx.x;
    slot[it] = -1;
    if (q < M) {
      int c[3];
      for (int d = 0; d < 3; d++) {
        // the position: X, or Y + D with displacements as the state
        const double s = (Y ? Y[d * M + q] + X[d * M + q] : X[d * M + q]) / h;
        int64_t cd = isfinite(s) ? (int64_t)floor(s) : 0;
        c[d] = d == 2 ? wrap_cell(cd, nz) : (int)(cd & (int64_t)(n - 1));   // periodic wrap (n a power of two)
      }
      const uint32_t k = cell_key(c[0], c[1], c[2], log2nt), ko = keys_id[q];
      keys_id[q] = k;
      knew[it] = k;
      if (k != ko) {
        tile_moved |= (k >> 9) != (ko >> 9);
        if (listing) slot[it] = (int)atomicAdd(&nloc, 1u);
      }
    }
  }
  const bool any_tile = __syncthreads_or(tile_moved) != 0;
  if (threadIdx.x == 0) {
    base = listing && nloc > 0 ? atomicAdd(&st[BS_NMOV], nloc) : 0u;
    if (any_tile) st[BS_TILES] = 1u;
    if (rebuild && blockIdx.x == 0) st[BS_FULL] = 1u;
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kSortItems; it++) {
    if (slot[it] >= 0) {
      const uint32_t j = base + (uint32_t)slot[it];
      const int64_t q = b0 + (int64_t)it * kSortThreads + threadIdx.x;
      if (j < (uint32_t)kMoverCap) {
        mov[MV_Q * kMoverCap + j] = (int32_t)q;
        mov[MV_KEY * kMoverCap + j] = (int32_t)knew[it];
        mov[MV_POS * kMoverCap + j] = inv[q];
      } else {
        st[BS_FULL] = 1u;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t *__restrict__ keys, int64_t M,
                                                    int shift, int radix, uint32_t *__restrict__ hist, int nblk,
                                                    const uint32_t *__restrict__ bin_state) {
  if (full_off(bin_state)) return;
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
                                                          uint32_t *__restrict__ dtot,
                                                          const uint32_t *__restrict__ bin_state) {
  if (full_off(bin_state)) return;
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
// records each marker's sorted position (inv).  vin null: the values are the
// positions in kin (the marker ids of the first pass).
__global__ __launch_bounds__(256) void k_radix_scatter(const uint32_t *__restrict__ kin,
                                                       const int32_t *__restrict__ vin,
                                                       uint32_t *__restrict__ kout,
                                                       int32_t *__restrict__ vout, int64_t M, int shift,
                                                       int bits, const uint32_t *__restrict__ hist,
                                                       const uint32_t *__restrict__ dtot, int nblk,
                                                       int32_t *__restrict__ inv,
                                                       const uint32_t *__restrict__ bin_state) {
  if (full_off(bin_state)) return;
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
    val[it] = i < M ? (vin ? vin[i] : (int32_t)i) : 0;
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

// tile_start[t] = first sorted position whose key is >= t * 512, t in [0, ntiles]:
// after a full sort by search in the sorted keys; after an update, from the
// last value, plus the movers now in tiles below t, less those that were.
__global__ __launch_bounds__(256) void k_tile_start(const uint32_t *__restrict__ keys, int64_t M, int64_t ntiles,
                                                    int32_t *__restrict__ tile_start,
                                                    const uint32_t *__restrict__ bin_state,
                                                    const int32_t *__restrict__ mov) {
  if (worklist_off(bin_state)) return;
  const int64_t t = gtid();
  if (t > ntiles) return;
  if (bs_word(bin_state, BS_FULL) == 0u) {
    const uint32_t m = bs_word(bin_state, BS_NMOV), tile = (uint32_t)t;
    auto below = [&](const int32_t *k) {   // entries of the ascending keys k[0 .. m) in tiles below t
      uint32_t a = 0, b = m;
      while (a < b) {
        const uint32_t mid = (a + b) >> 1;
        if (((uint32_t)k[mid] >> 9) < tile) a = mid + 1;
        else b = mid;
      }
      return a;
    };
    const uint32_t in_now = below(mov + MS_KEY * kMoverCap), in_was = below(mov + MS_OLDKEY * kMoverCap);
    if (in_now != in_was) tile_start[t] += (int32_t)in_now - (int32_t)in_was;
    return;
  }
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
                                                           uint32_t *__restrict__ touch_bits,
                                                           const uint32_t *__restrict__ bin_state) {
  if (worklist_off(bin_state)) return;
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
                                                        int32_t *__restrict__ chunk_item0,
                                                        const uint32_t *__restrict__ bin_state) {
  if (worklist_off(bin_state)) return;
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
                                                          int32_t *__restrict__ chunk_item0,
                                                          const uint32_t *__restrict__ bin_state) {
  if (worklist_off(bin_state)) return;
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

// ------------------------------------------------- incremental update ----
__device__ __forceinline__ bool pair_less(uint32_t ka, uint32_t va, uint32_t kb, uint32_t vb) {
  return ka < kb || (ka == kb && va < vb);
}

// One block of 1024 threads: sort the movers by (new key, id) and their old
// positions, place each mover (its new position is its rank among the movers
// plus the stayers before it: the old entries before it, found within its
// tile's old range, less the movers among them), and record the range
// [lo, hi] of sorted positions that change.
__global__ __launch_bounds__(1024) void k_bin_fix(const uint32_t *__restrict__ K, const int32_t *__restrict__ V,
                                                  const int32_t *__restrict__ tile_start, uint32_t *__restrict__ st,
                                                  int32_t *__restrict__ mov) {
  if (update_off(st)) return;
  __shared__ uint64_t L[kMoverCap];
  __shared__ uint32_t Po[kMoverCap];
  __shared__ uint32_t lo_s, hi_s;
  const int m = (int)bs_word(st, BS_NMOV), tid = threadIdx.x;   // m <= kMoverCap: more set BS_FULL
  int np2 = 1;
  while (np2 < m) np2 <<= 1;
  for (int j = tid; j < np2; j += 1024) {
    if (j < m) {
      L[j] = ((uint64_t)(uint32_t)mov[MV_KEY * kMoverCap + j] << 32) | (uint32_t)mov[MV_Q * kMoverCap + j];
      Po[j] = (uint32_t)mov[MV_POS * kMoverCap + j];
    } else {
      L[j] = ~0ull;
      Po[j] = ~0u;
    }
  }
  if (tid == 0) {
    lo_s = ~0u;
    hi_s = 0u;
  }
  __syncthreads();
  // bitonic sorts, ascending
  for (int k = 2; k <= np2; k <<= 1)
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      for (int i = tid; i < np2; i += 1024) {
        const int ixj = i ^ jj;
        if (ixj > i) {
          const bool up = (i & k) == 0;
          const uint64_t a = L[i], b = L[ixj];
          if ((a > b) == up) {
            L[i] = b;
            L[ixj] = a;
          }
          const uint32_t pa = Po[i], pb = Po[ixj];
          if ((pa > pb) == up) {
            Po[i] = pb;
            Po[ixj] = pa;
          }
        }
      }
      __syncthreads();
    }
  int32_t *mkey = mov + MS_KEY * kMoverCap, *mval = mov + MS_VAL * kMoverCap, *mnew = mov + MS_NEW * kMoverCap,
          *mold = mov + MS_OLD * kMoverCap, *moldk = mov + MS_OLDKEY * kMoverCap;
  uint32_t lo = ~0u, hi = 0u;
  for (int j = tid; j < m; j += 1024) {
    const uint32_t kq = (uint32_t)(L[j] >> 32), q = (uint32_t)L[j];
    // old entries before (kq, q): all of the earlier tiles, then a search in its tile
    const uint32_t t = kq >> 9;
    uint32_t a = (uint32_t)tile_start[t], b = (uint32_t)tile_start[t + 1];
    while (a < b) {
      const uint32_t mid = (a + b) >> 1;
      if (pair_less(K[mid], (uint32_t)V[mid], kq, q)) a = mid + 1;
      else b = mid;
    }
    // movers among them: old positions below a
    uint32_t x = 0, y = (uint32_t)m;
    while (x < y) {
      const uint32_t mid = (x + y) >> 1;
      if (Po[mid] < a) x = mid + 1;
      else y = mid;
    }
    const uint32_t pn = (uint32_t)j + a - x;
    mkey[j] = (int32_t)kq;
    mval[j] = (int32_t)q;
    mnew[j] = (int32_t)pn;
    mold[j] = (int32_t)Po[j];
    moldk[j] = (int32_t)K[Po[j]];
    lo = min(lo, min(pn, Po[j]));
    hi = max(hi, max(pn, Po[j]));
  }
  atomicMin(&lo_s, lo);
  atomicMax(&hi_s, hi);
  __syncthreads();
  if (tid == 0) {
    st[BS_LO] = lo_s;
    st[BS_HI] = hi_s;
  }
}

// Sorted positions lo .. hi rewritten into (K2, V2): the movers at their new
// places, every other entry p shifted by the movers that leave before it and
// those that land before it.  inv follows every entry that moves.  (Outside
// [lo, hi] nothing moves: no mover lands before an entry below lo, or after
// one above hi.)
__global__ __launch_bounds__(256) void k_bin_merge(const uint32_t *__restrict__ K, const int32_t *__restrict__ V,
                                                   uint32_t *__restrict__ K2, int32_t *__restrict__ V2,
                                                   int32_t *__restrict__ inv, const uint32_t *__restrict__ st,
                                                   const int32_t *__restrict__ mov) {
  if (update_off(st)) return;
  const uint32_t m = bs_word(st, BS_NMOV), lo = bs_word(st, BS_LO), hi = bs_word(st, BS_HI);
  const uint32_t g = blockIdx.x * 256u + threadIdx.x, stride = gridDim.x * 256u;
  const int32_t *mkey = mov + MS_KEY * kMoverCap, *mval = mov + MS_VAL * kMoverCap,
                *mnew = mov + MS_NEW * kMoverCap, *mold = mov + MS_OLD * kMoverCap;
  for (uint32_t j = g; j < m; j += stride) {   // the movers
    const uint32_t pn = (uint32_t)mnew[j];
    K2[pn] = (uint32_t)mkey[j];
    V2[pn] = mval[j];
    inv[mval[j]] = (int32_t)pn;
  }
  for (uint32_t p = lo + g; p <= hi; p += stride) {
    // the entry at old position p: movers leaving before it
    uint32_t x = 0, y = m;
    while (x < y) {
      const uint32_t mid = (x + y) >> 1;
      if ((uint32_t)mold[mid] < p) x = mid + 1;
      else y = mid;
    }
    if (x < m && (uint32_t)mold[x] == p) continue;   // a mover's old place
    const uint32_t k = K[p];
    const int32_t v = V[p];
    // movers landing before it
    uint32_t a = 0, b = m;
    while (a < b) {
      const uint32_t mid = (a + b) >> 1;
      if (pair_less((uint32_t)mkey[mid], (uint32_t)mval[mid], k, (uint32_t)v)) a = mid + 1;
      else b = mid;
    }
    const uint32_t pn = p - x + a;
    K2[pn] = k;
    V2[pn] = v;
    if (pn != p) inv[v] = (int32_t)pn;
  }
}

// The rewritten range back into the sorted buffers.
__global__ __launch_bounds__(256) void k_bin_copyback(uint32_t *__restrict__ K, int32_t *__restrict__ V,
                                                      const uint32_t *__restrict__ K2,
                                                      const int32_t *__restrict__ V2,
                                                      const uint32_t *__restrict__ st) {
  if (update_off(st)) return;
  const uint32_t lo = bs_word(st, BS_LO), hi = bs_word(st, BS_HI);
  for (uint32_t p = lo + blockIdx.x * 256u + threadIdx.x; p <= hi; p += gridDim.x * 256u) {
    K[p] = K2[p];
    V[p] = V2[p];
  }
}

// The partition is current: clear the flags for the next binning.
__global__ void k_bin_end(uint32_t *__restrict__ st) {
  if (threadIdx.x == 0) {
    st[BS_FULL] = 0u;
    st[BS_NMOV] = 0u;
    st[BS_TILES] = 0u;
  }
}

hipError_t launch_bin(ib_ctx *c, const double *X) {
  PhaseScope ps(c, PH_BIN);
  const int64_t M = c->M;
  Workspace &ws = c->ws;
  uint32_t *st = ws.bin_state;
  const uint32_t *cst = st;
  const int sb = c->sorted_buf;   // fixed by the pass count: (sort_passes - 1) & 1
  if (M > 0) {
    const int bits = c->digit_bits, R = 1 << bits;
    const int nblk = (int)((M + kSortChunk - 1) / kSortChunk);
    hipLaunchKernelGGL(k_keys, dim3(nblk), dim3(kSortThreads), 0, c->stream, X,
                       c->mat.disp ? c->mat.X_ref : nullptr, M, c->h, c->n, c->nz, c->log2nt, ws.keys_id,
                       (const int32_t *)ws.inv, c->bin_reuse ? 0 : 1, st, ws.bin_mov);
    // full sort (BS_FULL): pass p reads the keys by marker id (p = 0) or pass
    // p - 1's output, and writes keys/vals[p & 1]; the last pass lands in sb
    for (int pass = 0; pass < c->sort_passes; pass++) {
      const int shift = pass * bits;
      const uint32_t *kin = pass == 0 ? ws.keys_id : ws.keys[(pass - 1) & 1];
      const int32_t *vin = pass == 0 ? nullptr : ws.vals[(pass - 1) & 1];
      hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kSortThreads), 0, c->stream, kin, M, shift, R, ws.hist,
                         nblk, cst);
      hipLaunchKernelGGL(k_radix_scan_digit, dim3(R), dim3(kSortThreads), 0, c->stream, ws.hist, nblk,
                         ws.hist + (int64_t)R * nblk, cst);
      hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(kSortThreads), 0, c->stream, kin, vin,
                         ws.keys[pass & 1], ws.vals[pass & 1], M, shift, bits, ws.hist,
                         ws.hist + (int64_t)R * nblk, nblk, pass == c->sort_passes - 1 ? ws.inv : nullptr, cst);
    }
    // incremental update (movers, no BS_FULL), through the other buffer
    const unsigned pgrid = (unsigned)std::min<int64_t>((M + 255) / 256, 2048);   // grid-stride over [lo, hi]
    hipLaunchKernelGGL(k_bin_fix, dim3(1), dim3(1024), 0, c->stream, (const uint32_t *)ws.keys[sb],
                       (const int32_t *)ws.vals[sb], (const int32_t *)ws.tile_start, st, ws.bin_mov);
    hipLaunchKernelGGL(k_bin_merge, dim3(pgrid), dim3(256), 0, c->stream, (const uint32_t *)ws.keys[sb],
                       (const int32_t *)ws.vals[sb], ws.keys[sb ^ 1], ws.vals[sb ^ 1], ws.inv, cst,
                       (const int32_t *)ws.bin_mov);
    hipLaunchKernelGGL(k_bin_copyback, dim3(pgrid), dim3(256), 0, c->stream, ws.keys[sb], ws.vals[sb],
                       (const uint32_t *)ws.keys[sb ^ 1], (const int32_t *)ws.vals[sb ^ 1], cst);
  }
  // tile ranges and work list (BS_FULL, or a mover changed tile)
  const int64_t nt = c->ntiles;
  hipLaunchKernelGGL(k_tile_start, dim3((unsigned)((nt + 1 + 255) / 256)), dim3(256), 0, c->stream,
                     ws.keys[sb], M, nt, ws.tile_start, cst, (const int32_t *)ws.bin_mov);
  const int nsb = (int)((nt + 1023) / 1024);
  int3 *tmp = (int3 *)ws.scan_tmp;
  hipLaunchKernelGGL(k_item_scan_blocks, dim3(nsb), dim3(1024), 0, c->stream, ws.tile_start, nt, c->log2nt,
                     c->ntz, c->chunk, tmp, ws.tile_nit, ws.tile_touch, ws.touch_bits, cst);
  hipLaunchKernelGGL(k_item_scan_top, dim3(1), dim3(1024), 0, c->stream, tmp, nsb, ws.nitems, c->nchunks,
                     ws.chunk_item0, cst);
  hipLaunchKernelGGL(k_item_scan_write, dim3(nsb), dim3(1024), 0, c->stream, ws.tile_nit, nt, ws.tile_touch,
                     ws.tile_start, c->chunk, tmp, ws.tile_item0, ws.item_tile, ws.split_list, ws.touch_list,
                     ws.chunk_item0, cst);
  hipLaunchKernelGGL(k_bin_end, dim3(1), dim3(64), 0, c->stream, st);
  return hipGetLastError();
}

int sort_hist_words(int64_t M, int digit_bits) {
  const int64_t nblk = (M + kSortChunk - 1) / kSortChunk;
  return (int)((int64_t)(1 << digit_bits) * (nblk + 1));
}

}  // namespace ib
