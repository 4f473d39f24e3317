// Force spreading, sub-step 2 (eq. discreteF), as an atomic-free gather.
//
// F(x) = sum_q F_q delta_h(x - X_q): a marker in cell c touches the 4^3 nodes
// c-1 .. c+2, so node j receives from cells j-2 .. j+1.  The grid is cut into
// 8^3-node tiles; the markers that can reach a tile are those of the 11^3
// cells around it: 121 cell rows, each a contiguous run of the sorted markers.
//
//   k_rowtab      per cell row, the sorted position of each x-boundary that a
//                 tile's 11-cell x-range can start or end at (two families,
//                 x = 8j - 2 and x = 8j + 1), so tiles need no searches;
//   k_tile_count  per tile, the length K of its marker list (121 rows);
//   k_tile_scan_* splits each tile's list into items of at most kSpreadItem
//                 markers and numbers them (a three-launch scan over the tiles);
//   k_spread      a persistent grid walks the items.  Each wave takes a
//                 quarter of an item; for one marker the 64 lanes own its 64
//                 stencil nodes, so no two lanes write the same node.  Lanes
//                 keep running sums in registers while consecutive markers
//                 share a cell and flush them into the wave's private LDS copy
//                 of the tile on a cell change; the four copies are added in a
//                 fixed order.  A tile with one item is written to the dense
//                 force grid; a split tile leaves one partial tile per item;
//   k_spread_reduce  adds a split tile's partials in item order into the grid.
// No atomics anywhere: results are bitwise reproducible.
#include "dev_common.h"
#include "ib_internal.h"

namespace ib {

constexpr int kSpreadThreads = 256;
constexpr int kRows = 121;          // (8 + 3)^2 cell rows per tile
constexpr int kSegs = kRows * 3;    // at most 3 wrapped pieces per row (n = 8)

// ------------------------------------------------------------- records ----
// Sorted marker records: fractional offset f = s - floor(s) per dimension
// (formed in FP64, stored in the fluid precision), spread force, cell x.
template <typename T>
__global__ __launch_bounds__(256) void k_prep(const int32_t *__restrict__ perm, const uint32_t *__restrict__ keys,
                                              const double *__restrict__ X, const double *__restrict__ F, int64_t M,
                                              double h, int mask, Rec<T> *__restrict__ recs) {
  const int64_t i = gtid();
  if (i >= M) return;
  const int64_t q = perm[i];
  Rec<T> r{};
  for (int d = 0; d < 3; d++) {
    const double s = X[d * M + q] / h;
    r.f[d] = (T)(s - floor(s));
    r.F[d] = F ? (T)F[d * M + q] : T(0);
  }
  r.cx = (int)(keys[i] & (uint32_t)mask);
  recs[i] = r;
}

__device__ __forceinline__ int lower_bound_u32(const uint32_t *__restrict__ a, int lo, int hi, uint32_t v) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// ------------------------------------------------------ boundary table ----
// rowtab[r * W + 2j] = first sorted position in row r with cell x >= 8j - 2,
// rowtab[r * W + 2j + 1] = first with x >= 8j + 1, for j in [0, n/8]; W = 2(n/8+1).
__global__ __launch_bounds__(256) void k_rowtab(const uint32_t *__restrict__ keys,
                                                const int32_t *__restrict__ row_start, int n, int log2n,
                                                int32_t *__restrict__ rowtab) {
  const int nj = n / 8 + 1;
  const int64_t e = gtid();
  if (e >= (int64_t)n * n * nj) return;
  const int r = (int)(e / nj), j = (int)(e - (int64_t)r * nj);
  const int rs = row_start[r], re = row_start[r + 1];
  int lo = rs, hi = rs;
  if (re > rs) {
    const uint32_t rowkey = (uint32_t)r << log2n;
    const int x0 = max(0, 8 * j - 2), x1 = min(n, 8 * j + 1);
    lo = lower_bound_u32(keys, rs, re, rowkey + (uint32_t)x0);
    hi = lower_bound_u32(keys, rs, re, rowkey + (uint32_t)x1);
  }
  rowtab[(int64_t)r * 2 * nj + 2 * j] = lo;
  rowtab[(int64_t)r * 2 * nj + 2 * j + 1] = hi;
}

// Sorted position of the first marker of a row with cell x >= x, for the
// boundaries a tile's x-range uses: 0, n, 8j - 2, 8j + 1.
__device__ __forceinline__ int row_bound(const int32_t *__restrict__ tab, int rs, int re, int n, int x) {
  if (x <= 0) return rs;
  if (x >= n) return re;
  if (((x + 2) & 7) == 0) return tab[2 * ((x + 2) >> 3)];
  return tab[2 * ((x - 1) >> 3) + 1];
}

// Pieces of the tile-relative x-range [-2, 8] of tile column T1 in one row:
// up to three runs [start, start + len) whose cell x maps to rel x = x + shift.
__device__ __forceinline__ int row_pieces(const int32_t *__restrict__ tab, int rs, int re, int n, int T1,
                                          int start[3], int len[3], int shift[3]) {
  if (re <= rs) return 0;
  int s = 0, rel = -2;
  const int mask = n - 1;
  while (rel <= 8) {
    const int c0 = (8 * T1 + rel) & mask;
    const int run = min(9 - rel, n - c0);
    const int a = row_bound(tab, rs, re, n, c0);
    const int b = row_bound(tab, rs, re, n, c0 + run);
    start[s] = a;
    len[s] = b - a;
    shift[s] = rel - c0;
    s++;
    rel += run;
  }
  return s;
}

__global__ __launch_bounds__(128) void k_tile_count(const int32_t *__restrict__ row_start,
                                                    const int32_t *__restrict__ rowtab, int n,
                                                    int32_t *__restrict__ tile_count) {
  const int nt = n >> 3, mask = n - 1, nj2 = 2 * (n / 8 + 1);
  const int tile = blockIdx.x;
  const int T1 = tile % nt, T2 = (tile / nt) % nt, T3 = tile / (nt * nt);
  int K = 0;
  if (threadIdx.x < kRows) {
    const int dy = threadIdx.x % 11 - 2, dz = threadIdx.x / 11 - 2;
    const int r = ((8 * T3 + dz) & mask) * n + ((8 * T2 + dy) & mask);
    int st[3], ln[3], sh[3];
    const int np = row_pieces(rowtab + (int64_t)r * nj2, row_start[r], row_start[r + 1], n, T1, st, ln, sh);
    for (int s = 0; s < np; s++) K += ln[s];
  }
  for (int o = 32; o >= 1; o >>= 1) K += __shfl_xor(K, o, 64);
  __shared__ int part[2];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = K;
  __syncthreads();
  if (threadIdx.x == 0) tile_count[tile] = part[0] + part[1];
}

// Items per tile (ceil(K / cap)), their numbering, the item -> tile map, each
// tile's first item, the base of a split tile's partials and the list of
// split tiles; three launches: per-block scans of 1024 tiles, a scan of the
// block totals, and the writes.  tile_flag: number of items (0: no force).
constexpr int kScanQ = 3;   // scanned per tile: items, partials (split tiles), split-tile count

__device__ __forceinline__ void scan1024(const int v[kScanQ], int off[kScanQ], int tot[kScanQ],
                                         int (*wsum)[16]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int incl[kScanQ];
  for (int k = 0; k < kScanQ; k++) {
    incl[k] = v[k];
    for (int o = 1; o < 64; o <<= 1) {
      const int x = __shfl_up(incl[k], o, 64);
      if (lane >= o) incl[k] += x;
    }
    if (lane == 63) wsum[k][w] = incl[k];
  }
  __syncthreads();
  for (int k = 0; k < kScanQ; k++) {
    int wb = 0;
    tot[k] = 0;
    for (int i = 0; i < 16; i++) {
      if (i < w) wb += wsum[k][i];
      tot[k] += wsum[k][i];
    }
    off[k] = wb + incl[k] - v[k];
  }
}

__device__ __forceinline__ void tile_items(const int32_t *tile_count, int t, int ntiles, int cap, int v[kScanQ]) {
  const int K = t < ntiles ? tile_count[t] : 0;
  const int it = (K + cap - 1) / cap;
  v[0] = it;
  v[1] = it > 1 ? it : 0;
  v[2] = it > 1 ? 1 : 0;
}

__global__ __launch_bounds__(1024) void k_tile_scan_blocks(const int32_t *__restrict__ tile_count, int ntiles,
                                                           int cap, int32_t *__restrict__ block_tot) {
  __shared__ int wsum[kScanQ][16];
  int v[kScanQ], off[kScanQ], tot[kScanQ];
  tile_items(tile_count, blockIdx.x * 1024 + threadIdx.x, ntiles, cap, v);
  scan1024(v, off, tot, wsum);
  if (threadIdx.x == 0)
    for (int k = 0; k < kScanQ; k++) block_tot[kScanQ * blockIdx.x + k] = tot[k];
}

// counts[0] = work items, counts[1] = split tiles
__global__ __launch_bounds__(1024) void k_tile_scan_top(int32_t *__restrict__ block_tot, int nblk,
                                                        int32_t *__restrict__ counts) {
  __shared__ int wsum[kScanQ][16];
  int carry[kScanQ] = {0, 0, 0};
  for (int base = 0; base < nblk; base += 1024) {
    const int b = base + threadIdx.x;
    int v[kScanQ], off[kScanQ], tot[kScanQ];
    for (int k = 0; k < kScanQ; k++) v[k] = b < nblk ? block_tot[kScanQ * b + k] : 0;
    scan1024(v, off, tot, wsum);
    __syncthreads();
    if (b < nblk)
      for (int k = 0; k < kScanQ; k++) block_tot[kScanQ * b + k] = carry[k] + off[k];
    for (int k = 0; k < kScanQ; k++) carry[k] += tot[k];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    counts[0] = carry[0];
    counts[1] = carry[2];
    counts[2] = 0;          // next work item for the spreading grid
  }
}

__global__ __launch_bounds__(1024) void k_tile_scan_write(const int32_t *__restrict__ tile_count, int ntiles,
                                                          int cap, const int32_t *__restrict__ block_off,
                                                          int32_t *__restrict__ tile_flag,
                                                          int32_t *__restrict__ tile_part,
                                                          int32_t *__restrict__ tile_item0,
                                                          int32_t *__restrict__ item_tile,
                                                          int32_t *__restrict__ split_list) {
  __shared__ int wsum[kScanQ][16];
  const int t = blockIdx.x * 1024 + threadIdx.x;
  int v[kScanQ], off[kScanQ], tot[kScanQ];
  tile_items(tile_count, t, ntiles, cap, v);
  scan1024(v, off, tot, wsum);
  if (t < ntiles) {
    const int i0 = block_off[kScanQ * blockIdx.x] + off[0];
    tile_flag[t] = v[0];
    tile_part[t] = block_off[kScanQ * blockIdx.x + 1] + off[1];
    tile_item0[t] = i0;
    for (int j = 0; j < v[0]; j++) item_tile[i0 + j] = t;
    if (v[2]) split_list[block_off[kScanQ * blockIdx.x + 2] + off[2]] = t;
  }
}

// ------------------------------------------------------------- spread ----
template <typename T>
struct SpreadSmem {
  T acc[4][3][512];               // per-wave tile accumulators
  T wgt[4][64][12];               // per-wave staging: 4 weights per dimension
  T frc[4][64][4];                // per-wave staging: force (padded)
  int rel[4][64];                 // per-wave staging: packed tile-relative cell
  int seg_start[kSegs];
  int seg_pref[kSegs + 1];
  int seg_shift[kSegs];           // relative x = cell x + shift
  int seg_yz[kSegs];              // packed relative (y, z)
};

__device__ __forceinline__ int pack_rel(int x, int y, int z) { return ((z + 4) << 10) | ((y + 4) << 5) | (x + 4); }

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__global__ __launch_bounds__(256) void k_spread(const int32_t *__restrict__ row_start,
                                                const int32_t *__restrict__ rowtab, const Rec<T> *__restrict__ recs,
                                                const int32_t *__restrict__ tile_count,
                                                const int32_t *__restrict__ tile_flag,
                                                const int32_t *__restrict__ tile_part,
                                                const int32_t *__restrict__ tile_item0,
                                                const int32_t *__restrict__ item_tile,
                                                int32_t *__restrict__ nitems, int n, T scale,
                                                T *__restrict__ Fgrid, T *__restrict__ partials) {
  __shared__ SpreadSmem<T> sm;
  __shared__ int s_item;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nt = n >> 3, mask = n - 1, nj2 = 2 * (n / 8 + 1);
  const int64_t G = (int64_t)n * n * n;
  const int W = nitems[0];
  const int oa = lane & 3, ob = (lane >> 2) & 3, oc = lane >> 4;
  // items are taken from a counter in index order (the grid is what fits on
  // the device at once); each item writes fixed locations, so the result does
  // not depend on which block takes which item
  int32_t *next = (int32_t *)nitems + 2;
  if (tid == 0) s_item = atomicAdd(next, 1);
  __syncthreads();
  for (int item = s_item; item < W;) {
    const int tile = item_tile[item];
    const int T1 = tile % nt, T2 = (tile / nt) % nt, T3 = tile / (nt * nt);
    if (tid < kRows) {
      const int dy = tid % 11 - 2, dz = tid / 11 - 2;
      const int r = ((8 * T3 + dz) & mask) * n + ((8 * T2 + dy) & mask);
      int st[3], ln[3], sh[3];
      const int np = row_pieces(rowtab + (int64_t)r * nj2, row_start[r], row_start[r + 1], n, T1, st, ln, sh);
      for (int s = 0; s < 3; s++) {
        sm.seg_start[tid * 3 + s] = s < np ? st[s] : 0;
        sm.seg_pref[tid * 3 + s] = s < np ? ln[s] : 0;
        sm.seg_shift[tid * 3 + s] = s < np ? sh[s] : 0;
        sm.seg_yz[tid * 3 + s] = pack_rel(0, dy, dz);
      }
    }
    __syncthreads();
    // exclusive prefix over the 363 piece lengths (wave 0), total in seg_pref[kSegs]
    if (w == 0) {
      int loc[6], sum = 0;
      for (int k = 0; k < 6; k++) {
        const int s = lane * 6 + k;
        loc[k] = s < kSegs ? sm.seg_pref[s] : 0;
        sum += loc[k];
      }
      int incl = sum;
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
      }
      int run = incl - sum;
      for (int k = 0; k < 6; k++) {
        const int s = lane * 6 + k;
        if (s < kSegs) sm.seg_pref[s] = run;
        run += loc[k];
      }
      if (lane == 63) sm.seg_pref[kSegs] = incl;
    }
    for (int e = tid; e < 4 * 3 * 512; e += kSpreadThreads) (&sm.acc[0][0][0])[e] = T(0);
    __syncthreads();

    // this item's share of the tile's list, split evenly among the tile's items,
    // then among the four waves
    const int K = sm.seg_pref[kSegs];
    const int nit = tile_flag[tile];
    const int jit = item - tile_item0[tile];
    const int lo = (int)((int64_t)K * jit / nit), hi = (int)((int64_t)K * (jit + 1) / nit);
    const int j0 = lo + (int)(((int64_t)(hi - lo) * w) >> 2);
    const int j1 = lo + (int)(((int64_t)(hi - lo) * (w + 1)) >> 2);

    auto locate = [&](int j) {       // piece holding list entry j: largest s with seg_pref[s] <= j
      int a = 0, b = kSegs - 1;
      while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (sm.seg_pref[mid] <= j) a = mid;
        else b = mid - 1;
      }
      return a;
    };
    T acc0 = 0, acc1 = 0, acc2 = 0;
    int cur = -1, cur_p = -1;
    // flush the running sums of cell `cur` and start cell rp
    auto switch_cell = [&](int rp) {
      if (cur_p >= 0) {
        sm.acc[w][0][cur_p] += acc0;
        sm.acc[w][1][cur_p] += acc1;
        sm.acc[w][2][cur_p] += acc2;
      }
      acc0 = acc1 = acc2 = T(0);
      cur = rp;
      const int px = (rp & 31) - 4 + oa - 1;
      const int py = ((rp >> 5) & 31) - 4 + ob - 1;
      const int pz = (rp >> 10) - 4 + oc - 1;
      cur_p = (px >= 0 && px < 8 && py >= 0 && py < 8 && pz >= 0 && pz < 8) ? (pz * 64 + py * 8 + px) : -1;
    };
    int sg = 0;
    Rec<T> rec{};
    if (j0 + lane < j1) {
      sg = locate(j0 + lane);
      rec = recs[sm.seg_start[sg] + (j0 + lane - sm.seg_pref[sg])];
    }
    for (int jb = j0; jb < j1; jb += 64) {
      const int cnt = min(64, j1 - jb);
      if (lane < cnt) {
        sm.rel[w][lane] = sm.seg_yz[sg] + (rec.cx + sm.seg_shift[sg]);   // x field: low 5 bits (+4 bias)
        T wv[4];
        for (int d = 0; d < 3; d++) {
          phi4<T>(rec.f[d], wv);
          sm.wgt[w][lane][4 * d + 0] = wv[0];
          sm.wgt[w][lane][4 * d + 1] = wv[1];
          sm.wgt[w][lane][4 * d + 2] = wv[2];
          sm.wgt[w][lane][4 * d + 3] = wv[3];
          sm.frc[w][lane][d] = rec.F[d];
        }
      }
      // issue the next chunk's record load before consuming this chunk; list
      // entries only move forward, so the piece index is advanced, not searched
      const int jn = jb + 64 + lane;
      if (jn < j1) {
        while (sm.seg_pref[sg + 1] <= jn) sg++;
        rec = recs[sm.seg_start[sg] + (jn - sm.seg_pref[sg])];
      }
      wave_sync_lds();
      int mm = 0;
      // four markers at a time: all their LDS reads issue together; the common
      // case (same cell as the running sum) needs no store in between
      for (; mm + 4 <= cnt; mm += 4) {
        const int r0 = sm.rel[w][mm], r1 = sm.rel[w][mm + 1], r2 = sm.rel[w][mm + 2], r3 = sm.rel[w][mm + 3];
        T wt[4], f0[4], f1[4], f2[4];
        for (int u = 0; u < 4; u++) {
          wt[u] = (sm.wgt[w][mm + u][oa] * sm.wgt[w][mm + u][4 + ob]) * sm.wgt[w][mm + u][8 + oc];
          f0[u] = sm.frc[w][mm + u][0];
          f1[u] = sm.frc[w][mm + u][1];
          f2[u] = sm.frc[w][mm + u][2];
        }
        const int rr[4] = {r0, r1, r2, r3};
        for (int u = 0; u < 4; u++) {
          if (rr[u] != cur) switch_cell(rr[u]);
          acc0 += f0[u] * wt[u];
          acc1 += f1[u] * wt[u];
          acc2 += f2[u] * wt[u];
        }
      }
      for (; mm < cnt; mm++) {
        const int rp = sm.rel[w][mm];
        if (rp != cur) switch_cell(rp);
        const T wt = (sm.wgt[w][mm][oa] * sm.wgt[w][mm][4 + ob]) * sm.wgt[w][mm][8 + oc];
        acc0 += sm.frc[w][mm][0] * wt;
        acc1 += sm.frc[w][mm][1] * wt;
        acc2 += sm.frc[w][mm][2] * wt;
      }
      wave_sync_lds();
    }
    if (cur_p >= 0) {
      sm.acc[w][0][cur_p] += acc0;
      sm.acc[w][1][cur_p] += acc1;
      sm.acc[w][2][cur_p] += acc2;
    }
    __syncthreads();

    // add the wave copies in a fixed order; store the tile or this item's partial
    const int base = ((8 * T3) * n + 8 * T2) * n + 8 * T1;
    T *part = nit > 1 ? partials + (int64_t)(tile_part[tile] + jit) * 3 * 512 : nullptr;
    for (int e = tid; e < 3 * 512; e += kSpreadThreads) {
      const int c = e >> 9, p = e & 511;
      const T v = (((sm.acc[0][c][p] + sm.acc[1][c][p]) + sm.acc[2][c][p]) + sm.acc[3][c][p]) * scale;
      if (part) {
        part[e] = v;
      } else {
        const int px = p & 7, py = (p >> 3) & 7, pz = p >> 6;
        Fgrid[c * G + base + ((int64_t)pz * n + py) * n + px] = v;
      }
    }
    if (tid == 0) s_item = atomicAdd(next, 1);
    __syncthreads();   // LDS is reused by the next item
    item = s_item;
  }
  (void)tile_count;
}

// Split tiles: add their partial tiles in item order into the force grid, so
// that every tile with force is dense there (a persistent grid over the list).
template <typename T>
__global__ __launch_bounds__(256) void k_spread_reduce(const int32_t *__restrict__ split_list,
                                                       const int32_t *__restrict__ counts,
                                                       const int32_t *__restrict__ tile_flag,
                                                       const int32_t *__restrict__ tile_part,
                                                       const T *__restrict__ partials, int n, T *__restrict__ Fgrid) {
  const int nt = n >> 3;
  const int64_t G = (int64_t)n * n * n;
  const int ns = counts[1];
  for (int s = blockIdx.x; s < ns; s += gridDim.x) {
    const int tile = split_list[s];
    const int f = tile_flag[tile];
    const T *pp = partials + (int64_t)tile_part[tile] * 3 * 512;
    const int T1 = tile % nt, T2 = (tile / nt) % nt, T3 = tile / (nt * nt);
    const int base = ((8 * T3) * n + 8 * T2) * n + 8 * T1;
    for (int e = threadIdx.x; e < 3 * 512; e += 256) {
      T v = T(0);
      for (int i = 0; i < f; i++) v += pp[(int64_t)i * 3 * 512 + e];
      const int c = e >> 9, p = e & 511;
      const int px = p & 7, py = (p >> 3) & 7, pz = p >> 6;
      Fgrid[c * G + base + ((int64_t)pz * n + py) * n + px] = v;
    }
  }
}

// Dense force grid for the ib_spread entry point: zero the tiles without force.
template <typename T>
__global__ __launch_bounds__(256) void k_spread_zero(const int32_t *__restrict__ tile_flag, int n,
                                                     T *__restrict__ Fgrid) {
  const int nt = n >> 3;
  const int tile = blockIdx.x;
  if (tile_flag[tile] != 0) return;
  const int T1 = tile % nt, T2 = (tile / nt) % nt, T3 = tile / (nt * nt);
  const int64_t G = (int64_t)n * n * n;
  const int base = ((8 * T3) * n + 8 * T2) * n + 8 * T1;
  for (int e = threadIdx.x; e < 3 * 512; e += 256) {
    const int c = e >> 9, p = e & 511;
    const int px = p & 7, py = (p >> 3) & 7, pz = p >> 6;
    Fgrid[c * G + base + ((int64_t)pz * n + py) * n + px] = T(0);
  }
}

template <typename T>
hipError_t launch_prep(ib_ctx *c, const double *X, const double *F) {
  if (c->M == 0) return hipSuccess;
  PhaseScope ps(c, PH_PREP);
  hipLaunchKernelGGL(k_prep<T>, dim3((unsigned)((c->M + 255) / 256)), dim3(256), 0, c->stream,
                     c->ws.vals[c->sorted_buf], c->ws.keys[c->sorted_buf], X, F, c->M, c->h, c->n - 1,
                     (Rec<T> *)c->ws.recs);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spread(ib_ctx *c, T *Fgrid, bool dense, double scale) {
  PhaseScope ps(c, PH_SPREAD);
  const int n = c->n, nt = n / 8, ntiles = nt * nt * nt;
  const int64_t ntab = (int64_t)n * n * (n / 8 + 1);
  hipLaunchKernelGGL(k_rowtab, dim3((unsigned)((ntab + 255) / 256)), dim3(256), 0, c->stream,
                     c->ws.keys[c->sorted_buf], c->ws.row_start, n, c->log2n, c->ws.rowtab);
  hipLaunchKernelGGL(k_tile_count, dim3(ntiles), dim3(128), 0, c->stream, c->ws.row_start, c->ws.rowtab, n,
                     c->ws.tile_count);
  const int nsb = (ntiles + 1023) / 1024;
  hipLaunchKernelGGL(k_tile_scan_blocks, dim3(nsb), dim3(1024), 0, c->stream, c->ws.tile_count, ntiles, kSpreadItem,
                     c->ws.scan_tmp);
  hipLaunchKernelGGL(k_tile_scan_top, dim3(1), dim3(1024), 0, c->stream, c->ws.scan_tmp, nsb, c->ws.nitems);
  hipLaunchKernelGGL(k_tile_scan_write, dim3(nsb), dim3(1024), 0, c->stream, c->ws.tile_count, ntiles, kSpreadItem,
                     c->ws.scan_tmp, c->ws.tile_flag, c->ws.tile_part, c->ws.tile_item0, c->ws.item_tile,
                     c->ws.split_list);
  hipLaunchKernelGGL(k_spread<T>, dim3(c->spread_grid), dim3(kSpreadThreads), 0, c->stream, c->ws.row_start,
                     c->ws.rowtab, (const Rec<T> *)c->ws.recs, c->ws.tile_count, c->ws.tile_flag, c->ws.tile_part,
                     c->ws.tile_item0, c->ws.item_tile, c->ws.nitems, n, (T)scale, Fgrid, (T *)c->ws.partials);
  hipLaunchKernelGGL(k_spread_reduce<T>, dim3(256), dim3(256), 0, c->stream, c->ws.split_list, c->ws.nitems,
                     c->ws.tile_flag, c->ws.tile_part, (const T *)c->ws.partials, n, Fgrid);
  if (dense) hipLaunchKernelGGL(k_spread_zero<T>, dim3(ntiles), dim3(256), 0, c->stream, c->ws.tile_flag, n, Fgrid);
  return hipGetLastError();
}

template hipError_t launch_prep<float>(ib_ctx *, const double *, const double *);
template hipError_t launch_prep<double>(ib_ctx *, const double *, const double *);
template hipError_t launch_spread<float>(ib_ctx *, float *, bool, double);
template hipError_t launch_spread<double>(ib_ctx *, double *, bool, double);

}  // namespace ib
