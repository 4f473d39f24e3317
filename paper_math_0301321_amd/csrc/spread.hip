// Force spreading, sub-step 2 (eq. discreteF), bitwise reproducible.
//
// F(x) = sum_q F_q delta_h(x - X_q): a marker in cell c touches the 4^3 nodes
// c-1 .. c+2.  Markers are binned by 8^3-cell tiles, so the nodes that one
// tile's markers touch lie in the tile's 11^3 halo (tile nodes -1 .. 9).
//
//   k_prep    sorted records: fractional offset f = s - floor(s) per dimension
//             (formed in FP64, stored in the fluid precision), force, key;
//   k_spread  single-wave blocks take the work items (up to kItem markers of
//             one tile) round robin.  Markers are staged 64 at a time as
//             F_c phi(f_x - a) and phi(f_y - b) phi(f_z - c);
//             then, for one marker, the 64 lanes own its 64 stencil nodes
//             (a, b, c), keep running sums in registers while consecutive
//             markers share a cell, and add them into the wave's 11^3 halo
//             accumulator in LDS on a cell change.  Each item's halo is
//             written, scaled, to its own partial buffer;
//   k_split_reduce  for tiles cut into several items, adds the items' halos
//             in item order into the first one;
//   k_spread_gather  one wave per tile: the force at a node is the sum of
//             the halo values of the tiles whose halos cover it (itself and
//             up to 7 neighbours), in a fixed order.
//             Tiles no halo reaches are marked untouched (and zeroed when a
//             dense grid is asked for).
// No floating-point atomics: every value is summed in a fixed order, so
// results are bitwise reproducible.
#include <algorithm>

#include "dev_common.h"
#include "ib_internal.h"

namespace ib {

// ------------------------------------------------------------- records ----
template <typename T>
__global__ __launch_bounds__(256) void k_prep(const int32_t *__restrict__ perm, const uint32_t *__restrict__ keys,
                                              const double *__restrict__ X, const double *__restrict__ F, int64_t M,
                                              double h, Rec<T> *__restrict__ recs) {
  const int64_t i = gtid();
  if (i >= M) return;
  const int64_t q = perm[i];
  Rec<T> r{};
  for (int d = 0; d < 3; d++) {
    const double s = X[d * M + q] / h;
    r.f[d] = (T)(s - floor(s));
    r.F[d] = F ? (T)F[d * M + q] : T(0);
  }
  r.key = keys[i];
  recs[i] = r;
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Vector of 16 bytes of the fluid precision, for LDS and global block copies.
template <typename T>
struct Vec16T;
template <>
struct Vec16T<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct Vec16T<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};

// Range [j0, j1) of the sorted markers that work item `item` covers: item j
// of a tile takes the tile's markers j kItem .. min((j + 1) kItem, K) - 1.
__device__ __forceinline__ void item_range(int item, const int32_t *__restrict__ tile_start,
                                           const int32_t *__restrict__ tile_item0,
                                           const int32_t *__restrict__ item_tile, int *j0, int *j1) {
  const int tile = item_tile[item];
  const int a = tile_start[tile] + (item - tile_item0[tile]) * kItem;
  *j0 = a;
  *j1 = min(a + kItem, tile_start[tile + 1]);
}

// ------------------------------------------------------------- spread ----
// Staged per marker and x-offset a: F_c phi(f_x - a) (c = 0..2) and the halo
// position of the marker's stencil origin.
template <typename T>
struct alignas(16) SpreadG {
  T g[3];
  int base;
};

template <typename T>
struct SpreadSmem {
  T acc[kPartStride];             // the wave's halo accumulator, [3][11^3] + pad
  SpreadG<T> g[64][4];            // staging: force times x-weights
  T wyz[64][16];                  // staging: y-weight times z-weight, index b * 4 + c
};

// Single-wave blocks; block b takes items b, b + grid, b + 2 grid, ...  The
// next item's range and first records are loaded before the current item's
// halo is written out, so their latency overlaps the write.
template <typename T>
__global__ __launch_bounds__(64) void k_spread(const int32_t *__restrict__ tile_start,
                                               const int32_t *__restrict__ tile_item0,
                                               const int32_t *__restrict__ item_tile,
                                               const int32_t *__restrict__ counts, const Rec<T> *__restrict__ recs,
                                               T scale, T *__restrict__ partials) {
  using V = typename Vec16T<T>::type;
  constexpr int kVec = 16 / sizeof(T);
  constexpr int kNV = kPartStride / kVec;
  __shared__ SpreadSmem<T> sm;
  const int lane = threadIdx.x;
  const int oa = lane & 3, ob = (lane >> 2) & 3, oc = lane >> 4;
  const int loff = oc * (kHalo * kHalo) + ob * kHalo + oa;   // the lane's node relative to the stencil origin
  const int W = counts[0];
  V *acc4 = (V *)sm.acc;
  int item = blockIdx.x;
  int j0 = 0, j1 = 0;
  Rec<T> rec{};
  if (item < W) {
    item_range(item, tile_start, tile_item0, item_tile, &j0, &j1);
    if (j0 + lane < j1) rec = recs[j0 + lane];
  }
  while (item < W) {
    for (int e = lane; e < kNV; e += 64) acc4[e] = V{};
    T a0 = 0, a1 = 0, a2 = 0;
    int cur = -1;
    // add the running sums of cell `cur` into the accumulator and start cell nb
    auto switch_cell = [&](int nb) {
      if (cur >= 0) {
        const int p = cur + loff;
        sm.acc[p] += a0;
        sm.acc[kHalo3 + p] += a1;
        sm.acc[2 * kHalo3 + p] += a2;
      }
      a0 = a1 = a2 = T(0);
      cur = nb;
    };
    for (int jb = j0; jb < j1; jb += 64) {
      const int cnt = min(64, j1 - jb);
      wave_sync_lds();   // the previous chunk's staging has been consumed
      if (lane < cnt) {
        T wx[4], wy[4], wz[4];
        phi4<T>(rec.f[0], wx);
        phi4<T>(rec.f[1], wy);
        phi4<T>(rec.f[2], wz);
        const int base = halo_base(rec.key);
#pragma unroll
        for (int a = 0; a < 4; a++) {
          SpreadG<T> g;
          g.g[0] = rec.F[0] * wx[a];
          g.g[1] = rec.F[1] * wx[a];
          g.g[2] = rec.F[2] * wx[a];
          g.base = base;
          sm.g[lane][a] = g;
        }
#pragma unroll
        for (int b = 0; b < 4; b++)
#pragma unroll
          for (int c = 0; c < 4; c++) sm.wyz[lane][b * 4 + c] = wy[b] * wz[c];
      }
      // issue the next chunk's record load before consuming this chunk
      if (jb + 64 + lane < j1) rec = recs[jb + 64 + lane];
      wave_sync_lds();
      int m = 0;
      // eight markers at a time: their LDS reads issue together
      for (; m + 8 <= cnt; m += 8) {
        SpreadG<T> g[8];
        T w[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
          g[u] = sm.g[m + u][oa];
          w[u] = sm.wyz[m + u][ob * 4 + oc];
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
          const int nb = __builtin_amdgcn_readfirstlane(g[u].base);
          if (nb != cur) switch_cell(nb);
          a0 += g[u].g[0] * w[u];
          a1 += g[u].g[1] * w[u];
          a2 += g[u].g[2] * w[u];
        }
      }
      for (; m < cnt; m++) {
        const SpreadG<T> g = sm.g[m][oa];
        const T w = sm.wyz[m][ob * 4 + oc];
        const int nb = __builtin_amdgcn_readfirstlane(g.base);
        if (nb != cur) switch_cell(nb);
        a0 += g.g[0] * w;
        a1 += g.g[1] * w;
        a2 += g.g[2] * w;
      }
    }
    switch_cell(-1);
    // next item: range and first records, in flight during the write-out
    const int nitem = item + (int)gridDim.x;
    int nj0 = 0, nj1 = 0;
    Rec<T> nrec{};
    if (nitem < W) {
      item_range(nitem, tile_start, tile_item0, item_tile, &nj0, &nj1);
      if (nj0 + lane < nj1) nrec = recs[nj0 + lane];
    }
    wave_sync_lds();
    V *out = (V *)(partials + (int64_t)item * kPartStride);
#pragma unroll 4
    for (int e = lane; e < kNV; e += 64) out[e] = acc4[e] * scale;
    item = nitem;
    j0 = nj0;
    j1 = nj1;
    rec = nrec;
    wave_sync_lds();   // the write-out has read the accumulator
  }
}

// Split tiles: add the halos of a tile's items, in item order, into its
// first item's halo.  Blocks take the tiles of the split-tile list round
// robin; each thread owns whole 16-byte vectors of the halo and loads four
// items ahead of the running sum.
template <typename T>
__global__ __launch_bounds__(256) void k_split_reduce(const int32_t *__restrict__ split_list,
                                                      const int32_t *__restrict__ counts,
                                                      const int32_t *__restrict__ tile_nit,
                                                      const int32_t *__restrict__ tile_item0,
                                                      T *__restrict__ partials) {
  using V = typename Vec16T<T>::type;
  constexpr int kNV = kPartStride / (16 / sizeof(T));
  const int nsplit = counts[1];
  for (int si = blockIdx.x; si < nsplit; si += gridDim.x) {
    const int tile = split_list[si];
    const int nit = tile_nit[tile];
    V *p0 = (V *)(partials + (int64_t)tile_item0[tile] * kPartStride);
    for (int e = threadIdx.x; e < kNV; e += 256) {
      V acc = p0[e];
      int j = 1;
      for (; j + 4 <= nit; j += 4) {
        V x[4];
#pragma unroll
        for (int u = 0; u < 4; u++) x[u] = p0[(int64_t)(j + u) * kNV + e];
#pragma unroll
        for (int u = 0; u < 4; u++) acc += x[u];
      }
      for (; j < nit; j++) acc += p0[(int64_t)j * kNV + e];
      p0[e] = acc;
    }
  }
}

// Halo source s = 0..10 along one dimension of a tile: s = 0, 1 come from the
// neighbour at offset -1 (its halo positions 9, 10 = this tile's nodes 0, 1),
// s = 2..9 from the tile itself (positions 1..8 = nodes 0..7), s = 10 from the
// neighbour at +1 (position 0 = node 7).
__device__ __forceinline__ int src_off(int s) { return s < 2 ? -1 : (s < 10 ? 0 : 1); }
__device__ __forceinline__ int src_pos(int s) { return s < 2 ? s + 9 : (s < 10 ? s - 1 : 0); }

constexpr int kSrcPerLane = (kHalo3 + 63) / 64;   // 21

// One wave per tile (four tiles per block).  For each component, every lane
// loads its share of the 11^3 sources (the neighbours' reduced halos; all
// loads in flight at once) into LDS; then each lane adds, for its nodes
// (x, y) = (l % 8, l / 8) on the 8 z-planes, the 1 to 8 sources that cover
// them in the order of the neighbour offset (z, then y, then x).  Tiles that
// no neighbour's markers reach are marked untouched (zeroed when dense).
template <typename T>
__global__ __launch_bounds__(256) void k_spread_gather(const int32_t *__restrict__ tile_nit,
                                                       const int32_t *__restrict__ tile_item0,
                                                       const T *__restrict__ partials, int n, int log2nt,
                                                       int64_t ntiles, int dense, T *__restrict__ Fgrid,
                                                       int32_t *__restrict__ tile_touch) {
  __shared__ T Vs[4][kHalo3];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t tile = (int64_t)blockIdx.x * 4 + w;
  if (tile >= ntiles) return;
  const int tmask = (1 << log2nt) - 1;
  const int T1 = (int)(tile & tmask), T2 = (int)((tile >> log2nt) & tmask), T3 = (int)(tile >> (2 * log2nt));
  int nb_nit = 0, nb_i0 = 0;
  if (lane < 27) {
    const int dx = lane % 3 - 1, dy = (lane / 3) % 3 - 1, dz = lane / 9 - 1;
    const int t2 = (((((T3 + dz) & tmask) << log2nt) | ((T2 + dy) & tmask)) << log2nt) | ((T1 + dx) & tmask);
    nb_nit = tile_nit[t2];
    nb_i0 = tile_item0[t2];
  }
  const bool any = __ballot(nb_nit > 0) != 0;
  const int64_t G = (int64_t)n * n * n;
  const int px = lane & 7, py = lane >> 3;
  T *dst = Fgrid + (((int64_t)(8 * T3) * n + 8 * T2 + py) * n + 8 * T1 + px);
  if (lane == 0) tile_touch[tile] = any ? 1 : 0;
  if (!any) {
    if (dense)
      for (int k = 0; k < 8; k++)
        for (int c = 0; c < 3; c++) dst[c * G + (int64_t)k * n * n] = T(0);
    return;
  }
  // offsets of the lane's sources s = lane + 64 i (-1: none)
  int soff[kSrcPerLane];
#pragma unroll
  for (int i = 0; i < kSrcPerLane; i++) {
    const int s = lane + 64 * i;
    const int sz = s / (kHalo * kHalo), r = s - sz * (kHalo * kHalo), sy = r / kHalo, sx = r - sy * kHalo;
    const int d27 = (src_off(sz) + 1) * 9 + (src_off(sy) + 1) * 3 + (src_off(sx) + 1);
    const int e = (src_pos(sz) * kHalo + src_pos(sy)) * kHalo + src_pos(sx);
    const int nd = __shfl(nb_nit, d27, 64), i0 = __shfl(nb_i0, d27, 64);
    soff[i] = (s < kHalo3 && nd > 0) ? i0 * kPartStride + e : -1;
  }
  // x and y sources of this lane's column, in offset order
  int xs[2], ys[2], nx = 0, ny = 0;
  if (px <= 1) xs[nx++] = px;
  xs[nx++] = px + 2;
  if (px == 7) xs[nx++] = 10;
  if (py <= 1) ys[ny++] = py;
  ys[ny++] = py + 2;
  if (py == 7) ys[ny++] = 10;
  T *Vw = Vs[w];
  for (int c = 0; c < 3; c++) {
    T v[kSrcPerLane];
#pragma unroll
    for (int i = 0; i < kSrcPerLane; i++) {
      const T x = partials[(soff[i] >= 0 ? soff[i] : 0) + c * kHalo3];
      v[i] = soff[i] >= 0 ? x : T(0);
    }
    wave_sync_lds();   // the previous component's sums have read the sources
#pragma unroll
    for (int i = 0; i < kSrcPerLane; i++) {
      const int s = lane + 64 * i;
      if (s < kHalo3) Vw[s] = v[i];
    }
    wave_sync_lds();
#pragma unroll
    for (int k = 0; k < 8; k++) {
      int zs[2], nz = 0;
      if (k <= 1) zs[nz++] = k;
      zs[nz++] = k + 2;
      if (k == 7) zs[nz++] = 10;
      T acc = T(0);
      for (int a = 0; a < nz; a++)
        for (int b = 0; b < ny; b++)
          for (int q = 0; q < nx; q++) acc += Vw[(zs[a] * kHalo + ys[b]) * kHalo + xs[q]];
      dst[c * G + (int64_t)k * n * n] = acc;
    }
  }
}

template <typename T>
hipError_t launch_prep(ib_ctx *c, const double *X, const double *F) {
  if (c->M == 0) return hipSuccess;
  PhaseScope ps(c, PH_PREP);
  hipLaunchKernelGGL(k_prep<T>, dim3((unsigned)((c->M + 255) / 256)), dim3(256), 0, c->stream,
                     c->ws.vals[c->sorted_buf], c->ws.keys[c->sorted_buf], X, F, c->M, c->h,
                     (Rec<T> *)c->ws.recs);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spread(ib_ctx *c, T *Fgrid, bool dense, double scale) {
  {
    PhaseScope ps(c, PH_SPREAD);
    if (c->M > 0)
      hipLaunchKernelGGL(k_spread<T>, dim3(c->item_grid), dim3(64), 0, c->stream, c->ws.tile_start, c->ws.tile_item0,
                         c->ws.item_tile, c->ws.nitems, (const Rec<T> *)c->ws.recs, (T)scale, (T *)c->ws.partials);
  }
  if (c->M > 0) {
    PhaseScope ps(c, PH_SPLIT);
    hipLaunchKernelGGL(k_split_reduce<T>, dim3((unsigned)std::min<int64_t>(c->ntiles, 4 * c->ncu)), dim3(256), 0,
                       c->stream, c->ws.split_list, c->ws.nitems, c->ws.tile_nit, c->ws.tile_item0,
                       (T *)c->ws.partials);
  }
  PhaseScope ps(c, PH_GATHER);
  hipLaunchKernelGGL(k_spread_gather<T>, dim3((unsigned)((c->ntiles + 3) / 4)), dim3(256), 0, c->stream,
                     c->ws.tile_nit, c->ws.tile_item0, (const T *)c->ws.partials, c->n, c->log2nt, c->ntiles,
                     dense ? 1 : 0, Fgrid, c->ws.tile_touch);
  return hipGetLastError();
}

template hipError_t launch_prep<float>(ib_ctx *, const double *, const double *);
template hipError_t launch_prep<double>(ib_ctx *, const double *, const double *);
template hipError_t launch_spread<float>(ib_ctx *, float *, bool, double);
template hipError_t launch_spread<double>(ib_ctx *, double *, bool, double);

}  // namespace ib
