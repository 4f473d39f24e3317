// Force spreading, sub-step 2 (eq. discreteF), bitwise reproducible.
//
// F(x) = sum_q F_q delta_h(x - X_q): a marker in cell c touches the 4^3 nodes
// c-1 .. c+2.  Markers are binned by 8^3-cell tiles, so the nodes that one
// tile's markers touch lie in the tile's 11^3 halo (tile nodes -1 .. 9).
//
//   k_prep    sorted records: fractional offset f = s - floor(s) per dimension
//             (formed in FP64, stored in the fluid precision), force, key;
//   k_spread  one single-wave block per chunk of the sorted markers (equal
//             chunks) streams the chunk, whose work items are its parts of
//             consecutive tiles.  Markers are staged in LDS 32 at a time as
//             F_c phi(f_x - a) and phi(f_y - b) phi(f_z - c); each of the 64
//             lanes owns one of a marker's 4^3 stencil nodes and keeps
//             running sums (vector ALU, FP32 or FP64) while consecutive
//             markers share a cell, adding them into the wave's 11^3 halo
//             accumulator in LDS on a cell change.  Each item's halo is
//             written, scaled, to its own partial buffer;
//   k_split_reduce  for tiles cut into several items, adds the items' halos
//             in item order into the first one;
//   k_spread_gather  one wave per touched tile (the binning lists the tiles
//             that some neighbour's markers reach): the force at a node is the
//             sum of the halo values of the tiles whose halos cover it (itself
//             and up to 7 neighbours), in a fixed order.  Untouched tiles are
//             zeroed only when a dense grid is asked for.
// No floating-point atomics: every value is summed in a fixed order, so
// results are bitwise reproducible.
#include <algorithm>

#include "dev_common.h"
#include "ib_internal.h"

namespace ib {

// ------------------------------------------------------------- records ----
template <typename T>
__global__ __launch_bounds__(256) void k_prep(const int32_t *__restrict__ perm, const uint32_t *__restrict__ keys,
                                              const double *__restrict__ X, const double *__restrict__ Y,
                                              const double *__restrict__ F, int64_t M, double h,
                                              Rec<T> *__restrict__ recs) {
  const int64_t i = gtid();
  if (i >= M) return;
  const int64_t q = perm[i];
  Rec<T> r{};
  for (int d = 0; d < 3; d++) {
    const double s = (Y ? Y[d * M + q] + X[d * M + q] : X[d * M + q]) / h;   // position: X or Y + D
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

// ------------------------------------------------------------- spread ----
// For one marker the 64 lanes of a wave own its 64 stencil nodes (a, b, c):
// lane a + 4b + 16c.  Each lane keeps running sums in registers while
// consecutive markers share a cell and adds them into the wave's 11^3 halo
// accumulator in LDS on a cell change.

// Staged per marker and x-offset a: F_c phi(f_x - a) (c = 0..2) and the cell key.
template <typename T>
struct alignas(16) SpreadG {
  T g[3];
  uint32_t key;
};

// Markers are staged kStage at a time: half a record batch, so that the
// staging and the accumulator fit eight waves per CU (FP32).
constexpr int kStage = 32;

template <typename T>
struct SpreadSmem {
  T acc[kPartStride];             // the wave's halo accumulator, [3][11^3] + pad
  SpreadG<T> g[kStage][4];        // staging: force times x-weights, [marker][a]
  T wyz[kStage][16];              // staging: y-weight times z-weight, [marker][b * 4 + c]
};

constexpr int kSpreadRing = 4;    // 64-marker batches of records in flight per wave

// Write a finished item's halo (scaled) to its partial buffer and clear the
// accumulator.  Out of line: it runs a few times per wave, and keeping it out
// of the unrolled loops keeps the kernel's code small.
template <typename T>
__device__ __noinline__ void spread_write_item(T *__restrict__ acc, T *__restrict__ out, T scale, int lane) {
  using V = typename Vec16T<T>::type;
  constexpr int kNV = kPartStride / (16 / sizeof(T));
  V *acc4 = (V *)acc;
  V *out4 = (V *)out;
  wave_sync_lds();
#pragma unroll 8
  for (int i = 0; i < kNV / 64; i++) out4[lane + 64 * i] = acc4[lane + 64 * i] * scale;
  wave_sync_lds();   // the write-out has read the accumulator
#pragma unroll 8
  for (int i = 0; i < kNV / 64; i++) acc4[lane + 64 * i] = V{};
  wave_sync_lds();
}

// Single-wave blocks, one per chunk of the sorted markers (all chunks hold the
// same number of markers, so the waves have the same work).  A wave streams
// its chunk in batches of 64 with kSpreadRing batches of records in flight
// (every load unconditional, so that the waits for them stay exact); its
// items (the chunk's parts of consecutive tiles) follow one another in the
// stream: at a tile change the finished item's halo is written out, scaled,
// and the accumulator cleared.
template <typename T>
__global__ __launch_bounds__(64) void k_spread(const int32_t *__restrict__ chunk_item0, int chunk, int64_t M,
                                               const Rec<T> *__restrict__ recs, T scale, T *__restrict__ partials) {
  using V = typename Vec16T<T>::type;
  constexpr int kNV = kPartStride / (16 / sizeof(T));
  static_assert(kNV % 64 == 0, "whole rounds of 64 lanes");
  __shared__ SpreadSmem<T> sm;
  const int lane = threadIdx.x;
  const int oa = lane & 3, ob = (lane >> 2) & 3, oc = lane >> 4;
  const int loff = oc * (kHalo * kHalo) + ob * kHalo + oa;   // the lane's node relative to the stencil origin
  const int64_t cs = (int64_t)blockIdx.x * chunk, ce = min(M, cs + chunk);
  int item = chunk_item0[blockIdx.x];
  V *acc4 = (V *)sm.acc;
  Rec<T> ring[kSpreadRing];
#pragma unroll
  for (int q = 0; q < kSpreadRing; q++) ring[q] = recs[min(cs + 64 * q + lane, ce - 1)];
#pragma unroll
  for (int i = 0; i < kNV / 64; i++) acc4[lane + 64 * i] = V{};
  T a0 = 0, a1 = 0, a2 = 0;
  uint32_t cur = 0xFFFFFFFFu;                           // key of the cell being summed
  // add the running sums of cell `cur` into the accumulator and start cell k
  auto switch_cell = [&](uint32_t k) {
    if (cur != 0xFFFFFFFFu) {
      const int p = halo_base(cur) + loff;
      sm.acc[p] += a0;
      sm.acc[kHalo3 + p] += a1;
      sm.acc[2 * kHalo3 + p] += a2;
      if ((k >> 9) != (cur >> 9)) {                     // the tile (item) is complete
        spread_write_item<T>(sm.acc, partials + (int64_t)item * kPartStride, scale, lane);
        item++;
      }
    }
    a0 = a1 = a2 = T(0);
    cur = k;
  };
  // one batch of 64 markers from ring slot r, which is then refilled with the
  // batch kSpreadRing batches ahead (the slots are never moved: a register
  // move would wait for the load in flight)
  auto batch = [&](Rec<T> &r, int64_t jb) {
    const int cnt64 = (int)max((int64_t)0, min((int64_t)64, ce - jb));
    // the lanes' weights, computed once for the whole batch
    T wx[4], wy[4], wz[4];
    phi4<T>(r.f[0], wx);
    phi4<T>(r.f[1], wy);
    phi4<T>(r.f[2], wz);
    const Rec<T> rr = r;
    r = recs[min(jb + 64 * kSpreadRing + lane, ce - 1)];
#pragma unroll
    for (int half = 0; half < 64 / kStage; half++) {
      const int cnt = min(kStage, cnt64 - half * kStage);
      if (cnt <= 0) break;
      wave_sync_lds();   // the previous staging has been consumed
      if (lane >= half * kStage && lane < half * kStage + cnt) {
        const int sl = lane - half * kStage;
#pragma unroll
        for (int a = 0; a < 4; a++) {
          SpreadG<T> g;
          g.g[0] = rr.F[0] * wx[a];
          g.g[1] = rr.F[1] * wx[a];
          g.g[2] = rr.F[2] * wx[a];
          g.key = rr.key;
          sm.g[sl][a] = g;
        }
#pragma unroll
        for (int b = 0; b < 4; b++)
#pragma unroll
          for (int c = 0; c < 4; c++) sm.wyz[sl][b * 4 + c] = wy[b] * wz[c];
      }
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
          const uint32_t k = __builtin_amdgcn_readfirstlane(g[u].key);
          if (k != cur) switch_cell(k);
          a0 += g[u].g[0] * w[u];
          a1 += g[u].g[1] * w[u];
          a2 += g[u].g[2] * w[u];
        }
      }
      for (; m < cnt; m++) {
        const SpreadG<T> g = sm.g[m][oa];
        const T w = sm.wyz[m][ob * 4 + oc];
        const uint32_t k = __builtin_amdgcn_readfirstlane(g.key);
        if (k != cur) switch_cell(k);
        a0 += g.g[0] * w;
        a1 += g.g[1] * w;
        a2 += g.g[2] * w;
      }
    }
  };
  static_assert(kSpreadRing == 4, "the batch loop below is unrolled for four ring slots");
  for (int64_t jb = cs; jb < ce; jb += 64 * kSpreadRing) {
    batch(ring[0], jb);
    batch(ring[1], jb + 64);
    batch(ring[2], jb + 128);
    batch(ring[3], jb + 192);
  }
  if (cur != 0xFFFFFFFFu) switch_cell(0xFFFFFFFEu);   // flush, and write out the last item (a different tile)
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
    // every vector of this thread at once (kNV / 256 of them), four items ahead
    constexpr int NE = kNV / 256;
    static_assert(NE * 256 == kNV, "whole vectors per thread");
    V acc[NE];
#pragma unroll
    for (int q = 0; q < NE; q++) acc[q] = p0[threadIdx.x + 256 * q];
    int j = 1;
    for (; j + 4 <= nit; j += 4) {
      V x[4][NE];
#pragma unroll
      for (int u = 0; u < 4; u++)
#pragma unroll
        for (int q = 0; q < NE; q++) x[u][q] = p0[(int64_t)(j + u) * kNV + threadIdx.x + 256 * q];
#pragma unroll
      for (int u = 0; u < 4; u++)
#pragma unroll
        for (int q = 0; q < NE; q++) acc[q] += x[u][q];
    }
    for (; j < nit; j++)
#pragma unroll
      for (int q = 0; q < NE; q++) acc[q] += p0[(int64_t)j * kNV + threadIdx.x + 256 * q];
#pragma unroll
    for (int q = 0; q < NE; q++) p0[threadIdx.x + 256 * q] = acc[q];
  }
}

// Halo source s = 0..10 along one dimension of a tile: s = 0, 1 come from the
// neighbour at offset -1 (its halo positions 9, 10 = this tile's nodes 0, 1),
// s = 2..9 from the tile itself (positions 1..8 = nodes 0..7), s = 10 from the
// neighbour at +1 (position 0 = node 7).
__host__ __device__ constexpr int src_off(int s) { return s < 2 ? -1 : (s < 10 ? 0 : 1); }
__host__ __device__ constexpr int src_pos(int s) { return s < 2 ? s + 9 : (s < 10 ? s - 1 : 0); }

constexpr int kSrcPerLane = (kHalo3 + 63) / 64;   // 21

// Source s of a tile's 11^3 sources (z, y, x = s / 121, (s / 11) % 11,
// s % 11): the neighbour d27 = (dz + 1) 9 + (dy + 1) 3 + (dx + 1) whose halo
// holds it and its position e there; the padding sources past 11^3 read
// position 0 of the tile itself and are never summed.  Formed arithmetically:
// a table lookup per source made the gather wait on 21 dependent loads per tile.
__device__ __forceinline__ void src_of(int s, int &d27, int &e) {
  const int sz = s / (kHalo * kHalo), r = s - sz * (kHalo * kHalo), sy = r / kHalo, sx = r - sy * kHalo;
  d27 = (src_off(sz) + 1) * 9 + (src_off(sy) + 1) * 3 + (src_off(sx) + 1);
  e = (src_pos(sz) * kHalo + src_pos(sy)) * kHalo + src_pos(sx);
  if (s >= kHalo3) {
    d27 = 13;
    e = 0;
  }
}

// Waves take the touched tiles of the binning's list (four per block, round
// robin).  For each component, every lane loads its share of the 11^3
// sources (the neighbours' reduced halos; all loads in flight at once) into
// LDS; then each lane adds, for its nodes (x, y) = (l % 8, l / 8) on the 8
// z-planes, the sources that cover them.  Per dimension a node has two source
// slots in ascending neighbour offset (offset -1 for nodes 0, 1; the tile
// itself; offset +1 for node 7), the second one empty for nodes 2..6; the 8
// slot combinations are added in the fixed order (z, y, x), an empty slot
// adding zero.
template <typename T>
__global__ __launch_bounds__(256) void k_spread_gather(const int32_t *__restrict__ touch_list,
                                                       const int32_t *__restrict__ counts,
                                                       const int32_t *__restrict__ tile_nit,
                                                       const int32_t *__restrict__ tile_item0,
                                                       const T *__restrict__ partials, int n, int nz, int log2nt,
                                                       int ntz, T *__restrict__ Fgrid) {
  __shared__ T Vs[4][kSrcPerLane * 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ntouch = counts[2];
  const int tmask = (1 << log2nt) - 1;
  const int64_t G = (int64_t)n * n * nz;
  const int px = lane & 7, py = lane >> 3;
  // source slots of this lane's column: x, y positions in the 11^3 source cube
  const int x0 = px <= 1 ? px : px + 2, x1 = px <= 1 ? px + 2 : 10;
  const int y0 = py <= 1 ? py : py + 2, y1 = py <= 1 ? py + 2 : 10;
  const bool hx1 = px <= 1 || px == 7, hy1 = py <= 1 || py == 7;
  T *Vw = Vs[w];
  // blocks in runs of 16 per XCD: neighbouring tiles read neighbouring parts of the same halos
  for (int li = xcd_runs<16>(blockIdx.x, gridDim.x) * 4 + w; li < ntouch; li += gridDim.x * 4) {
    const int tile = touch_list[li];
    const int T1 = tile & tmask, T2 = (tile >> log2nt) & tmask, T3 = tile >> (2 * log2nt);
    int nb_base = -1;                     // first halo value of neighbour `lane`, -1 without markers
    if (lane < 27) {
      const int dx = lane % 3 - 1, dy = (lane / 3) % 3 - 1, dz = lane / 9 - 1;
      const int t2 = (((((T3 + dz + ntz) % ntz) << log2nt) | ((T2 + dy) & tmask)) << log2nt) | ((T1 + dx) & tmask);
      if (tile_nit[t2] > 0) nb_base = tile_item0[t2] * kPartStride;
    }
    T *dst = Fgrid + (((int64_t)(8 * T3) * n + 8 * T2 + py) * n + 8 * T1 + px);
    int soff[kSrcPerLane];
#pragma unroll
    for (int i = 0; i < kSrcPerLane; i++) {
      const int sidx = lane + 64 * i;
      int d27, e;
      src_of(sidx, d27, e);
      const int b = __shfl(nb_base, d27, 64);
      soff[i] = b >= 0 ? b + e : -1;
    }
    for (int c = 0; c < 3; c++) {
      T v[kSrcPerLane];
#pragma unroll
      for (int i = 0; i < kSrcPerLane; i++) {
        const T x = partials[(soff[i] >= 0 ? soff[i] : 0) + c * kHalo3];
        v[i] = soff[i] >= 0 ? x : T(0);
      }
      wave_sync_lds();   // the previous component's sums have read the sources
#pragma unroll
      for (int i = 0; i < kSrcPerLane; i++) Vw[lane + 64 * i] = v[i];
      wave_sync_lds();
#pragma unroll
      for (int k = 0; k < 8; k++) {
        const int z0 = k <= 1 ? k : k + 2, z1 = k <= 1 ? k + 2 : 10;
        const bool hz1 = k <= 1 || k == 7;
        T acc = T(0);
#pragma unroll
        for (int a = 0; a < 2; a++) {
          const int zz = a ? z1 : z0;
#pragma unroll
          for (int b = 0; b < 2; b++) {
            const int yy = b ? y1 : y0;
#pragma unroll
            for (int q = 0; q < 2; q++) {
              const int xx = q ? x1 : x0;
              const T val = Vw[(zz * kHalo + yy) * kHalo + xx];
              const bool ok = (!a || hz1) && (!b || hy1) && (!q || hx1);
              acc += ok ? val : T(0);
            }
          }
        }
        dst[c * G + (int64_t)k * n * n] = acc;
      }
    }
  }
}

// Dense force grid for the ib_spread entry point: zero the tiles no spread
// force reaches.
template <typename T>
__global__ __launch_bounds__(256) void k_spread_zero(const int32_t *__restrict__ tile_touch, int n, int nz,
                                                     int log2nt, T *__restrict__ Fgrid) {
  const int tile = blockIdx.x;
  if (tile_touch[tile] != 0) return;
  const int tmask = (1 << log2nt) - 1;
  const int T1 = tile & tmask, T2 = (tile >> log2nt) & tmask, T3 = tile >> (2 * log2nt);
  const int64_t G = (int64_t)n * n * nz;
  const int base = ((8 * T3) * n + 8 * T2) * n + 8 * T1;
  for (int e = threadIdx.x; e < 3 * 512; e += 256) {
    const int c = e >> 9, p = e & 511;
    Fgrid[c * G + base + ((int64_t)(p >> 6) * n + ((p >> 3) & 7)) * n + (p & 7)] = T(0);
  }
}

template <typename T>
hipError_t launch_prep(ib_ctx *c, const double *X, const double *F) {
  if (c->M == 0) return hipSuccess;
  PhaseScope ps(c, PH_PREP);
  hipLaunchKernelGGL(k_prep<T>, dim3((unsigned)((c->M + 255) / 256)), dim3(256), 0, c->stream,
                     c->ws.vals[c->sorted_buf], c->ws.keys[c->sorted_buf], X,
                     c->mat.disp ? c->mat.X_ref : nullptr, F, c->M, c->h, (Rec<T> *)c->ws.recs);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spread(ib_ctx *c, T *Fgrid, bool dense, double scale) {
  {
    PhaseScope ps(c, PH_SPREAD);
    if (c->M > 0)
      hipLaunchKernelGGL(k_spread<T>, dim3(c->nchunks), dim3(64), 0, c->stream, c->ws.chunk_item0, c->chunk, c->M,
                         (const Rec<T> *)c->ws.recs, (T)scale, (T *)c->ws.partials);
  }
  if (c->M > 0) {
    PhaseScope ps(c, PH_SPLIT);
    hipLaunchKernelGGL(k_split_reduce<T>, dim3((unsigned)std::min<int64_t>(c->ntiles, 4 * c->ncu)), dim3(256), 0,
                       c->stream, c->ws.split_list, c->ws.nitems, c->ws.tile_nit, c->ws.tile_item0,
                       (T *)c->ws.partials);
  }
  PhaseScope ps(c, PH_GATHER);
  hipLaunchKernelGGL(k_spread_gather<T>, dim3((unsigned)std::min<int64_t>((c->ntiles + 3) / 4, 5 * c->ncu)),
                     dim3(256), 0, c->stream, c->ws.touch_list, c->ws.nitems, c->ws.tile_nit, c->ws.tile_item0,
                     (const T *)c->ws.partials, c->n, c->nz, c->log2nt, c->ntz, Fgrid);
  if (dense)
    hipLaunchKernelGGL(k_spread_zero<T>, dim3((unsigned)c->ntiles), dim3(256), 0, c->stream, c->ws.tile_touch, c->n,
                       c->nz, c->log2nt, Fgrid);
  return hipGetLastError();
}

template hipError_t launch_prep<float>(ib_ctx *, const double *, const double *);
template hipError_t launch_prep<double>(ib_ctx *, const double *, const double *);
template hipError_t launch_spread<float>(ib_ctx *, float *, bool, double);
template hipError_t launch_spread<double>(ib_ctx *, double *, bool, double);

}  // namespace ib
