// Force spreading, sub-step 2 (eq. discreteF), as an atomic-free gather.
//
// F(x) = sum_q F_q delta_h(x - X_q): a marker in cell c touches the 4^3 nodes
// c-1 .. c+2, so node j receives from cells j-2 .. j+1.  One block owns an
// 8^3 tile of nodes.  It lists the markers of the 11^3 cells that can reach
// the tile -- 121 cell rows, each a contiguous run of the sorted markers
// (two binary searches per row) -- and each wave walks an equal share of
// that list.  For one marker the 64 lanes of a wave own its 64 stencil
// nodes, so no two lanes write the same node; lanes keep the running sum in
// registers while consecutive markers share a cell and flush it to the
// wave's private LDS copy of the tile when the cell changes.  The four wave
// copies are added in a fixed order.  No atomics: the result is bitwise
// reproducible from run to run.
#include "dev_common.h"
#include "ib_internal.h"

namespace ib {

constexpr int kSpreadThreads = 256;
constexpr int kRows = 121;          // (8 + 3)^2 cell rows per tile
constexpr int kSegs = kRows * 3;    // at most 3 wrapped segments per row (n = 8)

// Sorted marker records: fractional offset f = s - floor(s) per dimension and
// the spread force, both in the fluid precision (f is formed in FP64).
template <typename T>
__global__ __launch_bounds__(256) void k_prep(const int32_t *__restrict__ perm, const double *__restrict__ X,
                                              const double *__restrict__ F, int64_t M, double h,
                                              T *__restrict__ frac, T *__restrict__ Fs) {
  const int64_t i = gtid();
  if (i >= M) return;
  const int64_t q = perm[i];
  for (int d = 0; d < 3; d++) {
    const double s = X[d * M + q] / h;
    frac[d * M + i] = (T)(s - floor(s));
    if (F) Fs[d * M + i] = (T)F[d * M + q];
  }
}

__device__ __forceinline__ int lower_bound_u32(const uint32_t *__restrict__ a, int lo, int hi, uint32_t v) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

template <typename T>
struct SpreadSmem {
  T acc[4][3][512];               // per-wave tile accumulators
  T wgt[4][64][12];               // per-wave staging: 4 weights per dimension
  T frc[4][64][3];                // per-wave staging: force
  int rel[4][64];                 // per-wave staging: packed tile-relative cell
  int seg_start[kSegs];
  int seg_pref[kSegs + 1];
  int seg_shift[kSegs];           // relative x = cell x + shift
  int seg_yz[kSegs];              // packed relative (y, z)
};

__device__ __forceinline__ int pack_rel(int x, int y, int z) { return ((z + 4) << 10) | ((y + 4) << 5) | (x + 4); }

template <typename T>
__global__ __launch_bounds__(256) void k_spread(const uint32_t *__restrict__ keys,
                                                const int32_t *__restrict__ row_start,
                                                const T *__restrict__ frac, const T *__restrict__ Fs,
                                                int n, int log2n, int64_t M, T inv_h3, int dense_zero,
                                                T *__restrict__ Fgrid, int32_t *__restrict__ tile_flag) {
  __shared__ SpreadSmem<T> sm;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nt = n >> 3;
  const int tile = blockIdx.x;
  const int T1 = tile % nt, T2 = (tile / nt) % nt, T3 = tile / (nt * nt);
  const int64_t G = (int64_t)n * n * n;
  const int mask = n - 1;

  // ---- list the markers of the 121 cell rows that reach the tile ----
  int any = 0;
  if (tid < kRows) {
    const int dy = tid % 11 - 2, dz = tid / 11 - 2;
    const int cy = (8 * T2 + dy) & mask, cz = (8 * T3 + dz) & mask;
    const int r = cz * n + cy;
    const int rs = row_start[r], re = row_start[r + 1];
    int s = 0, rel = -2;
    if (re > rs) {
      any = 1;
      const uint32_t rowkey = (uint32_t)r << log2n;
      while (rel <= 8) {
        const int c0 = (8 * T1 + rel) & mask;
        const int run = min(9 - rel, n - c0);
        const int a = lower_bound_u32(keys, rs, re, rowkey + (uint32_t)c0);
        const int b = lower_bound_u32(keys, a, re, rowkey + (uint32_t)(c0 + run));
        sm.seg_start[tid * 3 + s] = a;
        sm.seg_pref[tid * 3 + s] = b - a;
        sm.seg_shift[tid * 3 + s] = rel - c0;
        sm.seg_yz[tid * 3 + s] = pack_rel(0, dy, dz);
        s++;
        rel += run;
      }
    }
    for (; s < 3; s++) {
      sm.seg_start[tid * 3 + s] = 0;
      sm.seg_pref[tid * 3 + s] = 0;
      sm.seg_shift[tid * 3 + s] = 0;
      sm.seg_yz[tid * 3 + s] = pack_rel(0, 0, 0);
    }
  }
  any = __syncthreads_or(any);
  const int base = ((8 * T3) * n + 8 * T2) * n + 8 * T1;
  if (!any) {
    if (tid == 0) tile_flag[tile] = 0;
    if (dense_zero) {
      for (int e = tid; e < 3 * 512; e += kSpreadThreads) {
        const int c = e >> 9, p = e & 511;
        const int px = p & 7, py = (p >> 3) & 7, pz = p >> 6;
        Fgrid[c * G + base + ((int64_t)pz * n + py) * n + px] = T(0);
      }
    }
    return;
  }

  // exclusive prefix over the 363 segment counts (wave 0), total in seg_pref[kSegs]
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

  // ---- each wave accumulates an equal share of the list ----
  const int K = sm.seg_pref[kSegs];
  const int j0 = (int)(((int64_t)K * w) >> 2), j1 = (int)(((int64_t)K * (w + 1)) >> 2);
  const int oa = lane & 3, ob = (lane >> 2) & 3, oc = lane >> 4;
  T acc0 = 0, acc1 = 0, acc2 = 0;
  int cur = -1;         // packed relative cell of the running sum (wave-uniform)
  int cur_p = -1;       // this lane's tile node for cur, -1 if outside
  for (int jb = j0; jb < j1; jb += 64) {
    const int j = jb + lane;
    const int cnt = min(64, j1 - jb);
    if (lane < cnt) {
      // segment holding list entry j: largest s with seg_pref[s] <= j
      int lo = 0, hi = kSegs - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sm.seg_pref[mid] <= j) lo = mid;
        else hi = mid - 1;
      }
      const int i = sm.seg_start[lo] + (j - sm.seg_pref[lo]);
      const int cx = (int)(keys[i] & (uint32_t)mask);
      const int yz = sm.seg_yz[lo];
      sm.rel[w][lane] = yz + (cx + sm.seg_shift[lo]);   // x field occupies the low 5 bits (+4 bias)
      T wv[4];
      for (int d = 0; d < 3; d++) {
        phi4<T>(frac[d * M + i], wv);
        sm.wgt[w][lane][4 * d + 0] = wv[0];
        sm.wgt[w][lane][4 * d + 1] = wv[1];
        sm.wgt[w][lane][4 * d + 2] = wv[2];
        sm.wgt[w][lane][4 * d + 3] = wv[3];
        sm.frc[w][lane][d] = Fs[d * M + i];
      }
    }
    // wave-local staging: the wave's lanes wrote it; make it visible to the wave
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int mm = 0; mm < cnt; mm++) {
      const int rp = sm.rel[w][mm];
      if (rp != cur) {
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
      }
      const T wt = (sm.wgt[w][mm][oa] * sm.wgt[w][mm][4 + ob]) * sm.wgt[w][mm][8 + oc];
      acc0 += sm.frc[w][mm][0] * wt;
      acc1 += sm.frc[w][mm][1] * wt;
      acc2 += sm.frc[w][mm][2] * wt;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  if (cur_p >= 0) {
    sm.acc[w][0][cur_p] += acc0;
    sm.acc[w][1][cur_p] += acc1;
    sm.acc[w][2][cur_p] += acc2;
  }
  __syncthreads();

  // ---- add the wave copies in a fixed order and store the tile ----
  for (int e = tid; e < 3 * 512; e += kSpreadThreads) {
    const int c = e >> 9, p = e & 511;
    const T v = (((sm.acc[0][c][p] + sm.acc[1][c][p]) + sm.acc[2][c][p]) + sm.acc[3][c][p]) * inv_h3;
    const int px = p & 7, py = (p >> 3) & 7, pz = p >> 6;
    Fgrid[c * G + base + ((int64_t)pz * n + py) * n + px] = v;
  }
  if (tid == 0) tile_flag[tile] = 1;
}

template <typename T>
hipError_t launch_prep(ib_ctx *c, const double *X, const double *F) {
  if (c->M == 0) return hipSuccess;
  PhaseScope ps(c, PH_PREP);
  hipLaunchKernelGGL(k_prep<T>, dim3((unsigned)((c->M + 255) / 256)), dim3(256), 0, c->stream,
                     c->ws.vals[c->sorted_buf], X, F, c->M, c->h, (T *)c->ws.frac, (T *)c->ws.Fs);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spread(ib_ctx *c, T *Fgrid, bool dense_zero, double scale) {
  PhaseScope ps(c, PH_SPREAD);
  const int nt = c->n / 8;
  hipLaunchKernelGGL(k_spread<T>, dim3(nt * nt * nt), dim3(kSpreadThreads), 0, c->stream,
                     c->ws.keys[c->sorted_buf], c->ws.row_start, (const T *)c->ws.frac, (const T *)c->ws.Fs,
                     c->n, c->log2n, c->M, (T)scale, dense_zero ? 1 : 0, Fgrid, c->ws.tile_flag);
  return hipGetLastError();
}

template hipError_t launch_prep<float>(ib_ctx *, const double *, const double *);
template hipError_t launch_prep<double>(ib_ctx *, const double *, const double *);
template hipError_t launch_spread<float>(ib_ctx *, float *, bool, double);
template hipError_t launch_spread<double>(ib_ctx *, double *, bool, double);

}  // namespace ib
