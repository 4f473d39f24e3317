// Interpolation and marker move, sub-step 4 (eq. discreteX), and the two
// gathers of the adjoint step that share its stencil.
//
// k_interp: blocks of 256 threads take the work items of the binning (the
// part of one 8^3-cell tile inside one chunk of the sorted markers) round robin.  For each item the block
// stages the velocity on the tile's 11^3 halo (nodes -1 .. 9, wrapped) in LDS,
// three components per node; then each thread interpolates one marker at a
// time from LDS.  The weights come from the same X^n fractional offsets the
// spread used (eq. discreteX interpolates u^{n+1} at X^n).
//
// These gathers weight the grid values (fluid precision) with FP64 weights,
// formed from the FP64 positions, and sum in FP64, in both fluid precisions;
// the position update X += dt U is FP64.  Membrane markers lie far closer
// together than h and read the same grid values, so the differences of their
// velocities (which set the membrane's strain rates, and through them the
// stretch and bend forces) keep the grid values' relative accuracy only if
// the weights and sums do not round: with FP32 weights the second difference
// of U across three neighbouring markers would carry an FP32 rounding of U
// itself, orders of magnitude above the difference.
#include <algorithm>

#include "dev_common.h"
#include "ib_internal.h"

namespace ib {

struct Cell {
  int x, y, z;
};

// Cell of a key: tile * 512 + (lz * 8 + ly) * 8 + lx.
__device__ __forceinline__ Cell key_cell(uint32_t key, int log2nt) {
  const uint32_t tile = key >> 9, tmask = (1u << log2nt) - 1u;
  return Cell{(int)(((tile & tmask) << 3) | (key & 7u)), (int)((((tile >> log2nt) & tmask) << 3) | ((key >> 3) & 7u)),
              (int)(((tile >> (2 * log2nt)) << 3) | ((key >> 6) & 7u))};
}

__device__ __forceinline__ void wave_sync_lds_i() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// velocity of one halo node, padded to a 16-byte (FP32) or 32-byte (FP64) vector
template <typename T>
struct alignas(4 * sizeof(T)) U4 {
  T x, y, z, pad;
};

constexpr int kInterpThreads = 256;
constexpr int kInterpPer = 4;     // markers per thread per round

// Fractional offset s - floor(s), s = x / h, in FP64: the same value the
// force pass stores in the record (rounded there to the fluid precision).
__device__ __forceinline__ double frac_of(double x, double h) {
  const double s = x / h;
  return s - floor(s);
}

// One marker at position x (its cell is the record's key): interpolate u from
// the staged halo with FP64 weights, summing in FP64.
template <typename T>
__device__ __forceinline__ void interp_one(const U4<T> *uh, uint32_t key, const double x[3], double h, double &a0,
                                           double &a1, double &a2) {
  double wx[4], wy[4], wz[4];
  phi4<double>(frac_of(x[0], h), wx);
  phi4<double>(frac_of(x[1], h), wy);
  phi4<double>(frac_of(x[2], h), wz);
  const int base = halo_base(key);
  a0 = a1 = a2 = 0.0;
#pragma unroll
  for (int c3 = 0; c3 < 4; c3++) {
#pragma unroll
    for (int c2 = 0; c2 < 4; c2++) {
      const int row = base + c3 * (kHalo * kHalo) + c2 * kHalo;
      const double wyz = wy[c2] * wz[c3];
#pragma unroll
      for (int c1 = 0; c1 < 4; c1++) {
        const U4<T> v = uh[row + c1];
        const double wt = wx[c1] * wyz;
        a0 += (double)v.x * wt;
        a1 += (double)v.y * wt;
        a2 += (double)v.z * wt;
      }
    }
  }
}

// Per round a thread takes up to kInterpPer markers: all their cell-key and
// marker-id loads, and the halo loads, are issued together, then the position
// loads, so that an item costs a few memory round trips.
template <typename T, bool DISP>
__global__ __launch_bounds__(kInterpThreads) void k_interp(const int32_t *__restrict__ tile_start,
                                                           const int32_t *__restrict__ tile_item0,
                                                           const int32_t *__restrict__ item_tile, int chunk,
                                                           const int32_t *__restrict__ counts,
                                                           const int32_t *__restrict__ perm,
                                                           const uint32_t *__restrict__ keys, const T *__restrict__ u,
                                                           int n, int nz, int log2nt, int64_t M, double h,
                                                           double dt, const double *__restrict__ Xpos,
                                                           const double *__restrict__ Y, double *__restrict__ X,
                                                           double *__restrict__ U) {
  __shared__ U4<T> uh[kHalo3];
  const int tid = threadIdx.x;
  const int W = counts[0];
  const int mask = n - 1, tmask = (1 << log2nt) - 1;
  const int64_t G = (int64_t)n * n * nz;
  constexpr int kPer = (kHalo3 + kInterpThreads - 1) / kInterpThreads;
  // blocks in runs of 16 per XCD: neighbouring items (tiles) share halo rows in its L2
  for (int item = xcd_runs<16>(blockIdx.x, gridDim.x); item < W; item += gridDim.x) {
    const int tile = item_tile[item];
    int j0, j1;
    item_range(item, tile_start, tile_item0, item_tile, chunk, &j0, &j1);
    {
      // a tile that fits one round is taken whole by its first item's block:
      // its halo is staged once rather than once per chunk it meets
      const int ts = tile_start[tile], te = tile_start[tile + 1];
      if (te - ts <= kInterpThreads * kInterpPer) {
        if (item != tile_item0[tile]) continue;
        j0 = ts;
        j1 = te;
      }
    }
    const int x0 = 8 * (tile & tmask) - 1, y0 = 8 * ((tile >> log2nt) & tmask) - 1, z0 = 8 * (tile >> (2 * log2nt)) - 1;
    // every load below is issued unconditionally (indices clamped), so that
    // the waits for them are exact
    T hv[kPer][3];
#pragma unroll
    for (int i = 0; i < kPer; i++) {
      const int e = min(tid + kInterpThreads * i, kHalo3 - 1);
      const int hz = e / (kHalo * kHalo), r = e - hz * (kHalo * kHalo), hy = r / kHalo, hx = r - hy * kHalo;
      const int64_t p = ((int64_t)wrap_cell(z0 + hz, nz) * n + ((y0 + hy) & mask)) * n + ((x0 + hx) & mask);
      hv[i][0] = u[p];
      hv[i][1] = u[G + p];
      hv[i][2] = u[2 * G + p];
    }
    // first round's cell keys and ids, in flight with the halo loads
    uint32_t key[kInterpPer];
    int64_t q[kInterpPer];
#pragma unroll
    for (int m = 0; m < kInterpPer; m++) {
      const int j = min(j0 + tid + kInterpThreads * m, j1 - 1);
      key[m] = keys[j];
      q[m] = perm[j];
    }
    __syncthreads();   // the previous item's reads of the halo are done
#pragma unroll
    for (int i = 0; i < kPer; i++) {
      const int e = tid + kInterpThreads * i;
      if (e < kHalo3) {
        U4<T> v;
        v.x = hv[i][0];
        v.y = hv[i][1];
        v.z = hv[i][2];
        v.pad = T(0);
        uh[e] = v;
      }
    }
    __syncthreads();
    for (int jr = j0; jr < j1; jr += kInterpThreads * kInterpPer) {
      if (jr > j0) {
#pragma unroll
        for (int m = 0; m < kInterpPer; m++) {
          const int j = min(jr + tid + kInterpThreads * m, j1 - 1);
          key[m] = keys[j];
          q[m] = perm[j];
        }
      }
      // the state at step n (Xpos = X when moving: positions, or displacements
      // with Y the reference shape) for the weights and the move
      double xo[kInterpPer][3], yo[kInterpPer][3];
#pragma unroll
      for (int m = 0; m < kInterpPer; m++) {
        xo[m][0] = Xpos[q[m]];
        xo[m][1] = Xpos[M + q[m]];
        xo[m][2] = Xpos[2 * M + q[m]];
        if (DISP) {
          yo[m][0] = Y[q[m]];
          yo[m][1] = Y[M + q[m]];
          yo[m][2] = Y[2 * M + q[m]];
        }
      }
#pragma unroll
      for (int m = 0; m < kInterpPer; m++) {
        const int j = jr + tid + kInterpThreads * m;
        if (j < j1) {
          double a0, a1, a2;
          if (DISP) {
            const double pos[3] = {yo[m][0] + xo[m][0], yo[m][1] + xo[m][1], yo[m][2] + xo[m][2]};
            interp_one<T>(uh, key[m], pos, h, a0, a1, a2);
          } else {
            interp_one<T>(uh, key[m], xo[m], h, a0, a1, a2);
          }
          if (U) {
            U[q[m]] = a0;
            U[M + q[m]] = a1;
            U[2 * M + q[m]] = a2;
          }
          if (X) {
            X[q[m]] = xo[m][0] + dt * a0;
            X[M + q[m]] = xo[m][1] + dt * a1;
            X[2 * M + q[m]] = xo[m][2] + dt * a2;
          }
        }
      }
    }
  }
}

// ------------------------------------------------- adjoint gathers ----
// Both adjoint gathers take the work items like k_interp: a block stages the
// grid field on the item's tile halo in LDS (three components per node),
// then each thread takes one of the item's sorted markers at a time and sums
// its 4^3 stencil from LDS.  The sums are separable: per x row against the x
// weight and its derivative, then the rows against the y and z factors.  A
// tile that fits one block round is taken whole by its first item's block.
template <typename T, typename Body>
__device__ __forceinline__ void adj_items(U4<T> *uh, const int32_t *__restrict__ tile_start,
                                          const int32_t *__restrict__ tile_item0,
                                          const int32_t *__restrict__ item_tile, int chunk, int W,
                                          const T *__restrict__ g, int n, int nz, int log2nt, Body body) {
  const int tid = threadIdx.x;
  const int mask = n - 1, tmask = (1 << log2nt) - 1;
  const int64_t G = (int64_t)n * n * nz;
  constexpr int kPer = (kHalo3 + kInterpThreads - 1) / kInterpThreads;
  for (int item = xcd_runs<16>(blockIdx.x, gridDim.x); item < W; item += gridDim.x) {
    const int tile = item_tile[item];
    int j0, j1;
    item_range(item, tile_start, tile_item0, item_tile, chunk, &j0, &j1);
    {
      const int ts = tile_start[tile], te = tile_start[tile + 1];
      if (te - ts <= kInterpThreads * kInterpPer) {
        if (item != tile_item0[tile]) continue;
        j0 = ts;
        j1 = te;
      }
    }
    const int x0 = 8 * (tile & tmask) - 1, y0 = 8 * ((tile >> log2nt) & tmask) - 1, z0 = 8 * (tile >> (2 * log2nt)) - 1;
    T hv[kPer][3];
#pragma unroll
    for (int i = 0; i < kPer; i++) {   // every load issued (indices clamped) before the stores
      const int e = min(tid + kInterpThreads * i, kHalo3 - 1);
      const int hz = e / (kHalo * kHalo), r = e - hz * (kHalo * kHalo), hy = r / kHalo, hx = r - hy * kHalo;
      const int64_t p = ((int64_t)wrap_cell(z0 + hz, nz) * n + ((y0 + hy) & mask)) * n + ((x0 + hx) & mask);
      hv[i][0] = g[p];
      hv[i][1] = g[G + p];
      hv[i][2] = g[2 * G + p];
    }
    __syncthreads();   // the previous item's reads of the halo are done
#pragma unroll
    for (int i = 0; i < kPer; i++) {
      const int e = tid + kInterpThreads * i;
      if (e < kHalo3) {
        U4<T> v;
        v.x = hv[i][0];
        v.y = hv[i][1];
        v.z = hv[i][2];
        v.pad = T(0);
        uh[e] = v;
      }
    }
    __syncthreads();
    for (int j = j0 + tid; j < j1; j += kInterpThreads) body(j);
  }
}

// Weights and their derivatives of one marker (FP64, from its FP64 position).
struct StencilW {
  double wx[4], wy[4], wz[4], gx[4], gy[4], gz[4];
};
__device__ __forceinline__ StencilW stencil_w(const double *__restrict__ X, const double *__restrict__ Y, int64_t M,
                                              int64_t q, double h) {
  StencilW s;
  double x0 = X[q], x1 = X[M + q], x2 = X[2 * M + q];
  if (Y) {   // the position Y + D with displacements as the state: both loaded before either is used
    const double y0 = Y[q], y1 = Y[M + q], y2 = Y[2 * M + q];
    x0 = y0 + x0;
    x1 = y1 + x1;
    x2 = y2 + x2;
  }
  const double f0 = frac_of(x0, h), f1 = frac_of(x1, h), f2 = frac_of(x2, h);
  phi4<double>(f0, s.wx);
  phi4<double>(f1, s.wy);
  phi4<double>(f2, s.wz);
  dphi4<double>(f0, s.gx);
  dphi4<double>(f1, s.gy);
  dphi4<double>(f2, s.gz);
  return s;
}

// Adjoint of the interpolation and move.  With Ubar = dt Xbar (Xbar at n+1):
//   Xbar_q += sum_x (u^{n+1}(x) . Ubar_q) dPhi_q/dX_q      (phi' term)
// and Ubar is staged (sorted order, fluid precision) for the transpose of
// interpolation, a spread without the 1/h^3 factor.
// The gather is in FP64 (weights from the FP64 position X^n, as in k_interp).
template <typename T>
__global__ __launch_bounds__(kInterpThreads) void k_adj_interp(
    const int32_t *__restrict__ tile_start, const int32_t *__restrict__ tile_item0,
    const int32_t *__restrict__ item_tile, int chunk, const int32_t *__restrict__ counts,
    const uint32_t *__restrict__ keys, const int32_t *__restrict__ perm, Rec<T> *__restrict__ recs,
    const T *__restrict__ u, int n, int nz, int log2nt, int64_t M, double h, double dt,
    const double *__restrict__ X, const double *__restrict__ Y, double *__restrict__ Xbar) {
  __shared__ U4<T> uh[kHalo3];
  adj_items<T>(uh, tile_start, tile_item0, item_tile, chunk, counts[0], u, n, nz, log2nt, [&](int j) {
    const uint32_t key = keys[j];
    const int64_t q = perm[j];
    const double xb0 = Xbar[q], xb1 = Xbar[M + q], xb2 = Xbar[2 * M + q];
    const double ub0 = dt * xb0, ub1 = dt * xb1, ub2 = dt * xb2;
    // stage Ubar as the record's force: the transpose of interpolation is a spread
    recs[j].F[0] = (T)ub0;
    recs[j].F[1] = (T)ub1;
    recs[j].F[2] = (T)ub2;
    const StencilW w = stencil_w(X, Y, M, q, h);
    const int base = halo_base(key);
    double g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
    for (int c3 = 0; c3 < 4; c3++) {
#pragma unroll
      for (int c2 = 0; c2 < 4; c2++) {
        const int row = base + c3 * (kHalo * kHalo) + c2 * kHalo;
        double sw = 0, sg = 0;
#pragma unroll
        for (int c1 = 0; c1 < 4; c1++) {
          const U4<T> v = uh[row + c1];
          const double uU = (double)v.x * ub0 + (double)v.y * ub1 + (double)v.z * ub2;
          sw += w.wx[c1] * uU;
          sg += w.gx[c1] * uU;
        }
        g0 += (w.wy[c2] * w.wz[c3]) * sg;
        g1 += (w.gy[c2] * w.wz[c3]) * sw;
        g2 += (w.wy[c2] * w.gz[c3]) * sw;
      }
    }
    Xbar[q] = xb0 + g0 / h;
    Xbar[M + q] = xb1 + g1 / h;
    Xbar[2 * M + q] = xb2 + g2 / h;
  });
}

// Adjoint of the spreading, with Fbar = scale_F * ubar^n (scale_F = dt/rho):
//   fbar_q = sum_x Fbar(x) Phi_q / h^3,
//   Xbar_q += sum_x (Fbar(x) . f_q) dPhi_q/dX_q / h^3.
// The gather is in FP64 (weights from the FP64 position X^n, as in k_interp):
// fbar feeds the elastic Hessian, whose stretch and bend parts difference it
// across neighbouring markers.
template <typename T>
__global__ __launch_bounds__(kInterpThreads) void k_adj_spread(
    const int32_t *__restrict__ tile_start, const int32_t *__restrict__ tile_item0,
    const int32_t *__restrict__ item_tile, int chunk, const int32_t *__restrict__ counts,
    const uint32_t *__restrict__ keys, const int32_t *__restrict__ perm, const T *__restrict__ ub,
    const double *__restrict__ F, int n, int nz, int log2nt, int64_t M, double scale, double h,
    const double *__restrict__ X, const double *__restrict__ Y, double *__restrict__ Xbar,
    double *__restrict__ fbar) {
  __shared__ U4<T> uh[kHalo3];
  adj_items<T>(uh, tile_start, tile_item0, item_tile, chunk, counts[0], ub, n, nz, log2nt, [&](int j) {
    const uint32_t key = keys[j];
    const int64_t q = perm[j];
    const double f0 = F[q], f1 = F[M + q], f2 = F[2 * M + q];
    const double xb0 = Xbar[q], xb1 = Xbar[M + q], xb2 = Xbar[2 * M + q];   // read with the others
    const StencilW w = stencil_w(X, Y, M, q, h);
    const int base = halo_base(key);
    double a0 = 0, a1 = 0, a2 = 0, g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
    for (int c3 = 0; c3 < 4; c3++) {
#pragma unroll
      for (int c2 = 0; c2 < 4; c2++) {
        const int row = base + c3 * (kHalo * kHalo) + c2 * kHalo;
        double s0 = 0, s1 = 0, s2 = 0, sf = 0, sg = 0;
#pragma unroll
        for (int c1 = 0; c1 < 4; c1++) {
          const U4<T> v = uh[row + c1];
          const double b0 = v.x, b1 = v.y, b2 = v.z;
          const double Ff = b0 * f0 + b1 * f1 + b2 * f2;
          s0 += w.wx[c1] * b0;
          s1 += w.wx[c1] * b1;
          s2 += w.wx[c1] * b2;
          sf += w.wx[c1] * Ff;
          sg += w.gx[c1] * Ff;
        }
        const double wyz = w.wy[c2] * w.wz[c3];
        a0 += wyz * s0;
        a1 += wyz * s1;
        a2 += wyz * s2;
        g0 += wyz * sg;
        g1 += (w.gy[c2] * w.wz[c3]) * sf;
        g2 += (w.wy[c2] * w.gz[c3]) * sf;
      }
    }
    fbar[q] = scale * a0;
    fbar[M + q] = scale * a1;
    fbar[2 * M + q] = scale * a2;
    Xbar[q] = xb0 + scale * g0 / h;
    Xbar[M + q] = xb1 + scale * g1 / h;
    Xbar[2 * M + q] = xb2 + scale * g2 / h;
  });
}

template <typename T>
hipError_t launch_interp(ib_ctx *c, const T *u, const double *X_pos, double *X_inout, double *U_out, double dt) {
  if (c->M == 0) return hipSuccess;
  PhaseScope ps(c, PH_INTERP);
  // 16 blocks per CU (4 resident in FP32, 3 in FP64): a block takes a few
  // items, so blocks that draw light items leave early and the rest queue
  // behind them (measured: 68 us at 256^3 + 1.5M markers against 82 with one
  // resident round)
  const int grid = (int)std::min<int64_t>(c->item_cap, (int64_t)c->ncu * 16);
  // the displacement form (positions Y + X) as its own kernel, so that the
  // position form holds no registers for Y
  hipLaunchKernelGGL((c->mat.disp ? k_interp<T, true> : k_interp<T, false>), dim3(grid), dim3(kInterpThreads), 0,
                     c->stream, c->ws.tile_start, c->ws.tile_item0, c->ws.item_tile, c->chunk, c->ws.nitems,
                     c->ws.vals[c->sorted_buf], c->ws.keys[c->sorted_buf], u, c->n, c->nz, c->log2nt, c->M, c->h, dt,
                     X_pos, c->mat.disp ? c->mat.X_ref : nullptr, X_inout, U_out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_interp(ib_ctx *c, const T *u_np1, const double *X_n, double *Xbar) {
  if (c->M == 0) return hipSuccess;
  PhaseScope ps(c, PH_ADJ_INTERP);
  const int grid = (int)std::min<int64_t>(c->item_cap, (int64_t)c->ncu * 16);   // as k_interp
  hipLaunchKernelGGL(k_adj_interp<T>, dim3(grid), dim3(kInterpThreads), 0, c->stream, c->ws.tile_start,
                     c->ws.tile_item0, c->ws.item_tile, c->chunk, c->ws.nitems, c->ws.keys[c->sorted_buf],
                     c->ws.vals[c->sorted_buf], (Rec<T> *)c->ws.recs, u_np1, c->n, c->nz, c->log2nt, c->M, c->h,
                     c->p.dt, X_n, c->mat.disp ? c->mat.X_ref : nullptr, Xbar);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_spread(ib_ctx *c, const T *ubar_n, const double *F, const double *X_n, double *Xbar,
                             double *fbar) {
  if (c->M == 0) return hipSuccess;
  PhaseScope ps(c, PH_ADJ_SPREAD);
  const double scale = (c->p.dt / c->p.rho) / (c->h * c->h * c->h);
  const int grid = (int)std::min<int64_t>(c->item_cap, (int64_t)c->ncu * 16);   // as k_interp
  hipLaunchKernelGGL(k_adj_spread<T>, dim3(grid), dim3(kInterpThreads), 0, c->stream, c->ws.tile_start,
                     c->ws.tile_item0, c->ws.item_tile, c->chunk, c->ws.nitems, c->ws.keys[c->sorted_buf],
                     c->ws.vals[c->sorted_buf], ubar_n, F, c->n, c->nz, c->log2nt, c->M, scale, c->h, X_n,
                     c->mat.disp ? c->mat.X_ref : nullptr, Xbar, fbar);
  return hipGetLastError();
}

template hipError_t launch_interp<float>(ib_ctx *, const float *, const double *, double *, double *, double);
template hipError_t launch_interp<double>(ib_ctx *, const double *, const double *, double *, double *, double);
template hipError_t launch_adj_interp<float>(ib_ctx *, const float *, const double *, double *);
template hipError_t launch_adj_interp<double>(ib_ctx *, const double *, const double *, double *);
template hipError_t launch_adj_spread<float>(ib_ctx *, const float *, const double *, const double *, double *,
                                             double *);
template hipError_t launch_adj_spread<double>(ib_ctx *, const double *, const double *, const double *, double *,
                                              double *);

// Diagnostics (Sec. 5): displacement of chosen markers along given unit
// directions, disp[i] = (X[idx[i]] - X0[idx[i]]) . dir[i], and its running
// maximum magnitude env[i].  Indices outside [0, M) give NaN and leave env.
__global__ __launch_bounds__(256) void k_probe(const double *__restrict__ X, const double *__restrict__ X0,
                                               int64_t M, const int32_t *__restrict__ idx,
                                               const double *__restrict__ dir, int64_t count,
                                               double *__restrict__ disp, double *__restrict__ env) {
  const int64_t i = gtid();
  if (i >= count) return;
  const int64_t q = idx[i];
  if (q < 0 || q >= M) {
    if (disp) disp[i] = __builtin_nan("");
    return;
  }
  double d = 0.0;
  for (int c = 0; c < 3; c++) d += (X[c * M + q] - X0[c * M + q]) * dir[c * count + i];
  if (disp) disp[i] = d;
  if (env) env[i] = fmax(env[i], fabs(d));
}

hipError_t launch_probe(ib_ctx *c, const double *X, const double *X0, const int32_t *idx, const double *dir,
                        int64_t count, double *disp, double *env) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_probe, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, c->stream, X, X0, c->M, idx, dir,
                     count, disp, env);
  return hipGetLastError();
}

}  // namespace ib
