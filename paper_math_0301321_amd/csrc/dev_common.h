// Device helpers shared by the IB kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ib {

template <typename T>
struct cplx {
  T x, y;
};

__device__ __forceinline__ uint64_t lanemask_lt() {
  const uint32_t lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ uint32_t bitrev(uint32_t v, int bits) {
  return __brev(v) >> (32 - bits);
}

// The four 4-point weights phi(1+f), phi(f), phi(1-f), phi(2-f) for a node
// offset f in [0, 1) (nodes floor(s)-1 .. floor(s)+2).  On [0,1] the two middle
// weights share one square root, sqrt(1 + 4f - 4f^2), and the outer ones follow
// from phi(r) = 1/2 - phi(2 - |r|) on [1, 2] (Sec. 3.2, definition of phi).
template <typename T>
__device__ __forceinline__ void phi4(T f, T w[4]) {
  const T q = sqrt(T(1) + T(4) * f - T(4) * f * f);
  const T w1 = (T(3) - T(2) * f + q) * T(0.125);
  const T w2 = (T(1) + T(2) * f + q) * T(0.125);
  w[0] = T(0.5) - w2;
  w[1] = w1;
  w[2] = w2;
  w[3] = T(0.5) - w1;
}

// Derivatives d/ds of the same four weights, phi'(s - j) for j = c-1 .. c+2.
template <typename T>
__device__ __forceinline__ void dphi4(T f, T g[4]) {
  const T q = sqrt(T(1) + T(4) * f - T(4) * f * f);
  const T dq = (T(2) - T(4) * f) / q;            // d/df sqrt(1 + 4f - 4f^2)
  const T d1 = (T(-2) + dq) * T(0.125);          // d/df phi(f)
  const T d2 = (T(2) + dq) * T(0.125);           // d/df phi(1 - f)
  g[0] = -d2;
  g[1] = d1;
  g[2] = d2;
  g[3] = -d1;
}

__device__ __forceinline__ int64_t gtid() {
  return (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
}

// Block index remapped so that each XCD (8 per device; the dispatcher deals
// blocks to them round-robin) runs one contiguous range of logical blocks and
// neighbouring blocks share its L2.  A bijection of [0, nblk) for any nblk.
__device__ __forceinline__ int xcd_block(int b, int nblk) {
  const int q = nblk >> 3, r = nblk & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

// Block index remapped so that each XCD runs groups of R consecutive logical
// blocks, the groups dealt to the XCDs in turn: neighbouring blocks share an
// L2 while every XCD still sees every part of the index range.  Blocks past
// the last whole round of 8 R keep their index.  A bijection of [0, nblk).
template <int R>
__device__ __forceinline__ int xcd_runs(int b, int nblk) {
  const int full = nblk / (8 * R) * (8 * R);
  if (b >= full) return b;
  const int x = b & 7, j = b >> 3;
  return (j / R) * (8 * R) + x * R + (j % R);
}

}  // namespace ib
