// Register-resident FFT passes of the Navier-Stokes update (eqs. discreteNS1-2)
// for n = 32, 64, 128, 256 along x and y, and nz = n or n / 2 along z (the
// cube, or the half-cube of Sec. 4).
//
// A length-n transform is split as n = R1 * R2 (four-step): each of the
// P = min(R1, R2) threads that own a pencil holds n / P values in registers,
// does length-R1 DFTs in registers, multiplies by exp(-2 pi i s k1 / n),
// exchanges once through LDS, and does length-R2 DFTs in registers.  The
// inverse of a transform done with (R1, R2) uses (R2, R1), which leaves every
// value in the register slot it started from.
//
// Five passes over HBM, each reading and writing its array once:
//   k_xf_rhs   r = u - dt (upwind advection) + (dt/rho) F for a block of
//              rows, kept in LDS, then transformed (two real rows packed as
//              one complex pencil), writing modes kx = 0 .. n/2 to
//              spec[c][kx][z][y], z < nz (runs of 128 bytes along y);
//   k_y        forward or inverse along y (contiguous pencils);
//   k_z_solve  forward along z for all three components of a (kx, y-block),
//              the diagonal viscous solve and the projection per mode in
//              registers, inverse along z;
//   k_xi       inverse along x, real rows, scaled by 1/(n^2 nz).
// Along z of length nz = n / s the twiddles, eigenvalues and gradient
// symbols are those of length n at stride s (exp(-2 pi i k / nz) is the
// n-table's entry s k), so one set of tables serves both lengths.
#include "dev_common.h"
#include "ib_internal.h"

namespace ib {
namespace {

// cos(2 pi k / 32) for k = 0 .. 8 (FP64, correctly rounded); the rest by symmetry.
__host__ __device__ constexpr double cos32(int k) {
  k &= 31;
  if (k > 16) k = 32 - k;
  const bool neg = k > 8;
  if (neg) k = 16 - k;
  double v = 0.0;
  switch (k) {
    case 0: v = 1.0; break;
    case 1: v = 0.9807852804032304; break;
    case 2: v = 0.9238795325112867; break;
    case 3: v = 0.8314696123025452; break;
    case 4: v = 0.7071067811865476; break;
    case 5: v = 0.5555702330196022; break;
    case 6: v = 0.3826834323650898; break;
    case 7: v = 0.19509032201612828; break;
    default: v = 0.0; break;
  }
  return neg ? -v : v;
}
__host__ __device__ constexpr double sin32(int k) { return cos32(k - 8); }

// cos(2 pi k / 24) for k = 0 .. 6 (FP64, correctly rounded); the rest by symmetry.
__host__ __device__ constexpr double cos24(int k) {
  k %= 24;
  if (k < 0) k += 24;
  if (k > 12) k = 24 - k;
  const bool neg = k > 6;
  if (neg) k = 12 - k;
  double v = 0.0;
  switch (k) {
    case 0: v = 1.0; break;
    case 1: v = 0.9659258262890683; break;
    case 2: v = 0.8660254037844386; break;
    case 3: v = 0.7071067811865476; break;
    case 4: v = 0.5; break;
    case 5: v = 0.25881904510252074; break;
    default: v = 0.0; break;
  }
  return neg ? -v : v;
}
__host__ __device__ constexpr double sin24(int k) { return cos24(k - 6); }

template <int R>
__host__ __device__ constexpr int brev_c(int i) {
  int r = 0;
  for (int b = 1, rb = R >> 1; b < R; b <<= 1, rb >>= 1)
    if (i & b) r |= rb;
  return r;
}

// 16-byte vector of the fluid precision, and its complex values
template <typename T>
struct V16;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <>
struct V16<float> {
  using type = f32x4;
  __device__ static __forceinline__ cplx<float> c(const f32x4 &a, int m) {
    return m == 0 ? cplx<float>{a.x, a.y} : cplx<float>{a.z, a.w};
  }
};
template <>
struct V16<double> {
  using type = f64x2;
  __device__ static __forceinline__ cplx<double> c(const f64x2 &a, int) { return cplx<double>{a.x, a.y}; }
};
template <typename T>
using Vec16 = typename V16<T>::type;

// 1 / x: in FP32 the hardware reciprocal refined by one Newton step
// r + r (1 - x r) (the hardware value alone, within 1 ulp but not centred,
// biased the solve measurably); a division in FP64.
__device__ __forceinline__ float recip(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(fmaf(-x, r, 1.0f), r, r);
}
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return cplx<T>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// In-register DFT of length R (1 .. 32, a power of two) on v[0 .. R), natural
// order in and out.
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_reg2(cplx<T> *v) {
#pragma unroll
  for (int i = 0; i < R; i++) {
    const int j = brev_c<R>(i);
    if (i < j) {
      const cplx<T> t = v[i];
      v[i] = v[j];
      v[j] = t;
    }
  }
#pragma unroll
  for (int len = 2; len <= R; len <<= 1) {
#pragma unroll
    for (int i0 = 0; i0 < R; i0 += len) {
#pragma unroll
      for (int k = 0; k < len / 2; k++) {
        const int m = k * (32 / len);   // angle 2 pi k / len = 2 pi m / 32
        const cplx<T> b = v[i0 + k + len / 2];
        cplx<T> tb;
        if (m == 0) {
          tb = b;
        } else if (m == 8) {             // times -i (forward) or +i (inverse)
          tb = INV ? cplx<T>{-b.y, b.x} : cplx<T>{b.y, -b.x};
        } else {
          const T wr = (T)cos32(m), wi = INV ? (T)sin32(m) : (T)(-sin32(m));
          tb = cplx<T>{b.x * wr - b.y * wi, b.x * wi + b.y * wr};
        }
        const cplx<T> a = v[i0 + k];
        v[i0 + k] = cplx<T>{a.x + tb.x, a.y + tb.y};
        v[i0 + k + len / 2] = cplx<T>{a.x - tb.x, a.y - tb.y};
      }
    }
  }
}

// In-register DFT of length R = 3 Q (Q a power of two, R | 24): the three
// decimated sequences v[3m + r] transformed with length Q, then combined,
// X[k] = sum_r W^{r k} Y_r[k mod Q], W = exp(-+2 pi i / R).
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_reg3(cplx<T> *v) {
  constexpr int Q = R / 3;
  static_assert(3 * Q == R && 24 % R == 0, "R = 3, 6, 12 or 24");
  cplx<T> a[3][Q];
#pragma unroll
  for (int r = 0; r < 3; r++)
#pragma unroll
    for (int m = 0; m < Q; m++) a[r][m] = v[3 * m + r];
#pragma unroll
  for (int r = 0; r < 3; r++) dft_reg2<T, Q, INV>(a[r]);
#pragma unroll
  for (int k = 0; k < R; k++) {
    const int km = k % Q;
    cplx<T> acc = a[0][km];
#pragma unroll
    for (int r = 1; r < 3; r++) {
      const int e = ((r * k) % R) * (24 / R);     // the angle 2 pi r k / R in 24ths of a turn
      const T wr = (T)cos24(e), wi = INV ? (T)sin24(e) : (T)(-sin24(e));
      const cplx<T> b = a[r][km];
      acc.x += b.x * wr - b.y * wi;
      acc.y += b.x * wi + b.y * wr;
    }
    v[k] = acc;
  }
}

// In-register DFT of length R: a power of two up to 32, or 3 times one (R | 24).
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_reg(cplx<T> *v) {
  if constexpr (R % 3 == 0) dft_reg3<T, R, INV>(v);
  else dft_reg2<T, R, INV>(v);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Copy a table of n values into LDS, the block's nthreads threads in turn
// (the caller synchronises before the first read).  Table reads inside the
// transforms and the solve then wait on LDS, not on the vector cache.
template <typename V>
__device__ __forceinline__ void stage_table(V *dst, const V *__restrict__ src, int n, int nthreads) {
  for (int i = (int)threadIdx.x; i < n; i += nthreads) dst[i] = src[i];
}

// Four-step transform of one pencil of length N = R1 R2 by P = min(R1, R2) threads.
//   in : v[i R1 + j]  = x[(t + P i) + R2 j],   i < R2/P, j < R1
//   out: v[i R2 + k2] = X[(t + P i) + R1 k2],  i < R1/P, k2 < R2
// xch: R1 (R2 + 1) LDS values private to the pencil.  BLOCK: the pencil's
// threads span several waves (block barrier) instead of one (wave barrier).
// tw holds exp(-2 pi i k / (TS N)); the transform reads it at stride TS.
template <typename T, int R1, int R2, bool INV, bool BLOCK, int TS = 1>
struct Fft4 {
  static constexpr int N = R1 * R2;
  static constexpr int P = R1 < R2 ? R1 : R2;
  static constexpr int E = N / P;
  static constexpr int XS = R2 + 1;
  __device__ static __forceinline__ void sync() {
    if (BLOCK) __syncthreads();
    else wave_sync();
  }
  __device__ static __forceinline__ void run(cplx<T> *v, int t, cplx<T> *xch, const cplx<T> *__restrict__ tw) {
#pragma unroll
    for (int i = 0; i < R2 / P; i++) dft_reg<T, R1, INV>(v + i * R1);
#pragma unroll
    for (int i = 0; i < R2 / P; i++) {
      const int s = t + P * i;
#pragma unroll
      for (int k1 = 1; k1 < R1; k1++) {
        cplx<T> w = tw[s * k1 * TS];
        if (INV) w.y = -w.y;
        v[i * R1 + k1] = cmul(v[i * R1 + k1], w);
      }
    }
    sync();   // xch is free (earlier users of it have finished)
#pragma unroll
    for (int i = 0; i < R2 / P; i++)
#pragma unroll
      for (int k1 = 0; k1 < R1; k1++) xch[k1 * XS + t + P * i] = v[i * R1 + k1];
    sync();
#pragma unroll
    for (int i = 0; i < R1 / P; i++)
#pragma unroll
      for (int s = 0; s < R2; s++) v[i * R2 + s] = xch[(t + P * i) * XS + s];
#pragma unroll
    for (int i = 0; i < R1 / P; i++) dft_reg<T, R2, INV>(v + i * R2);
  }
};

// Blocks go to XCDs in contiguous ranges (xcd_block): neighbouring z-planes
// then share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nblk) { return xcd_block(b, nblk); }

// --------------------------------------------- pass x, block shapes ----
template <typename T>
struct XfCfg {
  static constexpr int YB = sizeof(T) == 4 ? 16 : 8;   // rows per block: 128-byte runs of complex
};
// rows per block of the inverse x pass (16 in FP32: reads of 128-byte runs
// outweigh the occupancy that fewer rows would give)
template <typename T>
struct XiCfg {
  static constexpr int YB = XfCfg<T>::YB;
};
// rows per block of the forward x pass with the right-hand side: 8 keeps the
// staged rows and their y halo within a third of the LDS, so that several
// blocks share a CU and hide each other's load latency
template <typename T>
struct XrCfg {
  static constexpr int YB = 8;
};

template <typename T, int R1, int R2, int YB_ = XfCfg<T>::YB>
struct XfSmem {
  static constexpr int N = R1 * R2, YB = YB_, NP = 3 * YB / 2;
  static constexpr int US = N + 8;     // staged row stride: rows of one wave's pencils fall in different banks
  static constexpr int OS = YB + 1;    // output staging stride (complex values)
  static constexpr int HR = YB + 2;    // staged u rows per component (y halo of one row each side)
  static constexpr size_t U = sizeof(T) * 3 * HR * US;
  static constexpr size_t X = sizeof(cplx<T>) * NP * R1 * (R2 + 1);
  static constexpr size_t O = sizeof(cplx<T>) * 3 * (N / 2 + 1) * OS;
  static constexpr size_t XO = X > O ? X : O;
  static constexpr size_t BYTES = U > XO ? U : XO;   // forward pass: staged u, exchange, output staging
  static constexpr size_t BYTES_INV = XO;            // inverse pass: input staging, exchange
};

// Raw buffer access to the spectrum: a per-thread byte offset plus a uniform
// one, so that no per-value 64-bit address stays live in registers.  Offsets
// past num_records read 0 and drop stores.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t spec_rsrc(const void *p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ cplx<float> bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float) {
  return __builtin_bit_cast(cplx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ cplx<double> bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, double) {
  return __builtin_bit_cast(cplx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, cplx<float> v) {
  using B = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(B, v), r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, cplx<double> v) {
  using B = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(B, v), r, (int)voff, (int)soff, 0);
}

// 16-byte raw buffer load: offsets at or past the buffer's size read 0
// without a memory access.
template <typename T>
__device__ __forceinline__ Vec16<T> bload16(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  return __builtin_bit_cast(Vec16<T>, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, 0, 0));
}

// ------------------------------------------------ pass x, forward + RHS ----
// One block per (YB y rows, z), all three components.
//  1. Stage u of the rows y0-1 .. y0+YB (the outer two only with advection).
//     The same round of loads fetches this thread's first z neighbours,
//     tile flags and force, so that their latency overlaps the staging.
//  2. Right-hand side of eq. discreteNS1 per 16-byte run of one component:
//     r = u - dt (upwind advection) + f_scale F.  x and y neighbours come from
//     the staged rows, z neighbours and F from global memory; F is read only
//     in tiles the spreading touched (fmode 1), everywhere (2) or nowhere (0).
//     Upwind difference per direction: u_k (u_k > 0 ? u - u_minus : u_plus - u),
//     zero when u_k = 0, the sum scaled by dt/h once.
//  3. r replaces u in LDS; rows are transformed two per complex pencil and
//     modes kx = 0 .. n/2 written to spec[c][kx][z][y] (runs of YB complex
//     values along y).
// r never goes to HBM.
template <typename T, int R1, int R2, int YB, bool CONV>
__global__ __launch_bounds__(3 * YB / 2 * (R1 < R2 ? R1 : R2)) void k_xf_rhs(
    const T *__restrict__ u, const T *__restrict__ Fg, const uint32_t *__restrict__ touch_bits, int fmode,
    T dt_inv_h, T f_scale, const cplx<T> *__restrict__ tw, cplx<T> *__restrict__ spec, int nz) {
  using F4 = Fft4<T, R1, R2, false, false>;
  using SM = XfSmem<T, R1, R2, YB>;
  using V = Vec16<T>;
  constexpr int N = R1 * R2, P = F4::P, E = F4::E, NP = 3 * YB / 2;
  constexpr int NH = N / 2 + 1, mask = N - 1, NT = NP * P, US = SM::US, OS = SM::OS, HR = SM::HR;
  constexpr int EPC = 16 / sizeof(T), CPR = N / EPC;
  constexpr int64_t NN = (int64_t)N * N;
  const int64_t G = NN * nz;
  constexpr int RUNS = 3 * YB * CPR / NT;              // r runs per thread
  static_assert(RUNS * NT == 3 * YB * CPR, "runs must divide among the threads");
  constexpr int GMAX = sizeof(T) == 4 ? 8 : 4;
  constexpr int GR = RUNS < GMAX ? RUNS : GMAX;        // runs whose global loads are issued together
  static_assert(RUNS % GR == 0, "whole groups");
  __shared__ __attribute__((aligned(16))) unsigned char smem[SM::BYTES];
  T *us = (T *)smem;                                   // [3][HR][US] u, row y0 - 1 + lr
  __shared__ cplx<T> tw_s[N];
  stage_table(tw_s, tw, N, NT);   // read after the staging barrier
  const int nyb = N / YB;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int y0 = (b % nyb) * YB, z = b / nyb;
  const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;   // periodic z neighbours
  const int tid = threadIdx.x;
  constexpr uint32_t TB = sizeof(T);
  const __amdgpu_buffer_rsrc_t urs = spec_rsrc(u, (uint32_t)(3 * G * TB));
  const uint32_t fbytes = fmode ? (uint32_t)(3 * G * TB) : 0u;
  const __amdgpu_buffer_rsrc_t frs = spec_rsrc(Fg, fbytes);
  const int nt = N >> 3;
  // run k of this thread: staged row `row` (component row / YB, y = y0 + row % YB),
  // 16 bytes at x4; returns the run's byte offset in plane z = 0
  auto run_at = [&](int k, int &row, int &x4) {
    const int e = tid + k * NT;
    row = e / CPR;
    x4 = e % CPR;
    const int c = row / YB, y = y0 + row % YB;
    return (uint32_t)((c * G + (int64_t)y * N + x4 * EPC) * TB);
  };
  // the touched flags of the block's row of tiles (one word: the rows y0 .. y0+7
  // are one tile row, and a tile row of n <= 256 lies within one 32-bit word)
  static_assert(YB == 8 && N <= 256, "one tile row per block");
  const int trow = ((z >> 3) * nt + (y0 >> 3)) * nt;
  const uint32_t tbits = fmode == 1 ? touch_bits[trow >> 5] >> (trow & 31) : 0u;
  auto has_force = [&](int k) {
    if (fmode != 1) return fmode == 2;
    int row, x4;
    run_at(k, row, x4);
    return ((tbits >> ((x4 * EPC) >> 3)) & 1u) != 0;
  };
  V vzm[GR], vzp[GR], fv[GR];
  bool has[RUNS];
  auto issue = [&](int g0) {
#pragma unroll
    for (int k = 0; k < GR; k++) {
      int row, x4;
      const uint32_t at = run_at(g0 + k, row, x4);
      if (CONV) {
        vzm[k] = bload16<T>(urs, at + (uint32_t)(zm * NN * TB));
        vzp[k] = bload16<T>(urs, at + (uint32_t)(zp * NN * TB));
      }
      fv[k] = bload16<T>(frs, has[g0 + k] ? at + (uint32_t)(z * NN * TB) : fbytes);
    }
  };
  // 1. stage u: all 16-byte loads issued before the LDS stores
  {
#pragma unroll
    for (int k = 0; k < RUNS; k++) has[k] = has_force(k);
    constexpr int RS = CONV ? HR : YB, TOT = 3 * RS * CPR, IT = (TOT + NT - 1) / NT;
    V tmp[IT];
    auto split = [&](int e, int &c, int &lr, int &x4) {
      const int row = e / CPR;
      x4 = e % CPR;
      c = row / RS;
      lr = row % RS + (CONV ? 0 : 1);
    };
#pragma unroll
    for (int k = 0; k < IT; k++) {
      const int e = tid + k * NT;
      if (TOT % NT == 0 || e < TOT) {
        int c, lr, x4;
        split(e, c, lr, x4);
        const int y = (y0 + lr - 1) & mask;
        tmp[k] = bload16<T>(urs, (uint32_t)((c * G + ((int64_t)z * N + y) * N + x4 * EPC) * TB));
      }
    }
    issue(0);
#pragma unroll
    for (int k = 0; k < IT; k++) {
      const int e = tid + k * NT;
      if (TOT % NT == 0 || e < TOT) {
        int c, lr, x4;
        split(e, c, lr, x4);
        *(V *)(us + (c * HR + lr) * US + x4 * EPC) = tmp[k];
      }
    }
  }
  __syncthreads();
  // 2. r of this thread's runs
  V out[RUNS];
#pragma unroll
  for (int g0 = 0; g0 < RUNS; g0 += GR) {
    if (g0 > 0) issue(g0);
#pragma unroll
    for (int k = 0; k < GR; k++) {
      int row, x4;
      run_at(g0 + k, row, x4);
      const int c = row / YB, lr = row % YB + 1;
      const T *urow = us + (c * HR + lr) * US;
      const V uc = *(const V *)(urow + x4 * EPC);
      V r = uc;
      if (CONV) {
        V uk[3], vym, vyp;
#pragma unroll
        for (int cc = 0; cc < 3; cc++) uk[cc] = *(const V *)(us + (cc * HR + lr) * US + x4 * EPC);
        vym = *(const V *)(urow - US + x4 * EPC);
        vyp = *(const V *)(urow + US + x4 * EPC);
        const T xl = urow[(x4 * EPC - 1) & mask], xr = urow[(x4 * EPC + EPC) & mask];
        // backward x differences d[i] = u[i] - u[i-1]; the forward one of i is d[i+1]
        T dm[EPC + 1];
        dm[0] = uc[0] - xl;
#pragma unroll
        for (int i = 1; i < EPC; i++) dm[i] = uc[i] - uc[i - 1];
        dm[EPC] = xr - uc[EPC - 1];
#pragma unroll
        for (int i = 0; i < EPC; i++) {
          const T ucc = uc[i];
          const T dx = uk[0][i] > T(0) ? dm[i] : dm[i + 1];
          const T dy = uk[1][i] > T(0) ? ucc - vym[i] : vyp[i] - ucc;
          const T dz = uk[2][i] > T(0) ? ucc - vzm[k][i] : vzp[k][i] - ucc;
          const T acc = uk[0][i] * dx + uk[1][i] * dy + uk[2][i] * dz;
          r[i] = ucc - dt_inv_h * acc;
        }
      }
#pragma unroll
      for (int i = 0; i < EPC; i++) {
        T ri = r[i] + f_scale * fv[k][i];
        asm volatile("" : "+v"(ri));   // materialise r here, so this group's loads die before the next
        out[g0 + k][i] = ri;
      }
    }
  }
  __syncthreads();   // every staged u value has been read
#pragma unroll
  for (int k = 0; k < RUNS; k++) {
    int row, x4;
    run_at(k, row, x4);
    *(V *)(us + row * US + x4 * EPC) = out[k];         // [3][YB][US] r
  }
  __syncthreads();
  // 3. this thread's values of its pencil (rows 2rp, 2rp+1 of component c)
  const int p = tid / P, t = tid % P;
  const int c = p / (YB / 2), rp = p % (YB / 2);
  cplx<T> v[E];
#pragma unroll
  for (int i = 0; i < R2 / P; i++)
#pragma unroll
    for (int j = 0; j < R1; j++) {
      const int x = (t + P * i) + R2 * j;
      v[i * R1 + j] = cplx<T>{us[(c * YB + 2 * rp) * US + x], us[(c * YB + 2 * rp + 1) * US + x]};
    }
  __syncthreads();   // the staged rows are dead; the buffer becomes pencil exchange space
  cplx<T> *xch = (cplx<T> *)smem + p * R1 * (R2 + 1);
  F4::run(v, t, xch, tw_s);
  // spectra of the two real rows: A = (Z[k] + conj Z[-k]) / 2, B = (Z[k] - conj Z[-k]) / 2i
  wave_sync();
#pragma unroll
  for (int i = 0; i < R1 / P; i++)
#pragma unroll
    for (int k2 = 0; k2 < R2; k2++) xch[(t + P * i) + R1 * k2] = v[i * R2 + k2];
  wave_sync();
  constexpr int KM = (NH + P - 1) / P;
  cplx<T> A[KM], B[KM];
#pragma unroll
  for (int m = 0; m < KM; m++) {
    const int k = t + P * m;
    if (k < NH) {
      const cplx<T> zk = xch[k], zn = xch[(N - k) & mask];
      A[m] = cplx<T>{T(0.5) * (zk.x + zn.x), T(0.5) * (zk.y - zn.y)};
      B[m] = cplx<T>{T(0.5) * (zk.y + zn.y), T(0.5) * (zn.x - zk.x)};
    }
  }
  __syncthreads();
  cplx<T> *outs = (cplx<T> *)smem;                     // [3][NH][OS]
#pragma unroll
  for (int m = 0; m < KM; m++) {
    const int k = t + P * m;
    if (k < NH) {
      outs[(c * NH + k) * OS + 2 * rp] = A[m];
      outs[(c * NH + k) * OS + 2 * rp + 1] = B[m];
    }
  }
  __syncthreads();
  for (int e = tid; e < 3 * NH * YB; e += NT) {
    const int yy = e % YB, ck = e / YB, k = ck % NH, cc = ck / NH;
    spec[(((int64_t)cc * NH + k) * nz + z) * N + y0 + yy] = outs[ck * OS + yy];
  }
}

// ---------------------------------------------------------------- pass y ----
template <typename T, int R1, int R2, bool INV>
__global__ __launch_bounds__(256) void k_y(cplx<T> *__restrict__ spec, int64_t npencils,
                                           const cplx<T> *__restrict__ tw) {
  using F4 = Fft4<T, R1, R2, INV, false>;
  constexpr int N = R1 * R2, P = F4::P, E = F4::E, PPB = 256 / P;
  __shared__ cplx<T> xch[PPB * R1 * (R2 + 1)];
  __shared__ cplx<T> tw_s[N];
  stage_table(tw_s, tw, N, 256);
  __syncthreads();
  const int lp = threadIdx.x / P, t = threadIdx.x % P;
  const int64_t pen = (int64_t)blockIdx.x * PPB + lp;
  if (pen >= npencils) return;       // whole pencils only: the exchange is wave-local
  cplx<T> *g = spec + pen * N;
  cplx<T> v[E];
#pragma unroll
  for (int i = 0; i < R2 / P; i++)
#pragma unroll
    for (int j = 0; j < R1; j++) v[i * R1 + j] = g[(t + P * i) + R2 * j];
  F4::run(v, t, xch + lp * R1 * (R2 + 1), tw_s);
#pragma unroll
  for (int i = 0; i < R1 / P; i++)
#pragma unroll
    for (int k2 = 0; k2 < R2; k2++) g[(t + P * i) + R1 * k2] = v[i * R2 + k2];
}

// ------------------------------------------------- pass z with the solve ----
// z transforms of length NZ = R1 R2 on a grid of NY x NY x NZ nodes (NZ = NY,
// NY / 2 or 3 NY / 4) with the tables of length NZ (twz, lamz, sgz), which the
// block stages in LDS; the x and y modes read the tables of length NY (lam, sg).
template <typename T, int R1, int R2, int NY>
__global__ __launch_bounds__(XfCfg<T>::YB *(R1 < R2 ? R1 : R2), sizeof(T) == 4 ? 2 : 1) void k_z_solve(
    cplx<T> *__restrict__ spec, const cplx<T> *__restrict__ twz, const T *__restrict__ lamz,
    const T *__restrict__ sgz, const T *__restrict__ lam, const T *__restrict__ sg, T nu_dt) {
  constexpr int NZ = R1 * R2;
  using Ff = Fft4<T, R1, R2, false, true>;
  using Fi = Fft4<T, R2, R1, true, true>;
  constexpr int P = Ff::P, E = Ff::E, YB = XfCfg<T>::YB, NH = NY / 2 + 1;
  // per-y exchange space, padded to 2 (mod 32) values so that the 16 y's and
  // neighbouring t's of a wave fall in distinct LDS banks
  constexpr int XS0 = (R1 * (R2 + 1) > R2 * (R1 + 1)) ? R1 * (R2 + 1) : R2 * (R1 + 1);
  constexpr int XSZ = XS0 + ((2 - XS0 % 32) + 32) % 32;
  __shared__ cplx<T> xch[YB * XSZ];
  __shared__ cplx<T> twz_s[NZ];
  __shared__ T lamz_s[NZ], sgz_s[NZ];
  stage_table(twz_s, twz, NZ, YB * P);
  stage_table(lamz_s, lamz, NZ, YB * P);
  stage_table(sgz_s, sgz, NZ, YB * P);
  __syncthreads();
  const int nyb = NY / YB;
  const int kx = blockIdx.x / nyb, y0 = (blockIdx.x % nyb) * YB;
  const int yy = threadIdx.x % YB, t = threadIdx.x / YB;
  constexpr uint32_t CB = sizeof(cplx<T>);
  constexpr uint32_t cs = (uint32_t)NH * NZ * NY * CB;              // component stride, bytes
  const __amdgpu_buffer_rsrc_t rs = spec_rsrc(spec, 3 * cs);
  const uint32_t voff = ((uint32_t)(kx * NZ + t) * NY + y0 + yy) * CB;  // (kx, z = t, y)
  cplx<T> v[3][E];
#pragma unroll
  for (int c = 0; c < 3; c++)
#pragma unroll
    for (int i = 0; i < R2 / P; i++)
#pragma unroll
      for (int j = 0; j < R1; j++)
        v[c][i * R1 + j] = bload(rs, voff, c * cs + (uint32_t)((P * i + R2 * j) * NY) * CB, T(0));
#pragma unroll
  for (int c = 0; c < 3; c++) Ff::run(v[c], t, xch + yy * XSZ, twz_s);
  // per mode (kx, ky, kz): w = r^/(1 + nu dt lambda), then remove the s-component
  const int ky = y0 + yy;
  const T lxy = lam[kx] + lam[ky];
  const T s0 = sg[kx], s1 = sg[ky];
#pragma unroll
  for (int i = 0; i < R1 / P; i++) {
#pragma unroll
    for (int k2 = 0; k2 < R2; k2++) {
      const int e = i * R2 + k2;
      const int kz = (t + P * i) + R1 * k2;
      const T rden = recip(T(1) + nu_dt * (lxy + lamz_s[kz]));
      const T s2 = sgz_s[kz];
      cplx<T> w0{v[0][e].x * rden, v[0][e].y * rden};
      cplx<T> w1{v[1][e].x * rden, v[1][e].y * rden};
      cplx<T> w2{v[2][e].x * rden, v[2][e].y * rden};
      const T ss = s0 * s0 + s1 * s1 + s2 * s2;
      if (ss > T(0)) {
        const T rss = recip(ss);
        const T dr = (s0 * w0.x + s1 * w1.x + s2 * w2.x) * rss;
        const T di = (s0 * w0.y + s1 * w1.y + s2 * w2.y) * rss;
        w0.x -= s0 * dr; w0.y -= s0 * di;
        w1.x -= s1 * dr; w1.y -= s1 * di;
        w2.x -= s2 * dr; w2.y -= s2 * di;
      }
      v[0][e] = w0;
      v[1][e] = w1;
      v[2][e] = w2;
    }
  }
  // each component stored as soon as it is transformed back, so that its
  // stores drain while the next component's transform runs
#pragma unroll
  for (int c = 0; c < 3; c++) {
    Fi::run(v[c], t, xch + yy * XSZ, twz_s);
#pragma unroll
    for (int i = 0; i < R2 / P; i++)
#pragma unroll
      for (int j = 0; j < R1; j++) bstore(rs, voff, c * cs + (uint32_t)((P * i + R2 * j) * NY) * CB, v[c][i * R1 + j]);
  }
}

// ------------------------------------------------------ pass x, inverse ----
template <typename T, int R1, int R2, int YB>
__global__ __launch_bounds__(3 * YB / 2 * (R1 < R2 ? R1 : R2)) void k_xi(
    const cplx<T> *__restrict__ spec, const cplx<T> *__restrict__ tw, T scale, T *__restrict__ u, int nz) {
  using F4 = Fft4<T, R1, R2, true, false>;
  constexpr int N = R1 * R2, P = F4::P, E = F4::E, NP = 3 * YB / 2;
  constexpr int NH = N / 2 + 1, NT = NP * P;
  const int64_t G = (int64_t)N * N * nz;
  __shared__ __attribute__((aligned(16))) unsigned char smem[XfSmem<T, R1, R2, YB>::BYTES_INV];
  constexpr int OS = XfSmem<T, R1, R2, YB>::OS;
  cplx<T> *stage = (cplx<T> *)smem;                   // [3][NH][OS]
  const int nyb = N / YB;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int y0 = (b % nyb) * YB, z = b / nyb;
  const int tid = threadIdx.x;
  __shared__ cplx<T> tw_s[N];
  stage_table(tw_s, tw, N, NT);   // read after the staging barrier
  {
    // 16-byte loads of the (c, kx) runs along y, all issued before the LDS stores
    using V = Vec16<T>;
    constexpr int CPC = 16 / sizeof(cplx<T>), CPRUN = YB / CPC, TOT = 3 * NH * CPRUN, IT = (TOT + NT - 1) / NT;
    V tmp[IT];
#pragma unroll
    for (int k = 0; k < IT; k++) {
      const int e = tid + k * NT;
      if (e < TOT) {
        const int q = e % CPRUN, ck = e / CPRUN, kk = ck % NH, cc = ck / NH;
        tmp[k] = *(const V *)(spec + (((int64_t)cc * NH + kk) * nz + z) * N + y0 + q * CPC);
      }
    }
#pragma unroll
    for (int k = 0; k < IT; k++) {
      const int e = tid + k * NT;
      if (e < TOT) {
        const int q = e % CPRUN, ck = e / CPRUN;
#pragma unroll
        for (int m = 0; m < CPC; m++) stage[ck * OS + q * CPC + m] = V16<T>::c(tmp[k], m);
      }
    }
  }
  __syncthreads();
  const int p = tid / P, t = tid % P;
  const int c = p / (YB / 2), rp = p % (YB / 2);
  // Z[k] = A[k] + i B[k] with A, B the Hermitian spectra of rows 2rp, 2rp+1
  cplx<T> v[E];
#pragma unroll
  for (int i = 0; i < R2 / P; i++)
#pragma unroll
    for (int j = 0; j < R1; j++) {
      const int k = (t + P * i) + R2 * j;
      const bool hi = k > N / 2;
      const int kk = hi ? N - k : k;
      cplx<T> a = stage[(c * NH + kk) * OS + 2 * rp];
      cplx<T> bb = stage[(c * NH + kk) * OS + 2 * rp + 1];
      if (hi) {
        a.y = -a.y;
        bb.y = -bb.y;
      }
      v[i * R1 + j] = cplx<T>{a.x - bb.y, a.y + bb.x};
    }
  __syncthreads();   // staging is dead; the buffer becomes pencil exchange space
  F4::run(v, t, (cplx<T> *)smem + p * R1 * (R2 + 1), tw_s);
  T *ra = u + c * G + ((int64_t)z * N + y0 + 2 * rp) * N;
#pragma unroll
  for (int i = 0; i < R1 / P; i++)
#pragma unroll
    for (int k2 = 0; k2 < R2; k2++) {
      const int x = (t + P * i) + R1 * k2;
      ra[x] = v[i * R2 + k2].x * scale;
      ra[N + x] = v[i * R2 + k2].y * scale;
    }
}

// --------------------------------------- passes y and x, inverse, merged ----
// One 1024-thread block per (component, z) plane: the inverse y transforms of
// its n/2 + 1 kx pencils (each contiguous in the spectrum), kept in registers
// (two pencils per 16-thread slot; the kx = n/2 pencil by slot 0 into LDS),
// then for each half of the y rows an LDS transpose [y][kx] and the inverse x
// transforms, two real rows per complex pencil, written as rows of u.  The
// spectrum is read once and u written once: one pass over HBM for the two
// transforms.  n = 256 (R1 = R2 = 16) in FP32: the plane's spectrum (264 KB)
// fits the block's registers, the transpose of half the rows its LDS.
template <typename T, int R1, int R2>
struct YxiCfg {
  static constexpr int N = R1 * R2, NH = N / 2 + 1, P = R1 < R2 ? R1 : R2;
  static constexpr int SLOTS = 1024 / P;           // pencil slots of the block
  static constexpr int HALF = N / 2;               // y rows per transpose
  static constexpr int TS = NH;                    // transpose row stride (complex)
  static constexpr size_t XCH = sizeof(cplx<T>) * SLOTS * R1 * (R2 + 1);   // pencil exchange space
  static constexpr size_t TB = sizeof(cplx<T>) * HALF * TS;                // transpose, over the exchange space
  static constexpr size_t BYTES = (XCH > TB ? XCH : TB) + sizeof(cplx<T>) * N;   // + the kx = n/2 pencil
  static_assert(2 * SLOTS + 1 == NH && HALF == 2 * SLOTS, "two pencils per slot (and one more), two rows per x pencil");
};

template <typename T, int R1, int R2>
__global__ __launch_bounds__(1024) void k_yxi(const cplx<T> *__restrict__ spec, const cplx<T> *__restrict__ tw,
                                              T scale, T *__restrict__ u, int nz) {
  using C = YxiCfg<T, R1, R2>;
  using F4 = Fft4<T, R1, R2, true, false>;
  constexpr int N = C::N, NH = C::NH, P = C::P, E = F4::E, TS = C::TS;
  static_assert(R2 / P == 1 && R1 / P == 1, "square four-step factors");
  __shared__ __attribute__((aligned(16))) unsigned char smem[C::BYTES];
  __shared__ cplx<T> tw_s[N];
  stage_table(tw_s, tw, N, 1024);
  __syncthreads();
  const int64_t G = (int64_t)N * N * nz;
  const int c = blockIdx.x / nz, z = blockIdx.x % nz;
  const int s = threadIdx.x / P, t = threadIdx.x % P;
  cplx<T> *xch = (cplx<T> *)smem + s * R1 * (R2 + 1);
  cplx<T> *tr = (cplx<T> *)smem;                   // [HALF][TS] after the y transforms
  cplx<T> *nyq = (cplx<T> *)(smem + (C::XCH > C::TB ? C::XCH : C::TB));   // [N] the kx = n/2 pencil
  auto pencil = [&](int kx) { return spec + (((int64_t)c * NH + kx) * nz + z) * N; };
  // 1. inverse y transforms: kx = n/2 by slot 0 (into LDS), then pencils s and
  // s + SLOTS (kx) of every slot, kept in registers
  if (s == 0) {   // lanes 0 .. P-1 of wave 0 (the pencil's exchange is wave-local)
    cplx<T> vn[E];
    const cplx<T> *gn = pencil(N / 2);
#pragma unroll
    for (int j = 0; j < R1; j++) vn[j] = gn[t + R2 * j];
    F4::run(vn, t, xch, tw_s);
#pragma unroll
    for (int k2 = 0; k2 < R2; k2++) nyq[t + R1 * k2] = vn[k2];
  }
  cplx<T> va[E], vb[E];
  {
    const cplx<T> *ga = pencil(s);
#pragma unroll
    for (int j = 0; j < R1; j++) va[j] = ga[t + R2 * j];
  }
  F4::run(va, t, xch, tw_s);                          // y = t + R1 k2 in slot k2
  {
    const cplx<T> *gb = pencil(s + C::SLOTS);
#pragma unroll
    for (int j = 0; j < R1; j++) vb[j] = gb[t + R2 * j];
  }
  F4::run(vb, t, xch, tw_s);
  // 2. per half of the rows: transpose to [y][kx], inverse x transforms of
  // row pairs (2r, 2r + 1), r = s, and the rows written out
#pragma unroll
  for (int h = 0; h < 2; h++) {
    int th = threadIdx.x;
    asm volatile("" : "+v"(th));   // addresses formed anew in each half
    const int sh = th / P, tt = th % P;   // s and t
    __syncthreads();   // the previous half's exchange space is free
#pragma unroll
    for (int k2 = 0; k2 < R2 / 2; k2++) {
      const int yl = tt + R1 * k2;                  // row within the half
      tr[yl * TS + sh] = va[k2 + h * R2 / 2];
      tr[yl * TS + sh + C::SLOTS] = vb[k2 + h * R2 / 2];
    }
    __syncthreads();
    const int r0 = 2 * sh;
    cplx<T> v[E];
#pragma unroll
    for (int j = 0; j < R1; j++) {
      const int k = tt + R2 * j;
      const bool hi = k > N / 2;
      const int kk = hi ? N - k : k;
      cplx<T> a = kk == N / 2 ? nyq[h * C::HALF + r0] : tr[r0 * TS + kk];
      cplx<T> b = kk == N / 2 ? nyq[h * C::HALF + r0 + 1] : tr[(r0 + 1) * TS + kk];
      if (hi) {
        a.y = -a.y;
        b.y = -b.y;
      }
      v[j] = cplx<T>{a.x - b.y, a.y + b.x};
    }
    __syncthreads();   // the transpose is consumed: its space becomes exchange space
    F4::run(v, tt, xch, tw_s);
    T *ra = u + c * G + ((int64_t)z * N + h * C::HALF + r0) * N;
#pragma unroll
    for (int k2 = 0; k2 < R2; k2++) {
      const int x = tt + R1 * k2;
      ra[x] = v[k2].x * scale;
      ra[N + x] = v[k2].y * scale;
    }
  }
}

// The merged inverse y + x pass serves n = 256 in FP32.
template <typename T, int R1, int R2>
constexpr bool yx_merged() {
  return sizeof(T) == 4 && R1 == 16 && R2 == 16;
}

// (R1, R2): factors of n (x and y); (Z1, Z2): factors of nz (z).
template <typename T, int R1, int R2, int Z1, int Z2>
hipError_t run_reg(ib_ctx *c, const T *u_in, const T *Fg, int fmode, int convect, double f_scale, T *u_out) {
  constexpr int N = R1 * R2, P = R1 < R2 ? R1 : R2, YB = XfCfg<T>::YB, NH = N / 2 + 1;
  constexpr int NZ = Z1 * Z2, PZ = Z1 < Z2 ? Z1 : Z2;
  const int nz = c->nz;
  if (c->n != N || nz != NZ) return hipErrorInvalidValue;
  cplx<T> *spec = (cplx<T> *)c->ws.spec;
  const cplx<T> *tw = (const cplx<T> *)c->ws.tw;
  const int64_t npen = (int64_t)3 * NH * NZ;
  const unsigned ny = (unsigned)((npen + 256 / P - 1) / (256 / P));
  {
    PhaseScope ps(c, PH_RHS_FFT_X);
    const int fm = Fg ? fmode : 0;
    const T dtih = (T)c->p.dt * (T)(1.0 / c->h);
    constexpr int YR = XrCfg<T>::YB;
    if (convect)
      hipLaunchKernelGGL((k_xf_rhs<T, R1, R2, YR, true>), dim3(NZ * (N / YR)), dim3(3 * YR / 2 * P), 0, c->stream,
                         u_in, Fg, c->ws.touch_bits, fm, dtih, (T)f_scale, tw, spec, nz);
    else
      hipLaunchKernelGGL((k_xf_rhs<T, R1, R2, YR, false>), dim3(NZ * (N / YR)), dim3(3 * YR / 2 * P), 0, c->stream,
                         u_in, Fg, c->ws.touch_bits, fm, dtih, (T)f_scale, tw, spec, nz);
  }
  {
    PhaseScope ps(c, PH_FFT_Y);
    hipLaunchKernelGGL((k_y<T, R1, R2, false>), dim3(ny), dim3(256), 0, c->stream, spec, npen, tw);
  }
  {
    PhaseScope ps(c, PH_FFT_Z_SOLVE);
    hipLaunchKernelGGL((k_z_solve<T, Z1, Z2, N>), dim3(NH * (N / YB)), dim3(YB * PZ), 0, c->stream, spec,
                       (const cplx<T> *)c->ws.twz, (const T *)c->ws.lamz, (const T *)c->ws.sgradz,
                       (const T *)c->ws.lam, (const T *)c->ws.sgrad, (T)(c->p.mu * c->p.dt / c->p.rho));
  }
  if constexpr (yx_merged<T, R1, R2>()) {
    PhaseScope ps(c, PH_FFT_YX_INV);
    hipLaunchKernelGGL((k_yxi<T, R1, R2>), dim3(3 * NZ), dim3(1024), 0, c->stream, (const cplx<T> *)spec, tw,
                       (T)(1.0 / (double)c->G), u_out, nz);
    return hipGetLastError();
  }
  {
    PhaseScope ps(c, PH_FFT_Y_INV);
    hipLaunchKernelGGL((k_y<T, R1, R2, true>), dim3(ny), dim3(256), 0, c->stream, spec, npen, tw);
  }
  {
    PhaseScope ps(c, PH_FFT_X_INV);
    constexpr int YI = XiCfg<T>::YB;
    hipLaunchKernelGGL((k_xi<T, R1, R2, YI>), dim3(NZ * (N / YI)), dim3(3 * YI / 2 * P), 0, c->stream, spec, tw,
                       (T)(1.0 / (double)c->G), u_out, nz);
  }
  return hipGetLastError();
}

}  // namespace

bool fluid_reg_supported(int n, int nz) {
  return (n == 32 || n == 64 || n == 128 || n == 256) && (nz == n || 2 * nz == n || 4 * nz == 3 * n);
}

template <typename T>
hipError_t launch_fluid_reg(ib_ctx *c, const T *u_in, const T *Fg, int fmode, int convect, double f_scale,
                            T *u_out) {
  // z factors: nz = n (cube), n / 2 (half-cube), 3 n / 4 (a factor 3 along z)
  const int zk = c->nz == c->n ? 0 : (2 * c->nz == c->n ? 1 : 2);
  switch (c->n) {
    case 32:
      return zk == 0 ? run_reg<T, 8, 4, 8, 4>(c, u_in, Fg, fmode, convect, f_scale, u_out)
           : zk == 1 ? run_reg<T, 8, 4, 4, 4>(c, u_in, Fg, fmode, convect, f_scale, u_out)
                     : run_reg<T, 8, 4, 12, 2>(c, u_in, Fg, fmode, convect, f_scale, u_out);
    case 64:
      return zk == 0 ? run_reg<T, 8, 8, 8, 8>(c, u_in, Fg, fmode, convect, f_scale, u_out)
           : zk == 1 ? run_reg<T, 8, 8, 8, 4>(c, u_in, Fg, fmode, convect, f_scale, u_out)
                     : run_reg<T, 8, 8, 12, 4>(c, u_in, Fg, fmode, convect, f_scale, u_out);
    case 128:
      return zk == 0 ? run_reg<T, 16, 8, 16, 8>(c, u_in, Fg, fmode, convect, f_scale, u_out)
           : zk == 1 ? run_reg<T, 16, 8, 8, 8>(c, u_in, Fg, fmode, convect, f_scale, u_out)
                     : run_reg<T, 16, 8, 24, 4>(c, u_in, Fg, fmode, convect, f_scale, u_out);
    case 256:
      return zk == 0 ? run_reg<T, 16, 16, 16, 16>(c, u_in, Fg, fmode, convect, f_scale, u_out)
           : zk == 1 ? run_reg<T, 16, 16, 16, 8>(c, u_in, Fg, fmode, convect, f_scale, u_out)
                     : run_reg<T, 16, 16, 24, 8>(c, u_in, Fg, fmode, convect, f_scale, u_out);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_fluid_reg<float>(ib_ctx *, const float *, const float *, int, int, double, float *);
template hipError_t launch_fluid_reg<double>(ib_ctx *, const double *, const double *, int, int, double, double *);

}  // namespace ib
