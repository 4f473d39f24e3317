// Navier-Stokes update, sub-step 3 (eqs. discreteNS1-2), by FFT.
//
// With r = u^n - dt sum_k u_k D_k^{+-} u^n + (dt/rho) F^n (explicit part of
// eq. discreteNS1, upwind as in Sec. 3.2), the implicit part is diagonal in
// Fourier space: mode m has symbols lambda = sum_d (4/h^2) sin^2(pi m_d/n) for
// -sum_k D+_k D-_k and i s_d, s_d = sin(2 pi m_d/n)/h, for D0_d, so
//   w = r^ / (1 + (mu dt/rho) lambda),   u^{n+1}^ = w - s (s.w)/|s|^2
// (w itself when s = 0).  The transform runs in five passes over HBM:
//   x: real rows -> half spectrum (n/2+1 modes), stored [c][kx][z][y];
//   y: contiguous pencils;  z: all three components of a (kx, y-block) at
//   once, forward FFT, solve/projection, inverse FFT in one kernel;
//   y inverse;  x inverse (Hermitian completion, real output, 1/n^3).
// Each pass stages a block of pencils in LDS (row stride n+1 against bank
// conflicts) and runs radix-2 butterflies there; twiddles are FP64 values
// rounded to the fluid precision.
#include "dev_common.h"
#include "ib_internal.h"

namespace ib {

constexpr int kFftThreads = 256;
constexpr int kFftCap = 4096;   // complex values of payload per x / y block
constexpr int kFftBuf = kFftCap + kFftCap / 8;   // payload plus the n+1 row padding (n >= 8)

// ---------------------------------------------------------------- RHS ----
template <typename T>
__global__ __launch_bounds__(256) void k_rhs(const T *__restrict__ u, const T *__restrict__ Fg,
                                             const int32_t *__restrict__ tile_touch, int n, int log2n, T dt,
                                             T dt_rho, T h, int convect, int fmode, T *__restrict__ r) {
  const int64_t G = (int64_t)n << (2 * log2n);
  const int64_t p = gtid();
  if (p >= G) return;
  const int mask = n - 1;
  const int x = (int)(p & mask), y = (int)((p >> log2n) & mask), z = (int)(p >> (2 * log2n));
  const T uk[3] = {u[p], u[G + p], u[2 * G + p]};
  int64_t pm[3], pp[3];
  if (convect) {
    const int64_t rowz = (int64_t)z << (2 * log2n), rowy = (int64_t)y << log2n;
    pm[0] = rowz + rowy + ((x - 1) & mask);
    pp[0] = rowz + rowy + ((x + 1) & mask);
    pm[1] = rowz + ((int64_t)((y - 1) & mask) << log2n) + x;
    pp[1] = rowz + ((int64_t)((y + 1) & mask) << log2n) + x;
    pm[2] = ((int64_t)((z - 1) & mask) << (2 * log2n)) + rowy + x;
    pp[2] = ((int64_t)((z + 1) & mask) << (2 * log2n)) + rowy + x;
  }
  // fmode: 0 no force, 1 force in the tiles the spread marked, 2 dense force field
  bool hasF = fmode == 2;
  if (fmode == 1) {
    const int nt = n >> 3;
    hasF = tile_touch[((z >> 3) * nt + (y >> 3)) * nt + (x >> 3)] != 0;
  }
  for (int c = 0; c < 3; c++) {
    const T *uc = u + c * G;
    T rv = uk[c];
    if (convect) {
      T acc = T(0);
      for (int k = 0; k < 3; k++) {
        if (uk[k] > T(0)) acc += uk[k] * ((uk[c] - uc[pm[k]]) / h);
        else if (uk[k] < T(0)) acc += uk[k] * ((uc[pp[k]] - uk[c]) / h);
      }
      rv = rv - dt * acc;
    }
    if (hasF) rv = rv + dt_rho * Fg[c * G + p];
    r[c * G + p] = rv;
  }
}

// ---------------------------------------------------------- LDS FFT ----
// In-place radix-2 decimation-in-time FFT of np pencils of length n held in
// LDS at buf[p * ps + k], each already in bit-reversed order.  Forward uses
// exp(-2 pi i k / n) (table tw, n/2 entries), inverse its conjugate.
template <typename T>
__device__ __forceinline__ void lds_fft_dit(cplx<T> *buf, int n, int log2n, int np, int ps,
                                            const cplx<T> *__restrict__ tw, bool inverse) {
  const int half_n = n >> 1;
  const int total = np * half_n;
  for (int s = 1; s <= log2n; s++) {
    const int half = 1 << (s - 1);
    const int tstep = n >> s;
    for (int b = threadIdx.x; b < total; b += kFftThreads) {
      const int p = b >> (log2n - 1);
      const int j = b & (half_n - 1);
      const int k = j & (half - 1);
      const int i0 = p * ps + ((j >> (s - 1)) << s) + k;
      const int i1 = i0 + half;
      cplx<T> wv = tw[k * tstep];
      if (inverse) wv.y = -wv.y;
      const cplx<T> a = buf[i0], bb = buf[i1];
      const T xr = bb.x * wv.x - bb.y * wv.y;
      const T xi = bb.x * wv.y + bb.y * wv.x;
      buf[i1] = cplx<T>{a.x - xr, a.y - xi};
      buf[i0] = cplx<T>{a.x + xr, a.y + xi};
    }
    __syncthreads();
  }
}

// ---- pass x, forward: real rows (c, z, y0 .. y0+yb) -> spec[c][kx][z][y] ----
template <typename T>
__global__ __launch_bounds__(256) void k_fft_x_fwd(const T *__restrict__ r, int n, int log2n, int yb,
                                                   const cplx<T> *__restrict__ tw, cplx<T> *__restrict__ spec) {
  __shared__ cplx<T> buf[kFftBuf];
  const int ps = n + 1, nh = n / 2 + 1, mask = n - 1;
  const int nyb = n / yb;
  const int b = blockIdx.x;
  const int y0 = (b % nyb) * yb, z = (b / nyb) % n, c = b / (nyb * n);
  const T *src = r + (((int64_t)c * n + z) * n + y0) * n;
  for (int e = threadIdx.x; e < yb * n; e += kFftThreads) {
    const int row = e >> log2n, x = e & mask;
    buf[row * ps + (int)bitrev((uint32_t)x, log2n)] = cplx<T>{src[e], T(0)};
  }
  __syncthreads();
  lds_fft_dit<T>(buf, n, log2n, yb, ps, tw, false);
  for (int e = threadIdx.x; e < nh * yb; e += kFftThreads) {
    const int kx = e / yb, row = e - kx * yb;
    spec[(((int64_t)c * nh + kx) * n + z) * n + y0 + row] = buf[row * ps + kx];
  }
}

// ---- pass y (forward or inverse): contiguous pencils of length n ----
template <typename T>
__global__ __launch_bounds__(256) void k_fft_y(cplx<T> *__restrict__ spec, int64_t npencils, int n, int log2n,
                                               int pb, const cplx<T> *__restrict__ tw, int inverse) {
  __shared__ cplx<T> buf[kFftBuf];
  const int ps = n + 1, mask = n - 1;
  const int64_t p0 = (int64_t)blockIdx.x * pb;
  const int np = (int)min((int64_t)pb, npencils - p0);
  cplx<T> *g = spec + p0 * n;
  for (int e = threadIdx.x; e < np * n; e += kFftThreads) {
    const int p = e >> log2n, k = e & mask;
    buf[p * ps + (int)bitrev((uint32_t)k, log2n)] = g[e];
  }
  __syncthreads();
  lds_fft_dit<T>(buf, n, log2n, np, ps, tw, inverse != 0);
  for (int e = threadIdx.x; e < np * n; e += kFftThreads) {
    const int p = e >> log2n, k = e & mask;
    g[e] = buf[p * ps + k];
  }
}

// ---- pass z with the solve: block (kx, y0 .. y0+yb), all z, 3 components ----
template <typename T, int CAP>
__global__ __launch_bounds__(256) void k_fft_z_solve(cplx<T> *__restrict__ spec, int n, int log2n, int yb,
                                                     const cplx<T> *__restrict__ tw, const T *__restrict__ lam,
                                                     const T *__restrict__ sg, T nu_dt) {
  __shared__ cplx<T> buf[CAP];
  const int ps = n + 1, nh = n / 2 + 1, mask = n - 1;
  const int nyb = n / yb;
  const int kx = blockIdx.x / nyb, y0 = (blockIdx.x % nyb) * yb;
  const int np = 3 * yb;
  const int64_t cstride = (int64_t)nh * n * n;
  // element e = ((c * n + z) * yb + row): global runs of yb values per (c, z)
  for (int e = threadIdx.x; e < np * n; e += kFftThreads) {
    const int row = e % yb, cz = e / yb, z = cz & mask, c = cz >> log2n;
    const cplx<T> v = spec[c * cstride + ((int64_t)kx * n + z) * n + y0 + row];
    buf[(c * yb + row) * ps + (int)bitrev((uint32_t)z, log2n)] = v;
  }
  __syncthreads();
  lds_fft_dit<T>(buf, n, log2n, np, ps, tw, false);
  // solve / projection for every (row, kz)
  for (int e = threadIdx.x; e < yb * n; e += kFftThreads) {
    const int row = e >> log2n, kz = e & mask;
    const int ky = y0 + row;
    const T lm = (lam[kx] + lam[ky]) + lam[kz];
    const T den = T(1) + nu_dt * lm;
    const T s0 = sg[kx], s1 = sg[ky], s2 = sg[kz];
    cplx<T> wv[3];
    for (int c = 0; c < 3; c++) {
      const cplx<T> v = buf[(c * yb + row) * ps + kz];
      wv[c] = cplx<T>{v.x / den, v.y / den};
    }
    const T ss = s0 * s0 + s1 * s1 + s2 * s2;
    if (ss > T(0)) {
      const T dr = (s0 * wv[0].x + s1 * wv[1].x + s2 * wv[2].x) / ss;
      const T di = (s0 * wv[0].y + s1 * wv[1].y + s2 * wv[2].y) / ss;
      wv[0].x -= s0 * dr; wv[0].y -= s0 * di;
      wv[1].x -= s1 * dr; wv[1].y -= s1 * di;
      wv[2].x -= s2 * dr; wv[2].y -= s2 * di;
    }
    for (int c = 0; c < 3; c++) buf[(c * yb + row) * ps + kz] = wv[c];
  }
  __syncthreads();
  // bit-reversal permutation in place (pairs k < rev(k) swap)
  for (int e = threadIdx.x; e < np * n; e += kFftThreads) {
    const int p = e >> log2n, k = e & mask;
    const int rk = (int)bitrev((uint32_t)k, log2n);
    if (k < rk) {
      const cplx<T> t = buf[p * ps + k];
      buf[p * ps + k] = buf[p * ps + rk];
      buf[p * ps + rk] = t;
    }
  }
  __syncthreads();
  lds_fft_dit<T>(buf, n, log2n, np, ps, tw, true);
  for (int e = threadIdx.x; e < np * n; e += kFftThreads) {
    const int row = e % yb, cz = e / yb, z = cz & mask, c = cz >> log2n;
    spec[c * cstride + ((int64_t)kx * n + z) * n + y0 + row] = buf[(c * yb + row) * ps + z];
  }
}

// ---- pass x, inverse: half spectrum -> real rows, scaled by 1/n^3 ----
template <typename T>
__global__ __launch_bounds__(256) void k_fft_x_inv(const cplx<T> *__restrict__ spec, int n, int log2n, int yb,
                                                   const cplx<T> *__restrict__ tw, T scale, T *__restrict__ u) {
  __shared__ cplx<T> buf[kFftBuf];
  const int ps = n + 1, nh = n / 2 + 1, mask = n - 1;
  const int nyb = n / yb;
  const int b = blockIdx.x;
  const int y0 = (b % nyb) * yb, z = (b / nyb) % n, c = b / (nyb * n);
  for (int e = threadIdx.x; e < nh * yb; e += kFftThreads) {
    const int kx = e / yb, row = e - kx * yb;
    const cplx<T> v = spec[(((int64_t)c * nh + kx) * n + z) * n + y0 + row];
    buf[row * ps + (int)bitrev((uint32_t)kx, log2n)] = v;
    if (kx > 0 && kx < n / 2)   // Hermitian completion X[n-k] = conj X[k]
      buf[row * ps + (int)bitrev((uint32_t)(n - kx), log2n)] = cplx<T>{v.x, -v.y};
  }
  __syncthreads();
  lds_fft_dit<T>(buf, n, log2n, yb, ps, tw, true);
  T *dst = u + (((int64_t)c * n + z) * n + y0) * n;
  for (int e = threadIdx.x; e < yb * n; e += kFftThreads) {
    const int row = e >> log2n, x = e & mask;
    dst[e] = buf[row * ps + x].x * scale;
  }
}

// ------------------------------------------------------------ launch ----
template <typename T>
hipError_t launch_rhs(ib_ctx *c, const T *u, const T *Fgrid, int fmode, int convect, double f_scale, T *r) {
  PhaseScope ps(c, PH_RHS);
  const double dt = c->p.dt;
  hipLaunchKernelGGL(k_rhs<T>, dim3((unsigned)((c->G + 255) / 256)), dim3(256), 0, c->stream, u, Fgrid,
                     c->ws.tile_touch, c->n, c->log2n, (T)dt, (T)f_scale, (T)c->h, convect, Fgrid ? fmode : 0, r);
  return hipGetLastError();
}

static int pow2_floor(int v) {
  int p = 1;
  while (p * 2 <= v) p *= 2;
  return p;
}

template <typename T>
hipError_t launch_fluid_solve(ib_ctx *c, const T *r, T *u_out) {
  const int n = c->n, L2 = c->log2n, nh = n / 2 + 1;
  cplx<T> *spec = (cplx<T> *)c->ws.spec;
  const cplx<T> *tw = (const cplx<T> *)c->ws.tw;
  const int yb = std::min(n, kFftCap / n);
  {  // x forward
    PhaseScope ps(c, PH_FFT_X);
    hipLaunchKernelGGL(k_fft_x_fwd<T>, dim3(3 * n * (n / yb)), dim3(kFftThreads), 0, c->stream, r, n, L2, yb, tw,
                       spec);
  }
  // y forward
  const int pb = kFftCap / n;
  const int64_t npen = (int64_t)3 * nh * n;
  const unsigned ny = (unsigned)((npen + pb - 1) / pb);
  {
    PhaseScope ps(c, PH_FFT_Y);
    hipLaunchKernelGGL(k_fft_y<T>, dim3(ny), dim3(kFftThreads), 0, c->stream, spec, npen, n, L2, pb, tw, 0);
  }
  // z forward, solve, z inverse
  constexpr int ZCAP = sizeof(T) == 4 ? 8192 : 4096;
  const int ybz = std::min(n, pow2_floor(ZCAP / (3 * (n + 1))));
  const T nu_dt = (T)(c->p.mu * c->p.dt / c->p.rho);
  {
    PhaseScope ps(c, PH_FFT_Z_SOLVE);
    hipLaunchKernelGGL((k_fft_z_solve<T, ZCAP>), dim3(nh * (n / ybz)), dim3(kFftThreads), 0, c->stream, spec, n,
                       L2, ybz, tw, (const T *)c->ws.lam, (const T *)c->ws.sgrad, nu_dt);
  }
  // y inverse
  {
    PhaseScope ps(c, PH_FFT_Y_INV);
    hipLaunchKernelGGL(k_fft_y<T>, dim3(ny), dim3(kFftThreads), 0, c->stream, spec, npen, n, L2, pb, tw, 1);
  }
  // x inverse
  {
    PhaseScope ps(c, PH_FFT_X_INV);
    hipLaunchKernelGGL(k_fft_x_inv<T>, dim3(3 * n * (n / yb)), dim3(kFftThreads), 0, c->stream, spec, n, L2, yb,
                       tw, (T)(1.0 / (double)c->G), u_out);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fluid(ib_ctx *c, const T *u_in, const T *Fg, int fmode, int convect, double f_scale, T *u_out) {
  if (fluid_reg_supported(c->n, c->nz)) return launch_fluid_reg<T>(c, u_in, Fg, fmode, convect, f_scale, u_out);
  hipError_t e = launch_rhs<T>(c, u_in, Fg, fmode, convect, f_scale, (T *)c->ws.r);
  if (e != hipSuccess) return e;
  return launch_fluid_solve<T>(c, (const T *)c->ws.r, u_out);
}

template hipError_t launch_fluid<float>(ib_ctx *, const float *, const float *, int, int, double, float *);
template hipError_t launch_fluid<double>(ib_ctx *, const double *, const double *, int, int, double, double *);
template hipError_t launch_rhs<float>(ib_ctx *, const float *, const float *, int, int, double, float *);
template hipError_t launch_rhs<double>(ib_ctx *, const double *, const double *, int, int, double, double *);
template hipError_t launch_fluid_solve<float>(ib_ctx *, const float *, float *);
template hipError_t launch_fluid_solve<double>(ib_ctx *, const double *, double *);

// Adjoint of the upwind advection for the time step's adjoint (convect = 1),
// linearised at u^n with every branch frozen at the side u_k(x) selects (no
// term where u_k(x) = 0).  With the advection A_c(x) = sum_k u_k(x) D_k u_c(x),
// a perturbation d changes it by sum_k [d_k D_k u_c + u_k D_k d_c]; the
// transpose applied to a cotangent r, gathered at each point y, is
//   out_c(y) = sum_c' r_c'(y) D_c u_c'(y)
//            + sum_k [b_k(y) - b_k(y + e_k) - f_k(y) + f_k(y - e_k)],
// b_k(x) = u_k(x) r_c(x) / h where u_k(x) > 0, f_k(x) the same where
// u_k(x) < 0.  The step's adjoint is then ubar = r - dt out.
//
// One thread per run of E = 16 / sizeof(T) consecutive x values of one row:
// the three components of u and r at the run, its y and z neighbour rows
// (16-byte loads) and its two x neighbours, all loads issued before use.
// r is read and ubar written (out of place), so no point's result waits for
// its neighbours' reads.
template <typename T>
struct AdvVec;
template <>
struct AdvVec<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct AdvVec<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};

template <typename T>
__global__ __launch_bounds__(256) void k_adv_adjoint(const T *__restrict__ u, const T *__restrict__ r, int n,
                                                     int nz, int log2n, T inv_h, T dt, T *__restrict__ ubar) {
  using V = typename AdvVec<T>::type;
  constexpr int E = 16 / sizeof(T);
  const int64_t G = (int64_t)nz << (2 * log2n);
  const int64_t e = gtid();                                    // run index
  if (e * E >= G) return;
  const int mask = n - 1;
  const int64_t p0 = e * E;                                     // first point of the run
  const int x0 = (int)(p0 & mask), y = (int)((p0 >> log2n) & mask), z = (int)(p0 >> (2 * log2n));
  const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;   // periodic z neighbours
  const int64_t zo = (int64_t)z << (2 * log2n), row = zo + ((int64_t)y << log2n);
  const int64_t rym = zo + ((int64_t)((y - 1) & mask) << log2n), ryp = zo + ((int64_t)((y + 1) & mask) << log2n);
  const int64_t rzm = ((int64_t)zm << (2 * log2n)) + ((int64_t)y << log2n);
  const int64_t rzp = ((int64_t)zp << (2 * log2n)) + ((int64_t)y << log2n);
  const int xl = (x0 - 1) & mask, xr = (x0 + E) & mask;
  // [comp][0: centre, 1: y-1, 2: y+1, 3: z-1, 4: z+1] runs, and the x neighbours
  V U[3][5], R[3][5];
  T ul[3], ur[3], rl[3], rr[3];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    const T *uk = u + k * G, *rk = r + k * G;
    U[k][0] = *(const V *)(uk + row + x0);
    U[k][1] = *(const V *)(uk + rym + x0);
    U[k][2] = *(const V *)(uk + ryp + x0);
    U[k][3] = *(const V *)(uk + rzm + x0);
    U[k][4] = *(const V *)(uk + rzp + x0);
    R[k][0] = *(const V *)(rk + row + x0);
    R[k][1] = *(const V *)(rk + rym + x0);
    R[k][2] = *(const V *)(rk + ryp + x0);
    R[k][3] = *(const V *)(rk + rzm + x0);
    R[k][4] = *(const V *)(rk + rzp + x0);
    ul[k] = uk[row + xl];
    ur[k] = uk[row + xr];
    rl[k] = rk[row + xl];
    rr[k] = rk[row + xr];
  }
  V out[3];
#pragma unroll
  for (int i = 0; i < E; i++) {
    // neighbours of point i along direction d: minus (m) and plus (p)
    auto um = [&](int k, int d) { return d == 0 ? (i == 0 ? ul[k] : U[k][0][i - 1]) : U[k][2 * d - 1][i]; };
    auto up = [&](int k, int d) { return d == 0 ? (i == E - 1 ? ur[k] : U[k][0][i + 1]) : U[k][2 * d][i]; };
    auto rm = [&](int k, int d) { return d == 0 ? (i == 0 ? rl[k] : R[k][0][i - 1]) : R[k][2 * d - 1][i]; };
    auto rp = [&](int k, int d) { return d == 0 ? (i == E - 1 ? rr[k] : R[k][0][i + 1]) : R[k][2 * d][i]; };
#pragma unroll
    for (int c = 0; c < 3; c++) {
      T acc = T(0);
      const T uc = U[c][0][i];
#pragma unroll
      for (int cp = 0; cp < 3; cp++) {
        const T v = U[cp][0][i];
        const T D = uc > T(0) ? (v - um(cp, c)) * inv_h : (uc < T(0) ? (up(cp, c) - v) * inv_h : T(0));
        acc += R[cp][0][i] * D;
      }
      const T rcp = R[c][0][i];
#pragma unroll
      for (int k = 0; k < 3; k++) {
        const T at = U[k][0][i], uup = up(k, k), udn = um(k, k);
        if (at > T(0)) acc += at * rcp * inv_h;
        if (uup > T(0)) acc -= uup * rp(c, k) * inv_h;
        if (at < T(0)) acc -= at * rcp * inv_h;
        if (udn < T(0)) acc += udn * rm(c, k) * inv_h;
      }
      out[c][i] = rcp - dt * acc;
    }
  }
#pragma unroll
  for (int c = 0; c < 3; c++) *(V *)(ubar + c * G + row + x0) = out[c];
}

// ubar = rbar - dt (dA/du)^T rbar at u^n; rbar and ubar are distinct arrays.
template <typename T>
hipError_t launch_adv_adjoint(ib_ctx *c, const T *u_n, const T *rbar, T *ubar) {
  PhaseScope ps(c, PH_ADJ_ADVECT);
  constexpr int E = 16 / sizeof(T);
  if (c->n % E != 0) return hipErrorInvalidValue;
  const unsigned g = (unsigned)((c->G / E + 255) / 256);
  hipLaunchKernelGGL(k_adv_adjoint<T>, dim3(g), dim3(256), 0, c->stream, u_n, rbar, c->n, c->nz, c->log2n,
                     (T)(1.0 / c->h), (T)c->p.dt, ubar);
  return hipGetLastError();
}

template hipError_t launch_adv_adjoint<float>(ib_ctx *, const float *, const float *, float *);
template hipError_t launch_adv_adjoint<double>(ib_ctx *, const double *, const double *, double *);

}  // namespace ib
