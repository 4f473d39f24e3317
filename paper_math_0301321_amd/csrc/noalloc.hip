// ib_fluid_noalloc: the Navier-Stokes update of ib_fluid (eqs. discreteNS1-2,
// solved by FFT, Sec. 3.2) without a context, for callers that cannot
// allocate device memory.  Its spectrum and tables live in `scratch`, a
// file-scope device array of kNoAllocBytes that every GPU the library runs on
// holds until the process ends.  Host code never passes the array's name to a
// kernel (in host code it is a stand-in, not a device address): the device
// address comes from hipGetSymbolAddress, once per device, and is kept in
// g_scratch_dev[].  Calls that overlap on one GPU share the array and race.
#include <math.h>

#include <mutex>
#include <string>

#include "dev_common.h"
#include "ib_internal.h"

namespace ib {
void set_context_free_error(const std::string &msg);
}

using namespace ib;

static constexpr size_t kNoAllocBytes = size_t(32) << 20;   // 32 MiB

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
constexpr double kPiD = 3.14159265358979323846;

std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of this device's scratch array (the device must be current).
hipError_t scratch_for(int dev, void **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

// Twiddles exp(-2 pi i k / n), eigenvalues (4/h^2) sin^2(pi m / n) and gradient
// symbols sin(2 pi m / n) / h (exactly 0 at m = 0, n/2) for one transform
// length n: the tables ib_create computes on the host, here in FP64 on the
// device and rounded once.
template <typename T>
__global__ __launch_bounds__(256) void k_fluid_tables(int n, double h, T *__restrict__ tw, T *__restrict__ lam,
                                                      T *__restrict__ sg) {
  const int k = (int)gtid();
  if (k >= n) return;
  const double a = 2.0 * kPiD * (double)k / (double)n;
  tw[2 * k] = (T)cos(a);
  tw[2 * k + 1] = (T)(-sin(a));
  const double sh = sin(kPiD * (double)k / (double)n);
  lam[k] = (T)((4.0 / (h * h)) * sh * sh);
  sg[k] = (k == 0 || 2 * k == n) ? T(0) : (T)(sin(a) / h);
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

template <typename T>
int fluid_noalloc(const ib_params *p, int nz, T *u, const T *F) {
  const int n = p->n;
  const size_t ts = sizeof(T);
  const size_t spec_b = align256((size_t)3 * (n / 2 + 1) * n * nz * 2 * ts);
  const size_t tw_b = align256((size_t)2 * n * ts), tab_b = align256((size_t)n * ts);
  const size_t twz_b = align256((size_t)2 * nz * ts), tabz_b = align256((size_t)nz * ts);
  const size_t need = spec_b + tw_b + 2 * tab_b + twz_b + 2 * tabz_b;
  if (need > kNoAllocBytes) {
    set_context_free_error("ib_fluid_noalloc: " + std::to_string(n) + " x " + std::to_string(n) + " x " +
                           std::to_string(nz) + " in this precision needs " + std::to_string(need) +
                           " bytes of scratch; the limit is " + std::to_string(kNoAllocBytes));
    return IB_ENOTSUP;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess && (dev < 0 || dev >= kMaxDevices)) e = hipErrorInvalidDevice;
  void *base = nullptr;
  if (e == hipSuccess) e = scratch_for(dev, &base);
  if (e != hipSuccess) {
    set_context_free_error(std::string("ib_fluid_noalloc: scratch address: ") + hipGetErrorString(e));
    return IB_EDEVICE;
  }
  // a context on the stack: no allocation, its workspace pointers into the scratch
  ib_ctx c;
  c.p = *p;
  c.p.nz = nz;
  c.n = n;
  c.nz = nz;
  c.G = (int64_t)n * n * nz;
  c.h = p->L / n;
  c.fp32 = sizeof(T) == 4;
  c.stream = (hipStream_t)p->stream;
  unsigned char *b = (unsigned char *)base;
  c.ws.spec = b;
  c.ws.tw = b + spec_b;
  c.ws.lam = b + spec_b + tw_b;
  c.ws.sgrad = b + spec_b + tw_b + tab_b;
  unsigned char *bz = b + spec_b + tw_b + 2 * tab_b;
  c.ws.twz = bz;
  c.ws.lamz = bz + twz_b;
  c.ws.sgradz = bz + twz_b + tabz_b;
  hipLaunchKernelGGL(k_fluid_tables<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, n, c.h,
                     (T *)c.ws.tw, (T *)c.ws.lam, (T *)c.ws.sgrad);
  e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_fluid_tables<T>, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, c.stream, nz, c.h,
                       (T *)c.ws.twz, (T *)c.ws.lamz, (T *)c.ws.sgradz);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = launch_fluid_reg<T>(&c, u, F, F ? 2 : 0, p->convect, p->dt / p->rho, u);
  if (e != hipSuccess) {
    set_context_free_error(std::string("ib_fluid_noalloc: launch failed: ") + hipGetErrorString(e));
    return IB_EDEVICE;
  }
  return IB_OK;
}

}  // namespace

extern "C" int ib_fluid_noalloc(const ib_params *p, void *u, const void *F_grid) {
  if (!p || !u) {
    set_context_free_error("ib_fluid_noalloc: params and u are required");
    return IB_EINVAL;
  }
  const int n = p->n, nz = p->nz == 0 ? n : p->nz;
  if (!fluid_reg_supported(n, nz)) {
    set_context_free_error("ib_fluid_noalloc: n must be 32, 64, 128 or 256 and nz 0, n, n/2 or 3n/4");
    return IB_ENOTSUP;
  }
  if (!(p->L > 0.0) || !isfinite(p->L) || !(p->rho > 0.0) || !isfinite(p->rho) || !(p->mu >= 0.0) ||
      !isfinite(p->mu) || !(p->dt > 0.0) || !isfinite(p->dt) || (p->convect != 0 && p->convect != 1) ||
      (p->fluid_precision != IB_FLUID_FP64 && p->fluid_precision != IB_FLUID_FP32)) {
    set_context_free_error("ib_fluid_noalloc: need L > 0, rho > 0, mu >= 0, dt > 0 (finite), convect 0 or 1, "
                           "a valid fluid_precision");
    return IB_EINVAL;
  }
  set_context_free_error("");
  return p->fluid_precision == IB_FLUID_FP32
             ? fluid_noalloc<float>(p, nz, (float *)u, (const float *)F_grid)
             : fluid_noalloc<double>(p, nz, (double *)u, (const double *)F_grid);
}
