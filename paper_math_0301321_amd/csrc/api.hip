// C-ABI of the IB library: context creation, validation, workspace, tables
// and the entry points declared in include/ib.h.  Host code; every step of the
// method runs in the kernels of bin.hip, force.hip, spread.hip, fluid.hip and
// interp.hip, enqueued on the context's stream.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <string>
#include <vector>

#include "dev_common.h"
#include "ib_internal.h"

namespace ib {
int sort_hist_words(int64_t M, int digit_bits);
}

using namespace ib;

static thread_local std::string g_create_error;   // last error of a call without a context

void ib::set_context_free_error(const std::string &msg) { g_create_error = msg; }
static const double kPi = 3.14159265358979323846;

#define IB_TRY(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      c->err = std::string(#expr) + ": " + hipGetErrorString(e_);                            \
      return IB_EDEVICE;                                                                     \
    }                                                                                        \
  } while (0)

static int fail(ib_ctx *c, int code, const std::string &msg) {
  c->err = msg;
  return code;
}

// ------------------------------------------------------------ helpers ----
namespace {

__global__ void k_nonfinite_d(const double *__restrict__ a, int64_t n, int32_t *flag) {
  const int64_t i = gtid();
  if (i < n && !isfinite(a[i])) flag[0] = 1;
}
__global__ void k_nonfinite_f(const float *__restrict__ a, int64_t n, int32_t *flag) {
  const int64_t i = gtid();
  if (i < n && !isfinite(a[i])) flag[0] = 1;
}

template <typename A>
hipError_t dalloc(ib_ctx *c, A **p, int64_t count) {
  const size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(A);
  c->ws_bytes += (int64_t)bytes;
  return hipMalloc((void **)p, bytes);
}

hipError_t dalloc_bytes(ib_ctx *c, void **p, int64_t bytes) {
  c->ws_bytes += std::max<int64_t>(bytes, 1);
  return hipMalloc(p, (size_t)std::max<int64_t>(bytes, 1));
}

double drive_amp(const ib_ctx *c, double t) {
  if (c->n_drive == 0 || c->drive_A == 0.0) return 0.0;
  return c->drive_A * sin(2.0 * kPi * c->drive_freq * t);
}

// Twiddles, eigenvalues (4/h^2) sin^2(pi m / len) and gradient symbols
// sin(2 pi m / len) / h (exactly 0 at m = 0, len/2) for one transform length.
template <typename T>
hipError_t upload_tables_len(int len, double h, void *tw_d, void *lam_d, void *sg_d) {
  std::vector<T> tw(2 * len), lam(len), sg(len);
  for (int k = 0; k < len; k++) {
    const double a = 2.0 * kPi * (double)k / (double)len;
    tw[2 * k] = (T)cos(a);
    tw[2 * k + 1] = (T)(-sin(a));
  }
  for (int m = 0; m < len; m++) {
    const double sh = sin(kPi * (double)m / (double)len);
    lam[m] = (T)((4.0 / (h * h)) * sh * sh);
    sg[m] = (m == 0 || 2 * m == len) ? (T)0 : (T)(sin(2.0 * kPi * (double)m / (double)len) / h);
  }
  hipError_t e = hipMemcpy(tw_d, tw.data(), sizeof(T) * 2 * len, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(lam_d, lam.data(), sizeof(T) * len, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(sg_d, sg.data(), sizeof(T) * len, hipMemcpyHostToDevice);
  return e;
}

template <typename T>
hipError_t upload_tables(ib_ctx *c) {
  hipError_t e = upload_tables_len<T>(c->n, c->h, c->ws.tw, c->ws.lam, c->ws.sgrad);
  if (e == hipSuccess) e = upload_tables_len<T>(c->nz, c->h, c->ws.twz, c->ws.lamz, c->ws.sgradz);
  return e;
}

bool is_fin(double v) { return isfinite(v) != 0; }

void free_ws(ib_ctx *c) {
  Workspace &w = c->ws;
  void *ptrs[] = {w.keys[0], w.keys[1], w.vals[0], w.vals[1], w.keys_id, w.bin_state, w.bin_mov, w.hist, w.tile_start, w.recs, w.Flag, w.fb,
                  w.Fgrid, w.tile_nit, w.tile_item0, w.tile_touch, w.item_tile, w.chunk_item0, w.nitems, w.split_list, w.touch_list, w.scan_tmp, w.partials,
                  w.r, w.spec, w.nonfinite, w.tw, w.lam, w.sgrad, w.twz, w.lamz, w.sgradz, w.drive_idx, w.drive_dir,
                  w.sp_rowptr, w.sp_col,
                  w.sp_rest, w.inv, w.drive_slot, w.lat_pre, w.touch_bits};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  c->ws = Workspace{};
}

int checked(ib_ctx *c, const void *grid, bool grid_f32, const double *markers) {
  if (!c->check) return IB_OK;
  IB_TRY(hipStreamSynchronize(c->stream));
  IB_TRY(hipGetLastError());
  IB_TRY(hipMemsetAsync(c->ws.nonfinite, 0, sizeof(int32_t), c->stream));
  if (markers && c->M > 0)
    hipLaunchKernelGGL(k_nonfinite_d, dim3((unsigned)((3 * c->M + 255) / 256)), dim3(256), 0, c->stream, markers,
                       3 * c->M, c->ws.nonfinite);
  if (grid) {
    if (grid_f32)
      hipLaunchKernelGGL(k_nonfinite_f, dim3((unsigned)((3 * c->G + 255) / 256)), dim3(256), 0, c->stream,
                         (const float *)grid, 3 * c->G, c->ws.nonfinite);
    else
      hipLaunchKernelGGL(k_nonfinite_d, dim3((unsigned)((3 * c->G + 255) / 256)), dim3(256), 0, c->stream,
                         (const double *)grid, 3 * c->G, c->ws.nonfinite);
  }
  int32_t bad = 0;
  IB_TRY(hipMemcpyAsync(&bad, c->ws.nonfinite, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  IB_TRY(hipStreamSynchronize(c->stream));
  if (bad) return fail(c, IB_ENONFINITE, "non-finite value in an output");
  return IB_OK;
}

}  // namespace

static void graph_release(ib_ctx *c);

// ------------------------------------------------------------- create ----
extern "C" int ib_create(const ib_params *p, const ib_elastic *e, ib_ctx **out) {
  if (!out) {
    g_create_error = "ib_create: out is NULL";
    return IB_EINVAL;
  }
  *out = nullptr;
  if (!p || !e) {
    g_create_error = "ib_create: params or elastic is NULL";
    return IB_EINVAL;
  }
  const int n = p->n;
  if (n < 8 || n > 512 || (n & (n - 1)) != 0) {
    g_create_error = "ib_create: n must be a power of two in [8, 512]";
    return IB_ENOTSUP;
  }
  const int nz = p->nz == 0 ? n : p->nz;
  if (nz != n && !fluid_reg_supported(n, nz)) {
    g_create_error = "ib_create: nz must be 0 or n, or n/2 or 3n/4 with n in [32, 256]";
    return IB_ENOTSUP;
  }
  if (!(p->L > 0.0) || !is_fin(p->L) || !(p->rho > 0.0) || !is_fin(p->rho) || !(p->mu >= 0.0) || !is_fin(p->mu) ||
      !(p->dt > 0.0) || !is_fin(p->dt)) {
    g_create_error = "ib_create: need L > 0, rho > 0, mu >= 0, dt > 0 (finite)";
    return IB_EINVAL;
  }
  if (p->fluid_precision != IB_FLUID_FP64 && p->fluid_precision != IB_FLUID_FP32) {
    g_create_error = "ib_create: fluid_precision must be IB_FLUID_FP64 or IB_FLUID_FP32";
    return IB_EINVAL;
  }
  if (p->convect != 0 && p->convect != 1) {
    g_create_error = "ib_create: convect must be 0 or 1";
    return IB_EINVAL;
  }
  if (p->displacement != 0 && p->displacement != 1) {
    g_create_error = "ib_create: displacement must be 0 or 1";
    return IB_EINVAL;
  }
  const int64_t M = p->n_markers;
  if (M < 0 || M >= (int64_t)INT32_MAX) {
    g_create_error = "ib_create: n_markers out of range";
    return IB_EINVAL;
  }
  if (M > 0 && (!e->w || !e->k || !e->X_ref)) {
    g_create_error = "ib_create: w, k and X_ref are required when n_markers > 0";
    return IB_EINVAL;
  }
  if (e->n_lattices < 0 || e->n_lattices > kMaxLattices || (e->n_lattices > 0 && !e->lattices)) {
    g_create_error = "ib_create: n_lattices must be in [0, 16] with a lattice array";
    return IB_EINVAL;
  }
  std::vector<std::pair<int64_t, int64_t>> spans;
  for (int l = 0; l < e->n_lattices; l++) {
    const ib_lattice &L = e->lattices[l];
    if (L.first < 0 || L.n1 < 1 || L.n2 < 1 || L.first + (int64_t)L.n1 * L.n2 > M || (L.periodic2 && L.n2 < 3) ||
        !is_fin(L.Ks) || !is_fin(L.Kb)) {
      g_create_error = "ib_create: lattice " + std::to_string(l) +
                       " out of range (need first + n1*n2 <= M, n2 >= 3 when periodic, finite moduli)";
      return IB_EINVAL;
    }
    spans.push_back({L.first, L.first + (int64_t)L.n1 * L.n2});
  }
  std::sort(spans.begin(), spans.end());
  for (size_t i = 1; i < spans.size(); i++)
    if (spans[i].first < spans[i - 1].second) {
      g_create_error = "ib_create: lattices overlap";
      return IB_EINVAL;
    }
  if (e->n_springs < 0 || (e->n_springs > 0 && (!e->spring_ab || !e->spring_rest)) || !is_fin(e->K_spring)) {
    g_create_error = "ib_create: bad springs";
    return IB_EINVAL;
  }
  const int64_t S = e->n_springs;
  for (int64_t s = 0; s < S; s++) {
    const int64_t a = e->spring_ab[s], b = e->spring_ab[S + s];
    if (a < 0 || a >= M || b < 0 || b >= M || a == b || !(e->spring_rest[s] >= 0.0) || !is_fin(e->spring_rest[s])) {
      g_create_error = "ib_create: spring " + std::to_string(s) + " has a bad index or rest length";
      return IB_EINVAL;
    }
  }
  if (e->n_drive < 0 || (e->n_drive > 0 && (!e->drive_idx || !e->drive_dir)) || !is_fin(e->drive_A) ||
      !is_fin(e->drive_freq)) {
    g_create_error = "ib_create: bad drive";
    return IB_EINVAL;
  }
  const int64_t D = e->n_drive;
  {
    std::vector<int32_t> di(e->drive_idx, e->drive_idx + D);
    for (int32_t v : di)
      if (v < 0 || v >= M) {
        g_create_error = "ib_create: drive index out of range";
        return IB_EINVAL;
      }
    std::sort(di.begin(), di.end());
    if (std::adjacent_find(di.begin(), di.end()) != di.end()) {
      g_create_error = "ib_create: drive indices must be distinct";
      return IB_EINVAL;
    }
  }

  ib_ctx *c = new ib_ctx();
  c->p = *p;
  c->p.nz = nz;
  c->n = n;
  while ((1 << c->log2n) < n) c->log2n++;
  c->nz = nz;
  c->G = (int64_t)n * n * nz;
  c->M = M;
  c->h = p->L / n;
  c->fp32 = p->fluid_precision == IB_FLUID_FP32;
  c->stream = (hipStream_t)p->stream;
  const char *chk = getenv("IB_CHECK");
  c->check = chk && chk[0] == '1';
  c->log2nt = c->log2n - 3;
  c->ntz = nz / 8;
  c->ntiles = ((int64_t)1 << (2 * c->log2nt)) * c->ntz;
  c->n_springs = S;
  c->n_drive = D;
  c->drive_A = e->drive_A;
  c->drive_freq = e->drive_freq;
  int key_bits = 9;                       // the cell within its tile, then the tile index
  while (((int64_t)1 << (key_bits - 9)) < c->ntiles) key_bits++;
  c->sort_passes = (key_bits + 7) / 8;
  c->digit_bits = (key_bits + c->sort_passes - 1) / c->sort_passes;
  c->sorted_buf = (c->sort_passes - 1) & 1;   // the last radix pass writes keys/vals[(passes - 1) & 1]

  Material &mt = c->mat;
  mt.w = e->w;
  mt.k = e->k;
  mt.X_ref = e->X_ref;
  mt.kappa = e->kappa;
  mt.M = M;
  mt.K_spring = e->K_spring;
  mt.disp = p->displacement;
  mt.lat.n = e->n_lattices;
  for (int l = 0; l < e->n_lattices; l++) {
    const ib_lattice &L = e->lattices[l];
    mt.lat.l[l] = LatticeDev{L.first, L.n1, L.n2, L.periodic2 ? 1 : 0, L.Ks, L.Kb};
  }

  const size_t ts = c->fp32 ? 4 : 8;
  const int64_t nh = n / 2 + 1;
  Workspace &w = c->ws;
  hipError_t err = hipSuccess;
  auto chk_alloc = [&](hipError_t x) {
    if (err == hipSuccess) err = x;
  };
  chk_alloc(dalloc(c, &w.keys[0], M));
  chk_alloc(dalloc(c, &w.keys[1], M));
  chk_alloc(dalloc(c, &w.vals[0], M));
  chk_alloc(dalloc(c, &w.vals[1], M));
  chk_alloc(dalloc(c, &w.keys_id, M));
  chk_alloc(dalloc(c, &w.bin_state, BS_WORDS));
  chk_alloc(dalloc(c, &w.bin_mov, MV_ARRAYS * kMoverCap));
  chk_alloc(dalloc(c, &w.hist, sort_hist_words(M, c->digit_bits)));
  chk_alloc(dalloc(c, &w.tile_start, c->ntiles + 1));
  chk_alloc(dalloc(c, &w.inv, M));
  chk_alloc(dalloc_bytes(c, &w.recs, M * (int64_t)(c->fp32 ? sizeof(Rec<float>) : sizeof(Rec<double>))));
  chk_alloc(dalloc(c, &w.Flag, 3 * M));
  chk_alloc(dalloc(c, &w.fb, 3 * M));
  chk_alloc(dalloc_bytes(c, &w.Fgrid, 3 * c->G * (int64_t)ts));
  {
    // work list: every tile with markers has one item more than the chunk
    // boundaries inside it
    const int64_t ntiles = c->ntiles;
    // spreading waves resident at once: 24 KB of LDS per wave in FP32, 48 KB in FP64
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
      hipDeviceProp_t prop;
      if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
        c->ncu = prop.multiProcessorCount;
    }
    c->item_grid = c->ncu * (c->fp32 ? 8 : 4);   // spreading waves: as many as fit in LDS at once
    c->chunk = (int)std::max<int64_t>(256, (M + c->item_grid - 1) / std::max(1, c->item_grid));
    c->nchunks = (int)((M + c->chunk - 1) / c->chunk);
    c->item_cap = std::min<int64_t>(ntiles, M) + c->nchunks + 1;
    if (c->item_cap * (int64_t)kPartStride >= (int64_t)INT32_MAX) {
      g_create_error = "ib_create: too many markers for the spreading work list at this grid size";
      free_ws(c);
      delete c;
      return IB_ENOTSUP;
    }
    chk_alloc(dalloc(c, &w.tile_nit, ntiles));
    chk_alloc(dalloc(c, &w.tile_item0, ntiles));
    chk_alloc(dalloc(c, &w.tile_touch, ntiles));
    chk_alloc(dalloc(c, &w.touch_bits, (ntiles + 31) / 32));
    chk_alloc(dalloc(c, &w.item_tile, c->item_cap));
    chk_alloc(dalloc(c, &w.chunk_item0, c->nchunks + 1));
    chk_alloc(dalloc(c, &w.nitems, 3));
    chk_alloc(dalloc(c, &w.split_list, ntiles));
    chk_alloc(dalloc(c, &w.touch_list, ntiles));
    chk_alloc(dalloc(c, &w.scan_tmp, 3 * ((ntiles + 1023) / 1024)));
    chk_alloc(dalloc_bytes(c, &w.partials, c->item_cap * kPartStride * (int64_t)ts));
  }
  if (!fluid_reg_supported(n, nz)) chk_alloc(dalloc_bytes(c, &w.r, 3 * c->G * (int64_t)ts));   // the fused path keeps r in LDS
  chk_alloc(dalloc_bytes(c, &w.spec, 3 * nh * (int64_t)n * nz * 2 * (int64_t)ts));
  chk_alloc(dalloc(c, &w.nonfinite, 1));
  chk_alloc(dalloc_bytes(c, &w.tw, 2 * (int64_t)n * (int64_t)ts));
  chk_alloc(dalloc_bytes(c, &w.lam, (int64_t)n * (int64_t)ts));
  chk_alloc(dalloc_bytes(c, &w.sgrad, (int64_t)n * (int64_t)ts));
  chk_alloc(dalloc_bytes(c, &w.twz, 2 * (int64_t)nz * (int64_t)ts));
  chk_alloc(dalloc_bytes(c, &w.lamz, (int64_t)nz * (int64_t)ts));
  chk_alloc(dalloc_bytes(c, &w.sgradz, (int64_t)nz * (int64_t)ts));
  chk_alloc(dalloc(c, &w.drive_idx, D));
  chk_alloc(dalloc(c, &w.drive_dir, 3 * D));
  if (err != hipSuccess) {
    g_create_error = std::string("ib_create: device allocation failed: ") + hipGetErrorString(err);
    free_ws(c);
    delete c;
    return err == hipErrorOutOfMemory ? IB_ENOMEM : IB_EDEVICE;
  }
  {
    // no partition yet: the first binning sorts in full
    uint32_t st0[BS_WORDS] = {};
    st0[BS_FULL] = 1u;
    chk_alloc(hipMemcpy(w.bin_state, st0, sizeof(st0), hipMemcpyHostToDevice));
  }
  if (D > 0) {
    chk_alloc(hipMemcpy(w.drive_idx, e->drive_idx, sizeof(int32_t) * D, hipMemcpyHostToDevice));
    chk_alloc(hipMemcpy(w.drive_dir, e->drive_dir, sizeof(double) * 3 * D, hipMemcpyHostToDevice));
    std::vector<int32_t> slot(M, -1);
    for (int64_t j = 0; j < D; j++) slot[e->drive_idx[j]] = (int32_t)j;
    chk_alloc(dalloc(c, &w.drive_slot, M));
    if (err == hipSuccess)
      chk_alloc(hipMemcpy(w.drive_slot, slot.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice));
  }
  if (S > 0) {
    // spring adjacency in CSR, neighbours of each marker in spring order
    std::vector<int32_t> rowptr(M + 1, 0), col(2 * S);
    std::vector<double> rest(2 * S);
    for (int64_t s = 0; s < S; s++) {
      rowptr[e->spring_ab[s] + 1]++;
      rowptr[e->spring_ab[S + s] + 1]++;
    }
    for (int64_t q = 0; q < M; q++) rowptr[q + 1] += rowptr[q];
    std::vector<int32_t> fill(rowptr.begin(), rowptr.end() - 1);
    for (int64_t s = 0; s < S; s++) {
      const int32_t a = e->spring_ab[s], b = e->spring_ab[S + s];
      col[fill[a]] = b;
      rest[fill[a]++] = e->spring_rest[s];
      col[fill[b]] = a;
      rest[fill[b]++] = e->spring_rest[s];
    }
    chk_alloc(dalloc(c, &w.sp_rowptr, M + 1));
    chk_alloc(dalloc(c, &w.sp_col, 2 * S));
    chk_alloc(dalloc(c, &w.sp_rest, 2 * S));
    if (err == hipSuccess) {
      chk_alloc(hipMemcpy(w.sp_rowptr, rowptr.data(), sizeof(int32_t) * (M + 1), hipMemcpyHostToDevice));
      chk_alloc(hipMemcpy(w.sp_col, col.data(), sizeof(int32_t) * 2 * S, hipMemcpyHostToDevice));
      chk_alloc(hipMemcpy(w.sp_rest, rest.data(), sizeof(double) * 2 * S, hipMemcpyHostToDevice));
    }
    mt.sp_rowptr = w.sp_rowptr;
    mt.sp_col = w.sp_col;
    mt.sp_rest = w.sp_rest;
  }
  {
    bool moduli = false;
    for (int l = 0; l < e->n_lattices; l++) moduli = moduli || e->lattices[l].Ks != 0.0 || e->lattices[l].Kb != 0.0;
    if (moduli && M > 0) {
      chk_alloc(dalloc(c, &w.lat_pre, (int64_t)kLatPre * M));
      mt.lat_pre = w.lat_pre;
      if (err == hipSuccess) err = launch_lattice_pre(c);
      if (err == hipSuccess) err = hipStreamSynchronize(c->stream);
    }
  }
  if (err == hipSuccess) err = c->fp32 ? upload_tables<float>(c) : upload_tables<double>(c);
  if (err != hipSuccess) {
    g_create_error = std::string("ib_create: upload failed: ") + hipGetErrorString(err);
    free_ws(c);
    delete c;
    return err == hipErrorOutOfMemory ? IB_ENOMEM : IB_EDEVICE;
  }
  *out = c;
  return IB_OK;
}

extern "C" void ib_destroy(ib_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  graph_release(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (auto &r : c->trec) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  free_ws(c);
  delete c;
}

// ------------------------------------------------------ instrumentation ----
static const char *kPhaseNames[PH_COUNT] = {"bin", "force", "prep", "spread", "split", "gather", "rhs", "fft_x", "fft_y",
                                            "fft_z_solve", "fft_y_inv", "fft_x_inv", "interp", "adj_interp",
                                            "adj_spread", "hessvec", "rhs_fft_x", "adj_advect", "fft_yx_inv"};

static void timers_fold(ib_ctx *c) {
  if (c->tused == 0) return;
  (void)hipStreamSynchronize(c->stream);
  for (size_t i = 0; i < c->tused; i++) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, c->trec[i].a, c->trec[i].b) == hipSuccess) {
      c->tms[c->trec[i].phase] += ms;
      c->tcalls[c->trec[i].phase] += 1;
    }
  }
  c->tused = 0;
}

void ib::timer_begin(ib_ctx *c, int phase) {
  if (!c->timing || !((c->tmask >> phase) & 1u)) {
    c->tskip = true;
    return;
  }
  c->tskip = false;
  if (c->tused == c->trec.size()) {
    TimerRec r{phase, nullptr, nullptr};
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) {
      c->timing = false;
      return;
    }
    c->trec.push_back(r);
  }
  c->trec[c->tused].phase = phase;
  (void)hipEventRecord(c->trec[c->tused].a, c->stream);
}

void ib::timer_end(ib_ctx *c) {
  if (!c->timing || c->tskip) return;
  (void)hipEventRecord(c->trec[c->tused].b, c->stream);
  if (++c->tused >= 8192) timers_fold(c);
}

extern "C" int ib_timers_enable(ib_ctx *c, int on) {
  if (!c) return IB_EINVAL;
  timers_fold(c);
  for (int i = 0; i < PH_COUNT; i++) {
    c->tms[i] = 0.0;
    c->tcalls[i] = 0;
  }
  c->timing = on != 0;
  return IB_OK;
}

extern "C" int ib_timers_select(ib_ctx *c, uint32_t mask) {
  if (!c) return IB_EINVAL;
  c->tmask = mask;
  return IB_OK;
}

extern "C" int ib_timers_read(ib_ctx *c, double *ms, int64_t *calls, int max) {
  if (!c || max < 0 || (max > 0 && (!ms || !calls))) return IB_EINVAL;
  timers_fold(c);
  for (int i = 0; i < max && i < IB_N_TIMERS; i++) {
    ms[i] = i < PH_COUNT ? c->tms[i] : 0.0;
    calls[i] = i < PH_COUNT ? c->tcalls[i] : 0;
  }
  return IB_OK;
}

extern "C" const char *ib_timer_name(int i) { return (i >= 0 && i < PH_COUNT) ? kPhaseNames[i] : nullptr; }

extern "C" int ib_set_material(ib_ctx *c, const double *w, const double *k, const double *X_ref,
                               const double *kappa) {
  if (!c) return IB_EINVAL;
  if (w) c->mat.w = w;
  if (k) c->mat.k = k;
  if (X_ref) c->mat.X_ref = X_ref;
  if (kappa) c->mat.kappa = kappa;
  graph_release(c);   // a captured step holds the material pointers
  if (w || X_ref) IB_TRY(launch_lattice_pre(c));   // reference-shape constants follow X_ref and w
  return IB_OK;
}

extern "C" int ib_set_stream(ib_ctx *c, void *stream) {
  if (!c) return IB_EINVAL;
  c->stream = (hipStream_t)stream;
  return IB_OK;
}

extern "C" const char *ib_last_error(const ib_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }

extern "C" int64_t ib_workspace_bytes(const ib_ctx *c) { return c ? c->ws_bytes : 0; }

// -------------------------------------------------------- entry points ----
// The four sub-steps of Sec. 3.2 as kernel launches on c->stream.
template <typename T>
static hipError_t step_launches(ib_ctx *c, double *X, T *u, double amp, double *F_lag_out) {
  hipError_t e = launch_bin(c, X);
  if (e == hipSuccess) e = launch_force_rec<T>(c, X, amp, F_lag_out);
  if (e == hipSuccess) e = launch_spread<T>(c, (T *)c->ws.Fgrid, false, 1.0 / (c->h * c->h * c->h));
  if (e == hipSuccess) e = launch_fluid<T>(c, u, (const T *)c->ws.Fgrid, 1, c->p.convect, c->p.dt / c->p.rho, u);
  if (e == hipSuccess) e = launch_interp<T>(c, u, X, X, nullptr, c->p.dt);
  return e;
}

static void graph_release(ib_ctx *c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
  c->graph_force = nullptr;
  c->graph_force_args.clear();
  c->graph_key[0] = c->graph_key[1] = c->graph_key[2] = nullptr;
}

// Capture the step's launches for these pointers into c->graph / c->graph_exec
// and find the force kernel's node, whose drive amplitude changes per step.
template <typename T>
static int graph_capture(ib_ctx *c, double *X, T *u, double amp, double *F_lag_out) {
  graph_release(c);
  if (!c->cap_stream) IB_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  // the capture stream starts after the work already queued on the context's stream
  hipStream_t user = c->stream;
  IB_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  c->stream = c->cap_stream;
  const hipError_t el = step_launches<T>(c, X, u, amp, F_lag_out);
  c->stream = user;
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(c->cap_stream, &g);
  if (el != hipSuccess || ee != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(c, IB_EDEVICE, std::string("ib_step: graph capture failed: ") +
                                   hipGetErrorString(el != hipSuccess ? el : ee));
  }
  c->graph = g;
  size_t nn = 0;
  IB_TRY(hipGraphGetNodes(g, nullptr, &nn));
  std::vector<hipGraphNode_t> nodes(nn);
  if (nn) IB_TRY(hipGraphGetNodes(g, nodes.data(), &nn));
  const void *fk = force_rec_kernel<T>(c->mat.disp != 0);
  for (hipGraphNode_t nd : nodes) {
    hipGraphNodeType ty;
    IB_TRY(hipGraphNodeGetType(nd, &ty));
    if (ty != hipGraphNodeTypeKernel) continue;
    hipKernelNodeParams kp{};
    IB_TRY(hipGraphKernelNodeGetParams(nd, &kp));
    if (kp.func == fk) {
      c->graph_force = nd;
      c->graph_force_params = kp;
    }
  }
  if (c->M > 0 && !c->graph_force) {
    graph_release(c);
    return fail(c, IB_EDEVICE, "ib_step: the captured graph has no force kernel node");
  }
  if (c->graph_force) {
    // argument pointers: the graph's own values, except the amplitude
    if (!c->graph_force_params.kernelParams) {
      graph_release(c);
      return fail(c, IB_EDEVICE, "ib_step: the captured force node has no argument list");
    }
    c->graph_force_args.assign(c->graph_force_params.kernelParams,
                               c->graph_force_params.kernelParams + kForceRecArgs);
    c->graph_force_args[kForceRecAmpArg] = &c->graph_amp;
    c->graph_force_params.kernelParams = c->graph_force_args.data();
    c->graph_amp = amp;
  }
  IB_TRY(hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0));
  c->graph_key[0] = X;
  c->graph_key[1] = u;
  c->graph_key[2] = F_lag_out;
  c->graph_captures++;
  return IB_OK;
}

template <typename T>
static int step_graph(ib_ctx *c, double *X, T *u, double t, double *F_lag_out) {
  const double amp = drive_amp(c, t);
  if (!c->graph_exec || c->graph_key[0] != X || c->graph_key[1] != u || c->graph_key[2] != F_lag_out) {
    const int rc = graph_capture<T>(c, X, u, amp, F_lag_out);
    if (rc != IB_OK) return rc;
  } else if (c->graph_force && amp != c->graph_amp) {
    c->graph_amp = amp;
    IB_TRY(hipGraphExecKernelNodeSetParams(c->graph_exec, c->graph_force, &c->graph_force_params));
  }
  IB_TRY(hipGraphLaunch(c->graph_exec, c->stream));
  c->graph_launches++;
  return IB_OK;
}

template <typename T>
static int step_impl(ib_ctx *c, double *X, T *u, double t, double *F_lag_out) {
  // the graph is bypassed while the timers record events or IB_CHECK synchronises
  if (c->graph_on && !c->timing && !c->check) return step_graph<T>(c, X, u, t, F_lag_out);
  IB_TRY(step_launches<T>(c, X, u, drive_amp(c, t), F_lag_out));
  return checked(c, u, c->fp32, X);
}

extern "C" int ib_step(ib_ctx *c, double *X, void *u, double t, double *F_lag_out) {
  if (!c) return IB_EINVAL;
  if ((!X && c->M > 0) || !u) return fail(c, IB_EINVAL, "ib_step: X and u are required");
  c->err.clear();
  return c->fp32 ? step_impl<float>(c, X, (float *)u, t, F_lag_out)
                 : step_impl<double>(c, X, (double *)u, t, F_lag_out);
}

extern "C" int ib_bin_reuse(ib_ctx *c, int on) {
  if (!c) return IB_EINVAL;
  if (on != 0 && on != 1) return fail(c, IB_EINVAL, "ib_bin_reuse: on must be 0 or 1");
  if (c->bin_reuse != (on != 0)) graph_release(c);   // a captured step holds the choice
  c->bin_reuse = on != 0;
  return IB_OK;
}

extern "C" int ib_graph_enable(ib_ctx *c, int on) {
  if (!c) return IB_EINVAL;
  c->err.clear();
  if (!on) graph_release(c);
  c->graph_on = on != 0;
  return IB_OK;
}

extern "C" int ib_graph_stats(const ib_ctx *c, int64_t *captures, int64_t *launches) {
  if (!c || !captures || !launches) return IB_EINVAL;
  *captures = c->graph_captures;
  *launches = c->graph_launches;
  return IB_OK;
}

extern "C" int ib_force(ib_ctx *c, const double *X, double t, double *F_lag) {
  if (!c) return IB_EINVAL;
  if (c->M > 0 && (!X || !F_lag)) return fail(c, IB_EINVAL, "ib_force: X and F_lag are required");
  c->err.clear();
  IB_TRY(launch_force(c, X, drive_amp(c, t), F_lag));
  return checked(c, nullptr, false, F_lag);
}

template <typename T>
static int spread_impl(ib_ctx *c, const double *X, const double *F, T *Fg) {
  IB_TRY(launch_bin(c, X));
  IB_TRY(launch_prep<T>(c, X, F));
  IB_TRY(launch_spread<T>(c, Fg, true, 1.0 / (c->h * c->h * c->h)));
  return checked(c, Fg, c->fp32, nullptr);
}

extern "C" int ib_spread(ib_ctx *c, const double *X, const double *F_lag, void *F_grid) {
  if (!c) return IB_EINVAL;
  if (!F_grid || (c->M > 0 && (!X || !F_lag))) return fail(c, IB_EINVAL, "ib_spread: X, F_lag, F_grid required");
  c->err.clear();
  return c->fp32 ? spread_impl<float>(c, X, F_lag, (float *)F_grid)
                 : spread_impl<double>(c, X, F_lag, (double *)F_grid);
}

template <typename T>
static int interp_impl(ib_ctx *c, const double *X, const T *u, double *U) {
  IB_TRY(launch_bin(c, X));
  IB_TRY(launch_prep<T>(c, X, nullptr));
  IB_TRY(launch_interp<T>(c, u, X, nullptr, U, 0.0));
  return checked(c, nullptr, false, U);
}

extern "C" int ib_interp(ib_ctx *c, const double *X, const void *u, double *U) {
  if (!c) return IB_EINVAL;
  if (!u || (c->M > 0 && (!X || !U))) return fail(c, IB_EINVAL, "ib_interp: X, u, U required");
  c->err.clear();
  return c->fp32 ? interp_impl<float>(c, X, (const float *)u, U) : interp_impl<double>(c, X, (const double *)u, U);
}

template <typename T>
static int fluid_impl(ib_ctx *c, T *u, const T *Fg) {
  IB_TRY(launch_fluid<T>(c, u, Fg, 2, c->p.convect, c->p.dt / c->p.rho, u));
  return checked(c, u, c->fp32, nullptr);
}

extern "C" int ib_fluid(ib_ctx *c, void *u, const void *F_grid) {
  if (!c) return IB_EINVAL;
  if (!u) return fail(c, IB_EINVAL, "ib_fluid: u required");
  c->err.clear();
  return c->fp32 ? fluid_impl<float>(c, (float *)u, (const float *)F_grid)
                 : fluid_impl<double>(c, (double *)u, (const double *)F_grid);
}

extern "C" int ib_bin(ib_ctx *c, const double *X, uint32_t *keys_sorted, int32_t *perm) {
  if (!c) return IB_EINVAL;
  if (c->M > 0 && (!X || !keys_sorted || !perm)) return fail(c, IB_EINVAL, "ib_bin: X, keys, perm required");
  c->err.clear();
  IB_TRY(launch_bin(c, X));
  if (c->M > 0) {
    IB_TRY(hipMemcpyAsync(keys_sorted, c->ws.keys[c->sorted_buf], sizeof(uint32_t) * c->M, hipMemcpyDeviceToDevice,
                          c->stream));
    IB_TRY(hipMemcpyAsync(perm, c->ws.vals[c->sorted_buf], sizeof(int32_t) * c->M, hipMemcpyDeviceToDevice,
                          c->stream));
  }
  return checked(c, nullptr, false, nullptr);
}

template <typename T>
static int adjoint_impl(ib_ctx *c, const double *X_n, const T *u_n, const T *u_np1, double t, double *Xbar,
                        T *ubar, double *kbar) {
  // forward quantities at X^n: binning, weights, force f^n
  IB_TRY(launch_bin(c, X_n));
  IB_TRY(launch_force_rec<T>(c, X_n, drive_amp(c, t), c->ws.Flag));
  // interpolation / move: phi' term into Xbar, stage Ubar = dt Xbar
  IB_TRY(launch_adj_interp<T>(c, u_np1, X_n, Xbar));
  // transpose of interpolation: ubar_tot = ubar + S(Ubar) h^3
  IB_TRY(launch_spread<T>(c, (T *)c->ws.Fgrid, false, 1.0));
  // the NS operator is symmetric: rbar = Lop ubar_tot.  With advection rbar
  // goes to the force grid (its first pass has read the force by the time its
  // last pass writes), and the advection's transpose forms ubar from it below;
  // without, rbar is ubar^n
  T *rbar = c->p.convect ? (T *)c->ws.Fgrid : ubar;
  IB_TRY(launch_fluid<T>(c, ubar, (const T *)c->ws.Fgrid, 1, 0, 1.0, rbar));
  // transpose of spreading (fbar) and its phi' term, then the force Jacobian
  IB_TRY(launch_adj_spread<T>(c, rbar, c->ws.Flag, X_n, Xbar, c->ws.fb));
  IB_TRY(launch_hessvec(c, X_n, c->ws.fb, Xbar, kbar));
  // with advection, r = u - dt A(u) + ...: ubar^n = rbar - dt (dA/du)^T rbar at u^n
  if (c->p.convect) IB_TRY(launch_adv_adjoint<T>(c, u_n, (const T *)rbar, ubar));
  return checked(c, ubar, c->fp32, Xbar);
}

extern "C" int ib_adjoint_step_u(ib_ctx *c, const double *X_n, const void *u_n, const void *u_np1, double t,
                                 double *Xbar, void *ubar, double *kbar) {
  if (!c) return IB_EINVAL;
  if (!u_np1 || !ubar || (c->M > 0 && (!X_n || !Xbar || !kbar)))
    return fail(c, IB_EINVAL, "ib_adjoint_step: X_n, u_np1, Xbar, ubar, kbar required");
  if (c->p.convect && !u_n) return fail(c, IB_EINVAL, "ib_adjoint_step_u: convect = 1 needs u_n");
  c->err.clear();
  return c->fp32 ? adjoint_impl<float>(c, X_n, (const float *)u_n, (const float *)u_np1, t, Xbar, (float *)ubar, kbar)
                 : adjoint_impl<double>(c, X_n, (const double *)u_n, (const double *)u_np1, t, Xbar, (double *)ubar,
                                        kbar);
}

extern "C" int ib_probe(ib_ctx *c, const double *X, const double *X0, const int32_t *idx, const double *dir,
                        int64_t count, double *disp, double *env) {
  if (!c) return IB_EINVAL;
  if (count < 0 || (count > 0 && (!X || !X0 || !idx || !dir)))
    return fail(c, IB_EINVAL, "ib_probe: count >= 0 and X, X0, idx, dir are required");
  c->err.clear();
  IB_TRY(launch_probe(c, X, X0, idx, dir, count, disp, env));
  if (c->check) IB_TRY(hipStreamSynchronize(c->stream));
  return IB_OK;
}

extern "C" int ib_adjoint_step(ib_ctx *c, const double *X_n, const void *u_np1, double t, double *Xbar,
                               void *ubar, double *kbar) {
  if (!c) return IB_EINVAL;
  if (c->p.convect != 0)
    return fail(c, IB_ENOTSUP, "ib_adjoint_step: convect = 1 needs u^n: use ib_adjoint_step_u");
  return ib_adjoint_step_u(c, X_n, nullptr, u_np1, t, Xbar, ubar, kbar);
}
